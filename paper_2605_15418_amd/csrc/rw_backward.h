// Backward (adjoint G1) kernels of the ray-wave hybrid PSF: the a.e.
// derivative of the forward with the drawn sample indices held fixed.
//
//   k_psf_cograd      dL/dI (Eq. 5 with closed-form alpha, or the caller's) ->
//                     cogradient of the kept modes 2 dI U / (Psi(kx) Psi(ky))
//   k_grid_cols_bwd / k_grid_rows_bwd   adjoint of the grid FFT and crop:
//                     B_l = sum_k exp(-2 pi i k.l / nf) G_k  (full nf x nf grid)
//   (the ray-wave interface adjoint k_doe_bwd2 lives in rw_doe.h)
//   k_dmaps           dL/dt -> dL/dphi, dL/dA
//   k_trace_bwd       reverse sweep over the per-surface checkpoints; local
//                     Jacobians of each Newton/Snell step by dual numbers
//   k_lens_map        per-surface sums -> normalised lens-parameter gradients
#pragma once
#include "rw_kernels.h"

#define RW_LENSG_SLOTS 128
// Cogradient components per incident ray at the DOE: position (3), direction (3),
// optical path, sensor z, then the frame: u (3), v (3) as explicit vectors and
// the torque (3) of an infinitesimal rotation of the whole frame (u, v, n).
#define RW_RAYGRAD 17
#define RW_LENSG_SENSOR (RW_MAX_SURF * 8)

namespace rw {

// ------------------------------------------------------- loss cogradient ---
template <class Tg>
__global__ __launch_bounds__(256) void k_psf_cograd(const float* dpsf, const float* psf,
                                                    const float* target, const double* alpha,
                                                    const C2<Tg>* U, const double* psi_hat,
                                                    int Q, int pair0, int npairs, C2<Tg>* G) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t Q2 = (size_t)Q * Q;
  if (i >= (size_t)npairs * Q2) return;
  const int pair = pair0 + (int)(i / Q2);
  const size_t o = (size_t)pair * Q2 + i % Q2;
  const int r = (int)((i % Q2) / Q), c = (int)(i % Q);
  double dI;
  if (dpsf) {
    dI = dpsf[o];
  } else {
    const double a = alpha[pair];
    dI = 2.0 * a * (a * psf[o] - target[o]);
  }
  const double sc = 2.0 * dI / (psi_hat[r] * psi_hat[c]);
  G[o] = {(Tg)(sc * U[o].re), (Tg)(sc * U[o].im)};
}

// Column pass of the adjoint: for each kept column c (k_x), the Q kept k_y
// modes are placed at k_y mod nf and transformed with exp(-i ...) over all
// nf rows l_y.  Output T2[pair][c][l_y].
template <class Tg, int NF>
__global__ __launch_bounds__(256) void k_grid_cols_bwd(const C2<Tg>* G, const C2<Tg>* tw, int Q,
                                                       int pair0, int npairs, C2<Tg>* t2) {
  constexpr int E = NF / 64;
  const int lane = threadIdx.x & 63;
  const size_t col = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= (size_t)npairs * Q) return;
  const int pair = pair0 + (int)(col / Q), c = (int)(col % Q);
  C2<Tg> x[E];
#pragma unroll
  for (int n2 = 0; n2 < E; ++n2) {
    const int n = lane + 64 * n2;
    int r = -1;
    if (n < Q / 2) r = n + Q / 2;
    else if (n >= NF - Q / 2) r = n - NF + Q / 2;
    x[n2] = r >= 0 ? G[((size_t)pair * Q + r) * Q + c] : C2<Tg>{Tg(0), Tg(0)};
  }
  group_fft<Tg, 64, E, -1>(x, lane, tw);
  const int base = E * bitrev(lane, 6);
  C2<Tg>* dst = t2 + ((size_t)pair * Q + c) * NF;
#pragma unroll
  for (int k2 = 0; k2 < E; ++k2) dst[base + k2] = x[k2];
}

// Row pass: for each grid row l_y, the Q kept k_x values are transformed over
// all nf columns l_x.  Output B[pair][l_y][l_x].
template <class Tg, int NF>
__global__ __launch_bounds__(256) void k_grid_rows_bwd(const C2<Tg>* t2, const C2<Tg>* tw, int Q,
                                                       int pair0, int npairs, C2<Tg>* B) {
  constexpr int E = NF / 64;
  const int lane = threadIdx.x & 63;
  const size_t row = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= (size_t)npairs * NF) return;
  const int pair = pair0 + (int)(row / NF), ly = (int)(row % NF);
  C2<Tg> x[E];
#pragma unroll
  for (int n2 = 0; n2 < E; ++n2) {
    const int n = lane + 64 * n2;
    int c = -1;
    if (n < Q / 2) c = n + Q / 2;
    else if (n >= NF - Q / 2) c = n - NF + Q / 2;
    x[n2] = c >= 0 ? t2[((size_t)pair * Q + c) * NF + ly] : C2<Tg>{Tg(0), Tg(0)};
  }
  group_fft<Tg, 64, E, -1>(x, lane, tw);
  const int base = E * bitrev(lane, 6);
  C2<Tg>* dst = B + ((size_t)pair * NF + ly) * NF;
#pragma unroll
  for (int k2 = 0; k2 < E; ++k2) dst[base + k2] = x[k2];
}

struct WaveletAdj {    // cogradients of one wavelet's inputs
  C2<double> g_w;      // dL/dw (cogradient of the Eq. 1 weight)
  double g_phi0, g_wx, g_wy, g_dz;
};

// Cogradient of the incident state from the wavelets of one ray (sensor next):
// hit point, incident tangential wavevector, optical path, sensor z, and the
// torque sum_i d_i x dL/dd_i of the emitted directions, the cogradient of a
// rotation of the frame (u, v, n) at fixed tangential wavevectors.
struct IncAcc {
  double gp[3], gkin[2], gopl, gzs, tq[3];
};

// Cogradient of the emitted secondary direction (planar DOE, sensor next).
__device__ __forceinline__ void direction_cograd(const DoeArgs& a, const RayCtx& c,
                                                 const Secondary& sec, const WaveletAdj& wa,
                                                 double gds[3]) {
  const DevCfg& cfg = *a.cfg;
  const DevPair& pr = a.pairs[c.pair];
  const double ns = pr.n_med[cfg.ns_idx];
  const double k0 = c.k0;
  const double Xc[3] = {pr.pc[0], pr.pc[1], a.live->sensor_z};
  // phi0 = k0 (OPL + ns ds . (Xc - p)),  w = k0 ns psf_pitch (ds_x, ds_y)
  for (int i = 0; i < 3; ++i) gds[i] = k0 * ns * wa.g_phi0 * (Xc[i] - c.p[i]);
  gds[0] += k0 * ns * cfg.psf_pitch * wa.g_wx;
  gds[1] += k0 * ns * cfg.psf_pitch * wa.g_wy;
  gds[2] += wa.g_dz * (sec.dsz >= 0 ? 1.0 : -1.0);
}

// dL/dK of the secondary's tangential wavevector from its direction cogradient:
// ds = (Ku u + Kv v + sgn kz n) / k_out, kz = sqrt(k_out^2 - Ku^2 - Kv^2), sgn = -1
// after a reflective DOE.
__device__ __forceinline__ void wavevector_cograd(const RayCtx& c, const Secondary& sec,
                                                  const double gds[3], double& gKu,
                                                  double& gKv) {
  const double gu = gds[0] * c.u[0] + gds[1] * c.u[1] + gds[2] * c.u[2];
  const double gv = gds[0] * c.v[0] + gds[1] * c.v[1] + gds[2] * c.v[2];
  const double gn = c.sgn * (gds[0] * c.n[0] + gds[1] * c.n[1] + gds[2] * c.n[2]);
  gKu = (gu - gn * sec.Ku / sec.kz) / c.k_out;
  gKv = (gv - gn * sec.Kv / sec.kz) / c.k_out;
}

__device__ __forceinline__ void incident_from_wavelet(const DoeArgs& a, const RayCtx& c,
                                                      const Secondary& sec,
                                                      const WaveletAdj& wa, IncAcc& acc) {
  const DevCfg& cfg = *a.cfg;
  const DevPair& pr = a.pairs[c.pair];
  const double ns = pr.n_med[cfg.ns_idx];
  const double k0 = c.k0;
  const double ds[3] = {sec.dsx, sec.dsy, sec.dsz};
  acc.gopl += k0 * wa.g_phi0;
  for (int i = 0; i < 3; ++i) acc.gp[i] -= k0 * ns * wa.g_phi0 * ds[i];
  acc.gzs += k0 * ns * wa.g_phi0 * ds[2];
  double gds[3], gKu, gKv;
  direction_cograd(a, c, sec, wa, gds);
  wavevector_cograd(c, sec, gds, gKu, gKv);
  acc.gkin[0] += gKu;
  acc.gkin[1] += gKv;
  acc.tq[0] += ds[1] * gds[2] - ds[2] * gds[1];
  acc.tq[1] += ds[2] * gds[0] - ds[0] * gds[2];
  acc.tq[2] += ds[0] * gds[1] - ds[1] * gds[0];
}

// Inputs of one surface step of the trace adjoints: p_in, d_in and the surface's
// (z, c, k, A4, A6, A8, A10).
constexpr int kNT = 13;

// Entries per record of the tiled interpolation's results (value, d/dx, d/dy, pad).
constexpr int kInterpStride = 4;

// Sum over the 64 lanes of a wave (butterfly: every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
  v += xor_lane<32>(v);
  v += xor_lane<16>(v);
  v += xor_lane<8>(v);
  v += xor_lane<4>(v);
  v += xor_lane<2>(v);
  v += xor_lane<1>(v);
  return v;
}

// ------------------------------------- secondaries through post-DOE surfaces ---
// Adjoint of the conventional trace of every secondary ray through the surfaces
// between the DOE and the sensor, for the lens-parameter gradient (the DOE
// adjoint covers the weights; with such surfaces it leaves the geometry here).
// One wave per incident ray, its lanes over the ray's record slots: the
// secondary is re-traced in FP64 with its entry state before every surface,
// its wavelet cogradient formed from the forward's record value and the tiled
// interpolation, then taken back through the sensor step (analytic) and each
// surface (dual numbers of the 13 inputs of a step, as in the incident trace
// adjoint).  Adds, per ray, the cogradients of the hit point, the incident
// tangential wavevector, the optical path, the sensor z and the frame torque to
// the DOE adjoint's; the surfaces' own parameters go to lensg.
constexpr int kPostMax = 4;     // refracting surfaces after the DOE

template <class Tg>
__global__ __launch_bounds__(256) void k_post_bwd(DoeArgs a) {
  const DevCfg& cfg = *a.cfg;
  const int lane = threadIdx.x & 63;
  const size_t w = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= a.nray) return;                                   // uniform over the wave
  const size_t gid = a.ray0 + w;
  if (a.st[7 * a.n_total + gid] == 0.0) return;
  const RayCtx c = a.ctx[gid];
  const DevPair& pr = a.pairs[c.pair];
  const int sd = cfg.s_doe, S = cfg.n_surf, npost = S - sd - 1;
  const int M = cfg.pad * c.P;
  const double ns = pr.n_med[S], k0 = c.k0;
  const double Xc[3] = {pr.pc[0], pr.pc[1], a.live->sensor_z};
  const double cell = cfg.nf / (2.0 * RW_PI);
  double gp[3] = {0, 0, 0}, gkin[2] = {0, 0}, gopl = 0.0, gzs = 0.0, tq[3] = {0, 0, 0};
  double gsurf[kPostMax][7];
  for (int j = 0; j < kPostMax; ++j)
    for (int f = 0; f < 7; ++f) gsurf[j][f] = 0.0;
  const int nslot = a.full ? M * M : cfg.N;
  for (int i = lane; i < nslot; i += 64) {
    int J = i;
    if (!a.full) J = a.jdraw[gid * cfg.N + i];
    if (J < 0) continue;
    const size_t slot = (gid - a.ray0) * (size_t)a.emit + i;
    const C2<Tg> rv = ((const C2<Tg>*)a.rec_val)[slot];
    if (is_none(rv)) continue;
    const int jx = J / M - M / 2, jy = J % M - M / 2;
    const double Ku = c.kin_u + c.dk * jx, Kv = c.kin_v + c.dk * jy;
    const double kz = sqrt(c.k_out * c.k_out - Ku * Ku - Kv * Kv);
    double ds[3], p[3], d[3], pe[kPostMax][3], de[kPostMax][3];
    for (int q = 0; q < 3; ++q) {
      ds[q] = (Ku * c.u[q] + Kv * c.v[q] + c.sgn * kz * c.n[q]) / c.k_out;
      p[q] = c.p[q];
      d[q] = ds[q];
    }
    bool ok = true;
    for (int j = 0; j < npost && ok; ++j) {
      const int s = sd + 1 + j;
      for (int q = 0; q < 3; ++q) { pe[j][q] = p[q]; de[j][q] = d[q]; }
      const Surf<double> sf = surf_of<double>(a.live->s[s]);
      double t;
      ok = intersect(sf, p, d, t);
      if (!ok) break;
      for (int q = 0; q < 3; ++q) p[q] += t * d[q];
      double nrm[3];
      surface_normal(sf, p[0], p[1], nrm);
      ok = refract(d, nrm, pr.n_med[s] / pr.n_med[s + 1]);
    }
    if (!ok) continue;                 // the forward kept no record for it either
    // wavelet cogradients from the record value cv = w |d_z| e^{i phi0}
    const C2<Tg>* q3 = (const C2<Tg>*)a.interp + kInterpStride * slot;
    const double g0r = q3[0].re, g0i = q3[0].im, dxr = q3[1].re, dxi = q3[1].im,
                 dyr = q3[2].re, dyi = q3[2].im;
    const double cr = rv.re, ci = rv.im;
    const double dza = fabs(d[2]);
    const double g_wx = -(cr * dxr + ci * dxi) * cell, g_wy = -(cr * dyr + ci * dyi) * cell;
    const double g_phi0 = -(g0r * ci - g0i * cr), g_dz = (g0r * cr + g0i * ci) / dza;
    // sensor step: phi0 = k0 (OPL + ns d.(Xc - p)), w = k0 ns pitch (d_x, d_y), |d_z|
    double g_p[3], g_d[3];
    for (int q = 0; q < 3; ++q) {
      g_p[q] = -k0 * ns * g_phi0 * d[q];
      g_d[q] = k0 * ns * g_phi0 * (Xc[q] - p[q]);
    }
    g_d[0] += k0 * ns * cfg.psf_pitch * g_wx;
    g_d[1] += k0 * ns * cfg.psf_pitch * g_wy;
    g_d[2] += g_dz * (d[2] >= 0 ? 1.0 : -1.0);
    const double g_o = k0 * g_phi0;
    gopl += g_o;
    gzs += k0 * ns * g_phi0 * d[2];
    // back through the surfaces, last first
    for (int j = npost - 1; j >= 0; --j) {
      const int s = sd + 1 + j;
      typedef Dual<kNT> D;
      D pd[3], dd[3];
      for (int q = 0; q < 3; ++q) {
        pd[q] = dvar<kNT>(pe[j][q], q);
        dd[q] = dvar<kNT>(de[j][q], 3 + q);
      }
      const DevSurf& dsf = a.live->s[s];
      Surf<D> sf;
      sf.z = dvar<kNT>(dsf.z, 6);
      sf.c = dvar<kNT>(dsf.c, 7);
      sf.k = dvar<kNT>(dsf.k, 8);
      sf.A4 = dvar<kNT>(dsf.A4, 9);
      sf.A6 = dvar<kNT>(dsf.A6, 10);
      sf.A8 = dvar<kNT>(dsf.A8, 11);
      sf.A10 = dvar<kNT>(dsf.A10, 12);
      sf.gh = dconst<kNT>(dsf.gh);
      sf.gw = dconst<kNT>(dsf.gw);
      D tt;
      intersect(sf, pd, dd, tt);
      D qq[3];
      for (int q = 0; q < 3; ++q) qq[q] = pd[q] + tt * dd[q];
      const D dopl = tt * pr.n_med[s];
      D nrm[3];
      surface_normal(sf, qq[0], qq[1], nrm);
      refract(dd, nrm, dconst<kNT>(pr.n_med[s] / pr.n_med[s + 1]));
      double gin[kNT];
      for (int k = 0; k < kNT; ++k) {
        double v = g_o * dopl.d[k];
        for (int q = 0; q < 3; ++q) v += g_p[q] * qq[q].d[k] + g_d[q] * dd[q].d[k];
        gin[k] = v;
      }
      for (int q = 0; q < 3; ++q) { g_p[q] = gin[q]; g_d[q] = gin[3 + q]; }
      for (int f = 0; f < 7; ++f) gsurf[j][f] += gin[6 + f];
    }
    // at the DOE: origin p, direction ds = (Ku u + Kv v + kz n) / k_out
    for (int q = 0; q < 3; ++q) gp[q] += g_p[q];
    const double gu = g_d[0] * c.u[0] + g_d[1] * c.u[1] + g_d[2] * c.u[2];
    const double gv = g_d[0] * c.v[0] + g_d[1] * c.v[1] + g_d[2] * c.v[2];
    const double gn = g_d[0] * c.n[0] + g_d[1] * c.n[1] + g_d[2] * c.n[2];
    gkin[0] += (gu - gn * Ku / kz) / c.k_out;
    gkin[1] += (gv - gn * Kv / kz) / c.k_out;
    tq[0] += ds[1] * g_d[2] - ds[2] * g_d[1];
    tq[1] += ds[2] * g_d[0] - ds[0] * g_d[2];
    tq[2] += ds[0] * g_d[1] - ds[1] * g_d[0];
  }
  double v[10] = {gp[0], gp[1], gp[2], gkin[0], gkin[1], gopl, gzs, tq[0], tq[1], tq[2]};
  for (int q = 0; q < 10; ++q) v[q] = wave_sum(v[q]);
  for (int j = 0; j < npost; ++j)
    for (int f = 0; f < 7; ++f) {
      const double sum = wave_sum(gsurf[j][f]);
      if (lane == 0 && sum != 0.0) atomicAdd(&a.lensg[(sd + 1 + j) * 8 + f], sum);
    }
  if (lane == 0) {
    // one writer per ray: add to what the DOE adjoint stored
    const double lf = c.k0 * c.n_in;
    double add[RW_RAYGRAD];
    for (int q = 0; q < 3; ++q) {
      add[q] = v[q];
      add[3 + q] = lf * (v[3] * c.u[q] + v[4] * c.v[q]);
      add[8 + q] = lf * v[3] * c.d[q];
      add[11 + q] = lf * v[4] * c.d[q];
      add[14 + q] = v[7 + q];
    }
    add[6] = v[5];
    add[7] = v[6];
    for (int q = 0; q < RW_RAYGRAD; ++q) a.raygrad[(size_t)q * a.n_total + gid] += add[q];
  }
}

// ------------------------------------------ type-2 interpolation, tiled ---
// Results per record: B, dB/dx, dB/dy and a pad (kInterpStride), so that a
// record fills one aligned 32-byte sector (FP32) of the scattered stores.

// Cogradient of every secondary-ray record of the forward (sorted by bin):
// the sensor-grid cogradient B interpolated with the ES kernel at the record's
// grid coordinate, and with the kernel's derivative along x and along y.  One
// block per 2 x 2 bins stages every grid cell its records' footprints reach
// in LDS; one lane per record; results go to the record's slot.
// A block whose records a focusing system has concentrated takes a slice of
// them: k_interp_slices cuts a block's records into S = ceil(records / target)
// <= kInterpSlices slices (target about 1/2048 of the launch's); the block of
// the first launch takes slice 0, the blocks of the second the listed slices
// 1 .. S - 1 (each result goes to its own record's slot: no atomics).
__host__ __device__ constexpr int interp_side(int bin, int w) { return 2 * bin + 2 * ((w + 1) / 2); }
constexpr int kInterpSlices = 255;   // most slices of one block (a byte per block)

static __global__ __launch_bounds__(256) void k_interp_slices(const unsigned long long* offsets,
                                                       BinGeom g, int pair0, int npairs,
                                                       unsigned long long target,
                                                       unsigned char* slices, uint2* heavy,
                                                       unsigned int* n_heavy) {
  const int nsb = g.nb / 2, nt = nsb * nsb;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)npairs * nt) return;
  const int pl = (int)(i / nt), t = (int)(i % nt);
  const unsigned long long* off = offsets + (size_t)(pair0 + pl) * g.keys;
  unsigned long long n = 0;
  for (int q = 0; q < 4; ++q) {
    const int k = bin_key((t / nsb) * 2 + q / 2, (t % nsb) * 2 + q % 2, g);
    n += off[k + 1] - off[k];
  }
  const int S = (int)min((unsigned long long)kInterpSlices, max(1ull, (n + target - 1) / target));
  slices[i] = (unsigned char)S;
  if (S > 1) {
    const unsigned int b = atomicAdd(n_heavy, (unsigned int)(S - 1));
    for (int k = 1; k < S; ++k) heavy[b + k - 1] = make_uint2((unsigned int)i, (unsigned int)k);
  }
}

template <class Tg, int w>
__device__ __forceinline__ void interp_tile(const void* srt_pos, const unsigned int* srt_idx,
                                            const unsigned long long* offsets, const BinGeom& g,
                                            double beta, int pair, int tile_i, int slice, int S,
                                            const C2<Tg>* adj, C2<Tg>* out) {
  using U = typename RecPos<Tg>::T;
  extern __shared__ unsigned char s_raw[];
  C2<Tg>* cells = (C2<Tg>*)s_raw;
  __shared__ unsigned long long s_beg[4], s_pre[5];
  constexpr int half = (w + 1) / 2;
  const int side = interp_side(g.bin, w);
  const int nsb = g.nb / 2;
  const int sby = tile_i / nsb, sbx = tile_i % nsb;
  const int X0 = sbx * 2 * g.bin - half, Y0 = sby * 2 * g.bin - half;
  const C2<Tg>* gp = adj + (size_t)pair * g.nf * g.nf;
  __syncthreads();                              // LDS reuse across the tiles of a block
  // cells staged 8 per lane at a time: the loads are issued before the stores
  for (int i0 = threadIdx.x; i0 < side * side; i0 += 8 * blockDim.x) {
    C2<Tg> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * (int)blockDim.x;
      const int cy = i / side, cx = i - cy * side;
      if (i < side * side)
        v[u] = gp[(size_t)((Y0 + cy) & (g.nf - 1)) * g.nf + ((X0 + cx) & (g.nf - 1))];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * (int)blockDim.x;
      if (i < side * side) cells[i] = v[u];
    }
  }
  if (threadIdx.x < 4) {
    const int by = sby * 2 + (int)threadIdx.x / 2, bx = sbx * 2 + (int)threadIdx.x % 2;
    const int k = bin_key(by, bx, g);
    const unsigned long long* off = offsets + (size_t)pair * g.keys;
    s_beg[threadIdx.x] = off[k];
    s_pre[threadIdx.x + 1] = off[k + 1] - off[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s_pre[0] = 0;
    for (int i = 1; i <= 4; ++i) s_pre[i] += s_pre[i - 1];
  }
  __syncthreads();
  const U* pos = (const U*)srt_pos;
  const Tg tw = (Tg)(2.0 / w), bet = (Tg)beta;
  // this slice's records
  const unsigned long long nall = s_pre[4];
  const unsigned long long jlo = nall * (unsigned long long)slice / (unsigned long long)S;
  const unsigned long long ntot = nall * (unsigned long long)(slice + 1) / (unsigned long long)S;
  // the position and slot of the next record are loaded before the current one
  // is interpolated
  int b = 0;                                        // monotonic over the lane's records
  auto rec_of = [&](unsigned long long j) {
    while (j >= s_pre[b + 1]) ++b;
    return s_beg[b] + (j - s_pre[b]);
  };
  U nx = 0, ny = 0;
  unsigned int nid = 0;
  if (jlo + threadIdx.x < ntot) {
    const unsigned long long r = rec_of(jlo + threadIdx.x);
    nx = pos[2 * r]; ny = pos[2 * r + 1]; nid = srt_idx[r];
  }
  for (unsigned long long j = jlo + threadIdx.x; j < ntot; j += blockDim.x) {
    const U px = nx, py = ny;
    const unsigned int slot = nid;
    if (j + blockDim.x < ntot) {
      const unsigned long long r = rec_of(j + blockDim.x);
      nx = pos[2 * r]; ny = pos[2 * r + 1]; nid = srt_idx[r];
    }
    const double gx = turns_to_cells(px, g.nf), gy = turns_to_cells(py, g.nf);
    const int lx0 = (int)ceil(gx - 0.5 * w), ly0 = (int)ceil(gy - 0.5 * w);
    Tg kx[w], dkx[w];
#pragma unroll
    for (int i = 0; i < w; ++i) {
      kx[i] = Tg(0); dkx[i] = Tg(0);
      const Tg tx = (Tg)((double)(lx0 + i) - gx) * tw;
      const Tg ax = Tg(1) - tx * tx;
      if (ax > Tg(0)) {
        const Tg sx = sqrt(ax);
        kx[i] = (Tg)exp(bet * (sx - Tg(1)));
        dkx[i] = -kx[i] * bet * tx / sx * tw;
      }
    }
    double g0r = 0, g0i = 0, dxr = 0, dxi = 0, dyr = 0, dyi = 0;
    const C2<Tg>* base = cells + (ly0 - Y0) * side + (lx0 - X0);
#pragma unroll
    for (int jj = 0; jj < w; ++jj) {
      const Tg ty = (Tg)((double)(ly0 + jj) - gy) * tw;
      const Tg ay = Tg(1) - ty * ty;
      if (!(ay > Tg(0))) continue;
      const Tg sy = sqrt(ay);
      const Tg ky = (Tg)exp(bet * (sy - Tg(1)));
      const Tg dky = -ky * bet * ty / sy * tw;
      const C2<Tg>* row = base + jj * side;
      Tg s0r = 0, s0i = 0, s1r = 0, s1i = 0;
#pragma unroll
      for (int i = 0; i < w; ++i) {
        const C2<Tg> v = row[i];
        s0r += kx[i] * v.re; s0i += kx[i] * v.im;
        s1r += dkx[i] * v.re; s1i += dkx[i] * v.im;
      }
      g0r += (double)(ky * s0r); g0i += (double)(ky * s0i);
      dxr += (double)(ky * s1r); dxi += (double)(ky * s1i);
      dyr += (double)(dky * s0r); dyi += (double)(dky * s0i);
    }
    C2<Tg>* o = out + kInterpStride * (size_t)slot;
    o[0] = {(Tg)g0r, (Tg)g0i};
    o[1] = {(Tg)dxr, (Tg)dxi};
    o[2] = {(Tg)dyr, (Tg)dyi};
    o[3] = {Tg(0), Tg(0)};
  }
}

// slices: S per (pair of the group, block of 2 x 2 bins); heavy: null for the
// launch over every block (slice 0), else the list of further slices.
template <class Tg, int w>
__global__ __launch_bounds__(256) void k_interp_tiles(const void* srt_pos,
                                                      const unsigned int* srt_idx,
                                                      const unsigned long long* offsets,
                                                      BinGeom g, double beta, int pair0,
                                                      const C2<Tg>* adj, C2<Tg>* out,
                                                      const unsigned char* slices,
                                                      const uint2* heavy,
                                                      const unsigned int* n_heavy) {
  const int nt = (g.nb / 2) * (g.nb / 2);
  if (!heavy) {
    interp_tile<Tg, w>(srt_pos, srt_idx, offsets, g, beta, pair0 + blockIdx.y, blockIdx.x, 0,
                       slices[(size_t)blockIdx.y * nt + blockIdx.x], adj, out);
    return;
  }
  const unsigned int n = *n_heavy;
  for (unsigned int e = blockIdx.x; e < n; e += gridDim.x) {
    const uint2 h = heavy[e];
    interp_tile<Tg, w>(srt_pos, srt_idx, offsets, g, beta, pair0 + (int)(h.x / nt),
                       (int)(h.x % nt), (int)h.y, slices[h.x], adj, out);
  }
}

// ---------------------------------------------------- dL/dt -> dphi, dA ---
template <class Tg>
__global__ void k_dmaps(const float* phase, const float* amp, const C2<Tg>* gt, float* dphi,
                        float* damp, int n, int two_phase) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s, c;
  sincos((double)phase[i], &s, &c);
  const double gr = gt[i].re, gi = gt[i].im;
  if (two_phase) {
    // t = e^{i phi1} + e^{i phi2}: dL/dphi_k = Im(conj(e^{i phi_k}) g)
    double s2, c2;
    sincos((double)amp[i], &s2, &c2);
    dphi[i] = (float)(c * gi - s * gr);
    damp[i] = (float)(c2 * gi - s2 * gr);
    return;
  }
  const double a = amp[i];
  // t = A e^{i phi}: dL/dphi = Im(conj(t) g), dL/dA = Re(conj(e^{i phi}) g)
  dphi[i] = (float)(a * (c * gi - s * gr));
  damp[i] = (float)(c * gr + s * gi);
}

// ------------------------------------------------------- trace adjoint ---
// One surface step as a function of (p_in, d_in) and the surface's
// (z, c, k, A4, A6, A8, A10); dual numbers give its Jacobian columns (kNT).

static __global__ __launch_bounds__(256) void k_trace_bwd(const DevCfg* cfg, const DevPair* pairs,
                                                   const DevLive* live, const double* st,
                                                   const double* ck, const double* raygrad,
                                                   size_t n_total, size_t ray0, size_t nray,
                                                   double* lensg) {
  const size_t wi = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = wi < nray;
  const size_t gid = ray0 + (active ? wi : 0);
  const int sd = cfg->s_doe;
  double gsurf[RW_MAX_SURF][7];
  for (int s = 0; s < RW_MAX_SURF; ++s)
    for (int f = 0; f < 7; ++f) gsurf[s][f] = 0.0;
  double gzs = 0.0;
  if (active && st[7 * n_total + gid] != 0.0) {
    const int pair = (int)(gid / cfg->R2);
    const DevPair& pr = pairs[pair];
    double gp[3], gd[3], gu[3], gv[3], gtq[3];
    for (int i = 0; i < 3; ++i) {
      gp[i] = raygrad[i * n_total + gid];
      gd[i] = raygrad[(3 + i) * n_total + gid];
      gu[i] = raygrad[(8 + i) * n_total + gid];
      gv[i] = raygrad[(11 + i) * n_total + gid];
      gtq[i] = raygrad[(14 + i) * n_total + gid];
    }
    const double gopl = raygrad[6 * n_total + gid];
    gzs = raygrad[7 * n_total + gid];
    for (int s = sd; s >= 0; --s) {
      const double* c = ck + (size_t)s * 8 * n_total;
      typedef Dual<kNT> D;
      D p[3], d[3];
      for (int i = 0; i < 3; ++i) {
        p[i] = dvar<kNT>(c[i * n_total + gid], i);
        d[i] = dvar<kNT>(c[(3 + i) * n_total + gid], 3 + i);
      }
      const DevSurf& ds = live->s[s];
      Surf<D> sf;
      sf.z = dvar<kNT>(ds.z, 6);
      sf.c = dvar<kNT>(ds.c, 7);
      sf.k = dvar<kNT>(ds.k, 8);
      sf.A4 = dvar<kNT>(ds.A4, 9);
      sf.A6 = dvar<kNT>(ds.A6, 10);
      sf.A8 = dvar<kNT>(ds.A8, 11);
      sf.A10 = dvar<kNT>(ds.A10, 12);
      sf.gh = dconst<kNT>(ds.gh);
      sf.gw = dconst<kNT>(ds.gw);
      D tt;
      if (!intersect(sf, p, d, tt)) break;
      D q[3];
      for (int i = 0; i < 3; ++i) q[i] = p[i] + tt * d[i];
      const D dopl = tt * pr.n_med[s];
      if (s < sd) {
        D nrm[3];
        surface_normal(sf, q[0], q[1], nrm);
        refract(d, nrm, dconst<kNT>(pr.n_med[s] / pr.n_med[s + 1]));
      }
      // adjoint of the step: g_in[k] = sum_out g_out . d(out)/d(in_k)
      double gin[kNT];
      for (int k = 0; k < kNT; ++k) {
        double v = gopl * dopl.d[k];
        for (int i = 0; i < 3; ++i) v += gp[i] * q[i].d[k] + gd[i] * d[i].d[k];
        gin[k] = v;
      }
      if (s == sd && !cfg->planar) {
        // the tangent frame at the hit of a curved DOE: n from the sag gradient,
        // u the normalised projection of x on the tangent plane, v = n x u
        D n[3], u[3], v[3];
        surface_normal(sf, q[0], q[1], n);
        D ux = 1.0 - n[0] * n[0], uy = -(n[0] * n[1]), uz = -(n[0] * n[2]);
        const D iu = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
        u[0] = ux * iu; u[1] = uy * iu; u[2] = uz * iu;
        v[0] = n[1] * u[2] - n[2] * u[1];
        v[1] = n[2] * u[0] - n[0] * u[2];
        v[2] = n[0] * u[1] - n[1] * u[0];
        for (int k = 0; k < kNT; ++k) {
          // rotation of the frame induced by input k: w = (a x da) / 2 summed over u, v, n
          double w[3] = {0.0, 0.0, 0.0}, g = 0.0;
          const D* fr[3] = {u, v, n};
          for (int f = 0; f < 3; ++f) {
            const D* a3 = fr[f];
            w[0] += a3[1].v * a3[2].d[k] - a3[2].v * a3[1].d[k];
            w[1] += a3[2].v * a3[0].d[k] - a3[0].v * a3[2].d[k];
            w[2] += a3[0].v * a3[1].d[k] - a3[1].v * a3[0].d[k];
          }
          for (int i = 0; i < 3; ++i)
            g += gu[i] * u[i].d[k] + gv[i] * v[i].d[k] + 0.5 * gtq[i] * w[i];
          gin[k] += g;
        }
      }
      for (int i = 0; i < 3; ++i) { gp[i] = gin[i]; gd[i] = gin[3 + i]; }
      for (int f = 0; f < 7; ++f) gsurf[s][f] += gin[6 + f];
    }
  }
  // wave reductions, one atomic per wave and slot
  for (int s = 0; s <= sd; ++s)
    for (int f = 0; f < 7; ++f) {
      const double v = wave_sum(gsurf[s][f]);
      if ((threadIdx.x & 63) == 0 && v != 0.0) atomicAdd(&lensg[s * 8 + f], v);
    }
  const double v = wave_sum(gzs);
  if ((threadIdx.x & 63) == 0 && v != 0.0) atomicAdd(&lensg[RW_LENSG_SENSOR], v);
}

static __global__ void k_lens_map(const DevCfg* cfg, const DevParam* prm, const double* lensg,
                           float* d_lens) {
  const int i = threadIdx.x;
  if (i >= cfg->n_params) return;
  const int s = prm[i].surface, f = prm[i].field;
  double g;
  if (f < 6) {
    g = lensg[s * 8 + 1 + f];      // curv, conic, A4, A6, A8, A10 -> slots 1..6
  } else {
    g = lensg[RW_LENSG_SENSOR];    // a gap moves every later surface and the sensor
    for (int t = s + 1; t < cfg->n_surf; ++t) g += lensg[t * 8 + 0];
  }
  d_lens[i] = (float)(prm[i].scale * g);
}

}  // namespace rw
