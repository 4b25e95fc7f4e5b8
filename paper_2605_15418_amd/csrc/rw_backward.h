// Backward (adjoint G1) kernels of the ray-wave hybrid PSF: the a.e.
// derivative of the forward with the drawn sample indices held fixed.
//
//   k_psf_cograd      dL/dI (Eq. 3 with closed-form alpha, or the caller's) ->
//                     cogradient of the kept modes 2 dI U / (Psi(kx) Psi(ky))
//   k_grid_cols_bwd / k_grid_rows_bwd   adjoint of the grid FFT and crop:
//                     B_l = sum_k exp(-2 pi i k.l / nf) G_k  (full nf x nf grid)
//   k_doe_bwd         per incident ray: recompute the patch spectrum and the
//                     draws, interpolate B and its kernel derivative at each
//                     wavelet, chain through Eq. 2 and Eq. 1 (with the S = sum|U~|
//                     term of p_mag), the patch-centre reference, the inverse
//                     FFT and the bilinear gather (LDS-tiled scatter into dL/dt),
//                     and produce the cogradient of the incident ray state
//   k_dmaps           dL/dt -> dL/dphi, dL/dA
//   k_trace_bwd       reverse sweep over the per-surface checkpoints; local
//                     Jacobians of each Newton/Snell step by dual numbers
//   k_lens_map        per-surface sums -> normalised lens-parameter gradients
#pragma once
#include "rw_kernels.h"

#define RW_LENSG_SLOTS 128
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

// ------------------------------------------------- interpolation (type 2) ---
// g0 = sum_l B_l psi(l - x), dx = sum_l B_l psi'(l_x - x_x) psi(l_y - x_y), dy likewise.
template <class Prec>
__device__ __forceinline__ void interp_adj(const DevCfg& cfg, const C2<typename Prec::Tg>* B,
                                           int pair, typename Prec::Tp gx, typename Prec::Tp gy,
                                           C2<double>& g0, C2<double>& dx, C2<double>& dy) {
  using Tg = typename Prec::Tg;
  using Tp = typename Prec::Tp;
  const int nf = cfg.nf, w = cfg.w;
  const int lx0 = (int)ceil(gx - (Tp)(0.5 * w)), ly0 = (int)ceil(gy - (Tp)(0.5 * w));
  const double tw = 2.0 / w, beta = cfg.beta;
  double kx[16], ky[16], dkx[16], dky[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i < w) {
      const double zx = (double)((Tp)(lx0 + i) - gx), zy = (double)((Tp)(ly0 + i) - gy);
      const double tx = zx * tw, ty = zy * tw;
      const double ax = 1.0 - tx * tx, ay = 1.0 - ty * ty;
      const double sx = ax > 0 ? sqrt(ax) : 0.0, sy = ay > 0 ? sqrt(ay) : 0.0;
      kx[i] = ax > 0 ? exp(beta * (sx - 1.0)) : 0.0;
      ky[i] = ay > 0 ? exp(beta * (sy - 1.0)) : 0.0;
      // d psi / dz = psi * beta * (-t / sqrt(1 - t^2)) * (2 / w)
      dkx[i] = ax > 0 ? -kx[i] * beta * tx / sx * tw : 0.0;
      dky[i] = ay > 0 ? -ky[i] * beta * ty / sy * tw : 0.0;
    }
  }
  g0 = {0, 0}; dx = {0, 0}; dy = {0, 0};
  const C2<Tg>* gp = B + (size_t)pair * nf * nf;
  for (int j = 0; j < w; ++j) {
    const C2<Tg>* row = gp + (size_t)((ly0 + j) & (nf - 1)) * nf;
    C2<double> s0 = {0, 0}, s1 = {0, 0};
    for (int i = 0; i < w; ++i) {
      const C2<Tg> b = row[(lx0 + i) & (nf - 1)];
      s0.re += kx[i] * b.re; s0.im += kx[i] * b.im;
      s1.re += dkx[i] * b.re; s1.im += dkx[i] * b.im;
    }
    g0.re += ky[j] * s0.re; g0.im += ky[j] * s0.im;
    dx.re += ky[j] * s1.re; dx.im += ky[j] * s1.im;
    dy.re += dky[j] * s0.re; dy.im += dky[j] * s0.im;
  }
}

struct WaveletAdj {    // cogradients of one wavelet's inputs
  C2<double> g_w;      // dL/dw (cogradient of the Eq. 1 weight)
  double g_phi0, g_wx, g_wy, g_dz;
};

// Forward quantities of one wavelet and the cogradients of its inputs.
template <class Prec>
__device__ __forceinline__ bool wavelet_adjoint(const DoeArgs& a, const RayCtx& c, int jx, int jy,
                                                C2<typename Prec::Tp> w, WaveletAdj& wa,
                                                Secondary& sec) {
  using Tp = typename Prec::Tp;
  using Tg = typename Prec::Tg;
  const DevCfg& cfg = *a.cfg;
  Tp phi0, wx, wy;
  double dza;
  if (!secondary_to_sensor<Prec>(a, c, jx, jy, phi0, wx, wy, dza, sec)) return false;
  const C2<Tp> e = cis<Tp>(wrap_2pi(phi0));
  const C2<Tp> cv = (w * e) * (Tp)dza;
  C2<double> g0, dx, dy;
  interp_adj<Prec>(cfg, (const C2<Tg>*)a.adj, c.pair, grid_coord(wx, cfg.nf),
                   grid_coord(wy, cfg.nf), g0, dx, dy);
  const C2<double> cd = {(double)cv.re, (double)cv.im};
  // dL/dc = g0 ; dL/dx_grid = -Re(c conj(dx))
  const double cell = cfg.nf / (2.0 * RW_PI);
  wa.g_wx = -(cd.re * dx.re + cd.im * dx.im) * cell;
  wa.g_wy = -(cd.re * dy.re + cd.im * dy.im) * cell;
  // dL/dphi0 = Re(conj(g0) i c) = -Im(conj(g0) c)
  wa.g_phi0 = -(g0.re * cd.im - g0.im * cd.re);
  // dL/d|d_z| = Re(conj(g0) c) / |d_z|
  wa.g_dz = (g0.re * cd.re + g0.im * cd.im) / dza;
  // dL/dw = conj(|d_z| e^{i phi0}) g0
  const double er = (double)e.re * dza, ei = (double)e.im * dza;
  wa.g_w = {er * g0.re + ei * g0.im, er * g0.im - ei * g0.re};
  return true;
}

// Cogradient of the incident state from one wavelet (planar DOE, sensor next).
struct IncAcc {
  double gp[3], gkin[2], gopl, gzs;
};

__device__ __forceinline__ void incident_from_wavelet(const DoeArgs& a, const RayCtx& c,
                                                      const Secondary& sec,
                                                      const WaveletAdj& wa, IncAcc& acc) {
  const DevCfg& cfg = *a.cfg;
  const DevPair& pr = a.pairs[c.pair];
  const double ns = pr.n_med[cfg.n_surf];
  const double k0 = c.k0;
  const double ds[3] = {sec.dsx, sec.dsy, sec.dsz};
  const double Xc[3] = {pr.pc[0], pr.pc[1], a.live->sensor_z};
  // phi0 = k0 (OPL + ns ds . (Xc - p)),  w = k0 ns psf_pitch (ds_x, ds_y)
  acc.gopl += k0 * wa.g_phi0;
  double gds[3];
  for (int i = 0; i < 3; ++i) {
    acc.gp[i] -= k0 * ns * wa.g_phi0 * ds[i];
    gds[i] = k0 * ns * wa.g_phi0 * (Xc[i] - c.p[i]);
  }
  acc.gzs += k0 * ns * wa.g_phi0 * ds[2];
  gds[0] += k0 * ns * cfg.psf_pitch * wa.g_wx;
  gds[1] += k0 * ns * cfg.psf_pitch * wa.g_wy;
  gds[2] += wa.g_dz * (ds[2] >= 0 ? 1.0 : -1.0);
  // ds = (Ku u + Kv v + kz n) / k_out, kz = sqrt(k_out^2 - Ku^2 - Kv^2)
  const double gu = gds[0] * c.u[0] + gds[1] * c.u[1] + gds[2] * c.u[2];
  const double gv = gds[0] * c.v[0] + gds[1] * c.v[1] + gds[2] * c.v[2];
  const double gn = gds[0] * c.n[0] + gds[1] * c.n[1] + gds[2] * c.n[2];
  acc.gkin[0] += (gu - gn * sec.Ku / sec.kz) / c.k_out;
  acc.gkin[1] += (gv - gn * sec.Kv / sec.kz) / c.k_out;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <class Prec, int M, bool kLDS>
__global__ __launch_bounds__(kThreads) void k_doe_bwd(DoeArgs a) {
  using Tf = typename Prec::Tf;
  using Tg = typename Prec::Tg;
  using Tp = typename Prec::Tp;
  constexpr int SM = M + 1;
  constexpr int C = (M * M) / kThreads;
  constexpr int L = 4, E = M / L;
  constexpr int DPT = 8;
  __shared__ C2<Tf> s_buf[kLDS ? M * SM : 1];
  __shared__ C2<Tf> s_tw[M];
  __shared__ double s_pref[kThreads];
  __shared__ double s_red[4];
  __shared__ int s_redi[4];
  __shared__ double s_acc[4][10];
  const DevCfg& cfg = *a.cfg;
  C2<Tf>* buf = kLDS ? s_buf : (C2<Tf>*)a.scratch + (size_t)blockIdx.x * M * SM;
  const C2<Tf>* tm = (const C2<Tf>*)a.tmap;
  C2<Tg>* gt = (C2<Tg>*)a.gt;
  for (int i = threadIdx.x; i < M; i += kThreads) s_tw[i] = ((const C2<Tf>*)a.tw)[i];
  __syncthreads();
  const int N = cfg.N, P = cfg.P, t = threadIdx.x;
  const int g = t >> 2, gl = t & 3, br = bitrev(gl, 2);
  const double inv_m2 = 1.0 / ((double)M * M);
  const int H = cfg.H, W = cfg.W;
  // bilinear tile in the rows of buf that the patch adjoint leaves free
  const int free_elems = (M - P) * SM;
  int T = P + 4;
  while (T > 0 && T * T > free_elems) --T;
  const bool use_tile = T >= 4;
  for (size_t wi = blockIdx.x; wi < a.nray; wi += gridDim.x) {
    const size_t gid = a.ray0 + wi;
    if (a.st[7 * a.n_total + gid] == 0.0) continue;
    RayCtx c;
    make_ctx(a, gid, c);
    patch_spectrum<Tf, M>(cfg, c, tm, buf, s_tw);
    IncAcc acc = {{0, 0, 0}, {0, 0}, 0, 0};
    double dLdS = 0.0;
    int kk[DPT];
    C2<Tf> gX[DPT];
#pragma unroll
    for (int q = 0; q < DPT; ++q) kk[q] = -1;
    double S = 0.0;
    if (cfg.sampling != 2) {
      double accw = 0.0;
      int lastpos = -1;
      for (int q = 0; q < C; ++q) {
        const int Lb = t * C + q;
        const double wgt = bin_weight<Tf, M>(c, buf, Lb, cfg.sampling);
        accw += wgt;
        if (wgt > 0.0) lastpos = Lb;
      }
      double excl;
      S = block_exclusive_scan(accw, s_red, excl);
      s_pref[t] = excl;
      const int lastpos_all = block_max_int(lastpos, s_redi);
      if (S > 0.0) {
        const double scale = S * inv_m2 / N;
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
          const int i = t + q * kThreads;
          if (i >= N) break;
          int J = -1;
          if (a.replay) {
            J = a.replay[gid * N + i];
          } else {
            const double Tv = draw_uniform(cfg.key0, cfg.key1, (uint32_t)i, (uint32_t)c.r,
                                           (uint32_t)c.pair, 0u) * S;
            int lo = 0, hi = kThreads - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (s_pref[mid] <= Tv) lo = mid; else hi = mid - 1;
            }
            double run = s_pref[lo];
            int lp = -1;
            for (int qq = 0; qq < C; ++qq) {
              const int Lb = lo * C + qq;
              const double wgt = bin_weight<Tf, M>(c, buf, Lb, cfg.sampling);
              run += wgt;
              if (wgt > 0.0) lp = Lb;
              if (run > Tv) { J = Lb; break; }
            }
            if (J < 0) J = lp >= 0 ? lp : lastpos_all;
          }
          if (J < 0) continue;
          const int jy = J / M - M / 2, jx = J % M - M / 2;
          const int kidx = (jy & (M - 1)) * SM + (jx & (M - 1));
          const C2<Tf> X = buf[kidx];
          const C2<Tf> ref = centre_ref<Tf>(jx, jy, P, M);
          const C2<Tf> U = X * ref;
          C2<Tp> w;
          double mag = 0.0;
          if (cfg.sampling == 0) {
            const Tf m = cabs_rn(X);
            if (!(m > Tf(0))) continue;
            mag = (double)m;
            const Tp f = (Tp)(scale / mag);
            w = {(Tp)U.re * f, (Tp)U.im * f};
          } else {
            w = {(Tp)U.re * (Tp)scale, (Tp)U.im * (Tp)scale};
          }
          WaveletAdj wa;
          Secondary sec;
          if (!wavelet_adjoint<Prec>(a, c, jx, jy, w, wa, sec)) continue;
          C2<double> gU;
          if (cfg.sampling == 0) {
            // w = (S / (M^2 N)) U/|U|
            const double hr = (double)U.re / mag, hi_ = (double)U.im / mag;
            dLdS += (wa.g_w.re * hr + wa.g_w.im * hi_) * inv_m2 / N;
            const double gr = wa.g_w.re * scale, gi = wa.g_w.im * scale;   // dL/d(U/|U|)
            const double im = -(gr * hi_ - gi * hr) / mag;   // -Im(conj(g) h) / |U|
            gU = {-im * hi_, im * hr};                         // times i h
          } else {
            gU = {wa.g_w.re * scale, wa.g_w.im * scale};
          }
          // U = X ref  ->  dL/dX = conj(ref) dL/dU
          const double rr = (double)ref.re, ri = (double)ref.im;
          kk[q] = kidx;
          gX[q] = {(Tf)(rr * gU.re + ri * gU.im), (Tf)(rr * gU.im - ri * gU.re)};
          if (a.want_lens) incident_from_wavelet(a, c, sec, wa, acc);
        }
      }
      dLdS = block_sum(dLdS, s_red);    // also orders every read of buf before the rewrite
      // S-term over every propagating bin (p_mag only): dL/dX_k += dL/dS X_k / |X_k|
      for (int q = 0; q < C; ++q) {
        const int Lb = t * C + q;
        const int jy = Lb / M - M / 2, jx = Lb % M - M / 2;
        const int kidx = (jy & (M - 1)) * SM + (jx & (M - 1));
        const C2<Tf> X = buf[kidx];
        C2<Tf> v = {Tf(0), Tf(0)};
        if (cfg.sampling == 0) {
          const double wgt = bin_weight<Tf, M>(c, buf, Lb, 0);
          if (wgt > 0.0) v = {(Tf)(dLdS * X.re / wgt), (Tf)(dLdS * X.im / wgt)};
        }
        buf[kidx] = v;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < DPT; ++q) {
        if (kk[q] >= 0) {
          atomicAdd(&buf[kk[q]].re, gX[q].re);
          atomicAdd(&buf[kk[q]].im, gX[q].im);
        }
      }
    } else {
      // FULL: every propagating bin is a wavelet with weight U~ / M^2.
      for (int q = 0; q < C; ++q) {
        const int Lb = t * C + q;
        const int jy = Lb / M - M / 2, jx = Lb % M - M / 2;
        const int kidx = (jy & (M - 1)) * SM + (jx & (M - 1));
        const double Ku = c.kin_u + c.dk * jx, Kv = c.kin_v + c.dk * jy;
        C2<Tf> out = {Tf(0), Tf(0)};
        if (Ku * Ku + Kv * Kv < c.k_out * c.k_out) {
          const C2<Tf> X = buf[kidx];
          const C2<Tf> ref = centre_ref<Tf>(jx, jy, P, M);
          const C2<Tf> U = X * ref;
          const C2<Tp> w = {(Tp)U.re * (Tp)inv_m2, (Tp)U.im * (Tp)inv_m2};
          WaveletAdj wa;
          Secondary sec;
          if (wavelet_adjoint<Prec>(a, c, jx, jy, w, wa, sec)) {
            const double gr = wa.g_w.re * inv_m2, gi = wa.g_w.im * inv_m2;
            const double rr = (double)ref.re, ri = (double)ref.im;
            out = {(Tf)(rr * gr + ri * gi), (Tf)(rr * gi - ri * gr)};
            if (a.want_lens) incident_from_wavelet(a, c, sec, wa, acc);
          }
        }
        buf[kidx] = out;
      }
    }
    __syncthreads();
    // Inverse transform dL/dU[n][m] = sum_k exp(+2 pi i (k_y n + k_x m) / M) dL/dX[k]:
    // columns first (keep n < P), then rows n < P (keep m < P).
    for (int col = g; col < M; col += kThreads / L) {
      C2<Tf> x[E];
#pragma unroll
      for (int n2 = 0; n2 < E; ++n2) x[n2] = buf[(gl + L * n2) * SM + col];
      group_fft<Tf, L, E, +1>(x, gl, s_tw);
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) {
        const int n = E * br + k2;
        if (n < P) buf[n * SM + col] = x[k2];
      }
    }
    __syncthreads();
    for (int row = g; row < P; row += kThreads / L) {
      C2<Tf> x[E];
#pragma unroll
      for (int n2 = 0; n2 < E; ++n2) x[n2] = buf[row * SM + gl + L * n2];
      group_fft<Tf, L, E, +1>(x, gl, s_tw);
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) {
        const int m = E * br + k2;
        if (m < P) buf[row * SM + m] = x[k2];
      }
    }
    __syncthreads();
    // Bilinear gather adjoint: dL/dt[pixel] += w_bilinear dL/dU[n][m].
    C2<Tf>* tile = buf + P * SM;
    const double cfx = (c.p[0] - cfg.x0) / cfg.pitch, cfy = (c.p[1] - cfg.y0) / cfg.pitch;
    const int tx0 = (int)floor(cfx) - T / 2, ty0 = (int)floor(cfy) - T / 2;
    if (use_tile) {
      for (int i = t; i < T * T; i += kThreads) tile[i] = {Tf(0), Tf(0)};
      __syncthreads();
    }
    double gpx = 0.0, gpy = 0.0;
    for (int s = t; s < P * P; s += kThreads) {
      const int m = s % P, n = s / P;
      const C2<Tf> gu = buf[n * SM + m];
      const double sm = (m - (P - 1) * 0.5) * cfg.pitch;
      const double sn = (n - (P - 1) * 0.5) * cfg.pitch;
      const double qx = c.p[0] + sm * c.u[0] + sn * c.v[0];
      const double qy = c.p[1] + sm * c.u[1] + sn * c.v[1];
      const double fx = (qx - cfg.x0) / cfg.pitch, fy = (qy - cfg.y0) / cfg.pitch;
      const double flx = floor(fx), fly = floor(fy);
      const int ix = (int)flx, iy = (int)fly;
      const Tf wx = (Tf)(fx - flx), wy = (Tf)(fy - fly);
      C2<Tf> tv[2][2];
#pragma unroll
      for (int dy = 0; dy < 2; ++dy) {
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const int x = ix + dx, y = iy + dy;
          const bool in = x >= 0 && x < W && y >= 0 && y < H;
          tv[dy][dx] = (a.want_lens && in) ? tm[(size_t)y * W + x] : C2<Tf>{Tf(0), Tf(0)};
          if (!in) continue;
          const Tf wgt = (dx ? wx : Tf(1) - wx) * (dy ? wy : Tf(1) - wy);
          const C2<Tf> v = gu * wgt;
          const int lx = x - tx0, ly = y - ty0;
          if (use_tile && lx >= 0 && lx < T && ly >= 0 && ly < T) {
            atomicAdd(&tile[ly * T + lx].re, v.re);
            atomicAdd(&tile[ly * T + lx].im, v.im);
          } else {
            atomicAdd(&gt[(size_t)y * W + x].re, (Tg)v.re);
            atomicAdd(&gt[(size_t)y * W + x].im, (Tg)v.im);
          }
        }
      }
      if (a.want_lens) {
        // dU/dfx, dU/dfy of the bilinear interpolant; planar DOE: q = p + s
        const C2<Tf> dUx = (tv[0][1] - tv[0][0]) * (Tf(1) - wy) + (tv[1][1] - tv[1][0]) * wy;
        const C2<Tf> dUy = (tv[1][0] - tv[0][0]) * (Tf(1) - wx) + (tv[1][1] - tv[0][1]) * wx;
        gpx += ((double)gu.re * dUx.re + (double)gu.im * dUx.im) / cfg.pitch;
        gpy += ((double)gu.re * dUy.re + (double)gu.im * dUy.im) / cfg.pitch;
      }
    }
    if (use_tile) {
      __syncthreads();
      for (int i = t; i < T * T; i += kThreads) {
        const C2<Tf> v = tile[i];
        const int x = tx0 + i % T, y = ty0 + i / T;
        if ((v.re != Tf(0) || v.im != Tf(0)) && x >= 0 && x < W && y >= 0 && y < H) {
          atomicAdd(&gt[(size_t)y * W + x].re, (Tg)v.re);
          atomicAdd(&gt[(size_t)y * W + x].im, (Tg)v.im);
        }
      }
    }
    if (a.want_lens) {
      // ray-level cogradient of the incident state
      double v[8] = {acc.gp[0] + gpx, acc.gp[1] + gpy, acc.gp[2], acc.gkin[0], acc.gkin[1],
                     acc.gopl, acc.gzs, 0.0};
#pragma unroll
      for (int k = 0; k < 7; ++k) v[k] = wave_sum(v[k]);
      if ((t & 63) == 0)
        for (int k = 0; k < 7; ++k) s_acc[t >> 6][k] = v[k];
      __syncthreads();
      if (t == 0) {
        double r[7];
        for (int k = 0; k < 7; ++k)
          r[k] = s_acc[0][k] + s_acc[1][k] + s_acc[2][k] + s_acc[3][k];
        const DevPair& pr = a.pairs[c.pair];
        const double f = c.k0 * pr.n_med[cfg.s_doe];
        const size_t n = a.n_total;
        a.raygrad[0 * n + gid] = r[0];
        a.raygrad[1 * n + gid] = r[1];
        a.raygrad[2 * n + gid] = r[2];
        // k_in,t = k0 n_in (d.u, d.v)
        for (int i = 0; i < 3; ++i)
          a.raygrad[(3 + i) * n + gid] = f * (r[3] * c.u[i] + r[4] * c.v[i]);
        a.raygrad[6 * n + gid] = r[5];
        a.raygrad[7 * n + gid] = r[6];
      }
    }
    __syncthreads();   // buf and the tile are reused by the next ray
  }
}

// ---------------------------------------------------- dL/dt -> dphi, dA ---
template <class Tg>
__global__ void k_dmaps(const float* phase, const float* amp, const C2<Tg>* gt, float* dphi,
                        float* damp, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s, c;
  sincos((double)phase[i], &s, &c);
  const double a = amp[i];
  const double gr = gt[i].re, gi = gt[i].im;
  // t = A e^{i phi}: dL/dphi = Im(conj(t) g), dL/dA = Re(conj(e^{i phi}) g)
  dphi[i] = (float)(a * (c * gi - s * gr));
  damp[i] = (float)(c * gr + s * gi);
}

// ------------------------------------------------------- trace adjoint ---
// One surface step as a function of (p_in, d_in) and the surface's
// (z, c, k, A4, A6, A8, A10); dual numbers give its Jacobian columns.
constexpr int kNT = 13;

__global__ __launch_bounds__(256) void k_trace_bwd(const DevCfg* cfg, const DevPair* pairs,
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
    double gp[3], gd[3];
    for (int i = 0; i < 3; ++i) {
      gp[i] = raygrad[i * n_total + gid];
      gd[i] = raygrad[(3 + i) * n_total + gid];
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

__global__ void k_lens_map(const DevCfg* cfg, const DevParam* prm, const double* lensg,
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
