// Kernels of the ray-wave hybrid PSF (forward path).
//
//   k_params     lens parameters -> live prescription (one thread)
//   k_tmap       complex transmission t = A exp(i phi) of the DOE map
//   k_trace      launch + conventional refractive trace to the DOE, with
//                per-surface checkpoints of the ray state (one thread per ray)
//   (the ray-wave interface kernels live in rw_doe.h)
//   k_rec_hist / k_rec_scan / k_rec_place / k_spread_tiles   binned type-1
//                NUFFT spreading of the Eq. 2 wavelets onto the 2x grid
//   k_grid_rows / k_grid_cols   grid FFT, deconvolution, crop, |U|^2
//   k_loss_pairs / k_loss_total Eq. 5 with the closed-form alpha per PSF
#pragma once
#include "rw_common.h"
#include "rw_fft.h"

namespace rw {

constexpr int kThreads = 256;
// Forward counters: alive rays, secondaries, rays ended by cause (no hit,
// aperture, TIR, outside the DOE), secondaries lost after the DOE, evanescent
// and total spectrum bins of the alive rays, alive rays per patch class.
enum { RW_ST_ALIVE = 0, RW_ST_SEC = 1, RW_ST_NOHIT = 2, RW_ST_APER = 3, RW_ST_TIR = 4,
       RW_ST_OUTSIDE = 5, RW_ST_LOST = 6, RW_ST_EVAN = 7, RW_ST_BINS = 8, RW_ST_CLASS0 = 9,
       RW_N_STATS = 13 };

// Tt: trace; Tf: patch spectrum; Tp: optical path and wavelet phase; Tg: sensor
// grid; Te: sine / cosine of the wavelet phase after its reduction to [0, 2 pi)
// in Tp (an FP32 evaluation of a reduced angle is accurate to ~1e-7 rad).
struct PrecFP64 {
  using Tt = double; using Tf = double; using Tp = double; using Tg = double; using Te = double;
};
struct PrecMIXED {
  using Tt = double; using Tf = float; using Tp = double; using Tg = float; using Te = float;
};
struct PrecFP32 {
  using Tt = float; using Tf = float; using Tp = float; using Tg = float; using Te = float;
};

// e^{i phi} of a wavelet phase: reduced in Tp, evaluated in Te.
template <class Prec>
__device__ __forceinline__ C2<typename Prec::Tp> wavelet_cis(typename Prec::Tp phi) {
  using Te = typename Prec::Te;
  using Tp = typename Prec::Tp;
  Te s, c;
  sincos_any((Te)wrap_2pi(phi), &s, &c);
  return {(Tp)c, (Tp)s};
}

// Gradient modes of the draws (the values of the C ABI's RW_GRAD_*): frozen
// draws (G1), Gumbel-softmax straight-through (G2), frozen draws with the
// sampling density held constant (G1 with p detached).
enum { kGradG1 = 0, kGradG2 = 1, kGradG1Detach = 2 };

struct DevCfg {
  int n_surf, s_doe, n_pairs, n_field, R, R2, P, M, N, Q, nf, w, sampling, H, W, n_params;
  int planar;              // DOE surface is a plane z = const: u = x, v = y, n = z
  double pitch, x0, y0, launch_z, launch_half, psf_pitch, beta;
  double inv_pitch;
  uint32_t key0, key1;
  int grad;                // gradient mode (kGrad*)
  double tau;              // G2 temperature
  int pad;                 // M / P
  int n_class;             // patch classes (1: every ray uses P)
  int class_p[4];          // candidate patch sides, largest first (class_p[0] = P)
  int class_n[4];          // draws per ray of each class (N, or N (P_k / P_0)^2)
  double curv_eps;         // curvature bound of the class rule
  double bw_k2;            // adaptive patch sizing: (2 pi K)^2 for K local periods (0: off)
  int reflective;          // secondaries leave back into the medium before the DOE
  int ns_idx;              // n_med index of the medium at the sensor
  int relay_n1;            // first DOE of a cascade: side of each ray's block of relayed
                           // secondaries on the second DOE's ray grid (0: no cascade)
};

struct DevPair {
  double lam, k0;
  double dir[3];
  double lc[2];            // launch centre
  double pc[2];            // PSF centre
  double n_med[RW_MAX_SURF + 1];   // n_med[s] = index before surface s; n_med[n_surf] at the sensor
};

struct DevParam { int surface, field; double scale; };

struct DevLive {
  DevSurf s[RW_MAX_SURF];
  double sensor_z;
};

// ----------------------------------------------------------- block scans ---
// Exclusive prefix over the 256 threads of a block; returns the total.
__device__ __forceinline__ double block_exclusive_scan(double v, double* s_tmp /*[4]*/,
                                                       double& excl) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double n = __shfl_up(inc, o, 64);
    if (lane >= o) inc += n;
  }
  if (lane == 63) s_tmp[wv] = inc;
  __syncthreads();
  double base = 0.0, tot = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i < wv) base += s_tmp[i];
    tot += s_tmp[i];
  }
  excl = base + inc - v;
  __syncthreads();
  return tot;
}

__device__ __forceinline__ double block_sum(double v, double* s_tmp /*[4]*/) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) s_tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
  __syncthreads();
  return t;
}

__device__ __forceinline__ int block_max_int(int v, int* s_tmp /*[4]*/) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) s_tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  const int t = max(max(s_tmp[0], s_tmp[1]), max(s_tmp[2], s_tmp[3]));
  __syncthreads();
  return t;
}

// -------------------------------------------------------------- k_params ---
static __global__ void k_params(const DevCfg* cfg, const DevSurf* base, double base_sensor_z,
                         const DevParam* prm, const float* values, DevLive* live) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int S = cfg->n_surf;
  double gap[RW_MAX_SURF];
  DevLive L;
  for (int s = 0; s < S; ++s) {
    L.s[s] = base[s];
    gap[s] = (s + 1 < S ? base[s + 1].z : base_sensor_z) - base[s].z;
  }
  for (int i = 0; i < cfg->n_params; ++i) {
    const double v = prm[i].scale * (double)values[i];
    DevSurf& s = L.s[prm[i].surface];
    switch (prm[i].field) {
      case 0: s.c = v; break;
      case 1: s.k = v; break;
      case 2: s.A4 = v; break;
      case 3: s.A6 = v; break;
      case 4: s.A8 = v; break;
      case 5: s.A10 = v; break;
      case 6: gap[prm[i].surface] = v; break;
    }
  }
  double z = base[0].z;
  for (int s = 0; s < S; ++s) {
    L.s[s].z = z;
    z += gap[s];
  }
  L.sensor_z = z;
  *live = L;
}

// ---------------------------------------------------------------- k_tmap ---
template <class Tf>
__global__ void k_tmap(const float* phase, const float* amp, C2<Tf>* tmap, int n, int two_phase) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Tf s, c;
  sincos_any((Tf)phase[i], &s, &c);
  if (two_phase) {                     // e^{i phi1} + e^{i phi2}, phi2 in the second map
    Tf s2, c2;
    sincos_any((Tf)amp[i], &s2, &c2);
    tmap[i] = {c + c2, s + s2};
    return;
  }
  const Tf a = (Tf)amp[i];
  tmap[i] = {a * c, a * s};
}

template <class T>
__global__ void k_zero(T* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = T(0);
}

// --------------------------------------------------------------- k_trace ---
// Ray state layout: st[c * n_total + ray], c = px, py, pz, dx, dy, dz, opl, alive.
// Checkpoint s (state entering surface s, s = 0..s_doe) at ck[(s * 8 + c) * n_total + ray].
// One count per wave and cause: the lanes whose ray ended by that cause.
__device__ __forceinline__ void count_cause(unsigned long long* stats, int mine) {
  for (int c = RW_ST_NOHIT; c <= RW_ST_OUTSIDE; ++c) {
    const unsigned long long m = __ballot(mine == c);
    if (m && (threadIdx.x & 63) == 0) atomicAdd(&stats[c], (unsigned long long)__popcll(m));
  }
}

template <class Tt>
__global__ __launch_bounds__(256) void k_trace(const DevCfg* cfg, const DevPair* pairs,
                                               const DevLive* live, double* st, double* ck,
                                               size_t n_total, int pair0, int npairs,
                                               unsigned long long* stats) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int R = cfg->R, R2 = cfg->R2;
  const bool in_range = idx < (size_t)npairs * R2;
  int cause = -1;
  if (in_range) {
    const int pair = pair0 + (int)(idx / R2);
    const int r = (int)(idx % R2);
    const size_t gid = (size_t)pair * R2 + r;
    const DevPair& pr = pairs[pair];
    const int ix = r % R, iy = r / R;
    const double gx = ((ix + 0.5) / R) * 2.0 - 1.0, gy = ((iy + 0.5) / R) * 2.0 - 1.0;
    Tt p[3] = {(Tt)(pr.lc[0] + gx * cfg->launch_half), (Tt)(pr.lc[1] + gy * cfg->launch_half),
               (Tt)cfg->launch_z};
    Tt d[3] = {(Tt)pr.dir[0], (Tt)pr.dir[1], (Tt)pr.dir[2]};
    Tt opl = d[0] * p[0] + d[1] * p[1] + d[2] * p[2];
    bool alive = true;
    const int sd = cfg->s_doe;
    for (int s = 0; s <= sd; ++s) {
      double* c = ck + (size_t)s * 8 * n_total;
      c[0 * n_total + gid] = p[0]; c[1 * n_total + gid] = p[1]; c[2 * n_total + gid] = p[2];
      c[3 * n_total + gid] = d[0]; c[4 * n_total + gid] = d[1]; c[5 * n_total + gid] = d[2];
      c[6 * n_total + gid] = opl; c[7 * n_total + gid] = alive ? 1.0 : 0.0;
      if (!alive) break;
      const DevSurf& ds = live->s[s];
      const Surf<Tt> sf = surf_of<Tt>(ds);
      Tt t;
      if (!intersect(sf, p, d, t)) { alive = false; cause = RW_ST_NOHIT; break; }
  #pragma unroll
      for (int i = 0; i < 3; ++i) p[i] += t * d[i];
      opl += (Tt)pr.n_med[s] * t;
      if (ds.semi_ap > 0 && (double)(p[0] * p[0] + p[1] * p[1]) > ds.semi_ap * ds.semi_ap) {
        alive = false; cause = RW_ST_APER; break;
      }
      if (s == sd) break;
      Tt nrm[3];
      surface_normal(sf, p[0], p[1], nrm);
      if (!refract(d, nrm, (Tt)(pr.n_med[s] / pr.n_med[s + 1]))) {
        alive = false; cause = RW_ST_TIR; break;
      }
    }
    if (alive) {
      const double fx = ((double)p[0] - cfg->x0) / cfg->pitch;
      const double fy = ((double)p[1] - cfg->y0) / cfg->pitch;
      alive = fx >= -0.5 && fx <= cfg->W - 0.5 && fy >= -0.5 && fy <= cfg->H - 0.5;
      if (!alive) cause = RW_ST_OUTSIDE;
    }
    st[0 * n_total + gid] = p[0]; st[1 * n_total + gid] = p[1]; st[2 * n_total + gid] = p[2];
    st[3 * n_total + gid] = d[0]; st[4 * n_total + gid] = d[1]; st[5 * n_total + gid] = d[2];
    st[6 * n_total + gid] = opl; st[7 * n_total + gid] = alive ? 1.0 : 0.0;
  }
  if (stats) count_cause(stats, cause);
}

// NaN / Inf anywhere in the inputs of a forward (flag[0] set to 1).
static __global__ void k_check_finite(const float* a, size_t na, const float* b, size_t nb,
                                      const float* c, size_t nc, const float* d, size_t nd,
                                      unsigned int* flag) {
  const size_t n = na + nb + nc + nd;
  bool bad = false;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    float v;
    if (i < na) v = a[i];
    else if (i < na + nb) v = b[i - na];
    else if (i < na + nb + nc) v = c[i - na - nb];
    else v = d[i - na - nb - nc];
    bad |= !isfinite(v);
  }
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

// ------------------------------------------------------------- DOE stage ---
struct RayCtx;

struct DoeArgs {
  const DevCfg* cfg;
  const DevPair* pairs;
  const DevLive* live;
  const double* st;
  size_t n_total;
  const void* tmap;          // C2<Tf> [H][W]
  const void* tw;            // C2<Tf> [M] exp(-2 pi i m / M)
  void* grid;                // C2<Tg> [n_pairs][nf][nf]
  void* rec_pos;             // RecPos<Tg> [n_slots][2]  (n_slots = rays x emit)
  void* rec_val;             // C2<Tg> [n_slots]
  int emit;                  // record slots per ray: N, or M*M in FULL sampling
  void* scratch;             // C2<Tf> per block [M][M+1] when the patch does not fit in LDS
  const int32_t* replay;
  int32_t* idx_out;
  unsigned long long* stats; // [0] alive rays, [1] secondaries
  unsigned long long* wctr;  // DOE work-item counters, one per XCD (zero at launch)
  size_t ray0, nray;         // rays [ray0, ray0 + nray) of the global order
  // backward-only
  const void* adj;           // C2<Tg> adjoint grid
  void* gt;                  // C2<Tg> [H][W] cogradient of t
  double* raygrad;           // [RW_RAYGRAD][n_total] cogradients of the incident state
  double* lensg;             // per-surface sums of the lens-parameter cogradient
  int want_lens;
  void* acc;                 // C2<Tg> [blocks][acc_side][acc_side] block-private dL/dt
  int acc_side;
  RayCtx* ctx;               // [n_total] frame and wavevectors at the DOE hit (alive rays)
  void* dlist;               // per block [N]: (bin, spectrum cogradient) of each draw
  const void* interp;        // C2<Tg> [n_slots][4] sensor-grid cogradient at each record (+ pad)
                             // (value, d/dx, d/dy), or null: interpolate in the kernel
  void* g2;                  // G2 per block: double [N][8] draw data, then [M*M] dL/dlog p
  unsigned char* ray_class;  // [n_total] patch class of every ray (0 for dead rays)
  int32_t* jdraw;            // [n_total][N] bins drawn by the forward (read by the backward)
  int full;                  // FULL sampling (every propagating bin, no draws)
  int cls;                   // class processed by this launch
  // two-DOE cascade
  double* relay;             // first DOE: ray state [10][relay_n] of the second DOE's
                             // incident rays (p, d, opl, alive, amplitude re, im), or null
  size_t relay_n;
  const DevCfg* cfg2;        // first DOE: the second DOE's configuration
  const double* ain;         // second DOE: incident amplitudes [2][n_total] (re, im), or null
  double* gain;              // backward: dL/d(incident amplitude) of the second DOE's rays
                             // [2][n_total of the second DOE] (written by its adjoint, read
                             // by the first DOE's as its draws' weight cogradients)
  const float* phase;        // the phase map [H][W] (adaptive patch sizing)
};

// Amplitude of a ray whose patch side is P: (P_0 / P)^2, P_0 the largest patch
// class side.  The rays' patches cover the DOE uniformly (Formalism), so on one
// ray grid every part of the DOE counts equally whatever the side of the
// patches over it.  A power of two (the sides are M / pad with M a power of two).
__device__ __forceinline__ double class_weight(const DevCfg& cfg, int P) {
  const double r = (double)cfg.class_p[0] / (double)P;
  return r * r;
}

// Frame and incident tangential wavevector at the DOE hit (double).
struct RayCtx {
  double p[3], d[3], opl;
  double u[3], v[3], n[3];
  double kin_u, kin_v, k0, k_out, n_in, n_out, dk, k2out;
  double S;                 // sampling normaliser (sum of weights), set by the forward
  double sgn;               // +1, or -1 after a reflective DOE (normal component flipped)
  int pair, r;
  int P, cls;               // patch side and class of this ray
  size_t gid;
};
constexpr int kCtxWords = (int)(sizeof(RayCtx) / 4);

// Adaptive patch sizing: |grad phi|^2 at the map pixel nearest (x, y), the pixel
// clamped one away from the edge; each axis takes the mean of its two one-pixel
// phase differences wrapped to [-pi, pi].  Every operation is rounded on its own
// (no contraction), so that the class decision is the oracle's.
__device__ __forceinline__ double wrap_phase(double d) {
  const double tp = 2.0 * RW_PI;
  return __dsub_rn(d, __dmul_rn(tp, rint(__ddiv_rn(d, tp))));
}

__device__ __forceinline__ double local_phase_gradient2(const float* ph, const DevCfg& cfg,
                                                        double x, double y) {
  const int W = cfg.W, H = cfg.H;
  const int jx = (int)fmin(fmax(rint(__ddiv_rn(__dsub_rn(x, cfg.x0), cfg.pitch)), 1.0), W - 2.0);
  const int jy = (int)fmin(fmax(rint(__ddiv_rn(__dsub_rn(y, cfg.y0), cfg.pitch)), 1.0), H - 2.0);
  const double c = ph[(size_t)jy * W + jx];
  const double two_p = __dmul_rn(2.0, cfg.pitch);
  const double gx = __ddiv_rn(__dadd_rn(wrap_phase(__dsub_rn((double)ph[(size_t)jy * W + jx + 1], c)),
                                        wrap_phase(__dsub_rn(c, (double)ph[(size_t)jy * W + jx - 1]))),
                              two_p);
  const double gy = __ddiv_rn(__dadd_rn(wrap_phase(__dsub_rn((double)ph[(size_t)(jy + 1) * W + jx], c)),
                                        wrap_phase(__dsub_rn(c, (double)ph[(size_t)(jy - 1) * W + jx]))),
                              two_p);
  return __dadd_rn(__dmul_rn(gx, gx), __dmul_rn(gy, gy));
}

__device__ __forceinline__ void make_ctx(const DoeArgs& a, size_t gid, RayCtx& c) {
  const DevCfg& cfg = *a.cfg;
  c.gid = gid;
  c.pair = (int)(gid / cfg.R2);
  c.r = (int)(gid % cfg.R2);
  const size_t n = a.n_total;
  for (int i = 0; i < 3; ++i) { c.p[i] = a.st[i * n + gid]; c.d[i] = a.st[(3 + i) * n + gid]; }
  c.opl = a.st[6 * n + gid];
  const DevPair& pr = a.pairs[c.pair];
  const DevSurf& sd = a.live->s[cfg.s_doe];
  const Surf<double> sf = surf_of<double>(sd);
  surface_normal(sf, c.p[0], c.p[1], c.n);
  // u = normalised projection of the global x axis on the tangent plane, v = n x u
  double ux = 1.0 - c.n[0] * c.n[0], uy = -c.n[0] * c.n[1], uz = -c.n[0] * c.n[2];
  const double iu = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
  c.u[0] = ux * iu; c.u[1] = uy * iu; c.u[2] = uz * iu;
  c.v[0] = c.n[1] * c.u[2] - c.n[2] * c.u[1];
  c.v[1] = c.n[2] * c.u[0] - c.n[0] * c.u[2];
  c.v[2] = c.n[0] * c.u[1] - c.n[1] * c.u[0];
  c.k0 = pr.k0;
  c.n_in = pr.n_med[cfg.s_doe];
  // a reflective DOE sends its secondaries back into the medium before it
  c.n_out = cfg.reflective ? c.n_in : pr.n_med[cfg.s_doe + 1];
  c.sgn = cfg.reflective ? -1.0 : 1.0;
  c.k_out = c.k0 * c.n_out;
  c.kin_u = c.k0 * c.n_in * (c.d[0] * c.u[0] + c.d[1] * c.u[1] + c.d[2] * c.u[2]);
  c.kin_v = c.k0 * c.n_in * (c.d[0] * c.v[0] + c.d[1] * c.v[1] + c.d[2] * c.v[2]);
  // patch class (Eq. 4): the largest candidate side D = P pitch with
  // arcsin(D / 2 R_loc) <= eps at the hit, else the smallest
  c.cls = 0;
  if (cfg.n_class > 1) {
    const double Rl = local_radius(sf, c.p[0], c.p[1]);
    c.cls = cfg.n_class - 1;
    for (int k = 0; k < cfg.n_class; ++k) {
      const double D = cfg.class_p[k] * cfg.pitch;
      if (isinf(Rl) || (D <= 2.0 * Rl && asin(D / (2.0 * Rl)) <= cfg.curv_eps)) {
        c.cls = k;
        break;
      }
    }
    if (cfg.bw_k2 > 0.0) {
      // adaptive patch sizing: the smallest side spanning K local periods of the
      // phase map (the largest where the map is flatter); the smaller side of
      // this rule and the curvature bound wins
      const double g2 = local_phase_gradient2(a.phase, cfg, c.p[0], c.p[1]);
      int kb = 0;
      for (int k = cfg.n_class - 1; k >= 0; --k) {
        const double D = __dmul_rn((double)cfg.class_p[k], cfg.pitch);
        if (__dmul_rn(__dmul_rn(D, D), g2) >= cfg.bw_k2) {
          kb = k;
          break;
        }
      }
      if (kb > c.cls) c.cls = kb;
    }
  }
  c.P = cfg.class_p[c.cls];
  c.dk = 2.0 * RW_PI / ((double)cfg.pad * c.P * cfg.pitch);
  c.k2out = __dmul_rn(c.k_out, c.k_out);
  c.S = 0.0;
}

// Context of every alive ray of [ray0, ray0 + nray), one thread per ray.
static __global__ __launch_bounds__(256) void k_ray_ctx(DoeArgs a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nray) return;
  const size_t gid = a.ray0 + i;
  if (a.st[7 * a.n_total + gid] == 0.0) {
    a.ray_class[gid] = 0;
    return;
  }
  RayCtx c;
  make_ctx(a, gid, c);
  a.ctx[gid] = c;
  a.ray_class[gid] = (unsigned char)c.cls;
}

// Copy of a ray's context into shared memory by the first kCtxWords threads
// (the caller synchronises).
__device__ __forceinline__ void load_ctx(const DoeArgs& a, size_t gid, RayCtx& dst) {
  if (threadIdx.x < kCtxWords)
    reinterpret_cast<uint32_t*>(&dst)[threadIdx.x] =
        reinterpret_cast<const uint32_t*>(a.ctx + gid)[threadIdx.x];
}


// Exponential-of-semicircle spreading kernel psi(z) = exp(beta (sqrt(1 - (2z/w)^2) - 1)).
template <class Tg>
__device__ __forceinline__ Tg es_kernel(Tg z, Tg two_over_w, Tg beta) {
  const Tg t = z * two_over_w;
  const Tg a = Tg(1) - t * t;
  return a > Tg(0) ? (Tg)exp(beta * (sqrt(a) - Tg(1))) : Tg(0);
}

struct Secondary {          // one weighted secondary ray at the sensor
  double dsx, dsy, dsz;     // direction after the DOE (for the adjoint)
  double Ku, Kv, kz;
  bool ok;
};

// Emission (direction from the tangential wavevector), conventional trace to the
// sensor, and the Eq. 2 phase / frequencies of the wavelet.
template <class Prec>
__device__ __forceinline__ bool secondary_to_sensor(const DoeArgs& a, const RayCtx& c, int jx,
                                                    int jy, typename Prec::Tp& phi0,
                                                    typename Prec::Tp& wx, typename Prec::Tp& wy,
                                                    double& dz_abs, Secondary& sec) {
  using Tt = typename Prec::Tt;
  using Tp = typename Prec::Tp;
  const DevCfg& cfg = *a.cfg;
  const DevPair& pr = a.pairs[c.pair];
  const double Ku = c.kin_u + c.dk * jx, Kv = c.kin_v + c.dk * jy;
  const double kz2 = c.k_out * c.k_out - Ku * Ku - Kv * Kv;
  if (!(kz2 > 0.0)) return false;
  const double kz = sqrt(kz2);
  const double ik = 1.0 / c.k_out;
  Tt d[3], p[3];
  const double skz = c.sgn * kz;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    d[i] = (Tt)((Ku * c.u[i] + Kv * c.v[i] + skz * c.n[i]) * ik);
    p[i] = (Tt)c.p[i];
  }
  sec.Ku = Ku; sec.Kv = Kv; sec.kz = kz;
  sec.dsx = (double)d[0]; sec.dsy = (double)d[1]; sec.dsz = (double)d[2];
  Tt opl = (Tt)c.opl;
  for (int s = cfg.s_doe + 1; s < cfg.n_surf; ++s) {
    const DevSurf& ds = a.live->s[s];
    const Surf<Tt> sf = surf_of<Tt>(ds);
    Tt t;
    if (!intersect(sf, p, d, t)) return false;
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] += t * d[i];
    opl += (Tt)pr.n_med[s] * t;
    if (ds.semi_ap > 0 && (double)(p[0] * p[0] + p[1] * p[1]) > ds.semi_ap * ds.semi_ap) return false;
    Tt nrm[3];
    surface_normal(sf, p[0], p[1], nrm);
    if (!refract(d, nrm, (Tt)(pr.n_med[s] / pr.n_med[s + 1]))) return false;
  }
  const Tt zs = (Tt)a.live->sensor_z;
  const Tt t = (zs - p[2]) / d[2];
  if (!(t > Tt(0))) return false;
  const Tt ns = (Tt)pr.n_med[cfg.ns_idx];
#pragma unroll
  for (int i = 0; i < 3; ++i) p[i] += t * d[i];
  opl += ns * t;
  const Tp k0 = (Tp)c.k0;
  const Tp dr = (Tp)d[0] * ((Tp)pr.pc[0] - (Tp)p[0]) + (Tp)d[1] * ((Tp)pr.pc[1] - (Tp)p[1]) +
                (Tp)d[2] * ((Tp)zs - (Tp)p[2]);
  phi0 = k0 * ((Tp)opl + (Tp)ns * dr);
  wx = k0 * (Tp)ns * (Tp)cfg.psf_pitch * (Tp)d[0];
  wy = k0 * (Tp)ns * (Tp)cfg.psf_pitch * (Tp)d[1];
  dz_abs = fabs((double)d[2]);
  sec.ok = true;
  return true;
}

// ---------------------------------------------------------- DOE cascade ---
// Two DOEs in sequence: a secondary of the first DOE is traced to the second
// DOE's surface, where it is an incident ray whose complex amplitude is its
// Eq. 1 weight and whose phase is its optical path.  Secondary i of ray
// (iy, ix) of the first DOE's launch grid becomes ray
// (iy n1 + i / n1, ix n1 + i % n1) of the second DOE's grid of side R n1.
__device__ __forceinline__ size_t relay_gid(const DevCfg& cfg, const DevCfg& c2, int pair, int r,
                                            int i) {
  const int n1 = cfg.relay_n1;
  const int iy = r / cfg.R, ix = r % cfg.R;
  return (size_t)pair * c2.R2 + (size_t)(iy * n1 + i / n1) * c2.R + (size_t)(ix * n1 + i % n1);
}

__device__ __forceinline__ void relay_put(const DoeArgs& a, size_t g, const double* p,
                                          const double* d, double opl, double are, double aim) {
  double* st = a.relay;
  const size_t n = a.relay_n;
#pragma unroll
  for (int k = 0; k < 3; ++k) { st[k * n + g] = p[k]; st[(3 + k) * n + g] = d[k]; }
  st[6 * n + g] = opl;
  st[7 * n + g] = 1.0;
  st[8 * n + g] = are;
  st[9 * n + g] = aim;
}

// A relay slot that carries no ray (dead incident ray, failed draw or trace).
__device__ __forceinline__ void relay_none(const DoeArgs& a, int pair, int r, int i) {
  const size_t g = relay_gid(*a.cfg, *a.cfg2, pair, r, i);
  const size_t n = a.relay_n;
  double* st = a.relay;
#pragma unroll
  for (int k = 0; k < 10; ++k) st[k * n + g] = k == 5 ? 1.0 : 0.0;
}

// Emission of the first DOE's secondary (jx, jy) with weight w, conventional
// trace through the surfaces between the DOEs (refracting) to the second DOE's
// surface (intersected only; its map is the stop), and the relay record.
template <class Prec>
__device__ __forceinline__ bool relay_secondary(const DoeArgs& a, const RayCtx& c, int jx, int jy,
                                                double wre, double wim, int i) {
  using Tt = typename Prec::Tt;
  const DevCfg& cfg = *a.cfg;
  const DevCfg& c2 = *a.cfg2;
  const DevPair& pr = a.pairs[c.pair];
  const double Ku = c.kin_u + c.dk * jx, Kv = c.kin_v + c.dk * jy;
  const double kz2 = c.k_out * c.k_out - Ku * Ku - Kv * Kv;
  bool ok = kz2 > 0.0;
  Tt d[3], p[3];
  Tt opl = (Tt)c.opl;
  if (ok) {
    const double kz = sqrt(kz2), ik = 1.0 / c.k_out;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      d[k] = (Tt)((Ku * c.u[k] + Kv * c.v[k] + kz * c.n[k]) * ik);
      p[k] = (Tt)c.p[k];
    }
    for (int s = cfg.s_doe + 1; s <= c2.s_doe; ++s) {
      const DevSurf& ds = a.live->s[s];
      const Surf<Tt> sf = surf_of<Tt>(ds);
      Tt t;
      if (!intersect(sf, p, d, t)) { ok = false; break; }
#pragma unroll
      for (int k = 0; k < 3; ++k) p[k] += t * d[k];
      opl += (Tt)pr.n_med[s] * t;
      if (ds.semi_ap > 0 && (double)(p[0] * p[0] + p[1] * p[1]) > ds.semi_ap * ds.semi_ap) {
        ok = false;
        break;
      }
      if (s == c2.s_doe) break;
      Tt nrm[3];
      surface_normal(sf, p[0], p[1], nrm);
      if (!refract(d, nrm, (Tt)(pr.n_med[s] / pr.n_med[s + 1]))) { ok = false; break; }
    }
    if (ok) {
      const double fx = ((double)p[0] - c2.x0) / c2.pitch;
      const double fy = ((double)p[1] - c2.y0) / c2.pitch;
      ok = fx >= -0.5 && fx <= c2.W - 0.5 && fy >= -0.5 && fy <= c2.H - 0.5;
    }
  }
  if (!ok) {
    relay_none(a, c.pair, c.r, i);
    return false;
  }
  const double pd[3] = {(double)p[0], (double)p[1], (double)p[2]};
  const double dd[3] = {(double)d[0], (double)d[1], (double)d[2]};
  relay_put(a, relay_gid(cfg, c2, c.pair, c.r, i), pd, dd, (double)opl, wre, wim);
  return true;
}

// Grid coordinate (in cells, [0, nf)) of a wavelet frequency.
template <class Tp>
__device__ __forceinline__ Tp grid_coord(Tp w, int nf) {
  const Tp turns = w * (Tp)(1.0 / (2.0 * RW_PI));
  return (turns - floor(turns)) * (Tp)nf;
}

// Secondary-ray record for the binned spreading: wavelet value and its grid
// coordinate as fixed-point turns (2^32 per period; 2^64 in the FP64 form).
template <class Tg> struct RecPos;
template <> struct RecPos<float> { using T = uint32_t; };
template <> struct RecPos<double> { using T = unsigned long long; };

template <class Tp, class U>
__device__ __forceinline__ U to_turns(Tp w) {
  const Tp turns = w * (Tp)(1.0 / (2.0 * RW_PI));
  const Tp frac = turns - floor(turns);                 // [0, 1]
  if constexpr (sizeof(U) == 4) {
    const uint64_t v = (uint64_t)((double)frac * 4294967296.0);
    return (U)(v & 0xffffffffull);
  } else {
    // 2^64 fixed point from a double in [0, 1]: 53 significant bits
    const double hi = (double)frac * 4294967296.0;
    const uint64_t h = (uint64_t)hi;
    const uint64_t l = (uint64_t)((hi - (double)h) * 4294967296.0);
    return (U)((h << 32) + l);
  }
}

template <class U> __device__ __forceinline__ double turns_to_cells(U v, int nf) {
  if constexpr (sizeof(U) == 4) return (double)v * ((double)nf / 4294967296.0);
  else return ((double)(v >> 11)) * ((double)nf / 9007199254740992.0);
}

template <class Prec>
__device__ __forceinline__ void put_record(const DoeArgs& a, size_t slot,
                                           C2<typename Prec::Tg> v, typename Prec::Tp wx,
                                           typename Prec::Tp wy) {
  using Tg = typename Prec::Tg;
  using U = typename RecPos<Tg>::T;
  U* pos = (U*)a.rec_pos;
  pos[2 * slot] = to_turns<typename Prec::Tp, U>(wx);
  pos[2 * slot + 1] = to_turns<typename Prec::Tp, U>(wy);
  ((C2<Tg>*)a.rec_val)[slot] = v;
}

// A slot that carries no secondary ray (dead incident ray, failed emission,
// evanescent FULL bin) holds a NaN value; binning skips it.  A valid ray keeps
// its record even when its value is exactly zero, so that the adjoint finds it.
template <class Tg>
__device__ __forceinline__ void put_none(const DoeArgs& a, size_t slot) {
  ((C2<Tg>*)a.rec_val)[slot] = {(Tg)NAN, (Tg)NAN};
}
template <class Tg> __device__ __forceinline__ bool is_none(const C2<Tg>& v) { return v.re != v.re; }

// Angle reference of the patch centre: U~_j = X_k exp(i pi (jx + jy)(P - 1) / M).
template <class Tf>
__device__ __forceinline__ C2<Tf> centre_ref(int jx, int jy, int P, int M) {
  int num = ((jx + jy) * (P - 1)) % (2 * M);
  if (num < 0) num += 2 * M;
  Tf s, c;
  sincospi_any((Tf)num / (Tf)M, &s, &c);
  return {c, s};
}

// ------------------------------------------------------- binned spreading ---
// Records are binned by (pair, BIN x BIN cells of the oversampled grid); one
// workgroup per TILE x TILE cells (TILE = 4 BIN) gathers the records of its own
// bins and of a one-bin margin (w / 2 <= BIN), accumulates the ES-kernel taps
// that fall inside its tile in LDS, and stores the tile: no global atomics.
//
// Bin keys run over super-bins of SB x SB bins (SB = 1 << sshift), bins of one
// super-bin contiguous, so the counting sort can go in two passes that both
// write long runs: records to their super-bin, then each super-bin's records to
// their bins (a one-pass scatter over all bins of a pair writes a few records
// per bin and workgroup, each its own partial line).
struct BinGeom {
  int nf, bin, shift;      // BIN = 1 << shift cells
  int nb;                  // bins per axis
  int keys;                // bins per pair
  int sshift;              // super-bin side = 1 << sshift bins (<= nb)
};

constexpr int kMaxSuper = 64;  // super-bins per pair

__host__ __device__ __forceinline__ int bin_key(int by, int bx, const BinGeom& g) {
  const int sm = (1 << g.sshift) - 1, ns = g.nb >> g.sshift;
  return ((((by >> g.sshift) * ns + (bx >> g.sshift)) << g.sshift | (by & sm)) << g.sshift) |
         (bx & sm);
}

__device__ __forceinline__ int rec_key(double gx, double gy, const BinGeom& g) {
  const int cx = min((int)gx, g.nf - 1), cy = min((int)gy, g.nf - 1);
  return bin_key(cy >> g.shift, cx >> g.shift, g);
}

template <class Tg>
__global__ __launch_bounds__(256) void k_rec_hist(const void* rec_pos, const void* rec_val,
                                                  size_t per_pair, int chunk, BinGeom g,
                                                  int pair0, unsigned int* counts) {
  using U = typename RecPos<Tg>::T;
  extern __shared__ unsigned int s_h[];
  const int pair_l = blockIdx.y;
  const size_t base = (size_t)pair_l * per_pair + (size_t)blockIdx.x * chunk;
  const size_t end = min(base + (size_t)chunk, (size_t)(pair_l + 1) * per_pair);
  for (int i = threadIdx.x; i < g.keys; i += blockDim.x) s_h[i] = 0;
  __syncthreads();
  const U* pos = (const U*)rec_pos;
  const C2<Tg>* val = (const C2<Tg>*)rec_val;
  for (size_t r = base + threadIdx.x; r < end; r += blockDim.x) {
    const C2<Tg> v = val[r];
    if (is_none(v)) continue;
    const int k = rec_key(turns_to_cells(pos[2 * r], g.nf), turns_to_cells(pos[2 * r + 1], g.nf), g);
    atomicAdd(&s_h[k], 1u);
  }
  __syncthreads();
  unsigned int* out = counts + (size_t)(pair0 + pair_l) * g.keys;
  for (int i = threadIdx.x; i < g.keys; i += blockDim.x)
    if (s_h[i]) atomicAdd(&out[i], s_h[i]);
}

// Exclusive scan of the bin counts (one workgroup); cursors start at the offsets,
// and the cursor of each super-bin (fpc bins) at its first bin's offset.  Then
// the work list of the second sort pass: work[i] = first workgroup of super-bin
// i (pair-major), each super-bin taking ceil(count / chunk) workgroups.
static __global__ __launch_bounds__(1024) void k_rec_scan(const unsigned int* counts, size_t n,
                                                   int fpc, int chunk,
                                                   unsigned long long* offsets,
                                                   unsigned long long* cursor,
                                                   unsigned long long* scursor,
                                                   unsigned int* work) {
  __shared__ unsigned long long s_w[16];
  __shared__ unsigned long long s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  auto block_scan = [&](unsigned long long v, unsigned long long& pre_out) {
    unsigned long long inc = v;
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long x = __shfl_up(inc, o, 64);
      if (lane >= o) inc += x;
    }
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    unsigned long long pre = s_carry;
    for (int k = 0; k < wv; ++k) pre += s_w[k];
    pre_out = pre + inc - v;
    __syncthreads();
    if (threadIdx.x == 1023) {
      unsigned long long tot = s_carry;
      for (int k = 0; k < 16; ++k) tot += s_w[k];
      s_carry = tot;
    }
    __syncthreads();
  };
  for (size_t b0 = 0; b0 < n; b0 += 1024) {
    const size_t i = b0 + threadIdx.x;
    unsigned long long ex;
    block_scan(i < n ? counts[i] : 0ull, ex);
    if (i < n) {
      offsets[i] = ex;
      cursor[i] = ex;
      if (i % fpc == 0) scursor[i / fpc] = ex;
    }
  }
  if (threadIdx.x == 0) { offsets[n] = s_carry; s_carry = 0; }
  __syncthreads();                       // offsets visible to the whole workgroup
  const size_t ns = n / fpc;
  for (size_t b0 = 0; b0 < ns; b0 += 1024) {
    const size_t i = b0 + threadIdx.x;
    unsigned long long nch = 0;
    if (i < ns) nch = (offsets[(i + 1) * fpc] - offsets[i * fpc] + chunk - 1) / chunk;
    unsigned long long ex;
    block_scan(nch, ex);
    if (i < ns) work[i] = (unsigned int)ex;
  }
  if (threadIdx.x == 0) work[ns] = (unsigned int)s_carry;
}

// Records per workgroup of either sort pass.
template <class Tg> struct RecChunk { static constexpr int C = sizeof(Tg) == 4 ? 2048 : 1024; };

// One counting-sort pass over a chunk of records.  kSuper: the records of a
// chunk of slots of one pair go to their super-bin (skipping empty slots; the
// slot goes along as the record's index when dst_idx is given).  Otherwise: a
// chunk of one super-bin's records (work-list item) goes to its bins.  The
// chunk is ranked by key in LDS (one atomic per record), every key reserves its
// range with one global atomic, and the chunk is staged in LDS in key order, so
// that each wave stores runs of consecutive records: whole lines, where the
// direct scatter of a record at a time left a partial line per record.
template <class Tg, bool kSuper>
__global__ __launch_bounds__(256) void k_rec_place(const void* src_pos, const void* src_val,
                                                   const unsigned int* src_idx, size_t per_pair,
                                                   const unsigned long long* offsets,
                                                   const unsigned int* work, BinGeom g,
                                                   int pair0, unsigned long long* cursor,
                                                   void* dst_pos, void* dst_val,
                                                   unsigned int* dst_idx) {
  using U = typename RecPos<Tg>::T;
  constexpr int C = RecChunk<Tg>::C, PER = C / 256;
  struct UP { U x, y; };
  __shared__ UP s_pos[C];
  __shared__ C2<Tg> s_val[C];
  __shared__ unsigned int s_idx[C];
  __shared__ unsigned char s_key[C];
  __shared__ unsigned int s_cnt[kMaxSuper], s_loc[kMaxSuper];
  __shared__ unsigned long long s_gb[kMaxSuper];
  __shared__ unsigned long long s_rng[2];
  __shared__ int s_item;
  const int fsh = 2 * g.sshift, fpc = 1 << fsh;
  const int nsx = g.nb >> g.sshift, ns = nsx * nsx;
  const int nk = kSuper ? ns : fpc;                     // keys of this pass (<= 64)
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < kMaxSuper) s_cnt[tid] = 0;
  if (tid == 0) {
    if constexpr (kSuper) {
      const size_t b0 = (size_t)blockIdx.y * per_pair + (size_t)blockIdx.x * C;
      s_rng[0] = b0;
      s_rng[1] = min(b0 + (size_t)C, (size_t)(blockIdx.y + 1) * per_pair);
      s_item = blockIdx.y * ns;
    } else {
      // work item: the super-bin i with work[i] <= blockIdx.x < work[i + 1]
      const unsigned int w = blockIdx.x;
      const int nitems = (int)per_pair;
      int item = -1;
      if (w < work[nitems]) {
        int lo = 0, hi = nitems;                        // work[lo] <= w < work[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (work[mid] <= w) lo = mid; else hi = mid;
        }
        item = lo;
        const int pl = item / ns, sb = item % ns;
        const unsigned long long* off = offsets + (size_t)(pair0 + pl) * g.keys + (size_t)sb * fpc;
        const unsigned long long b0 = off[0] + (unsigned long long)(w - work[item]) * C;
        s_rng[0] = b0;
        s_rng[1] = min(b0 + (unsigned long long)C, off[fpc]);
      }
      s_item = item;
    }
  }
  __syncthreads();
  const int item = s_item;
  if (item < 0) return;                                 // uniform over the workgroup
  const unsigned long long base = s_rng[0], end = s_rng[1];
  const U* pos = (const U*)src_pos;
  const C2<Tg>* val = (const C2<Tg>*)src_val;
  U px[PER], py[PER];
  C2<Tg> v[PER];
  unsigned int id[PER];
  int key[PER], rank[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const unsigned long long r = base + (unsigned long long)(j * 256 + tid);
    key[j] = -1;
    if (r < end) {
      v[j] = val[r];
      px[j] = pos[2 * r];
      py[j] = pos[2 * r + 1];
      id[j] = kSuper ? (unsigned int)r : (src_idx ? src_idx[r] : 0u);
    }
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const unsigned long long r = base + (unsigned long long)(j * 256 + tid);
    if (r < end && (!kSuper || !is_none(v[j]))) {
      const int k = rec_key(turns_to_cells(px[j], g.nf), turns_to_cells(py[j], g.nf), g);
      key[j] = kSuper ? k >> fsh : k & (fpc - 1);
      rank[j] = (int)atomicAdd(&s_cnt[key[j]], 1u);
    }
  }
  __syncthreads();
  if (tid < 64) {
    const unsigned int c = tid < nk ? s_cnt[tid] : 0u;
    unsigned int inc = c;
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned int x = __shfl_up(inc, o, 64);
      if (lane >= o) inc += x;
    }
    if (tid < nk) {
      s_loc[tid] = inc - c;
      unsigned long long* cur =
          kSuper ? cursor + (size_t)(pair0 + item / ns) * ns + tid
                 : cursor + (size_t)(pair0 + item / ns) * g.keys + (size_t)(item % ns) * fpc + tid;
      s_gb[tid] = c ? atomicAdd(cur, (unsigned long long)c) : 0ull;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if (key[j] >= 0) {
      const int p = (int)s_loc[key[j]] + rank[j];
      s_pos[p] = {px[j], py[j]};
      s_val[p] = v[j];
      s_idx[p] = id[j];
      s_key[p] = (unsigned char)key[j];
    }
  }
  __syncthreads();
  const int tot = (int)(s_loc[nk - 1] + s_cnt[nk - 1]);
  U* op = (U*)dst_pos;
  C2<Tg>* ov = (C2<Tg>*)dst_val;
  for (int t = tid; t < tot; t += 256) {
    const int k = s_key[t];
    const unsigned long long o = s_gb[k] + (unsigned long long)(t - (int)s_loc[k]);
    const UP q = s_pos[t];
    op[2 * o] = q.x;
    op[2 * o + 1] = q.y;
    ov[o] = s_val[t];
    if (dst_idx) dst_idx[o] = s_idx[t];
  }
}

__device__ __forceinline__ int bcast_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ float bcast_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double bcast_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float bcast_v(float v, int lane) { return bcast_f(v, lane); }
__device__ __forceinline__ double bcast_v(double v, int lane) { return bcast_d(v, lane); }

// LDS ordering between lanes of one wave (no other wave touches these arrays).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kSpreadWaves = 4;      // waves per spreading block (256 threads)
constexpr int kSpreadTarget = 8192;  // least records per slice of a heavy tile
constexpr int kSpreadSlices = 255;   // most slices of one tile (a byte per tile)
constexpr int kSpreadBatch = 32;     // queued records staged and added per round
constexpr int kSpreadQueue = 96;     // queue capacity: a batch plus one scan step

// Records in the 3 x 6 bins whose kernel footprints can reach bin row q of tile
// (ty, tx): the records wave q of the tile's block scans.
__device__ __forceinline__ unsigned long long strip_records(const unsigned long long* off,
                                                            const BinGeom& g, int ty, int tx,
                                                            int q) {
  unsigned long long n = 0;
  for (int i = 0; i < 18; ++i) {
    const int by = i / 6 - 1, bx = i % 6 - 1;
    const int bny = (ty * 4 + q + by + g.nb) % g.nb, bnx = (tx * 4 + bx + g.nb) % g.nb;
    const int k = bin_key(bny, bnx, g);
    n += off[k + 1] - off[k];
  }
  return n;
}

// Slices of every tile of a launch group (one thread per (pair, tile)): a tile
// whose busiest strip scans more than `target` records is cut into
// S = ceil(records / target) <= kSpreadSlices slices of its scan ranges.  The
// host sets target to max(kSpreadTarget, the group's records / 1024), so that
// only tiles far above their share of the launch are cut.
// slices[pair][tile] = S; slices 1 .. S - 1 of such tiles go to the list
// (entry: pair * tiles + tile, slice), their count to *n_heavy (zero at launch).
static __global__ __launch_bounds__(256) void k_spread_slices(const unsigned long long* offsets,
                                                       BinGeom g, int pair0, int npairs,
                                                       unsigned long long target,
                                                       unsigned char* slices, uint2* heavy,
                                                       unsigned int* n_heavy) {
  const int tile = 4 * g.bin, ntx = g.nf / tile, nt = ntx * ntx;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)npairs * nt) return;
  const int pl = (int)(i / nt), t = (int)(i % nt);
  const unsigned long long* off = offsets + (size_t)(pair0 + pl) * g.keys;
  unsigned long long nmax = 0;
  for (int q = 0; q < 4; ++q) nmax = max(nmax, strip_records(off, g, t / ntx, t % ntx, q));
  const int S = (int)min((unsigned long long)kSpreadSlices,
                         max(1ull, (nmax + target - 1) / target));
  slices[i] = (unsigned char)S;
  if (S > 1) {
    const unsigned int b = atomicAdd(n_heavy, (unsigned int)(S - 1));
    for (int k = 1; k < S; ++k) heavy[b + k - 1] = make_uint2((unsigned int)i, (unsigned int)k);
  }
}

// Static LDS of k_spread_tiles<Tg, w> besides the dynamic accumulator tile.
__host__ __device__ constexpr size_t spread_static_lds(size_t sz_g, int w) {
  return (size_t)kSpreadWaves * (kSpreadBatch * (2 * (size_t)w * sz_g + (2 * sz_g + 8 + 15) / 16 * 16) +
                                 kSpreadQueue * 4 * sz_g + (18 + 19) * 8) +
         256;   // slack for the compiler's alignment of the arrays
}

// Spreading of one tile (TILE x TILE cells, TILE = 4 BIN).  Wave q owns bin row
// q of the tile (a strip no other wave writes) and scans the records of the
// 3 x 6 bins whose kernel footprints can reach it (w / 2 <= BIN).  Records that
// meet the strip are queued; per 32 queued records the lanes evaluate the
// separable ES-kernel factors (x in the low half-wave, y in the high one) into
// LDS, then the wave walks the batch: for each record every lane adds one tap
// with a plain LDS read-modify-write (the taps of one record are distinct
// cells): no atomics.  Batches of 32 keep the block within a third of the LDS,
// three blocks per CU.
// A heavy tile (records concentrated by a focusing system) is cut into S
// slices of every wave's scan range (k_spread_slices): the tile's own block
// takes slice 0 and stores the tile; the blocks of the second launch (heavy
// != null) take the listed slices 1 .. S - 1 afterwards and add their tiles to
// the grid with atomics.
template <class Tg, int w>
__device__ __forceinline__ void spread_tile(const void* srt_pos, const void* srt_val,
                                            const unsigned long long* offsets, const BinGeom& g,
                                            double beta, int pair, int tile_i, int slice, int S,
                                            C2<Tg>* grid) {
  using U = typename RecPos<Tg>::T;
  constexpr int NW = kSpreadWaves, QN = kSpreadQueue, QB = kSpreadBatch;
  extern __shared__ unsigned char s_raw[];
  __shared__ Tg s_kx[NW][QB][w], s_ky[NW][QB][w];
  // per queued record: value and first-tap offsets, read by the wave as one entry
  struct alignas(16) RecEnt { C2<Tg> v; int dx, dy; };
  __shared__ RecEnt s_r[NW][QB];
  // queued record: its grid position and value (no global load when staged)
  struct QEnt { U px, py; C2<Tg> v; };
  __shared__ QEnt s_q[NW][QN];
  __shared__ unsigned long long s_beg[NW][18], s_pre[NW][19];
  const int tile = 4 * g.bin;                 // cells per tile side
  // row stride = w (mod 16): the w x w taps of one record (lane = i + w j)
  // fall on consecutive 8-byte bank slots, conflict-free for the stores
  const int ts = tile + w;
  C2<Tg>* acc = (C2<Tg>*)s_raw;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ntx = g.nf / tile;
  const int ty = tile_i / ntx, tx = tile_i % ntx;
  const int x0 = tx * tile, y0 = ty * tile;
  const int strip = g.bin, sy0 = wave * strip;  // tile rows owned by this wave
  __syncthreads();                              // LDS reuse across the tiles of a block
  for (int i = threadIdx.x; i < tile * ts; i += blockDim.x) acc[i] = {Tg(0), Tg(0)};
  const U* pos = (const U*)srt_pos;
  const C2<Tg>* val = (const C2<Tg>*)srt_val;
  const unsigned long long* off = offsets + (size_t)pair * g.keys;
  if (lane < 18) {
    const int by = lane / 6 - 1, bx = lane % 6 - 1;
    const int bny = (ty * 4 + wave + by + g.nb) % g.nb, bnx = (tx * 4 + bx + g.nb) % g.nb;
    const int k = bin_key(bny, bnx, g);
    s_beg[wave][lane] = off[k];
    s_pre[wave][lane + 1] = off[k + 1] - off[k];
  }
  __syncthreads();
  if (lane == 0) {
    s_pre[wave][0] = 0;
    for (int i = 1; i <= 18; ++i) s_pre[wave][i] += s_pre[wave][i - 1];
  }
  __syncthreads();
  const Tg two_w = Tg(2.0 / w), bet = (Tg)beta;
  // this slice's part of the wave's scan range
  const unsigned long long nall = s_pre[wave][18];
  const unsigned long long jlo = nall * (unsigned long long)slice / (unsigned long long)S;
  const unsigned long long ntot = nall * (unsigned long long)(slice + 1) / (unsigned long long)S;

  // stage queue entries [0, n) and add their taps to the strip
  auto process = [&](int n) {
    wave_lds_sync();
    const int q = lane & (QB - 1);                 // record of this lane
    const bool hi = lane >= QB;                    // low half: x factors, high half: y
    if (q < n) {
      const QEnt qe = s_q[wave][q];
      const double gx = turns_to_cells(qe.px, g.nf), gy = turns_to_cells(qe.py, g.nf);
      const int lx0 = (int)ceil(gx - 0.5 * w), ly0 = (int)ceil(gy - 0.5 * w);
      const double f = hi ? gy - ly0 : gx - lx0;
      Tg* kf = hi ? &s_ky[wave][q][0] : &s_kx[wave][q][0];
#pragma unroll
      for (int i = 0; i < w; ++i) kf[i] = es_kernel<Tg>((Tg)((double)i - f), two_w, bet);
      if (!hi) {
        RecEnt e;
        e.v = qe.v;
        // first tap relative to the tile origin, in [-w, nf - w): a tap lands in
        // the tile iff its offset is in [0, tile) (nf >= tile + w)
        e.dx = ((lx0 - x0 + w) & (g.nf - 1)) - w;
        e.dy = ((ly0 - y0 + w) & (g.nf - 1)) - w;
        s_r[wave][q] = e;
      }
    }
    wave_lds_sync();
    // entries are read RB at a time ahead of the accumulator updates, so that
    // each record costs one LDS round trip (the read-modify-write of its taps)
    constexpr int RB = 4;
    for (int k0 = 0; k0 < n; k0 += RB) {
      RecEnt e[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) e[u] = s_r[wave][min(k0 + u, n - 1)];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int k = k0 + u;
        if (k >= n) break;                         // wave-uniform
        const int dx = e[u].dx, dy = e[u].dy - sy0;
        const C2<Tg> v = e[u].v;
#pragma unroll
        for (int tap0 = 0; tap0 < w * w; tap0 += 64) {
          const int tap = tap0 + lane;
          if (tap < w * w) {
            const int i = tap % w, jj = tap / w;
            const int cx = dx + i, cy = dy + jj + sy0;
            if ((unsigned)cx < (unsigned)tile && (unsigned)(dy + jj) < (unsigned)strip) {
              const Tg kk = s_kx[wave][k][i] * s_ky[wave][k][jj];
              C2<Tg>& d = acc[cy * ts + cx];
              d.re += v.re * kk;
              d.im += v.im * kk;
            }
          }
        }
      }
    }
    wave_lds_sync();
  };

  int qn = 0;                                      // queued records (wave-uniform)
  int bin = 0;                                     // monotonic per lane across batches
  // the positions and values of the next 64 records are loaded before the
  // current ones are tested and queued
  U pxn = 0, pyn = 0;
  C2<Tg> vn{};
  auto fetch = [&](unsigned long long j) {
    if (j < ntot) {
      while (j >= s_pre[wave][bin + 1]) ++bin;
      const unsigned long long r = s_beg[wave][bin] + (j - s_pre[wave][bin]);
      pxn = pos[2 * r];
      pyn = pos[2 * r + 1];
      vn = val[r];
    }
  };
  fetch(jlo + lane);
  for (unsigned long long base = jlo; base < ntot; base += 64) {
    const unsigned long long j = base + lane;
    const U px = pxn, py = pyn;
    const C2<Tg> v = vn;
    fetch(j + 64);
    bool hit = false;
    if (j < ntot) {
      const double gx = turns_to_cells(px, g.nf), gy = turns_to_cells(py, g.nf);
      const int lx0 = (int)ceil(gx - 0.5 * w), ly0 = (int)ceil(gy - 0.5 * w);
      // footprint vs tile columns and vs this wave's strip rows (periodic)
      const int cx0 = (lx0 - x0) & (g.nf - 1);
      const int cy0 = (ly0 - y0 - sy0) & (g.nf - 1);
      hit = (cx0 < tile || cx0 + w > g.nf) && (cy0 < strip || cy0 + w > g.nf);
    }
    const unsigned long long m = __ballot(hit);
    const int pre = __popcll(m & ((1ull << lane) - 1ull));
    if (hit) s_q[wave][qn + pre] = QEnt{px, py, v};   // qn < QB: at most QB + 63 < QN entries
    qn += __popcll(m);
    while (qn >= QB) {                         // wave-uniform
      process(QB);
      // move the overflow (< 64 entries) to the front of the queue
      const int rest = qn - QB;
      QEnt t{};
      if (lane < rest) t = s_q[wave][QB + lane];
      wave_lds_sync();
      if (lane < rest) s_q[wave][lane] = t;
      qn = rest;
    }
  }
  if (qn > 0) process(qn);
  __syncthreads();
  C2<Tg>* gp = grid + (size_t)pair * g.nf * g.nf;
  for (int i = threadIdx.x; i < tile * tile; i += blockDim.x) {
    const int cy = i / tile, cx = i % tile;
    C2<Tg>& d = gp[(size_t)(y0 + cy) * g.nf + x0 + cx];
    const C2<Tg> v = acc[cy * ts + cx];
    if (slice == 0) {
      d = v;
    } else {
      atomicAdd(&d.re, v.re);
      atomicAdd(&d.im, v.im);
    }
  }
}

// slices: S per (pair of the group, tile), or null (one slice each); heavy:
// null for the launch over every tile (slice 0), else the list of further
// slices and its length, taken in turn by the blocks of the second launch.
template <class Tg, int w>
__global__ __launch_bounds__(256) void k_spread_tiles(const void* srt_pos, const void* srt_val,
                                                      const unsigned long long* offsets,
                                                      BinGeom g, double beta, int pair0,
                                                      C2<Tg>* grid, const unsigned char* slices,
                                                      const uint2* heavy,
                                                      const unsigned int* n_heavy) {
  const int nt = (g.nf / (4 * g.bin)) * (g.nf / (4 * g.bin));
  if (!heavy) {
    const int S = slices ? slices[(size_t)blockIdx.y * nt + blockIdx.x] : 1;
    spread_tile<Tg, w>(srt_pos, srt_val, offsets, g, beta, pair0 + blockIdx.y, blockIdx.x, 0, S,
                       grid);
    return;
  }
  const unsigned int n = *n_heavy;
  for (unsigned int e = blockIdx.x; e < n; e += gridDim.x) {
    const uint2 h = heavy[e];
    spread_tile<Tg, w>(srt_pos, srt_val, offsets, g, beta, pair0 + (int)(h.x / nt),
                       (int)(h.x % nt), (int)h.y, slices[h.x], grid);
  }
}

// ------------------------------------------------------------- grid FFT ---
// Row pass: one wavefront per grid row l_y, FFT (+i) over l_x, keep
// k_x in [-Q/2, Q/2) and store transposed: T1[pair][c][l_y], c = k_x + Q/2.
template <class Tg, int NF>
__global__ __launch_bounds__(256) void k_grid_rows_fwd(const C2<Tg>* grid, C2<Tg>* t1,
                                                       const C2<Tg>* tw, int Q, int pair0,
                                                       int npairs) {
  constexpr int E = NF / 64;
  const int lane = threadIdx.x & 63;
  const size_t row = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= (size_t)npairs * NF) return;
  const int pair = pair0 + (int)(row / NF), ly = (int)(row % NF);
  const C2<Tg>* src = grid + ((size_t)pair * NF + ly) * NF;
  C2<Tg> x[E];
#pragma unroll
  for (int n2 = 0; n2 < E; ++n2) x[n2] = src[lane + 64 * n2];
  group_fft<Tg, 64, E, +1>(x, lane, tw);
  const int base = E * bitrev(lane, 6);
#pragma unroll
  for (int k2 = 0; k2 < E; ++k2) {
    const int k = base + k2;
    const int ks = k < NF / 2 ? k : k - NF;
    if (ks >= -Q / 2 && ks < Q / 2)
      t1[((size_t)pair * Q + (ks + Q / 2)) * NF + ly] = x[k2];
  }
}

// Column pass: FFT (+i) over l_y for each kept column, deconvolve, crop, |U|^2.
template <class Tg, int NF>
__global__ __launch_bounds__(256) void k_grid_cols_fwd(const C2<Tg>* t1, const C2<Tg>* tw,
                                                       const double* psi_hat, int Q, int pair0,
                                                       int npairs, C2<Tg>* Uout, float* psf) {
  constexpr int E = NF / 64;
  const int lane = threadIdx.x & 63;
  const size_t col = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= (size_t)npairs * Q) return;
  const int pair = pair0 + (int)(col / Q), c = (int)(col % Q);
  const C2<Tg>* src = t1 + ((size_t)pair * Q + c) * NF;
  C2<Tg> x[E];
#pragma unroll
  for (int n2 = 0; n2 < E; ++n2) x[n2] = src[lane + 64 * n2];
  group_fft<Tg, 64, E, +1>(x, lane, tw);
  const int base = E * bitrev(lane, 6);
#pragma unroll
  for (int k2 = 0; k2 < E; ++k2) {
    const int k = base + k2;
    const int ks = k < NF / 2 ? k : k - NF;
    if (ks >= -Q / 2 && ks < Q / 2) {
      const int r = ks + Q / 2;
      const Tg sc = (Tg)(1.0 / (psi_hat[c] * psi_hat[r]));
      const C2<Tg> U = x[k2] * sc;
      const size_t o = ((size_t)pair * Q + r) * Q + c;
      Uout[o] = U;
      psf[o] = (float)((double)U.re * U.re + (double)U.im * U.im);
    }
  }
}

// Component-major ray state [8][n] -> ray-major [n][8].
static __global__ void k_export_state(const double* st, size_t n, double* out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 8 * n) return;
  const size_t ray = i / 8, c = i % 8;
  out[i] = st[c * n + ray];
}

// ------------------------------------------------------------------ loss ---
// Per pair: alpha = <I,T>/<I,I>, L_p = ||alpha I - T||^2 (Eq. 5, closed-form alpha).
static __global__ __launch_bounds__(256) void k_loss_pairs(const float* psf, const float* target,
                                                    int Q2, int pair0, double* alpha,
                                                    double* lossp) {
  __shared__ double s_red[4];
  const int pair = pair0 + blockIdx.x;
  const float* I = psf + (size_t)pair * Q2;
  const float* T = target + (size_t)pair * Q2;
  double ii = 0, it = 0;
  for (int i = threadIdx.x; i < Q2; i += blockDim.x) {
    ii += (double)I[i] * I[i];
    it += (double)I[i] * T[i];
  }
  ii = block_sum(ii, s_red);
  it = block_sum(it, s_red);
  const double al = ii > 0 ? it / ii : 0.0;
  double l = 0;
  for (int i = threadIdx.x; i < Q2; i += blockDim.x) {
    const double r = al * I[i] - T[i];
    l += r * r;
  }
  l = block_sum(l, s_red);
  if (threadIdx.x == 0) { alpha[pair] = al; lossp[pair] = l; }
}

static __global__ void k_loss_total(const double* lossp, int n_pairs, float* loss_out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < n_pairs; ++i) s += lossp[i];
    *loss_out = (float)s;
  }
}

}  // namespace rw
