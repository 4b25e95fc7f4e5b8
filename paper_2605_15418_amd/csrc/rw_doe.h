// Ray-wave interface kernels (forward and adjoint), one workgroup of 512
// threads per incident ray at a time, persistent over spatial blocks of rays.
//
// Per ray (Formalism, second paragraph; Eq. 1; Fig. 1c):
//   1. tangent frame, incident tangential wavevector
//   2. stage the DOE map tile under the patch in LDS (coalesced), bilinear
//      samples of t = A exp(i phi) -> zero-padded M x M patch
//   3. 2-D FFT: row transforms of the P nonzero rows, then column transforms;
//      each lane ends the column pass holding E consecutive bins of one column,
//      which is one chunk of the j_x-major inverse CDF: the chunk sums of the
//      sampling density come straight from registers
//   4. block scan of the chunk sums, N Philox draws (binary search over chunk
//      prefixes, then at most E bins), Eq. 1 weights, emission, trace to the
//      sensor, Eq. 2 wavelet -> record for the binned spreading
// The adjoint recomputes 1-4, interpolates the sensor-grid cogradient at every
// wavelet, forms the spectrum cogradient (drawn bins + the S = sum |U~| term),
// inverse-transforms it to the patch, and scatters the bilinear adjoint into an
// LDS tile that is added to a block-private accumulator covering the whole
// block of rays; the accumulator is flushed to dL/dt once per ray block.
#pragma once
#include <climits>

#include "rw_backward.h"

namespace rw {

constexpr int kDoeThreads = 512;

// threadIdx.x behind an empty asm: index arithmetic derived from it is redone
// where it is used instead of being hoisted out of the per-ray loops, which
// would keep dozens of per-lane addresses live across the whole kernel.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Lanes per M-point transform of a DOE workgroup.
__host__ __device__ constexpr int doe_lanes(int M) {
  return 2 * kDoeThreads / M < 2 ? 2 : (2 * kDoeThreads / M > M / 2 ? M / 2 : 2 * kDoeThreads / M);
}
// Patch buffer layout.  A 64-bit LDS store serves 16 lanes per cycle through
// 16 eight-byte bank slots, and the transforms' stores are runs of E outputs
// per lane, lanes E elements apart.  For M = 128 (E = 16) element (r, c) sits
// at r SM + 2 (r >> 4) + c + (c >> 4), SM = M + 8: one element of skew per 16
// columns and two per 16 rows put the 16 lanes of every row-pass and
// column-pass store (and load) into distinct slots.  Other M: rows of M + 1.
__host__ __device__ constexpr bool doe_skew(int M) { return M == 128; }
__host__ __device__ constexpr int doe_stride(int M) { return doe_skew(M) ? M + 8 : M + 1; }
__host__ __device__ constexpr int doe_buf_elems(int M) {
  return M * doe_stride(M) + (doe_skew(M) ? 16 : 0);
}

template <int M> struct DoeGeom {
  static constexpr int NT = kDoeThreads;
  static constexpr int L = doe_lanes(M);                                   // lanes per transform
  static constexpr int E = M / L;                                          // elements per lane
  static constexpr int G = NT / L;                                         // transform groups
  static constexpr bool kSkew = doe_skew(M);
  static constexpr int SM = doe_stride(M);                                 // buffer row stride
  static constexpr int SIZE = doe_buf_elems(M);                            // buffer elements
  static constexpr int NCH = M * L;                                        // CDF chunks of E bins
  static constexpr int LB = Log2<L>::v;
  static_assert(!kSkew || (E == 16 && L <= 16), "the skewed layout assumes runs of 16");
  // element offsets of row r and of column c
  __device__ static __forceinline__ int row(int r) { return r * SM + (kSkew ? 2 * (r >> 4) : 0); }
  __device__ static __forceinline__ int col(int c) { return kSkew ? c + (c >> 4) : c; }
  __device__ static __forceinline__ int at(int r, int c) { return row(r) + col(c); }
  // row / column a + o of a transform's input: runtime lane part a < L,
  // compile-time part o a multiple of L, so that the skew is o's alone.  (An
  // output run E b + k, k < E, is row(E b) + k SM, column col(E b) + k.)
  __device__ static __forceinline__ int row_split(int a, int o) {
    return (a + o) * SM + (kSkew ? 2 * (o >> 4) : 0);
  }
  __device__ static __forceinline__ int col_split(int a, int o) {
    return a + o + (kSkew ? (o >> 4) : 0);
  }
};

// Division of small non-negative integers (< 2^20) by a runtime divisor through
// a float reciprocal: (i + 1/2) / d stays at least 1/(2d) away from an integer,
// far beyond the float rounding error, so the truncation is exact.
struct FDiv {
  int d;
  float inv;
  __device__ __forceinline__ explicit FDiv(int dd) : d(dd), inv(1.0f / (float)dd) {}
  __device__ __forceinline__ int div(int i) const { return (int)(((float)i + 0.5f) * inv); }
};

__device__ __forceinline__ float inv_sqrt(float x) { return rsqrtf(x); }
__device__ __forceinline__ double inv_sqrt(double x) { return 1.0 / sqrt(x); }

// Propagating test of shifted bin (jx, jy): |k_in,t + kappa_j| < k_out, in FP64
// with every rounding explicit, so that all call sites take the same decision.
// For fixed jx the result is monotone in |K_v|, hence an interval of jy.
__device__ __forceinline__ bool propagating(const RayCtx& c, int jx, int jy) {
  const double Ku = __dadd_rn(c.kin_u, __dmul_rn(c.dk, (double)jx));
  const double Kv = __dadd_rn(c.kin_v, __dmul_rn(c.dk, (double)jy));
  return __dadd_rn(__dmul_rn(Ku, Ku), __dmul_rn(Kv, Kv)) < c.k2out;
}

// Propagating rows of column jx: jy in [lo, hi] (empty when lo > hi).  The
// closed-form ends are corrected with the exact predicate above.
struct Span { int lo, hi; };
__device__ __forceinline__ Span prop_span(const RayCtx& c, int jx, int M) {
  const double Ku = __dadd_rn(c.kin_u, __dmul_rn(c.dk, (double)jx));
  const double rem = __dsub_rn(c.k2out, __dmul_rn(Ku, Ku));
  if (!(rem > 0.0)) return {1, 0};
  const double r = sqrt(rem) / c.dk, mid = -c.kin_v / c.dk;
  int lo = (int)fmax(ceil(mid - r), (double)(-M / 2));
  int hi = (int)fmin(floor(mid + r), (double)(M / 2 - 1));
  if (lo > hi) {                       // rounding may leave one bin between the ends
    lo = (int)fmin(fmax(floor(mid), (double)(-M / 2)), (double)(M / 2 - 1));
    hi = lo - 1;
    if (propagating(c, jx, lo)) hi = lo;
    else if (lo + 1 <= M / 2 - 1 && propagating(c, jx, lo + 1)) hi = ++lo;
  }
  while (lo <= hi && !propagating(c, jx, lo)) ++lo;
  while (lo <= hi && !propagating(c, jx, hi)) --hi;
  if (lo > hi) return {1, 0};
  while (lo > -M / 2 && propagating(c, jx, lo - 1)) --lo;
  while (hi < M / 2 - 1 && propagating(c, jx, hi + 1)) ++hi;
  return {lo, hi};
}

// Map tile under the patch: TW x TW pixels from (tx0, ty0); zero outside the map.
struct TileRef { int tx0, ty0, tw; };

__device__ __forceinline__ TileRef tile_of(const DevCfg& cfg, const RayCtx& c) {
  const double fx = (c.p[0] - cfg.x0) * cfg.inv_pitch, fy = (c.p[1] - cfg.y0) * cfg.inv_pitch;
  const int tw = c.P + 4;
  return {(int)floor(fx) - c.P / 2 - 1, (int)floor(fy) - c.P / 2 - 1, tw};
}

// Batches of KB pixels per lane: all loads of a batch are issued before its
// LDS stores, so the map latency is paid once per batch.
template <class Tf>
__device__ __forceinline__ void stage_tile(const DevCfg& cfg, const TileRef& tr, const C2<Tf>* tm,
                                           C2<Tf>* tile) {
  constexpr int KB = 80 / (int)sizeof(C2<Tf>);
  const int n = tr.tw * tr.tw;
  const FDiv dv(tr.tw);
  for (int i0 = opaque_tid(); i0 < n; i0 += kDoeThreads * KB) {
    C2<Tf> v[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int i = i0 + k * kDoeThreads;
      const int q = dv.div(i);
      const int y = tr.ty0 + q, x = tr.tx0 + (i - q * tr.tw);
      v[k] = (i < n && x >= 0 && x < cfg.W && y >= 0 && y < cfg.H) ? tm[(size_t)y * cfg.W + x]
                                                                  : C2<Tf>{Tf(0), Tf(0)};
    }
#pragma unroll
    for (int k = 0; k < KB; ++k)
      if (i0 + k * kDoeThreads < n) tile[i0 + k * kDoeThreads] = v[k];
  }
}

// Bilinear sample (m, n) of the patch; the 2 x 2 stencil is read from the
// staged tile when it lies inside it, else from the map.
template <class Tf>
__device__ __forceinline__ C2<Tf> patch_sample_t(const DevCfg& cfg, const RayCtx& c,
                                                 const C2<Tf>* tm, const C2<Tf>* tile,
                                                 const TileRef& tr, int m, int n) {
  const double sm = (m - (c.P - 1) * 0.5) * cfg.pitch;
  const double sn = (n - (c.P - 1) * 0.5) * cfg.pitch;
  const double qx = c.p[0] + sm * c.u[0] + sn * c.v[0];
  const double qy = c.p[1] + sm * c.u[1] + sn * c.v[1];
  const double fx = (qx - cfg.x0) * cfg.inv_pitch, fy = (qy - cfg.y0) * cfg.inv_pitch;
  const double flx = floor(fx), fly = floor(fy);
  const int ix = (int)flx, iy = (int)fly;
  const Tf wx = (Tf)(fx - flx), wy = (Tf)(fy - fly);
  const int lx = ix - tr.tx0, ly = iy - tr.ty0;
  C2<Tf> t00, t01, t10, t11;
  if (tile && lx >= 0 && lx + 1 < tr.tw && ly >= 0 && ly + 1 < tr.tw) {
    const C2<Tf>* r0 = tile + ly * tr.tw + lx;
    t00 = r0[0]; t01 = r0[1]; t10 = r0[tr.tw]; t11 = r0[tr.tw + 1];
  } else {
    auto at = [&](int y, int x) {
      return (x >= 0 && x < cfg.W && y >= 0 && y < cfg.H) ? tm[(size_t)y * cfg.W + x]
                                                          : C2<Tf>{Tf(0), Tf(0)};
    };
    t00 = at(iy, ix); t01 = at(iy, ix + 1); t10 = at(iy + 1, ix); t11 = at(iy + 1, ix + 1);
  }
  return (t00 * (Tf(1) - wx) + t01 * wx) * (Tf(1) - wy) + (t10 * (Tf(1) - wx) + t11 * wx) * wy;
}

// Planar DOE: every sample of the patch sits at the same sub-pixel fraction;
// sample (m, n) interpolates pixels (ix0 + m + {0,1}, iy0 + n + {0,1}).
template <class Tf> struct PlanarPatch {
  int ix0, iy0;
  Tf wx, wy;
};
template <class Tf>
__device__ __forceinline__ PlanarPatch<Tf> planar_patch(const DevCfg& cfg, const RayCtx& c) {
  const double fx0 = (c.p[0] - cfg.x0) * cfg.inv_pitch - 0.5 * (c.P - 1);
  const double fy0 = (c.p[1] - cfg.y0) * cfg.inv_pitch - 0.5 * (c.P - 1);
  const double flx = floor(fx0), fly = floor(fy0);
  return {(int)flx, (int)fly, (Tf)(fx0 - flx), (Tf)(fy0 - fly)};
}

// Shared scratch of one workgroup.
// One draw's spectrum cogradient term (bin index k, -1: none).
template <class Tf> struct DrawEnt {
  C2<Tf> g;
  int k;
};
constexpr int kDrawLds = 256;   // draws per ray whose terms stay in LDS

// 256-point line transforms (M = 256, whose spectrum lives in a global buffer):
// batches of kLines256 lines staged in LDS, element i of a line at i + i / 16
// (one element of skew per 16) in lines kLS256 apart, so that the 16 lanes of
// a quarter-wave hit 16 distinct 8-byte bank slots in both passes and in the
// transposed column loads.
constexpr int kLines256 = 64;
constexpr int kLS256 = 273;
__device__ __forceinline__ int sk256(int i) { return i + (i >> 4); }

template <class Tf, int M, bool kLDS> struct DoeLds {
  C2<Tf> buf[kLDS ? DoeGeom<M>::SIZE : 1];
  C2<Tf> ls[M == 256 ? kLines256 * kLS256 : 1];   // staged lines (M = 256)
  C2<Tf> tw[M];
  double pref[DoeGeom<M>::NCH + 1];
  double red[16];
  int redi[16];
  double acc[8][16];
  Span span[M];             // propagating rows of each shifted column
  RayCtx ctx;
  DrawEnt<Tf> dl[kLDS ? kDrawLds : 1];   // adjoint: the draws' terms when N <= kDrawLds
};

// Sampling weight of a propagating bin: |X| (p_mag) or 1 (p_uni).  Float
// spectra take the hardware square root; the chunk sums and the draws'
// rescan of a chunk use this same function, which is all the inverse CDF
// needs from it.
__device__ __forceinline__ float samp_w(const C2<float>& x, int sampling) {
  return sampling == 0 ? __builtin_amdgcn_sqrtf(fmaf(x.re, x.re, x.im * x.im)) : 1.0f;
}
__device__ __forceinline__ double samp_w(const C2<double>& x, int sampling) {
  return sampling == 0 ? cabs_rn(x) : 1.0;
}

// 128-point transforms of the lines (rows or columns) of the patch buffer in
// two register passes, n = a + 16 b, k = k1 + 8 k2:
//   pass A, per (line, a): the 8-point DFT over b, times W_128^(a k1), back
//   into slots a + 16 k1;
//   pass B, per (line, k1): the 16-point DFT over the slots a + 16 k1, stored
//   to slot k1 + 8 k2 once every pass-B read is done.
// Inputs at or beyond nin are zero (nin = M / 2: the upper half of every
// 8-point input); outputs below nout are stored, and with zb the outputs nout
// and M - 1 are stored as zeros.  Row transforms run the lanes along the
// row, column transforms across 16 consecutive columns, so that the 64-bit
// stores of every quarter-wavefront land on distinct bank slots of the skewed
// layout.  Starts and ends with every lane's LDS traffic ordered.
template <class Tf, int M, int DIR, bool COLS>
__device__ __forceinline__ void line_fft2(C2<Tf>* buf, const C2<Tf>* tw, int nl, int nin,
                                          int nout, bool zb) {
  using Gm = DoeGeom<M>;
  static_assert(M == 128 && Gm::kSkew, "two-pass lines are 8 x 16 points in the skewed layout");
  constexpr int SM = Gm::SM;
  constexpr int RB = 16 * SM + 2;          // 16 rows further in the skewed layout
  const int tid = opaque_tid();
  const bool hz = 2 * nin == M;
  // pass A, two tasks per round: a lane's tasks touch disjoint slots, so the
  // loads of both are issued before either transform
  constexpr int step = COLS ? RB : 17;     // slot a + 16 b sits at base + b * step
  for (int t0 = tid; t0 < nl * 16; t0 += 2 * kDoeThreads) {
    C2<Tf> x[2][8];
    int base[2], av[2];
    bool on[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int t = t0 + j * kDoeThreads;
      on[j] = t < nl * 16;
      const int line = COLS ? (t & (M - 1)) : (t >> 4);
      av[j] = COLS ? (t >> 7) : (t & 15);
      base[j] = COLS ? av[j] * SM + Gm::col(line) : Gm::row(line) + av[j];
    }
    if (hz) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int b = 0; b < 8; ++b)
          x[j][b] = on[j] && b < 4 ? buf[base[j] + b * step] : C2<Tf>{Tf(0), Tf(0)};
#pragma unroll
      for (int j = 0; j < 2; ++j) reg_fft<Tf, 8, DIR, true>(x[j]);
    } else {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int b = 0; b < 8; ++b)
          x[j][b] = on[j] && av[j] + 16 * b < nin ? buf[base[j] + b * step]
                                                  : C2<Tf>{Tf(0), Tf(0)};
#pragma unroll
      for (int j = 0; j < 2; ++j) reg_fft<Tf, 8, DIR>(x[j]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int k1 = 1; k1 < 8; ++k1) {
        const C2<Tf> w0 = tw[(av[j] * k1) & (M - 1)];
        const C2<Tf> w = {w0.re, DIR > 0 ? -w0.im : w0.im};
        x[j][k1] = x[j][k1] * w;
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (on[j])
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) buf[base[j] + k1 * step] = x[j][k1];
  }
  __syncthreads();
  // pass B: at most two tasks per lane (nl * 8 <= 1024)
  constexpr int NT = 2;
  C2<Tf> z[NT][16];
  int ob[NT], k1s[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int t = tid + j * kDoeThreads;
    k1s[j] = -1;
    if (t < nl * 8) {
      const int line = COLS ? (t & (M - 1)) : (t >> 3), k1 = COLS ? (t >> 7) : (t & 7);
      // slots a + 16 k1 (a < 16) and outputs k1 + 8 k2
      const int ib = COLS ? 16 * k1 * SM + 2 * k1 + Gm::col(line) : Gm::row(line) + 17 * k1;
      constexpr int istep = COLS ? SM : 1;
#pragma unroll
      for (int a = 0; a < 16; ++a) z[j][a] = buf[ib + a * istep];
      reg_fft<Tf, 16, DIR>(z[j]);
      ob[j] = COLS ? k1 * SM + Gm::col(line) : Gm::row(line) + k1;
      k1s[j] = k1;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    if (k1s[j] < 0) continue;
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) {
      const int e = k1s[j] + 8 * k2;
      const int o = ob[j] + (COLS ? 8 * k2 * SM + 2 * (k2 >> 1) : 8 * k2 + (k2 >> 1));
      if (e < nout) buf[o] = z[j][k2];
      else if (zb && (e == nout || e == M - 1)) buf[o] = C2<Tf>{Tf(0), Tf(0)};
    }
  }
  __syncthreads();
}

// Copies between the global patch buffer (M = 256) and the staged lines, KB
// elements per lane in flight: every load of a batch is issued before its
// stores (one workgroup per CU leaves eight waves to hide the memory latency).
// Rows: staged line l <- buffer row r0 + l (elements m < nm of a line, zeros up
// to zl).  Columns: staged line l <- buffer column c0 + l (rows r < nr, zeros up
// to zl).
template <class Tf, bool kCols>
__device__ __forceinline__ void stage_lines256(C2<Tf>* ls, const C2<Tf>* buf, int sm, int o0,
                                               int nl, int nk, int zl) {
  constexpr int KB = 16;
  const int tid = opaque_tid();
  const int n = kCols ? zl * kLines256 : nl * 256;
  for (int i0 = tid; i0 < n; i0 += kDoeThreads * KB) {
    C2<Tf> v[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int i = i0 + k * kDoeThreads;
      const int l = kCols ? (i & 63) : (i >> 8), e = kCols ? (i >> 6) : (i & 255);
      v[k] = C2<Tf>{Tf(0), Tf(0)};
      if (i < n && e < nk && l < nl)
        v[k] = kCols ? buf[(size_t)e * sm + o0 + l] : buf[(size_t)(o0 + l) * sm + e];
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int i = i0 + k * kDoeThreads;
      const int l = kCols ? (i & 63) : (i >> 8), e = kCols ? (i >> 6) : (i & 255);
      if (i < n && e < zl && l < nl) ls[l * kLS256 + sk256(e)] = v[k];
    }
  }
}

// Inverse column pass of the adjoint (M = 256): staged line l <- column c0 + l of
// the spectrum cogradient, formed as the spectrum is loaded: the p_mag
// normaliser term fS X / |X| (plus the G2 term (g / |X| - d2s) X / |X|) on
// propagating bins, zero elsewhere; then the draws' terms of bins in these
// columns are added in LDS (entries dl[0..N), bin index k = row * sm + column).
template <class Tf>
__device__ __forceinline__ void stage_cograd256(C2<Tf>* ls, const C2<Tf>* buf, int sm, int c0,
                                                const Span* span, bool mag, Tf fS,
                                                const float* dlg, Tf d2s,
                                                const DrawEnt<Tf>* dl, int N) {
  constexpr int KB = 16, M = 256;
  const int tid = opaque_tid();
  for (int i0 = tid; i0 < M * kLines256; i0 += kDoeThreads * KB) {
    C2<Tf> v[KB];
    float g[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int i = i0 + k * kDoeThreads;
      const int l = i & 63, e = i >> 6;
      v[k] = C2<Tf>{Tf(0), Tf(0)};
      g[k] = 0.0f;
      if (i < M * kLines256) {
        v[k] = buf[(size_t)e * sm + c0 + l];
        if (dlg) g[k] = dlg[e * M + c0 + l];
      }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int i = i0 + k * kDoeThreads;
      if (i >= M * kLines256) break;
      const int l = i & 63, ky = i >> 6, kx = c0 + l;
      const int jx = kx < M / 2 ? kx : kx - M, jy = ky < M / 2 ? ky : ky - M;
      const Span sp = span[jx + M / 2];
      C2<Tf> out = {Tf(0), Tf(0)};
      if (mag && jy >= sp.lo && jy <= sp.hi) {
        const C2<Tf> X = v[k];
        const Tf m2 = X.re * X.re + X.im * X.im;
        if (m2 > Tf(0)) {
          const Tf im = inv_sqrt(m2);
          Tf f = fS * im;
          if (dlg) f += ((Tf)g[k] * im - d2s) * im;
          out = {X.re * f, X.im * f};
        }
      }
      ls[l * kLS256 + sk256(ky)] = out;
    }
  }
  if (dl) {
    __syncthreads();
    for (int i = tid; i < N; i += kDoeThreads) {
      const DrawEnt<Tf> e = dl[i];
      if (e.k < 0) continue;
      const int row = e.k / sm, col = e.k - row * sm;
      if (col < c0 || col >= c0 + kLines256) continue;
      atomicAdd(&ls[(col - c0) * kLS256 + sk256(row)].re, e.g.re);
      atomicAdd(&ls[(col - c0) * kLS256 + sk256(row)].im, e.g.im);
    }
  }
}

// 256-point transforms of nl staged lines in place (natural order in and out),
// n = a + 16 b, k = k1 + 16 k2: pass A, per (line, a), the 16-point DFT over b
// times W_256^(a k1), back into slots a + 16 k1; pass B, per (line, k1), the
// 16-point DFT over the slots a + 16 k1, stored to k1 + 16 k2 after a barrier.
// half: inputs 128.. are zero (the zero-padded half of a patch line).  Starts
// and ends with every lane's LDS traffic ordered.
template <class Tf, int DIR>
__device__ __forceinline__ void lds_fft256(C2<Tf>* ls, const C2<Tf>* tw, int nl, bool half) {
  const int tid = opaque_tid();
  __syncthreads();
  for (int t = tid; t < nl * 16; t += kDoeThreads) {
    C2<Tf>* L = ls + (t >> 4) * kLS256;
    const int a = t & 15;
    C2<Tf> x[16];
    if (half) {
#pragma unroll
      for (int b = 0; b < 16; ++b) x[b] = b < 8 ? L[sk256(a + 16 * b)] : C2<Tf>{Tf(0), Tf(0)};
      reg_fft<Tf, 16, DIR, true>(x);
    } else {
#pragma unroll
      for (int b = 0; b < 16; ++b) x[b] = L[sk256(a + 16 * b)];
      reg_fft<Tf, 16, DIR>(x);
    }
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) {
      const C2<Tf> w0 = tw[(a * k1) & 255];
      x[k1] = x[k1] * C2<Tf>{w0.re, DIR > 0 ? -w0.im : w0.im};
    }
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) L[sk256(a + 16 * k1)] = x[k1];
  }
  __syncthreads();
  constexpr int NT = kLines256 * 16 / kDoeThreads;     // pass-B tasks per lane
  C2<Tf> z[NT][16];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int t = tid + j * kDoeThreads;
    if (t < nl * 16) {
      const C2<Tf>* L = ls + (t >> 4) * kLS256;
      const int k1 = t & 15;
#pragma unroll
      for (int a = 0; a < 16; ++a) z[j][a] = L[sk256(a + 16 * k1)];
      reg_fft<Tf, 16, DIR>(z[j]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int t = tid + j * kDoeThreads;
    if (t < nl * 16) {
      C2<Tf>* L = ls + (t >> 4) * kLS256;
      const int k1 = t & 15;
#pragma unroll
      for (int k2 = 0; k2 < 16; ++k2) L[sk256(k1 + 16 * k2)] = z[j][k2];
    }
  }
  __syncthreads();
}

// Spectrum of the ray's patch into buf (natural order) and the per-chunk sums of
// the sampling density into s.pref[chunk] (before the scan).  Returns lastpos
// candidates through *lastpos (block maximum taken by the caller).
template <class Tf, int M, bool kCdf = true>
__device__ __forceinline__ void doe_spectrum(const DevCfg& cfg, const RayCtx& c,
                                             const C2<Tf>* tm, C2<Tf>* buf, const C2<Tf>* tw,
                                             double* chunk, Span* span, int sampling,
                                             int* lastpos, C2<Tf>* ls) {
  using Gm = DoeGeom<M>;
  constexpr int L = Gm::L, E = Gm::E, G = Gm::G, SM = Gm::SM;
  const int tid = opaque_tid();
  const int g = tid / L, gl = tid % L;
  const int br = bitrev(gl, Gm::LB);
  const int P = c.P;
  if constexpr (M == 256) {
    // rows: batches of kRB of the P nonzero rows.  The map pixels under a batch's
    // sample stencils (a band, from the affine sample map at the patch corners,
    // one pixel wider on each side than rounding could move it) are staged in
    // the upper lines of the staging area with coalesced loads, the samples read
    // them from there into the lower lines, and the transformed rows go to buf;
    // columns: batches of columns (rows < P in), chunk sums from the staged
    // outputs, the spectrum to buf
    const bool half = 2 * P == M;
    const int lgP = __builtin_ctz(P);
    constexpr int kRB = 32;
    constexpr int kBandCap = (kLines256 - kRB) * kLS256;
    C2<Tf>* band = ls + kRB * kLS256;
    for (int r0 = 0; r0 < P; r0 += kRB) {
      const int nr = min(kRB, P - r0);
      auto sample_f = [&](int m, int n, double& fx, double& fy) {
        const double sm_ = (m - (P - 1) * 0.5) * cfg.pitch, sn_ = (n - (P - 1) * 0.5) * cfg.pitch;
        fx = (c.p[0] + sm_ * c.u[0] + sn_ * c.v[0] - cfg.x0) * cfg.inv_pitch;
        fy = (c.p[1] + sm_ * c.u[1] + sn_ * c.v[1] - cfg.y0) * cfg.inv_pitch;
      };
      double xl = 1e300, xh = -1e300, yl = 1e300, yh = -1e300;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        double fx, fy;
        sample_f((cc & 1) ? P - 1 : 0, r0 + ((cc & 2) ? nr - 1 : 0), fx, fy);
        xl = fmin(xl, fx); xh = fmax(xh, fx);
        yl = fmin(yl, fy); yh = fmax(yh, fy);
      }
      const int bx0 = (int)floor(xl) - 1, by0 = (int)floor(yl) - 1;
      const int bw = (int)floor(xh) + 3 - bx0, bh = (int)floor(yh) + 3 - by0;
      const bool use_band = bw * bh <= kBandCap;
      __syncthreads();      // the previous batch's lines and band are read out
      if (use_band) {
        constexpr int KB = 10;
        const FDiv dW(bw);
        for (int i0 = tid; i0 < bw * bh; i0 += kDoeThreads * KB) {
          C2<Tf> v[KB];
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            const int i = i0 + k * kDoeThreads;
            v[k] = C2<Tf>{Tf(0), Tf(0)};
            if (i < bw * bh) {
              const int yy = dW.div(i), x = bx0 + i - yy * bw, y = by0 + yy;
              if (x >= 0 && x < cfg.W && y >= 0 && y < cfg.H) v[k] = tm[(size_t)y * cfg.W + x];
            }
          }
#pragma unroll
          for (int k = 0; k < KB; ++k)
            if (i0 + k * kDoeThreads < bw * bh) band[i0 + k * kDoeThreads] = v[k];
        }
        __syncthreads();
      }
      // bilinear samples, KS per lane with their reads issued together
      constexpr int KS = 8;
      for (int i0 = tid; i0 < nr * P; i0 += kDoeThreads * KS) {
        C2<Tf> q[KS][4];
        Tf wx[KS], wy[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
          const int i = i0 + k * kDoeThreads;
          const int n = r0 + (i >> lgP), m = i & (P - 1);
          double fx, fy;
          sample_f(m, n, fx, fy);
          const double flx = floor(fx), fly = floor(fy);
          const int ix = (int)flx, iy = (int)fly;
          wx[k] = (Tf)(fx - flx);
          wy[k] = (Tf)(fy - fly);
          if (use_band) {
            const int o = i < nr * P ? (iy - by0) * bw + (ix - bx0) : 0;
            q[k][0] = band[o];
            q[k][1] = band[o + 1];
            q[k][2] = band[o + bw];
            q[k][3] = band[o + bw + 1];
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int x = ix + (j & 1), y = iy + (j >> 1);
              q[k][j] = (i < nr * P && x >= 0 && x < cfg.W && y >= 0 && y < cfg.H)
                            ? tm[(size_t)y * cfg.W + x] : C2<Tf>{Tf(0), Tf(0)};
            }
          }
        }
#pragma unroll
        for (int k = 0; k < KS; ++k) {
          const int i = i0 + k * kDoeThreads;
          if (i >= nr * P) break;
          ls[(i >> lgP) * kLS256 + sk256(i & (P - 1))] =
              (q[k][0] * (Tf(1) - wx[k]) + q[k][1] * wx[k]) * (Tf(1) - wy[k]) +
              (q[k][2] * (Tf(1) - wx[k]) + q[k][3] * wx[k]) * wy[k];
        }
      }
      if (!half)
        for (int i = tid; i < nr * M; i += kDoeThreads)
          if ((i & 255) >= P) ls[(i >> 8) * kLS256 + sk256(i & 255)] = C2<Tf>{Tf(0), Tf(0)};
      lds_fft256<Tf, -1>(ls, tw, nr, half);
      for (int i = tid; i < nr * M; i += kDoeThreads) {
        const int l = i >> 8, k = i & 255;
        buf[Gm::row(r0 + l) + k] = ls[l * kLS256 + sk256(k)];
      }
    }
    for (int i = tid; i < M; i += kDoeThreads) span[i] = prop_span(c, i - M / 2, M);
    int lp = -1;
    for (int c0 = 0; c0 < M; c0 += kLines256) {
      __syncthreads();
      stage_lines256<Tf, true>(ls, buf, SM, c0, kLines256, P, half ? P : M);
      lds_fft256<Tf, -1>(ls, tw, kLines256, half);
      if constexpr (kCdf) {
        // chunk q of column col: E = 64 consecutive shifted rows, summed in the
        // spectrum's type in shifted-row order (the order of the draws' rescan)
        if (tid < kLines256 * (M / E)) {
          const int cl = tid & 63, q = tid >> 6;
          const int col = c0 + cl;
          const int jx = col < M / 2 ? col : col - M;
          const int jys0 = E * q, ky0 = (jys0 + M / 2) & (M - 1);
          const Span sp = span[jx + M / 2];
          Tf sum = Tf(0);
          int last = -1;
          // groups of EB bins read before they are summed (in order)
          constexpr int EB = 8;
          for (int q0 = 0; q0 < E; q0 += EB) {
            C2<Tf> xs[EB];
#pragma unroll
            for (int e = 0; e < EB; ++e) xs[e] = ls[cl * kLS256 + sk256(ky0 + q0 + e)];
#pragma unroll
            for (int e = 0; e < EB; ++e) {
              const int ky = ky0 + q0 + e;
              const int jy = ky < M / 2 ? ky : ky - M;
              Tf wgt = Tf(0);
              if (jy >= sp.lo && jy <= sp.hi) wgt = samp_w(xs[e], sampling);
              sum += wgt;
              if (wgt > Tf(0)) last = q0 + e;
            }
          }
          const int ch = ((jx + M / 2) * M + jys0) / E;
          chunk[ch] = (double)sum;
          if (last >= 0) lp = max(lp, ch * E + last);
        }
      }
      for (int i = tid; i < M * kLines256; i += kDoeThreads) {
        const int k = i >> 6, cl = i & 63;
        buf[Gm::row(k) + c0 + cl] = ls[cl * kLS256 + sk256(k)];
      }
    }
    *lastpos = lp;
    __syncthreads();
  } else {
  // the map tile goes into rows P.. of buf, which the row pass leaves untouched
  const TileRef tr = tile_of(cfg, c);
  C2<Tf>* tile = Gm::SIZE - Gm::row(P) >= tr.tw * tr.tw ? buf + Gm::row(P) : nullptr;
  if (tile) stage_tile<Tf>(cfg, tr, tm, tile);
  __syncthreads();
  // bilinear samples of the patch into rows 0..P-1, columns 0..P-1 of buf
  if (cfg.planar && tile) {
    const PlanarPatch<Tf> pp = planar_patch<Tf>(cfg, c);
    const int ox = pp.ix0 - tr.tx0, oy = pp.iy0 - tr.ty0;
    const Tf w00 = (Tf(1) - pp.wx) * (Tf(1) - pp.wy), w01 = pp.wx * (Tf(1) - pp.wy);
    const Tf w10 = (Tf(1) - pp.wx) * pp.wy, w11 = pp.wx * pp.wy;
    const int lgP = __builtin_ctz(P);                // P is a power of two
    for (int i = tid; i < P * P; i += kDoeThreads) {
      const int m = i & (P - 1), n = i >> lgP;
      const C2<Tf>* r0 = tile + (oy + n) * tr.tw + ox + m;
      buf[Gm::at(n, m)] = r0[0] * w00 + r0[1] * w01 + r0[tr.tw] * w10 + r0[tr.tw + 1] * w11;
    }
  } else {
    const int lgP = __builtin_ctz(P);
    for (int i = tid; i < P * P; i += kDoeThreads) {
      const int m = i & (P - 1), n = i >> lgP;
      buf[Gm::at(n, m)] = patch_sample_t<Tf>(cfg, c, tm, tile, tr, m, n);
    }
  }
  __syncthreads();
  int lp = -1;
  if constexpr (Gm::kSkew) {
    line_fft2<Tf, M, -1, false>(buf, tw, P, P, M, false);      // rows n < P, inputs m < P
    for (int i = opaque_tid(); i < M; i += kDoeThreads) span[i] = prop_span(c, i - M / 2, M);
    line_fft2<Tf, M, -1, true>(buf, tw, M, P, M, false);       // columns, inputs n < P
    // sampling weights of the chunks of E consecutive rows of a column; a
    // lane's two chunks are loaded together (M * M / E = 2 * kDoeThreads)
    static_assert(M * (M / E) == 2 * kDoeThreads, "two chunks per lane");
    if constexpr (kCdf) {
      C2<Tf> xv[2][E];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int t = tid + j * kDoeThreads;
        const int col = t & (M - 1), ky0 = E * (t / M);
        const int base = Gm::row(ky0) + Gm::col(col);
#pragma unroll
        for (int k2 = 0; k2 < E; ++k2) xv[j][k2] = buf[base + k2 * SM];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int t = tid + j * kDoeThreads;
        const int col = t & (M - 1), ky0 = E * (t / M);
        const int jx = col < M / 2 ? col : col - M;
        const int jys0 = (ky0 + M / 2) & (M - 1);
        const int ch = ((jx + M / 2) * M + jys0) / E;
        const Span sp = span[jx + M / 2];
        Tf sum = Tf(0);
        int last = -1;                                  // last bin of positive weight
#pragma unroll
        for (int k2 = 0; k2 < E; ++k2) {
          const int ky = ky0 + k2;
          const int jy = ky < M / 2 ? ky : ky - M;
          Tf wgt = Tf(0);
          if (jy >= sp.lo && jy <= sp.hi) wgt = samp_w(xv[j][k2], sampling);
          sum += wgt;
          if (wgt > Tf(0)) last = k2;
        }
        chunk[ch] = (double)sum;
        if (last >= 0) lp = max(lp, ch * E + last);
      }
    }
  } else {
    const bool half = 2 * P == M;     // pad factor 2: the upper half of every input is zero
    for (int row = g; row < P; row += G) {
      C2<Tf> x[E];
      if (half) {
#pragma unroll
        for (int n2 = 0; n2 < E; ++n2)
          x[n2] = n2 < E / 2 ? buf[Gm::row(row) + Gm::col_split(gl, L * n2)] : C2<Tf>{Tf(0), Tf(0)};
        group_fft<Tf, L, E, -1, true>(x, gl, tw);
      } else {
#pragma unroll
        for (int n2 = 0; n2 < E; ++n2) {
          const int m = gl + L * n2;
          x[n2] = m < P ? buf[Gm::row(row) + Gm::col_split(gl, L * n2)] : C2<Tf>{Tf(0), Tf(0)};
        }
        group_fft<Tf, L, E, -1>(x, gl, tw);
      }
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) buf[Gm::row(row) + Gm::col(E * br) + k2] = x[k2];
    }
    for (int i = opaque_tid(); i < M; i += kDoeThreads) span[i] = prop_span(c, i - M / 2, M);
    __syncthreads();
    for (int col = g; col < M; col += G) {
      C2<Tf> x[E];
      if (half) {
#pragma unroll
        for (int n2 = 0; n2 < E; ++n2)
          x[n2] = n2 < E / 2 ? buf[Gm::row_split(gl, L * n2) + Gm::col(col)] : C2<Tf>{Tf(0), Tf(0)};
        group_fft<Tf, L, E, -1, true>(x, gl, tw);
      } else {
#pragma unroll
        for (int n2 = 0; n2 < E; ++n2) {
          const int n = gl + L * n2;
          x[n2] = n < P ? buf[Gm::row_split(gl, L * n2) + Gm::col(col)] : C2<Tf>{Tf(0), Tf(0)};
        }
        group_fft<Tf, L, E, -1>(x, gl, tw);
      }
      // this lane now holds rows ky = E*br .. E*br + E - 1 of column col
      const int jx = col < M / 2 ? col : col - M;
      const int ky0 = E * br;
      const int jys0 = (ky0 + M / 2) & (M - 1);                  // shifted row of the first bin
      const int ch = ((jx + M / 2) * M + jys0) / E;              // chunk id (j_x-major)
      const Span sp = span[jx + M / 2];
      Tf s = Tf(0);
      int last = -1;
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) {
        const int ky = ky0 + k2;
        const int jy = ky < M / 2 ? ky : ky - M;
        buf[Gm::row(ky0) + k2 * SM + Gm::col(col)] = x[k2];
        Tf wgt = Tf(0);
        if (jy >= sp.lo && jy <= sp.hi) wgt = samp_w(x[k2], sampling);
        s += wgt;
        if (wgt > Tf(0)) last = k2;
      }
      chunk[ch] = (double)s;
      if (last >= 0) lp = max(lp, ch * E + last);
    }
  }
  *lastpos = lp;
  __syncthreads();
  }
}

// Wave-level prefix operations with DPP row shifts (lanes whose source lies
// outside their 16-lane row keep `old`) and the three row totals by readlane.
template <int CTRL> __device__ __forceinline__ int dpp_shr(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ double dpp_shr_d(double v) {   // 0 without source
  const long long b = __double_as_longlong(v);
  const int lo = dpp_shr<CTRL>(0, (int)(b & 0xffffffff));
  const int hi = dpp_shr<CTRL>(0, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ double wave_incl_sum(double v, int lane) {
  v += dpp_shr_d<0x111>(v);               // row_shr:1
  v += dpp_shr_d<0x112>(v);               // row_shr:2
  v += dpp_shr_d<0x114>(v);               // row_shr:4
  v += dpp_shr_d<0x118>(v);               // row_shr:8
  const double r0 = lane_d(v, 15), r1 = lane_d(v, 31), r2 = lane_d(v, 47);
  const int row = lane >> 4;
  return v + (row >= 1 ? r0 : 0.0) + (row >= 2 ? r1 : 0.0) + (row >= 3 ? r2 : 0.0);
}
// Maximum over the 64 lanes.
__device__ __forceinline__ int wave_max_i(int v) {
  v = max(v, dpp_shr<0x111>(v, v));
  v = max(v, dpp_shr<0x112>(v, v));
  v = max(v, dpp_shr<0x114>(v, v));
  v = max(v, dpp_shr<0x118>(v, v));
  return max(max(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
             max(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}

// Exclusive scan of the chunk sums in place, returning the total S, and the
// block maximum of lp (last bin of positive weight) through the same barrier.
template <int M>
__device__ __forceinline__ double chunk_scan(double* pref, double* red, int lp, int* redi,
                                             int& lp_all) {
  using Gm = DoeGeom<M>;
  constexpr int K = (Gm::NCH + kDoeThreads - 1) / kDoeThreads;
  const int t = threadIdx.x;
  double v[K], tot = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = t * K + k;
    v[k] = i < Gm::NCH ? pref[i] : 0.0;
    tot += v[k];
  }
  // block exclusive scan of the per-thread totals (8 waves)
  const int lane = t & 63, wv = t >> 6;
  const double inc = wave_incl_sum(tot, lane);
  const int wmax = wave_max_i(lp);
  if (lane == 63) { red[wv] = inc; redi[wv] = wmax; }
  __syncthreads();
  double base = 0.0, S = 0.0;
  int m = redi[0];
#pragma unroll
  for (int i = 0; i < kDoeThreads / 64; ++i) {
    if (i < wv) base += red[i];
    S += red[i];
    m = max(m, redi[i]);
  }
  double run = base + inc - tot;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = t * K + k;
    if (i < Gm::NCH) pref[i] = run;
    run += v[k];
  }
  if (t == 0) pref[Gm::NCH] = S;
  lp_all = m;
  __syncthreads();
  return S;
}

__device__ __forceinline__ double block_sum_d(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = 0.0;
  for (int i = 0; i < kDoeThreads / 64; ++i) m += red[i];
  __syncthreads();
  return m;
}

// Inverse-CDF draw: J = min{j : C_j > T} in j_x-major shifted order.
template <class Tf, int M>
__device__ __forceinline__ int draw_bin(const C2<Tf>* buf, const double* pref, const Span* span,
                                        double T, int sampling, int lastpos_all) {
  using Gm = DoeGeom<M>;
  constexpr int E = Gm::E, NCH = Gm::NCH;
  // chunk lo: the last with pref[lo] <= T (prefix sums are non-decreasing),
  // by a 4-way descent: three independent reads per level
  static_assert((NCH & (NCH - 1)) == 0 && NCH >= 4, "chunk count must be a power of two");
  constexpr bool kPow4 = (NCH & 0x55555555) != 0;
  int lo = 0;
  int width = NCH;                               // the chunk is in [lo, lo + width)
  if constexpr (!kPow4) {
    if (pref[NCH / 2] <= T) lo = NCH / 2;
    width = NCH / 2;
  }
  for (int step = width / 4; step >= 1; step /= 4) {
    const double p1 = pref[lo + step], p2 = pref[lo + 2 * step], p3 = pref[lo + 3 * step];
    lo += (p1 <= T ? step : 0) + (p2 <= T ? step : 0) + (p3 <= T ? step : 0);
  }
  const int base = lo * E;                       // linear bin of the chunk's first bin
  const int jx = base / M - M / 2;
  const int kx = jx & (M - 1);
  const Span sp = span[jx + M / 2];
  // double spectra continue the prefix; float spectra rescan the chunk in the
  // type and order of its chunk sum
  constexpr bool kDbl = sizeof(Tf) == sizeof(double);
  const double Tc = kDbl ? T : T - pref[lo];
  Tf run = kDbl ? (Tf)pref[lo] : Tf(0);
  int lp = -1;
  // the chunk's bins are read in groups before the scan (all in range)
  constexpr int EB = E < 16 ? E : 16;
  for (int q0 = 0; q0 < E; q0 += EB) {
    C2<Tf> xs[EB];
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      const int jy = (base % M) + q0 + q - M / 2;
      xs[q] = buf[Gm::at(jy & (M - 1), kx)];
    }
    for (int q = 0; q < EB; ++q) {
      const int jy = (base % M) + q0 + q - M / 2;
      Tf wgt = Tf(0);
      if (jy >= sp.lo && jy <= sp.hi) wgt = samp_w(xs[q], sampling);
      run += wgt;
      if (wgt > Tf(0)) lp = base + q0 + q;
      if ((double)run > Tc) return base + q0 + q;
    }
  }
  return lp >= 0 ? lp : lastpos_all;
}

// Work item = block of rb x rb launch-grid rays of one pair.
struct RayBlockIter {
  int rb, nbx, per_pair, R;
  long long chunk;          // items per chunk of the XCD work distribution (ItemQueue)
  __device__ __forceinline__ int count() const { return rb * rb; }
  // global ray id of ray k of item it (or -1 past the grid edge)
  __device__ __forceinline__ long long ray(long long it, int k, int pair0) const {
    const int pair = pair0 + (int)(it / per_pair);
    const int b = (int)(it % per_pair);
    const int by = b / nbx, bx = b % nbx;
    const int iy = by * rb + k / rb, ix = bx * rb + k % rb;
    if (iy >= R || ix >= R) return -1;
    return (long long)pair * R * R + (long long)iy * R + ix;
  }
};

// Work items of the persistent DOE workgroups, taken dynamically.  Workgroups
// are dispatched to the eight XCDs in turn (XCD = blockIdx % 8).  The item list
// is cut into chunks of C consecutive items dealt to the XCDs in turn (chunk k
// to XCD k % 8), and the workgroups of XCD x take the next item of its chunks,
// in order, from a counter of their own (zeroed before the launch): the items
// in flight on one XCD are neighbouring ray blocks, whose patches share map
// lines in that XCD's L2, and the work balances itself within the XCD.  With
// C = ceil(n / 8) each XCD owns one contiguous eighth (launches over many
// pairs, whose eighths hold the same mix of work); smaller chunks spread a
// single pair's rays of one patch class, which cluster in space, over all
// XCDs.  Other grid sizes share one counter over [0, n).  Returns n when done.
struct ItemQueue {
  unsigned long long* ctr;
  long long end, C, count;
  int x, xcd;
  __device__ __forceinline__ ItemQueue(unsigned long long* c, long long n, long long chunk) {
    const int G = gridDim.x;
    end = n;
    xcd = G % 8 == 0 && n >= G;
    if (xcd) {
      C = chunk < 1 ? 1 : chunk;
      x = blockIdx.x % 8;
      const long long nc = n / C, tail = n % C;
      count = C * (nc / 8 + (x < nc % 8 ? 1 : 0)) + (tail > 0 && nc % 8 == x ? tail : 0);
      ctr = c + x;
    } else {
      C = n;
      x = 0;
      count = n;
      ctr = c;
    }
  }
  // the workgroup's next item (every thread calls it; two barriers)
  __device__ __forceinline__ long long next(long long* slot) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const long long l = (long long)atomicAdd(ctr, 1ull);
      *slot = l >= count ? end : xcd ? ((l / C) * 8 + x) * C + l % C : l;
    }
    __syncthreads();
    return *slot;
  }
};

// ------------------------------------------------------------------ forward ---
// Two-DOE cascade (kCasc): 1 = the first DOE, whose secondaries become the
// second DOE's incident rays (relay records) instead of sensor records; 2 = the
// second DOE, whose incident rays carry a complex amplitude and whose draws take
// Philox stream 1; 0 = a single DOE.
template <class Prec, int M, bool kLDS, int kCasc = 0>
__global__ __launch_bounds__(kDoeThreads) void k_doe_fwd2(DoeArgs a, RayBlockIter itr,
                                                          long long n_items, int pair0) {
  using Tf = typename Prec::Tf;
  using Tg = typename Prec::Tg;
  using Tp = typename Prec::Tp;
  using Gm = DoeGeom<M>;
  constexpr int SM = Gm::SM;
  __shared__ DoeLds<Tf, M, kLDS> s;
  const DevCfg& cfg = *a.cfg;
  C2<Tf>* buf = kLDS ? s.buf : (C2<Tf>*)a.scratch + (size_t)blockIdx.x * Gm::SIZE;
  const C2<Tf>* tm = (const C2<Tf>*)a.tmap;
  for (int i = threadIdx.x; i < M; i += kDoeThreads) s.tw[i] = ((const C2<Tf>*)a.tw)[i];
  __syncthreads();
  // NS: sample slots per ray (the stride of the index arrays); N: draws of this
  // launch's patch class (NS unless the draws are scaled by class)
  const int NS = cfg.N, N = cfg.class_n[a.cls], t = threadIdx.x, emit = a.emit;
  const double inv_m2 = 1.0 / ((double)M * M);
  unsigned long long n_sec = 0, n_alive = 0, n_lost = 0, n_evan = 0, n_bins = 0;
  // rays in work-list order; the class, alive flag and context word (thread
  // t < kCtxWords) of the next ray are loaded while the current one runs
  const int cnt = itr.count();
  __shared__ long long s_item;
  ItemQueue queue(a.wctr, n_items, itr.chunk);
  long long it_n = queue.next(&s_item);
  int k_n = 0;
  long long gid_n = -1;
  int cls_n = -1;
  double alive_n = 0.0;
  uint32_t cw_n = 0;
  auto fetch = [&]() {
    gid_n = it_n < queue.end ? itr.ray(it_n, k_n, pair0) : -1;
    if (gid_n >= 0) {
      cls_n = a.ray_class[gid_n];
      alive_n = a.st[7 * a.n_total + gid_n];
      if (t < kCtxWords) cw_n = reinterpret_cast<const uint32_t*>(a.ctx + gid_n)[t];
    }
  };
  fetch();
  while (it_n < queue.end) {                   // uniform over the workgroup
    {
      const long long gid = gid_n;
      const int cls = cls_n;
      const double alive = alive_n;
      const uint32_t cw = cw_n;
      if (++k_n == cnt) { k_n = 0; it_n = queue.next(&s_item); }
      fetch();
      if (gid < 0 || cls != a.cls) continue;   // past the grid edge or other patch class
      const size_t slot0 = ((size_t)gid - a.ray0) * (size_t)emit;
      if (alive == 0.0) {
        for (int i = t; i < emit; i += kDoeThreads) {
          if constexpr (kCasc == 1) relay_none(a, (int)(gid / cfg.R2), (int)(gid % cfg.R2), i);
          else put_none<Tg>(a, slot0 + i);
        }
        if (a.idx_out && cfg.sampling != 2)
          for (int i = t; i < NS; i += kDoeThreads) a.idx_out[gid * NS + i] = -1;
        continue;
      }
      n_alive += (t == 0);
      if (t < kCtxWords) reinterpret_cast<uint32_t*>(&s.ctx)[t] = cw;
      __syncthreads();
      const RayCtx& c = s.ctx;
      const int t = opaque_tid();
      const int P = c.P;
      // class weight (P_0 / P)^2: on one ray grid every part of the DOE counts
      // equally whatever the patch side that covers it (a power of two: exact)
      const Tp fk = (Tp)class_weight(cfg, P);
      // incident amplitude at the second DOE of a cascade (1 otherwise)
      C2<Tp> ain = {Tp(1), Tp(0)};
      if constexpr (kCasc == 2) ain = {(Tp)a.ain[gid], (Tp)a.ain[a.n_total + gid]};
      int lp;
      doe_spectrum<Tf, M>(cfg, c, tm, buf, s.tw, s.pref, s.span, cfg.sampling, &lp, s.ls);
      if (t < M) {
        const Span sp = s.span[t];
        n_evan += (unsigned long long)(M - (sp.hi >= sp.lo ? sp.hi - sp.lo + 1 : 0));
      }
      n_bins += t == 0 ? (unsigned long long)M * M : 0ull;
      if (cfg.sampling == 2) {
        // slots beyond this class's M^2 bins (classes smaller than the largest)
        if constexpr (kCasc != 1)
          for (int Lb = M * M + t; Lb < emit; Lb += kDoeThreads) put_none<Tg>(a, slot0 + Lb);
        for (int Lb = t; Lb < M * M; Lb += kDoeThreads) {
          const int jx = Lb / M - M / 2, jy = Lb % M - M / 2;
          const Span sp = s.span[jx + M / 2];
          const bool prop = jy >= sp.lo && jy <= sp.hi;
          if constexpr (kCasc == 1) {
            if (!prop) {
              relay_none(a, c.pair, c.r, Lb);
              continue;
            }
            const C2<Tf> X = buf[Gm::at(jy & (M - 1), jx & (M - 1))];
            const C2<Tf> U = X * centre_ref<Tf>(jx, jy, P, M);
            const C2<Tp> w = C2<Tp>{(Tp)U.re * (Tp)inv_m2, (Tp)U.im * (Tp)inv_m2} * ain;
            const bool ok = relay_secondary<Prec>(a, c, jx, jy, (double)w.re, (double)w.im, Lb);
            n_sec += ok;
            n_lost += !ok;
            continue;
          } else {
            Tp phi0, wx, wy; double dza; Secondary sec;
            if (!prop || !secondary_to_sensor<Prec>(a, c, jx, jy, phi0, wx, wy, dza, sec)) {
              n_lost += prop;
              put_none<Tg>(a, slot0 + Lb);
              continue;
            }
            const C2<Tf> X = buf[Gm::at(jy & (M - 1), jx & (M - 1))];
            const C2<Tf> U = X * centre_ref<Tf>(jx, jy, P, M);
            C2<Tp> w = {(Tp)U.re * (Tp)inv_m2 * fk, (Tp)U.im * (Tp)inv_m2 * fk};
            if constexpr (kCasc == 2) w = w * ain;
            const C2<Tp> cv = (w * wavelet_cis<Prec>(phi0)) * (Tp)dza;
            put_record<Prec>(a, slot0 + Lb, C2<Tg>{(Tg)cv.re, (Tg)cv.im}, wx, wy);
            ++n_sec;
          }
        }
        __syncthreads();
        continue;
      }
      int lastpos_all;
      const double S = chunk_scan<M>(s.pref, s.red, lp, s.redi, lastpos_all);
      const double scale = S * inv_m2 / N;               // S or |Pi| over M^2 N
      if (t == 0) a.ctx[gid].S = S;                      // for the backward
      // slots beyond this class's draws carry nothing
      for (int i = N + t; i < NS; i += kDoeThreads) {
        if (a.idx_out) a.idx_out[gid * NS + i] = -1;
        if (a.jdraw) a.jdraw[gid * NS + i] = -1;
        if constexpr (kCasc == 1) relay_none(a, c.pair, c.r, i);
        else put_none<Tg>(a, slot0 + i);
      }
      for (int i = t; i < N; i += kDoeThreads) {
        int J = -1;
        if (S > 0.0) {
          if (a.replay) {
            J = a.replay[gid * NS + i];
          } else {
            const double T = draw_uniform(cfg.key0, cfg.key1, (uint32_t)i, (uint32_t)c.r,
                                          (uint32_t)c.pair, kCasc == 2 ? 1u : 0u) * S;
            J = draw_bin<Tf, M>(buf, s.pref, s.span, T, cfg.sampling, lastpos_all);
          }
        }
        if (a.idx_out) a.idx_out[gid * NS + i] = J;
        if (a.jdraw) a.jdraw[gid * NS + i] = J;
        bool ok = J >= 0;
        C2<Tp> w = {Tp(0), Tp(0)};
        int jx = 0, jy = 0;
        if (ok) {
          jx = J / M - M / 2; jy = J % M - M / 2;
          const C2<Tf> X = buf[Gm::at(jy & (M - 1), jx & (M - 1))];
          const C2<Tf> U = X * centre_ref<Tf>(jx, jy, P, M);
          if (cfg.sampling == 0) {
            const Tf mag = cabs_rn(X);
            ok = mag > Tf(0);
            const Tp f = ok ? (Tp)(scale / (double)mag) : Tp(0);
            w = {(Tp)U.re * f * fk, (Tp)U.im * f * fk};
          } else {
            w = {(Tp)U.re * (Tp)scale * fk, (Tp)U.im * (Tp)scale * fk};
          }
        }
        if constexpr (kCasc == 1) {
          if (!ok) {
            relay_none(a, c.pair, c.r, i);
            continue;
          }
          w = w * ain;
          ok = relay_secondary<Prec>(a, c, jx, jy, (double)w.re, (double)w.im, i);
          n_sec += ok;
          n_lost += !ok;
          continue;
        }
        Tp phi0, wx, wy; double dza; Secondary sec;
        if (ok) {
          ok = secondary_to_sensor<Prec>(a, c, jx, jy, phi0, wx, wy, dza, sec);
          n_lost += !ok;
        }
        if (!ok) {
          put_none<Tg>(a, slot0 + i);
          continue;
        }
        if constexpr (kCasc == 2) w = w * ain;
        const C2<Tp> cv = (w * wavelet_cis<Prec>(phi0)) * (Tp)dza;
        put_record<Prec>(a, slot0 + i, C2<Tg>{(Tg)cv.re, (Tg)cv.im}, wx, wy);
        ++n_sec;
      }
      __syncthreads();   // buf and pref are reused by the next ray
    }
  }
  if (a.stats) {
    if (n_alive) atomicAdd(&a.stats[RW_ST_ALIVE], n_alive);
    if (n_alive) atomicAdd(&a.stats[RW_ST_CLASS0 + a.cls], n_alive);
    if (n_sec) atomicAdd(&a.stats[RW_ST_SEC], n_sec);
    if (n_lost) atomicAdd(&a.stats[RW_ST_LOST], n_lost);
    if (n_evan) atomicAdd(&a.stats[RW_ST_EVAN], n_evan);
    if (n_bins) atomicAdd(&a.stats[RW_ST_BINS], n_bins);
  }
}

// ------------------------------------------------------------------ adjoint ---
// Type-2 interpolation of the sensor-grid cogradient B at one wavelet's grid
// coordinate, with the ES-kernel derivative for the two frequencies.  Two
// adjacent lanes share one wavelet: lane h takes the kernel rows j = h, h + 2,
// ...; the partial sums are exchanged so both lanes return the totals.  Every
// row loads WMAX cells unconditionally (indices wrap on the periodic grid) so
// that the loads of all rows are in flight together.
template <class Prec, int WMAX>
__device__ __forceinline__ void interp_adj_pair(const DevCfg& cfg,
                                                const C2<typename Prec::Tg>* B, int pair,
                                                typename Prec::Tp gx, typename Prec::Tp gy, int h,
                                                C2<double>& g0, C2<double>& dx, C2<double>& dy) {
  using Tg = typename Prec::Tg;
  using Tp = typename Prec::Tp;
  const int nf = cfg.nf, w = cfg.w;
  const int lx0 = (int)ceil(gx - (Tp)(0.5 * w)), ly0 = (int)ceil(gy - (Tp)(0.5 * w));
  const Tg tw = (Tg)(2.0 / w), beta = (Tg)cfg.beta;
  Tg kx[WMAX], dkx[WMAX];
#pragma unroll
  for (int i = 0; i < WMAX; ++i) {
    kx[i] = Tg(0); dkx[i] = Tg(0);
    if (i < w) {
      const Tg tx = (Tg)((double)((Tp)(lx0 + i) - gx)) * tw;
      const Tg ax = Tg(1) - tx * tx;
      if (ax > Tg(0)) {
        const Tg sx = sqrt(ax);
        kx[i] = (Tg)exp(beta * (sx - Tg(1)));
        dkx[i] = -kx[i] * beta * tx / sx * tw;
      }
    }
  }
  g0 = {0, 0}; dx = {0, 0}; dy = {0, 0};
  const C2<Tg>* gp = B + (size_t)pair * nf * nf;
  constexpr int RH = (WMAX + 1) / 2;                       // rows per lane
  constexpr int RBr = 16 / WMAX / (int)(sizeof(Tg) / 4);     // rows loaded together
  constexpr int RB = RBr < 1 ? 1 : (RBr > RH ? RH : RBr);
#pragma unroll
  for (int r0 = 0; r0 < RH; r0 += RB) {
    C2<Tg> v[RB][WMAX];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const C2<Tg>* row = gp + (size_t)((ly0 + 2 * (r0 + r) + h) & (nf - 1)) * nf;
#pragma unroll
      for (int i = 0; i < WMAX; ++i) v[r][i] = row[(lx0 + i) & (nf - 1)];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int j = 2 * (r0 + r) + h;
      const Tg ty = (Tg)((double)((Tp)(ly0 + j) - gy)) * tw;
      const Tg ay = Tg(1) - ty * ty;
      if (!(j < w && ay > Tg(0))) continue;
      const Tg sy = sqrt(ay);
      const Tg ky = (Tg)exp(beta * (sy - Tg(1)));
      const Tg dky = -ky * beta * ty / sy * tw;
      Tg s0r = 0, s0i = 0, s1r = 0, s1i = 0;
#pragma unroll
      for (int i = 0; i < WMAX; ++i) {
        s0r += kx[i] * v[r][i].re; s0i += kx[i] * v[r][i].im;
        s1r += dkx[i] * v[r][i].re; s1i += dkx[i] * v[r][i].im;
      }
      g0.re += (double)(ky * s0r); g0.im += (double)(ky * s0i);
      dx.re += (double)(ky * s1r); dx.im += (double)(ky * s1i);
      dy.re += (double)(dky * s0r); dy.im += (double)(dky * s0i);
    }
    // keep the next group's loads from being scheduled above this point
    __builtin_amdgcn_sched_barrier(0);
  }
  g0.re += xor_lane<1>(g0.re); g0.im += xor_lane<1>(g0.im);
  dx.re += xor_lane<1>(dx.re); dx.im += xor_lane<1>(dx.im);
  dy.re += xor_lane<1>(dy.re); dy.im += xor_lane<1>(dy.im);
}

// Cogradients of one wavelet's inputs (its weight w, phase, grid frequencies and
// obliquity) from the interpolated sensor-grid cogradient; called by both lanes
// of a pair with identical arguments.  The interpolation comes from the tiled
// pass when it covered this record (record slot `slot`, non-zero forward value),
// else it is done here.
// kAmp (second DOE of a cascade): the record also carries the ray's incident
// amplitude ain; g_a receives dL/d(ain) of this wavelet.
template <class Prec, bool kTiled, bool kAmp = false>
__device__ __forceinline__ bool wavelet_adjoint_pair(const DoeArgs& a, const RayCtx& c, int jx,
                                                     int jy, C2<typename Prec::Tp> w, int h,
                                                     size_t slot, WaveletAdj& wa, Secondary& sec,
                                                     C2<double> ain = {1.0, 0.0},
                                                     C2<double>* g_a = nullptr) {
  using Tp = typename Prec::Tp;
  using Tg = typename Prec::Tg;
  const DevCfg& cfg = *a.cfg;
  Tp phi0, wx, wy;
  double dza;
  if (!secondary_to_sensor<Prec>(a, c, jx, jy, phi0, wx, wy, dza, sec)) return false;
  const C2<Tp> e = wavelet_cis<Prec>(phi0);
  const C2<Tp> cv = (w * e) * (Tp)dza;
  C2<double> g0, dx, dy;
  bool tiled = kTiled;
  if (!kTiled && a.interp) tiled = !is_none(((const C2<Tg>*)a.rec_val)[slot]);
  if (tiled) {
    const C2<Tg>* q = (const C2<Tg>*)a.interp + kInterpStride * slot;
    const C2<Tg> q0 = q[0], q1 = q[1], q2 = q[2];
    g0 = {(double)q0.re, (double)q0.im};
    dx = {(double)q1.re, (double)q1.im};
    dy = {(double)q2.re, (double)q2.im};
  } else if constexpr (!kTiled) {
    const Tp gx = grid_coord(wx, cfg.nf), gy = grid_coord(wy, cfg.nf);
    if (cfg.w <= 8)
      interp_adj_pair<Prec, 8>(cfg, (const C2<Tg>*)a.adj, c.pair, gx, gy, h, g0, dx, dy);
    else
      interp_adj_pair<Prec, 16>(cfg, (const C2<Tg>*)a.adj, c.pair, gx, gy, h, g0, dx, dy);
  }
  // the record carries the class weight (P_0 / P)^2 (exact power of two)
  const double fk = class_weight(cfg, c.P);
  C2<double> cd = {(double)cv.re * fk, (double)cv.im * fk};
  double er = (double)e.re * dza * fk, ei = (double)e.im * dza * fk;
  if constexpr (kAmp) {
    // record = ain w E, E = e |d_z| fk: dL/d(ain) = conj(w E) g0, dL/dw = conj(ain E) g0
    const double wr = (double)w.re * er - (double)w.im * ei, wi = (double)w.re * ei + (double)w.im * er;
    *g_a = {wr * g0.re + wi * g0.im, wr * g0.im - wi * g0.re};
    cd = {cd.re * ain.re - cd.im * ain.im, cd.re * ain.im + cd.im * ain.re};
    const double r2 = er * ain.re - ei * ain.im, i2 = er * ain.im + ei * ain.re;
    er = r2;
    ei = i2;
  }
  const double cell = cfg.nf / (2.0 * RW_PI);
  wa.g_wx = -(cd.re * dx.re + cd.im * dx.im) * cell;
  wa.g_wy = -(cd.re * dy.re + cd.im * dy.im) * cell;
  wa.g_phi0 = -(g0.re * cd.im - g0.im * cd.re);
  wa.g_dz = (g0.re * cd.re + g0.im * cd.im) / dza;
  wa.g_w = {er * g0.re + ei * g0.im, er * g0.im - ei * g0.re};
  return true;
}

// First DOE of a cascade: the weight cogradient of its secondary i is dL/d(ain)
// of the second DOE's ray that the secondary became (the relay record); the
// secondary's direction follows from its bin alone, so nothing else flows back.
__device__ __forceinline__ bool relay_cograd(const DoeArgs& a, const RayCtx& c, int i,
                                             WaveletAdj& wa) {
  const size_t g = relay_gid(*a.cfg, *a.cfg2, c.pair, c.r, i);
  wa.g_phi0 = wa.g_wx = wa.g_wy = wa.g_dz = 0.0;
  if (a.relay[7 * a.relay_n + g] == 0.0) return false;
  wa.g_w = {a.gain[g], a.gain[a.relay_n + g]};
  return true;
}

// Spectrum cogradient of one draw, kept in global memory between the draw pass
// and the S-term pass (bin index k into the LDS spectrum, -1 for none).
// ------------------------------------------------ G2: straight-through ---
// Gumbel-softmax straight-through gradient of the p_mag draws (reparameterised
// sampling, Fig. 1c).  Draw i (bin J_i) keeps its hard value; its gradient flows
// through y_i = softmax((log p + z_i) / tau), z_i the Gumbel perturbations of
// its replica, regenerated conditioned on argmax = J_i (top-down construction
// of Maddison, Tarlow & Minka 2014): the maximum G*_i = Gumbel(u*_i) (log of
// the total mass is 0) sits at J_i, every other bin k takes the Gumbel
// log p_k - log(-log u_ik) truncated below G*_i.  With the draw's weight and
// wavevector relaxed to sum_k y_k w_k and sum_k y_k K_k,
//     g_ik = dL/dy_ik = <A_i, w_k> + <B_i, K_k>,  A = dL/dw, B = dL/dK,
//     dL/dlog p_k = (1/tau) sum_i y_ik (g_ik - <y_i, g_i>),
// and log p_k = log|U~_k| - log S sends X_k/|X_k| (dL/dlog p_k / |X_k| - D / S),
// D = sum_k dL/dlog p_k, into the spectrum cogradient.
// Uniforms: u*_i from counter (i >> 2, ray, pair, 2), u_ik from counter
// (k, ray, pair, 0x10000 | (i >> 2)), word i & 3, k the inverse-CDF bin index.
// With L = -log u, L* = -log u* (so G* = -log L*) and P_k = 1/p_k, the
// truncated score gives exp((phi_k - G*) / tau) = (1 + P_k L / L*)^(-1/tau)
// for k != J and 1 at J.
struct G2Bin {              // per-bin quantities of one ray
  bool live;
  float P, wr, wi, Ku, Kv;  // 1/p, weight w_k, wavevector K_k
};

template <class Tf, int M>
__device__ __forceinline__ G2Bin g2_bin(const RayCtx& c, const C2<Tf>* buf, const Span* span,
                                        int k, int P, float S, float wmag) {
  constexpr int SM = DoeGeom<M>::SM;
  const int jx = k / M - M / 2, jy = k % M - M / 2;
  const Span sp = span[jx + M / 2];
  G2Bin b;
  b.live = false;
  if (jy < sp.lo || jy > sp.hi) return b;
  const C2<Tf> X = buf[DoeGeom<M>::at(jy & (M - 1), jx & (M - 1))];
  const float m2 = (float)X.re * (float)X.re + (float)X.im * (float)X.im;
  if (!(m2 > 0.0f)) return b;
  const float im = rsqrtf(m2);
  const C2<Tf> U = X * centre_ref<Tf>(jx, jy, P, M);
  b.live = true;
  b.P = S * im;
  b.wr = (float)U.re * im * wmag;
  b.wi = (float)U.im * im * wmag;
  b.Ku = (float)(c.kin_u + c.dk * jx);
  b.Kv = (float)(c.kin_v + c.dk * jy);
  return b;
}

// The four uniforms u_ik of draws 4 gi .. 4 gi + 3 at bin k.
__device__ __forceinline__ void g2_uniforms(const DevCfg& cfg, const RayCtx& c, int k, int gi,
                                            float u[4]) {
  uint32_t w[4] = {(uint32_t)k, (uint32_t)c.r, (uint32_t)c.pair, 0x10000u | (uint32_t)gi};
  philox4x32_10(w, cfg.key0, cfg.key1);
#pragma unroll
  for (int q = 0; q < 4; ++q) u[q] = ((float)(w[q] >> 9) + 0.5f) * (1.0f / 8388608.0f);
}

// exp((phi - G*) / tau) of a bin that is not the drawn one.
__device__ __forceinline__ float g2_weight(float P, float u, float inv_ls, float itau, bool unit) {
  const float x = fmaf(P * -__logf(u), inv_ls, 1.0f);
  return unit ? __frcp_rn(x) : __expf(-itau * __logf(x));
}

// Per-block draw record of the G2 pass (floats): [0..1] A = dL/dw, [2..3]
// B = dL/dK, [4] J (bit pattern of an int, -1: no gradient), [5] 1/L*,
// [6] 1/Z, [7] <y, g>.
constexpr int kG2Rec = 8;

// Pass 1 (a wave per group of four draws): the softmax normaliser Z_i and
// <y_i, g_i> of every draw.  Pass 2 (a lane per bin, the S-term layout):
// dL/dlog p_k into dlg; returns D = sum_k dL/dlog p_k.
template <class Prec, int M>
__device__ double g2_passes(const DoeArgs& a, const RayCtx& c,
                            const C2<typename Prec::Tf>* buf, const Span* span, double S,
                            float* gd, float* dlg, double* red, float* lrec) {
  using Tf = typename Prec::Tf;
  const DevCfg& cfg = *a.cfg;
  const int N = cfg.class_n[a.cls], P = c.P;   // this class's draws (records beyond are unused)
  const int t = opaque_tid(), lane = t & 63, wv = t >> 6;
  constexpr int NW = kDoeThreads / 64;
  const float Sf = (float)S;
  const float wmag = (float)(S / ((double)M * M * N));
  const float itau = (float)(1.0 / cfg.tau);
  const bool unit = cfg.tau == 1.0;
  const int ng = (N + 3) / 4;
  for (int gi = wv; gi < ng; gi += NW) {
    float Ar[4], Ai[4], Bu[4], Bv[4], IL[4];
    int J[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 4 * gi + q;
      J[q] = -1;
      Ar[q] = Ai[q] = Bu[q] = Bv[q] = IL[q] = 0.0f;
      if (i < N) {
        const float* e = gd + (size_t)i * kG2Rec;
        J[q] = __float_as_int(e[4]);
        Ar[q] = e[0]; Ai[q] = e[1]; Bu[q] = e[2]; Bv[q] = e[3];
        const double us = draw_uniform(cfg.key0, cfg.key1, (uint32_t)i, (uint32_t)c.r,
                                       (uint32_t)c.pair, 2u);
        IL[q] = (float)(1.0 / -log(us));
      }
    }
    float Z[4] = {0, 0, 0, 0}, Sg[4] = {0, 0, 0, 0};
    for (int k = lane; k < M * M; k += 64) {
      const G2Bin b = g2_bin<Tf, M>(c, buf, span, k, P, Sf, wmag);
      if (!b.live) continue;
      float u[4];
      g2_uniforms(cfg, c, k, gi, u);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (J[q] < 0) continue;
        const float e = k == J[q] ? 1.0f : g2_weight(b.P, u[q], IL[q], itau, unit);
        const float g = Ar[q] * b.wr + Ai[q] * b.wi + Bu[q] * b.Ku + Bv[q] * b.Kv;
        Z[q] += e;
        Sg[q] += e * g;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double z = wave_sum((double)Z[q]), sg = wave_sum((double)Sg[q]);
      const int i = 4 * gi + q;
      if (lane == 0 && i < N) {
        float* e = gd + (size_t)i * kG2Rec;
        e[5] = IL[q];
        e[6] = z > 0.0 ? (float)(1.0 / z) : 0.0f;
        e[7] = z > 0.0 ? (float)(sg / z) : 0.0f;
      }
    }
  }
  __syncthreads();
  // pass 2 reads the draw records from LDS when a buffer is given (every lane
  // reads the same record at a time: broadcasts)
  const float* rec = gd;
  if (lrec) {
    for (int i = t; i < N * kG2Rec; i += kDoeThreads) lrec[i] = gd[i];
    __syncthreads();
    rec = lrec;
  }
  double Dsum = 0.0;
  const int kx = t % M;
  for (int ky = t / M; ky < M; ky += kDoeThreads / M) {
    const int jx = kx < M / 2 ? kx : kx - M, jy = ky < M / 2 ? ky : ky - M;
    const int k = (jx + M / 2) * M + (jy + M / 2);
    const G2Bin b = g2_bin<Tf, M>(c, buf, span, k, P, Sf, wmag);
    float acc = 0.0f;
    if (b.live) {
      for (int gi = 0; gi < ng; ++gi) {
        float u[4];
        g2_uniforms(cfg, c, k, gi, u);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 4 * gi + q;
          if (i >= N) break;
          const float* e = rec + (size_t)i * kG2Rec;
          const int J = __float_as_int(e[4]);
          if (J < 0) continue;
          const float y = (k == J ? 1.0f : g2_weight(b.P, u[q], e[5], itau, unit)) * e[6];
          const float g = e[0] * b.wr + e[1] * b.wi + e[2] * b.Ku + e[3] * b.Kv;
          acc += y * (g - e[7]);
        }
      }
    }
    const float dl = acc * itau;
    dlg[ky * M + kx] = dl;
    Dsum += dl;
  }
  return block_sum_d(Dsum, red);
}

// kTiled: the sensor-grid cogradient of every record comes from the tiled
// interpolation pass (one lane per secondary ray); otherwise the kernel
// interpolates it itself (two lanes per secondary ray share the kernel rows).
// kCasc: 1 = the first DOE of a cascade (draws' weight cogradients from the
// relayed rays), 2 = the second DOE (records carry the incident amplitude;
// writes dL/d(ain) per ray), 0 = a single DOE.
template <class Prec, int M, bool kLDS, bool kG2, bool kTiled, bool kFull, int kCasc = 0>
__global__ __launch_bounds__(kDoeThreads) void k_doe_bwd2(DoeArgs a, RayBlockIter itr,
                                                          long long n_items, int pair0) {
  using Tf = typename Prec::Tf;
  using Tg = typename Prec::Tg;
  using Tp = typename Prec::Tp;
  using Gm = DoeGeom<M>;
  constexpr int L = Gm::L, E = Gm::E, G = Gm::G, SM = Gm::SM;
  __shared__ DoeLds<Tf, M, kLDS> s;
  __shared__ int s_box[4];
  const DevCfg& cfg = *a.cfg;
  C2<Tf>* buf = kLDS ? s.buf : (C2<Tf>*)a.scratch + (size_t)blockIdx.x * Gm::SIZE;
  const C2<Tf>* tm = (const C2<Tf>*)a.tmap;
  C2<Tg>* gt = (C2<Tg>*)a.gt;
  // block-private accumulator of dL/dt over one ray block
  const int AS = a.acc_side;
  C2<Tg>* accm = (C2<Tg>*)a.acc + (size_t)blockIdx.x * AS * AS;
  for (int i = threadIdx.x; i < M; i += kDoeThreads) s.tw[i] = ((const C2<Tf>*)a.tw)[i];
  __syncthreads();
  const int NS = cfg.N, N = cfg.class_n[a.cls], t = threadIdx.x;
  static_assert(kDoeThreads % M == 0, "the S-term pass keeps one column per lane");
  const double inv_m2 = 1.0 / ((double)M * M);
  const int H = cfg.H, W = cfg.W;
  __shared__ long long s_item;
  ItemQueue queue(a.wctr, n_items, itr.chunk);
  for (long long it = queue.next(&s_item); it < queue.end; it = queue.next(&s_item)) {
    // anchor of the accumulator: the first live ray of the block
    if (t == 0) { s_box[0] = INT_MAX; s_box[1] = INT_MAX; s_box[2] = INT_MIN; s_box[3] = INT_MIN; }
    int ax0 = 0, ay0 = 0;
    bool have_anchor = false;
    for (int k = 0; k < itr.count() && !have_anchor; ++k) {
      const long long gid = itr.ray(it, k, pair0);
      if (gid < 0 || a.st[7 * a.n_total + gid] == 0.0 || a.ray_class[gid] != a.cls) continue;
      const double fx = (a.st[0 * a.n_total + gid] - cfg.x0) * cfg.inv_pitch;
      const double fy = (a.st[1 * a.n_total + gid] - cfg.y0) * cfg.inv_pitch;
      ax0 = (int)floor(fx) - AS / 2;
      ay0 = (int)floor(fy) - AS / 2;
      have_anchor = true;
    }
    __syncthreads();
    if (!have_anchor) continue;
    // the alive flag, class and context word (thread t < kCtxWords) of the
    // block's next ray are loaded while the current one runs
    const int cnt = itr.count();
    long long gid_n = itr.ray(it, 0, pair0);
    double alive_n = 0.0;
    int cls_n = -1;
    uint32_t cw_n = 0;
    auto fetch = [&]() {
      if (gid_n >= 0) {
        alive_n = a.st[7 * a.n_total + gid_n];
        cls_n = a.ray_class[gid_n];
        if (t < kCtxWords) cw_n = reinterpret_cast<const uint32_t*>(a.ctx + gid_n)[t];
      }
    };
    fetch();
    for (int k = 0; k < cnt; ++k) {
      const long long gid = gid_n;
      const double alive = alive_n;
      const int cls = cls_n;
      const uint32_t cw = cw_n;
      gid_n = k + 1 < cnt ? itr.ray(it, k + 1, pair0) : -1;
      fetch();
      if (gid < 0 || alive == 0.0 || cls != a.cls) continue;
      if (t < kCtxWords) reinterpret_cast<uint32_t*>(&s.ctx)[t] = cw;
      __syncthreads();
      const RayCtx& c = s.ctx;
      const int t = opaque_tid();
      const int g = t / L, gl = t % L, br = bitrev(gl, Gm::LB);
      const int P = c.P;
      const int T = P + 4;                                // bilinear tile side
      const bool use_tile = Gm::SIZE - Gm::row(P) >= T * T;
      const size_t slot0 = ((size_t)gid - a.ray0) * (size_t)a.emit;   // this ray's records
      // second DOE of a cascade: the ray's incident amplitude, and the sum of
      // dL/d(ain) over its wavelets
      C2<double> ain = {1.0, 0.0};
      if constexpr (kCasc == 2) ain = {a.ain[gid], a.ain[a.n_total + gid]};
      double gar = 0.0, gai = 0.0;
      // the forward's draws and normaliser (it records them for every sampled
      // ray): no CDF here
      const int jpre = !kFull && t < N ? a.jdraw[gid * NS + t] : -1;  // first draw of lane t
      int lp = -1;
      doe_spectrum<Tf, M, false>(cfg, c, tm, buf, s.tw, s.pref, s.span, cfg.sampling, &lp,
                                 s.ls);
      IncAcc acc = {{0, 0, 0}, {0, 0}, 0, 0, {0, 0, 0}};
      double dLdS = 0.0;
      constexpr int LPD = kTiled ? 1 : 2;   // lanes per secondary ray
      const int h = kTiled ? 0 : (t & 1);
      const bool lead = kTiled || h == 0;   // writes the draw's entries
      const bool side = kTiled || h == 1;   // accumulates the incident-state cogradient
      // M = 256: the normaliser and draw terms are formed as the inverse column
      // pass stages the spectrum (no extra pass over the global buffer)
      Tf fold_fS = Tf(0), fold_d2s = Tf(0);
      const float* fold_dlg = nullptr;
      const DrawEnt<Tf>* fold_dl = nullptr;
      if constexpr (!kFull) {
        const double S = c.S;
        DrawEnt<Tf>* gdl = (DrawEnt<Tf>*)a.dlist + (size_t)blockIdx.x * N;
        const bool dl_lds = kLDS && N <= kDrawLds;
        if (S > 0.0) {
          const double scale = S * inv_m2 / N;
#pragma unroll 1
          for (int i = t / LPD; i < N; i += kDoeThreads / LPD) {
            const int J = i == t ? jpre : a.jdraw[gid * NS + i];
            DrawEnt<Tf> ent = {{Tf(0), Tf(0)}, -1};
            double g2r[5] = {0.0, 0.0, 0.0, 0.0, -1.0};      // A, B, J of the G2 record
            if (J >= 0) {
              const int jx = J / M - M / 2, jy = J % M - M / 2;
              const int kidx = Gm::at(jy & (M - 1), jx & (M - 1));
              const C2<Tf> X = buf[kidx];
              const C2<Tf> ref = centre_ref<Tf>(jx, jy, P, M);
              const C2<Tf> U = X * ref;
              C2<Tp> w;
              double mag = 0.0;
              bool ok = true;
              if (cfg.sampling == 0) {
                const Tf m = cabs_rn(X);
                ok = m > Tf(0);
                mag = (double)m;
                const Tp f = ok ? (Tp)(scale / mag) : Tp(0);
                w = {(Tp)U.re * f, (Tp)U.im * f};
              } else {
                w = {(Tp)U.re * (Tp)scale, (Tp)U.im * (Tp)scale};
              }
              WaveletAdj wa;
              Secondary sec;
              if (ok) {
                if constexpr (kCasc == 1) {
                  ok = relay_cograd(a, c, i, wa);
                } else if constexpr (kCasc == 2) {
                  C2<double> ga;
                  ok = wavelet_adjoint_pair<Prec, kTiled, true>(a, c, jx, jy, w, h, slot0 + i, wa,
                                                                sec, ain, &ga);
                  if (ok && lead) { gar += ga.re; gai += ga.im; }
                } else {
                  ok = wavelet_adjoint_pair<Prec, kTiled>(a, c, jx, jy, w, h, slot0 + i, wa, sec);
                }
              }
              if (ok) {
                C2<double> gU;
                if (cfg.sampling == 0 && cfg.grad == kGradG1Detach) {
                  // p held constant: w = U scale / |X| with a constant factor
                  gU = {wa.g_w.re * scale / mag, wa.g_w.im * scale / mag};
                } else if (cfg.sampling == 0) {
                  const double hr = (double)U.re / mag, hi_ = (double)U.im / mag;
                  if (lead) dLdS += (wa.g_w.re * hr + wa.g_w.im * hi_) * inv_m2 / N;
                  const double gr = wa.g_w.re * scale, gi = wa.g_w.im * scale;
                  const double im = -(gr * hi_ - gi * hr) / mag;
                  gU = {-im * hi_, im * hr};
                } else {
                  gU = {wa.g_w.re * scale, wa.g_w.im * scale};
                }
                const double rr = (double)ref.re, ri = (double)ref.im;
                ent.k = kidx;
                ent.g = {(Tf)(rr * gU.re + ri * gU.im), (Tf)(rr * gU.im - ri * gU.re)};
                // with surfaces after the DOE the secondaries' geometry goes to k_post_bwd
                if (a.want_lens && side && cfg.s_doe + 1 == cfg.n_surf)
                  incident_from_wavelet(a, c, sec, wa, acc);
                if constexpr (kG2) {
                  if (lead) {
                    double gds[3];
                    direction_cograd(a, c, sec, wa, gds);
                    wavevector_cograd(c, sec, gds, g2r[2], g2r[3]);
                    g2r[0] = wa.g_w.re;
                    g2r[1] = wa.g_w.im;
                    g2r[4] = (double)J;
                  }
                }
              }
            }
            if (lead) {
              if (dl_lds) s.dl[i] = ent;
              else gdl[i] = ent;
            }
            if constexpr (kG2) {
              if (lead && cfg.sampling == 0) {
                float* e = (float*)a.g2 + (size_t)blockIdx.x * (N * kG2Rec + M * M) +
                           (size_t)i * kG2Rec;
#pragma unroll
                for (int q = 0; q < 4; ++q) e[q] = (float)g2r[q];
                e[4] = __int_as_float((int)g2r[4]);
              }
            }
          }
        }
        dLdS = block_sum_d(dLdS, s.red);     // orders every read of buf before the rewrite
        if constexpr (kCasc == 2) {
          gar = block_sum_d(gar, s.red);
          gai = block_sum_d(gai, s.red);
          if (t == 0) { a.gain[gid] = gar; a.gain[a.n_total + gid] = gai; }
        }
        double D2 = 0.0;                      // G2: sum of dL/dlog p
        const float* dlg = nullptr;           // G2: dL/dlog p per bin, [ky][kx]
        if constexpr (kG2) {
          if (cfg.sampling == 0 && S > 0.0) {
            float* gd = (float*)a.g2 + (size_t)blockIdx.x * (N * kG2Rec + M * M);
            float* dg = gd + (size_t)N * kG2Rec;
            // the CDF prefix buffer is free in the adjoint (it takes the recorded draws)
            float* lrec = N * kG2Rec * sizeof(float) <= sizeof(s.pref) ? (float*)s.pref : nullptr;
            D2 = g2_passes<Prec, M>(a, c, buf, s.span, S, gd, dg, s.red, lrec);
            dlg = dg;
          }
        }
        if constexpr (M == 256) {
          fold_fS = (Tf)dLdS;
          fold_dlg = dlg;
          fold_d2s = dlg ? (Tf)(D2 / S) : Tf(0);
          fold_dl = S > 0.0 ? gdl : nullptr;
        } else {
          // S-term (p_mag): dL/dX_k = dL/dS X_k / |X_k| on propagating bins;
          // each lane keeps one column (M divides the block size)
          {
            const int kx = t % M;
            const int jx = kx < M / 2 ? kx : kx - M;
            const Span sp = s.span[jx + M / 2];
            const bool mag = cfg.sampling == 0;
            const Tf fS = (Tf)dLdS;
            // batches of SB rows: a lane's bins are distinct, so every load of a
            // batch is issued before its stores
            constexpr int RS = kDoeThreads / M, SB = M / RS >= 8 ? 8 : (M / RS >= 1 ? M / RS : 1);
            for (int ky0 = t / M; ky0 < M; ky0 += SB * RS) {
              C2<Tf> xv[SB];
#pragma unroll
              for (int q = 0; q < SB; ++q) {
                const int ky = ky0 + q * RS;
                xv[q] = ky < M ? buf[Gm::at(ky, kx)] : C2<Tf>{Tf(0), Tf(0)};
              }
#pragma unroll
              for (int q = 0; q < SB; ++q) {
                const int ky = ky0 + q * RS;
                const int jy = ky < M / 2 ? ky : ky - M;
                const C2<Tf> X = xv[q];
                C2<Tf> v = {Tf(0), Tf(0)};
                if (mag && jy >= sp.lo && jy <= sp.hi) {
                  const Tf m2 = X.re * X.re + X.im * X.im;
                  if (m2 > Tf(0)) {
                    const Tf im = inv_sqrt(m2);
                    Tf f = fS * im;
                    if (kG2 && dlg) f += ((Tf)dlg[ky * M + kx] * im - (Tf)(D2 / S)) * im;
                    v = {X.re * f, X.im * f};
                  }
                }
                if (ky < M) buf[Gm::at(ky, kx)] = v;
              }
            }
          }
          __syncthreads();
          // draw terms: each entry is re-read by the lane that wrote it
          if (S > 0.0 && lead) {
#pragma unroll 1
            for (int i = t / LPD; i < N; i += kDoeThreads / LPD) {
              const DrawEnt<Tf> e = dl_lds ? s.dl[i] : gdl[i];
              if (e.k >= 0) {
                atomicAdd(&buf[e.k].re, e.g.re);
                atomicAdd(&buf[e.k].im, e.g.im);
              }
            }
          }
        }
      } else {
        // FULL: every bin once, LPD lanes per bin (with two, both lanes read the
        // bin before the first of them writes it)
#pragma unroll 1
        for (int idx = t / LPD; idx < M * M; idx += kDoeThreads / LPD) {
          const int ky = idx / M, kx = idx % M;
          const int jx = kx < M / 2 ? kx : kx - M, jy = ky < M / 2 ? ky : ky - M;
          const Span sp = s.span[jx + M / 2];
          C2<Tf> out = {Tf(0), Tf(0)};
          if (jy >= sp.lo && jy <= sp.hi) {
            const C2<Tf> X = buf[Gm::at(ky, kx)];
            const C2<Tf> ref = centre_ref<Tf>(jx, jy, P, M);
            const C2<Tf> U = X * ref;
            const C2<Tp> w = {(Tp)U.re * (Tp)inv_m2, (Tp)U.im * (Tp)inv_m2};
            WaveletAdj wa;
            Secondary sec;
            const int Lb = (jx + M / 2) * M + (jy + M / 2);
            const size_t slot = slot0 + (size_t)Lb;
            bool okw;
            if constexpr (kCasc == 1) {
              okw = relay_cograd(a, c, Lb, wa);
            } else if constexpr (kCasc == 2) {
              C2<double> ga;
              okw = wavelet_adjoint_pair<Prec, kTiled, true>(a, c, jx, jy, w, h, slot, wa, sec, ain,
                                                             &ga);
              if (okw && lead) { gar += ga.re; gai += ga.im; }
            } else {
              okw = wavelet_adjoint_pair<Prec, kTiled>(a, c, jx, jy, w, h, slot, wa, sec);
            }
            if (okw) {
              const double gr = wa.g_w.re * inv_m2, gi = wa.g_w.im * inv_m2;
              const double rr = (double)ref.re, ri = (double)ref.im;
              out = {(Tf)(rr * gr + ri * gi), (Tf)(rr * gi - ri * gr)};
              if (a.want_lens && side && cfg.s_doe + 1 == cfg.n_surf)
                incident_from_wavelet(a, c, sec, wa, acc);
            }
          }
          if (lead) buf[Gm::at(ky, kx)] = out;
        }
        if constexpr (kCasc == 2) {
          gar = block_sum_d(gar, s.red);
          gai = block_sum_d(gai, s.red);
          if (t == 0) { a.gain[gid] = gar; a.gain[a.n_total + gid] = gai; }
        }
      }
      __syncthreads();
      // inverse transform: columns (keep rows n < P), then rows n < P (keep m < P;
      // columns P and M - 1 become a zero border of the patch gradient)
      if constexpr (Gm::kSkew) {
        line_fft2<Tf, M, +1, true>(buf, s.tw, M, M, P, false);
        line_fft2<Tf, M, +1, false>(buf, s.tw, P, M, P, true);
      } else if constexpr (M == 256) {
        // batches staged in LDS: columns (all rows in, rows < P out), then the
        // rows < P (columns < P out, columns P and M - 1 as the zero border)
        C2<Tf>* ls = s.ls;
        for (int c0 = 0; c0 < M; c0 += kLines256) {
          if constexpr (kFull) stage_lines256<Tf, true>(ls, buf, SM, c0, kLines256, M, M);
          else stage_cograd256<Tf>(ls, buf, SM, c0, s.span, cfg.sampling == 0, fold_fS, fold_dlg,
                                   fold_d2s, fold_dl, N);
          lds_fft256<Tf, +1>(ls, s.tw, kLines256, false);
          for (int i = t; i < P * kLines256; i += kDoeThreads) {
            const int r = i >> 6, cl = i & 63;
            buf[Gm::row(r) + c0 + cl] = ls[cl * kLS256 + sk256(r)];
          }
          __syncthreads();
        }
        for (int r0 = 0; r0 < P; r0 += kLines256) {
          const int nr = min(kLines256, P - r0);
          stage_lines256<Tf, false>(ls, buf, SM, r0, nr, M, M);
          lds_fft256<Tf, +1>(ls, s.tw, nr, false);
          for (int i = t; i < nr * M; i += kDoeThreads) {
            const int l = i >> 8, m = i & 255;
            if (m < P) buf[Gm::row(r0 + l) + m] = ls[l * kLS256 + sk256(m)];
            else if (m == P || m == M - 1) buf[Gm::row(r0 + l) + m] = C2<Tf>{Tf(0), Tf(0)};
          }
          __syncthreads();
        }
      } else {
        for (int col = g; col < M; col += G) {
          C2<Tf> x[E];
#pragma unroll
          for (int n2 = 0; n2 < E; ++n2) x[n2] = buf[Gm::row_split(gl, L * n2) + Gm::col(col)];
          group_fft<Tf, L, E, +1>(x, gl, s.tw);
#pragma unroll
          for (int k2 = 0; k2 < E; ++k2) {
            const int n = E * br + k2;
            if (n < P) buf[Gm::row(E * br) + k2 * SM + Gm::col(col)] = x[k2];
          }
        }
        __syncthreads();
        for (int row = g; row < P; row += G) {
          C2<Tf> x[E];
#pragma unroll
          for (int n2 = 0; n2 < E; ++n2) x[n2] = buf[Gm::row(row) + Gm::col_split(gl, L * n2)];
          group_fft<Tf, L, E, +1>(x, gl, s.tw);
          // columns P and M - 1 become a zero border of the patch gradient
#pragma unroll
          for (int k2 = 0; k2 < E; ++k2) {
            const int m = E * br + k2;
            if (m < P) buf[Gm::row(row) + Gm::col(E * br) + k2] = x[k2];
            else if (m == P || m == M - 1) buf[Gm::row(row) + Gm::col(E * br) + k2] = C2<Tf>{Tf(0), Tf(0)};
          }
        }
      }
      // rows P and M - 1 too (the row pass touches rows < P only): the
      // bilinear adjoint below reads samples -1 and P through the wrap M - 1
      if (P < M - 1)
        for (int i = t; i < 2 * M; i += kDoeThreads)
          buf[Gm::at(i < M ? P : M - 1, i & (M - 1))] = C2<Tf>{Tf(0), Tf(0)};
      __syncthreads();
      // bilinear adjoint of the patch gather -> dL/dt, added to the block accumulator
      double gpx = 0.0, gpy = 0.0;
      // curved DOE: the samples sit at p + s_m u + s_n v, so the position
      // cogradient of each sample also moves u and v (xy parts)
      double gux = 0.0, guy = 0.0, gvx = 0.0, gvy = 0.0;
      if (cfg.planar && Gm::SIZE - Gm::row(P) >= T * T) {
        // gather form: pixel (ix0 + a, iy0 + b) collects the (up to) four samples
        // whose 2 x 2 stencils contain it; no atomics
        const PlanarPatch<Tf> pp = planar_patch<Tf>(cfg, c);
        const Tf w00 = (Tf(1) - pp.wx) * (Tf(1) - pp.wy), w01 = pp.wx * (Tf(1) - pp.wy);
        const Tf w10 = (Tf(1) - pp.wx) * pp.wy, w11 = pp.wx * pp.wy;
        const int P1 = P + 1;
        const int lx0 = pp.ix0 - ax0, ly0 = pp.iy0 - ay0;
        const bool inside = lx0 >= 0 && ly0 >= 0 && lx0 + P1 <= AS && ly0 + P1 <= AS;
        if (inside && t == 0) {
          atomicMin(&s_box[0], lx0); atomicMin(&s_box[1], ly0);
          atomicMax(&s_box[2], lx0 + P1); atomicMax(&s_box[3], ly0 + P1);
        }
        // samples -1 and P read the zero border (index -1 wraps to M - 1)
        auto gu = [&](int n, int m) { return buf[Gm::at(n & (M - 1), m & (M - 1))]; };
        const FDiv dP1(P1);
        auto pix = [&](int i, int& x, int& y) -> C2<Tf> {
          const int bb = dP1.div(i), aa = i - bb * P1;
          x = pp.ix0 + aa; y = pp.iy0 + bb;
          return gu(bb, aa) * w00 + gu(bb, aa - 1) * w01 + gu(bb - 1, aa) * w10 +
                 gu(bb - 1, aa - 1) * w11;
        };
        // Lens position gradient: sum over samples of <g_s, dU_s/dx> equals the
        // sum over pixels of <G'_p, t_p>, G' the bilinear adjoint with the
        // weights differentiated in the sub-pixel offset (x: wx, y: wy).
        const bool lens = a.want_lens != 0;
        // read before the accumulator stores: a global load after them would
        // wait for the stores to complete
        const double inv_pitch = cfg.inv_pitch;
        auto lens_term = [&](int i, const C2<Tf>& tp) {
          const int bb = dP1.div(i), aa = i - bb * P1;
          const C2<Tf> g00 = gu(bb, aa), g01 = gu(bb, aa - 1), g10 = gu(bb - 1, aa),
                       g11 = gu(bb - 1, aa - 1);
          const C2<Tf> gx = (g01 - g00) * (Tf(1) - pp.wy) + (g11 - g10) * pp.wy;
          const C2<Tf> gy = (g10 - g00) * (Tf(1) - pp.wx) + (g11 - g01) * pp.wx;
          gpx += (double)(gx.re * tp.re + gx.im * tp.im);
          gpy += (double)(gy.re * tp.re + gy.im * tp.im);
        };
        if (inside) {
          // the window lies inside the accumulator: batches of KB pixels per
          // lane; the accumulator and map loads of a batch are issued first,
          // then its samples are read from LDS once for both the pixel value
          // and the lens terms while those loads are in flight
          constexpr int KB = 9;
          for (int i0 = t; i0 < P1 * P1; i0 += kDoeThreads * KB) {
            int li[KB], mi[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
              const int i = i0 + k * kDoeThreads;
              li[k] = -1;
              mi[k] = -1;
              if (i < P1 * P1) {
                const int bb = dP1.div(i), aa = i - bb * P1;
                const int x = pp.ix0 + aa, y = pp.iy0 + bb;
                if (x >= 0 && x < W && y >= 0 && y < H) {
                  li[k] = (ly0 + bb) * AS + lx0 + aa;
                  mi[k] = y * W + x;
                }
              }
            }
            C2<Tg> old[KB];
            C2<Tf> tp[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
              if (li[k] >= 0) old[k] = accm[li[k]];
              tp[k] = (lens && mi[k] >= 0) ? tm[mi[k]] : C2<Tf>{Tf(0), Tf(0)};
            }
            C2<Tf> v[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
              v[k] = {Tf(0), Tf(0)};
              if (li[k] < 0) continue;
              const int i = i0 + k * kDoeThreads;
              const int bb = dP1.div(i), aa = i - bb * P1;
              const C2<Tf> g00 = gu(bb, aa), g01 = gu(bb, aa - 1), g10 = gu(bb - 1, aa),
                           g11 = gu(bb - 1, aa - 1);
              v[k] = g00 * w00 + g01 * w01 + g10 * w10 + g11 * w11;
              if (lens) {
                const C2<Tf> gx = (g01 - g00) * (Tf(1) - pp.wy) + (g11 - g10) * pp.wy;
                const C2<Tf> gy = (g10 - g00) * (Tf(1) - pp.wx) + (g11 - g01) * pp.wx;
                gpx += (double)(gx.re * tp[k].re + gx.im * tp[k].im);
                gpy += (double)(gy.re * tp[k].re + gy.im * tp[k].im);
              }
            }
            // every load of the batch is consumed before the stores, and none
            // is left in flight (vmcnt(0) alone: 0x0F70 keeps the export and
            // LDS counters unconstrained): a load pending behind the stores
            // would make later code wait for them
            __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
            for (int k = 0; k < KB; ++k) {
              if (li[k] < 0) continue;
              accm[li[k]] = {old[k].re + (Tg)v[k].re, old[k].im + (Tg)v[k].im};
            }
          }
        } else {
          for (int i = t; i < P1 * P1; i += kDoeThreads) {
            int x, y;
            const C2<Tf> v = pix(i, x, y);
            if (x < 0 || x >= W || y < 0 || y >= H) continue;
            if (lens) lens_term(i, tm[(size_t)y * W + x]);
            if (v.re == Tf(0) && v.im == Tf(0)) continue;
            atomicAdd(&gt[(size_t)y * W + x].re, (Tg)v.re);
            atomicAdd(&gt[(size_t)y * W + x].im, (Tg)v.im);
          }
        }
        gpx *= inv_pitch;
        gpy *= inv_pitch;
      } else {
      // general surface.  Sample (m, n) sits at the fractional map position
      // f(m, n) = xy(p + s_m u + s_n v) / pitch, affine in (m, n), and feeds the
      // pixels floor(f) + {0, 1} in each axis.  Gather form: every pixel of a
      // T x T tile around the patch inverts that map, visits the few samples
      // whose stencils contain it (each (pixel, sample) pair exactly once, with
      // the forward's own position arithmetic) and adds their sum to the block
      // accumulator with one read-modify-write; no atomics.  When the stencils
      // leave the tile (or the map is degenerate) every sample scatters its
      // stencil instead.
      const double cfx = (c.p[0] - cfg.x0) * cfg.inv_pitch, cfy = (c.p[1] - cfg.y0) * cfg.inv_pitch;
      const int tx0 = (int)floor(cfx) - T / 2, ty0 = (int)floor(cfy) - T / 2;
      const double jxm = cfg.pitch * c.u[0] * cfg.inv_pitch, jxn = cfg.pitch * c.v[0] * cfg.inv_pitch;
      const double jym = cfg.pitch * c.u[1] * cfg.inv_pitch, jyn = cfg.pitch * c.v[1] * cfg.inv_pitch;
      const double hc = (P - 1) * 0.5;
      const double ex = hc * (fabs(jxm) + fabs(jxn)), ey = hc * (fabs(jym) + fabs(jyn));
      const double det = jxm * jyn - jxn * jym;
      const bool gather = floor(cfx - ex - 1e-6) >= tx0 && floor(cfx + ex + 1e-6) + 1 < tx0 + T &&
                          floor(cfy - ey - 1e-6) >= ty0 && floor(cfy + ey + 1e-6) + 1 < ty0 + T &&
                          fabs(det) > 0.25;
      const bool lens = a.want_lens != 0;
      const int lgP = __builtin_ctz(P);
      // sample position arithmetic of the forward gather
      auto sample_pos = [&](int m, int n, double& fx, double& fy) {
        const double sm = (m - (P - 1) * 0.5) * cfg.pitch;
        const double sn = (n - (P - 1) * 0.5) * cfg.pitch;
        const double qx = c.p[0] + sm * c.u[0] + sn * c.v[0];
        const double qy = c.p[1] + sm * c.u[1] + sn * c.v[1];
        fx = (qx - cfg.x0) * cfg.inv_pitch;
        fy = (qy - cfg.y0) * cfg.inv_pitch;
      };
      if (gather) {
        if constexpr (M == 256) {
          // the patch gradient (rows and columns < P of the global buffer) into
          // the staged-line area, free after the inverse transforms
          constexpr int KC = 8;
          for (int i0 = t; i0 < P * P; i0 += kDoeThreads * KC) {
            C2<Tf> v[KC];
#pragma unroll
            for (int k = 0; k < KC; ++k) {
              const int i = i0 + k * kDoeThreads;
              v[k] = i < P * P ? buf[Gm::row(i >> lgP) + (i & (P - 1))] : C2<Tf>{Tf(0), Tf(0)};
            }
#pragma unroll
            for (int k = 0; k < KC; ++k)
              if (i0 + k * kDoeThreads < P * P) s.ls[i0 + k * kDoeThreads] = v[k];
          }
          __syncthreads();
        }
        auto gpatch = [&](int n, int m) -> C2<Tf> {
          if constexpr (M == 256) return s.ls[(n << lgP) + m];
          else return buf[Gm::at(n, m)];
        };
        const double i11 = jyn / det, i12 = -jxn / det, i21 = -jym / det, i22 = jxm / det;
        const double rm = fabs(i11) + fabs(i12) + 1e-7, rn = fabs(i21) + fabs(i22) + 1e-7;
        const int lx0 = tx0 - ax0, ly0 = ty0 - ay0;
        const bool inside = lx0 >= 0 && ly0 >= 0 && lx0 + T <= AS && ly0 + T <= AS;
        if (inside && t == 0) {
          atomicMin(&s_box[0], lx0); atomicMin(&s_box[1], ly0);
          atomicMax(&s_box[2], lx0 + T); atomicMax(&s_box[3], ly0 + T);
        }
        double lx_ = 0.0, ly_ = 0.0, lux = 0.0, luy = 0.0, lvx = 0.0, lvy = 0.0;
        // KB pixels per lane: their accumulator and map loads are issued first
        constexpr int KB = 6;
        const FDiv dT(T);
        for (int i0 = t; i0 < T * T; i0 += kDoeThreads * KB) {
          int li[KB];               // accumulator index; -1: off the map; -2: global atomics
          C2<Tg> old[KB];
          C2<Tf> tp[KB];
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            const int i = i0 + k * kDoeThreads;
            li[k] = -1;
            old[k] = {Tg(0), Tg(0)};
            tp[k] = {Tf(0), Tf(0)};
            if (i < T * T) {
              const int yy = dT.div(i), xx = i - yy * T;
              const int x = tx0 + xx, y = ty0 + yy;
              if (x >= 0 && x < W && y >= 0 && y < H) {
                li[k] = inside ? (ly0 + yy) * AS + lx0 + xx : -2;
                if (inside) old[k] = accm[li[k]];
                if (lens) tp[k] = tm[(size_t)y * W + x];
              }
            }
          }
          C2<Tf> vs[KB];
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            vs[k] = {Tf(0), Tf(0)};
            if (li[k] == -1) continue;
            const int i = i0 + k * kDoeThreads;
            const int yy = dT.div(i), xx = i - yy * T;
            const int X = tx0 + xx, Y = ty0 + yy;
            // lattice coordinates of the pixel; its samples lie within (rm, rn)
            const double dxp = X - cfx, dyp = Y - cfy;
            const double mc = i11 * dxp + i12 * dyp + hc, nc = i21 * dxp + i22 * dyp + hc;
            const int m0 = max(0, (int)ceil(mc - rm)), m1 = min(P - 1, (int)floor(mc + rm));
            const int n0 = max(0, (int)ceil(nc - rn)), n1 = min(P - 1, (int)floor(nc + rn));
            C2<Tf> v = {Tf(0), Tf(0)};
            for (int n = n0; n <= n1; ++n) {
              for (int m = m0; m <= m1; ++m) {
                double fx, fy;
                sample_pos(m, n, fx, fy);
                const double flx = floor(fx), fly = floor(fy);
                const int ddx = X - (int)flx, ddy = Y - (int)fly;
                if ((unsigned)ddx > 1u || (unsigned)ddy > 1u) continue;
                const Tf wx = (Tf)(fx - flx), wy = (Tf)(fy - fly);
                const Tf ax = ddx ? wx : Tf(1) - wx, ay = ddy ? wy : Tf(1) - wy;
                const C2<Tf> g = gpatch(n, m);
                v = v + g * (ax * ay);
                if (lens) {
                  // <g, t_pixel> times the derivative of this pixel's weight
                  const double q = (double)g.re * tp[k].re + (double)g.im * tp[k].im;
                  const double qx = q * (double)(ddx ? ay : -ay);
                  const double qy = q * (double)(ddy ? ax : -ax);
                  const double sm = (m - (P - 1) * 0.5) * cfg.pitch;
                  const double sn = (n - (P - 1) * 0.5) * cfg.pitch;
                  lx_ += qx; ly_ += qy;
                  lux += sm * qx; luy += sm * qy;
                  lvx += sn * qx; lvy += sn * qy;
                }
              }
            }
            vs[k] = v;
          }
          __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            if (li[k] >= 0) {
              accm[li[k]] = {old[k].re + (Tg)vs[k].re, old[k].im + (Tg)vs[k].im};
            } else if (li[k] == -2 && (vs[k].re != Tf(0) || vs[k].im != Tf(0))) {
              const int i = i0 + k * kDoeThreads;
              const int yy = dT.div(i), xx = i - yy * T;
              atomicAdd(&gt[(size_t)(ty0 + yy) * W + tx0 + xx].re, (Tg)vs[k].re);
              atomicAdd(&gt[(size_t)(ty0 + yy) * W + tx0 + xx].im, (Tg)vs[k].im);
            }
          }
        }
        const double ip = cfg.inv_pitch;
        gpx += lx_ * ip; gpy += ly_ * ip;
        gux += lux * ip; guy += luy * ip;
        gvx += lvx * ip; gvy += lvy * ip;
      } else {
      // scatter of every sample's 2 x 2 stencil into an LDS tile (M = 128) or
      // straight into dL/dt
      C2<Tf>* tile = buf + Gm::row(P);
      const bool tile_ok = M != 256 && use_tile;
      if (tile_ok) {
        for (int i = t; i < T * T; i += kDoeThreads) tile[i] = {Tf(0), Tf(0)};
        __syncthreads();
      }
      for (int smp = t; smp < P * P; smp += kDoeThreads) {
        const int m = smp & (P - 1), n = smp >> lgP;
        const C2<Tf> gu = buf[Gm::at(n, m)];
        double fx, fy;
        sample_pos(m, n, fx, fy);
        const double flx = floor(fx), fly = floor(fy);
        const int ix = (int)flx, iy = (int)fly;
        const Tf wx = (Tf)(fx - flx), wy = (Tf)(fy - fly);
        if (lens) {
          // <g, dU/dq> with the bilinear interpolant's xy derivative at q
          auto at = [&](int y, int x) {
            return (x >= 0 && x < W && y >= 0 && y < H) ? tm[(size_t)y * W + x]
                                                        : C2<Tf>{Tf(0), Tf(0)};
          };
          const C2<Tf> t00 = at(iy, ix), t01 = at(iy, ix + 1), t10 = at(iy + 1, ix),
                       t11 = at(iy + 1, ix + 1);
          const C2<Tf> dtx = (t01 - t00) * (Tf(1) - wy) + (t11 - t10) * wy;
          const C2<Tf> dty = (t10 - t00) * (Tf(1) - wx) + (t11 - t01) * wx;
          const double sm = (m - (P - 1) * 0.5) * cfg.pitch;
          const double sn = (n - (P - 1) * 0.5) * cfg.pitch;
          const double qx_ = ((double)gu.re * dtx.re + (double)gu.im * dtx.im) * cfg.inv_pitch;
          const double qy_ = ((double)gu.re * dty.re + (double)gu.im * dty.im) * cfg.inv_pitch;
          gpx += qx_; gpy += qy_;
          gux += sm * qx_; guy += sm * qy_;
          gvx += sn * qx_; gvy += sn * qy_;
        }
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const int x = ix + dx, y = iy + dy;
            if (!(x >= 0 && x < W && y >= 0 && y < H)) continue;
            const Tf wgt = (dx ? wx : Tf(1) - wx) * (dy ? wy : Tf(1) - wy);
            const C2<Tf> v = gu * wgt;
            const int lx = x - tx0, ly = y - ty0;
            if (tile_ok && lx >= 0 && lx < T && ly >= 0 && ly < T) {
              atomicAdd(&tile[ly * T + lx].re, v.re);
              atomicAdd(&tile[ly * T + lx].im, v.im);
            } else {
              atomicAdd(&gt[(size_t)y * W + x].re, (Tg)v.re);
              atomicAdd(&gt[(size_t)y * W + x].im, (Tg)v.im);
            }
          }
        }
      }
      if (tile_ok) {
        __syncthreads();
        const int lx0 = tx0 - ax0, ly0 = ty0 - ay0;
        const bool inside = lx0 >= 0 && ly0 >= 0 && lx0 + T <= AS && ly0 + T <= AS;
        if (inside && t == 0) {
          atomicMin(&s_box[0], lx0); atomicMin(&s_box[1], ly0);
          atomicMax(&s_box[2], lx0 + T); atomicMax(&s_box[3], ly0 + T);
        }
        for (int i = t; i < T * T; i += kDoeThreads) {
          const C2<Tf> v = tile[i];
          if (v.re == Tf(0) && v.im == Tf(0)) continue;
          const int x = tx0 + i % T, y = ty0 + i / T;
          if (x < 0 || x >= W || y < 0 || y >= H) continue;
          if (inside) {
            C2<Tg>& d = accm[(size_t)(ly0 + i / T) * AS + lx0 + i % T];
            d.re += (Tg)v.re;
            d.im += (Tg)v.im;
          } else {
            atomicAdd(&gt[(size_t)y * W + x].re, (Tg)v.re);
            atomicAdd(&gt[(size_t)y * W + x].im, (Tg)v.im);
          }
        }
      }
      }
      }
      // lens: per-wave sums of the incident-state cogradient into s.acc; lanes
      // 3..5 keep the frame they need, so that the combination can run after
      // the end-of-ray barrier while the other waves start the next ray
      double lf = 0.0, lu = 0.0, lv = 0.0, ld = 0.0;
      if (a.want_lens) {
        constexpr int NQ = 14;
        double v[NQ] = {acc.gp[0] + gpx, acc.gp[1] + gpy, acc.gp[2], acc.gkin[0], acc.gkin[1],
                        acc.gopl, acc.gzs, acc.tq[0], acc.tq[1], acc.tq[2], gux, guy, gvx, gvy};
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
        if ((t & 63) == 0)
          for (int q = 0; q < NQ; ++q) s.acc[t >> 6][q] = v[q];
        lf = c.k0 * c.n_in;
        if (t >= 3 && t < 6) {
          lu = c.u[t - 3];
          lv = c.v[t - 3];
        }
        if (t >= 8 && t < 14) ld = c.d[(t - 8) % 3];
      }
      __syncthreads();   // buf, tile and pref are reused by the next ray; s.acc is complete
      // component t < RW_RAYGRAD of the incident-state cogradient, one lane each
      // (s.acc is next written after several barriers of the next ray):
      // k_in,t = k0 n_in (d.u, d.v) feeds the direction d and the vectors u, v
      if (a.want_lens && t < RW_RAYGRAD) {
        auto tot = [&](int q) {
          double r = 0.0;
          for (int wv = 0; wv < kDoeThreads / 64; ++wv) r += s.acc[wv][q];
          return r;
        };
        double out;
        if (t < 3) out = tot(t);
        else if (t < 6) out = lf * (tot(3) * lu + tot(4) * lv);
        else if (t < 8) out = tot(t - 1);
        else if (t < 11) out = (t < 10 ? tot(10 + (t - 8)) : 0.0) + lf * tot(3) * ld;
        else if (t < 14) out = (t < 13 ? tot(12 + (t - 11)) : 0.0) + lf * tot(4) * ld;
        else out = tot(7 + (t - 14));
        a.raygrad[(size_t)t * a.n_total + gid] = out;
      }
    }
    // flush the accumulator over the touched box, clearing it for the next block
    const int bx0 = s_box[0], by0 = s_box[1], bx1 = s_box[2], by1 = s_box[3];
    if (bx0 < bx1 && by0 < by1) {
      const int bw = bx1 - bx0, bh = by1 - by0;
      // KF pixels per lane: their loads are all issued before any is used
      constexpr int KF = 8;
      const FDiv dW(bw);
      for (int i0 = t; i0 < bw * bh; i0 += kDoeThreads * KF) {
        C2<Tg> v[KF];
#pragma unroll
        for (int k = 0; k < KF; ++k) {
          const int i = i0 + k * kDoeThreads;
          v[k] = {Tg(0), Tg(0)};
          if (i < bw * bh) {
            const int r = dW.div(i);
            v[k] = accm[(size_t)(by0 + r) * AS + bx0 + i - r * bw];
          }
        }
#pragma unroll
        for (int k = 0; k < KF; ++k) {
          const int i = i0 + k * kDoeThreads;
          if (i >= bw * bh || (v[k].re == Tg(0) && v[k].im == Tg(0))) continue;
          const int r = dW.div(i), lx = bx0 + i - r * bw, ly = by0 + r;
          accm[(size_t)ly * AS + lx] = {Tg(0), Tg(0)};
          const int x = ax0 + lx, y = ay0 + ly;
          atomicAdd(&gt[(size_t)y * W + x].re, v[k].re);
          atomicAdd(&gt[(size_t)y * W + x].im, v[k].im);
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace rw
