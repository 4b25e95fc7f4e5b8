// Device-side building blocks of the ray-wave library: complex numbers,
// forward-mode dual numbers (for the local Jacobians of the trace adjoint),
// the Philox4x32-10 stream of the secondary-ray draws, and the templated
// conventional refractive trace (Newton ray-sag intersection, vector Snell).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define RW_MAX_SURF 8
#define RW_PI 3.14159265358979323846

namespace rw {

using ::ceil;
using ::exp;
using ::fabs;
using ::floor;
using ::sqrt;

// ---------------------------------------------------------------- complex ---
template <class T> struct C2 { T re, im; };
template <class T> __host__ __device__ __forceinline__ C2<T> mk(T a, T b) { return {a, b}; }
template <class T> __device__ __forceinline__ C2<T> operator+(C2<T> a, C2<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __device__ __forceinline__ C2<T> operator-(C2<T> a, C2<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __device__ __forceinline__ C2<T> operator*(C2<T> a, C2<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> __device__ __forceinline__ C2<T> operator*(C2<T> a, T s) { return {a.re * s, a.im * s}; }
template <class T> __device__ __forceinline__ C2<T> conj(C2<T> a) { return {a.re, -a.im}; }
template <class T, class U> __device__ __forceinline__ C2<T> cvt(C2<U> a) { return {T(a.re), T(a.im)}; }

__device__ __forceinline__ void sincos_any(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void sincos_any(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincospi_any(double x, double* s, double* c) { sincospi(x, s, c); }
__device__ __forceinline__ void sincospi_any(float x, float* s, float* c) { sincospif(x, s, c); }
template <class T> __device__ __forceinline__ C2<T> cis(T x) { T s, c; sincos_any(x, &s, &c); return {c, s}; }

// |z| evaluated with explicit rounding so that two evaluations of the same
// value always agree bit for bit (the sampler recomputes it).
__device__ __forceinline__ float cabs_rn(C2<float> z) {
  return __fsqrt_rn(__fmaf_rn(z.re, z.re, __fmul_rn(z.im, z.im)));
}
__device__ __forceinline__ double cabs_rn(C2<double> z) {
  return __dsqrt_rn(__fma_rn(z.re, z.re, __dmul_rn(z.im, z.im)));
}

// Reduce an angle to [0, 2 pi) in the precision it was accumulated in.
__device__ __forceinline__ double wrap_2pi(double x) {
  const double tp = 2.0 * RW_PI;
  return x - tp * floor(x / tp);
}
__device__ __forceinline__ float wrap_2pi(float x) {
  const float tp = 6.28318530717958647692f;
  return x - tp * floorf(x / tp);
}

// ------------------------------------------------------------ dual numbers ---
template <int NT> struct Dual {
  double v;
  double d[NT];
};
template <int NT> __device__ __forceinline__ Dual<NT> dconst(double v) {
  Dual<NT> r; r.v = v;
#pragma unroll
  for (int i = 0; i < NT; ++i) r.d[i] = 0.0;
  return r;
}
template <int NT> __device__ __forceinline__ Dual<NT> dvar(double v, int k) {
  Dual<NT> r = dconst<NT>(v); r.d[k] = 1.0; return r;
}
#define RW_DUAL_BIN(OP, VAL, DER)                                                           \
  template <int NT> __device__ __forceinline__ Dual<NT> operator OP(const Dual<NT>& a,   \
                                                                     const Dual<NT>& b) { \
    Dual<NT> r; r.v = VAL;                                                                \
    _Pragma("unroll") for (int i = 0; i < NT; ++i) r.d[i] = DER;                          \
    return r;                                                                             \
  }
RW_DUAL_BIN(+, a.v + b.v, a.d[i] + b.d[i])
RW_DUAL_BIN(-, a.v - b.v, a.d[i] - b.d[i])
RW_DUAL_BIN(*, a.v * b.v, a.d[i] * b.v + a.v * b.d[i])
template <int NT> __device__ __forceinline__ Dual<NT> operator/(const Dual<NT>& a, const Dual<NT>& b) {
  Dual<NT> r; r.v = a.v / b.v; const double ib = 1.0 / b.v;
#pragma unroll
  for (int i = 0; i < NT; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <int NT> __device__ __forceinline__ Dual<NT> operator-(const Dual<NT>& a) {
  Dual<NT> r; r.v = -a.v;
#pragma unroll
  for (int i = 0; i < NT; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int NT> __device__ __forceinline__ Dual<NT> operator+(const Dual<NT>& a, double b) { Dual<NT> r = a; r.v += b; return r; }
template <int NT> __device__ __forceinline__ Dual<NT> operator+(double b, const Dual<NT>& a) { return a + b; }
template <int NT> __device__ __forceinline__ Dual<NT> operator-(const Dual<NT>& a, double b) { Dual<NT> r = a; r.v -= b; return r; }
template <int NT> __device__ __forceinline__ Dual<NT> operator-(double b, const Dual<NT>& a) { return dconst<NT>(b) - a; }
template <int NT> __device__ __forceinline__ Dual<NT> operator*(const Dual<NT>& a, double b) {
  Dual<NT> r; r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <int NT> __device__ __forceinline__ Dual<NT> operator*(double b, const Dual<NT>& a) { return a * b; }
template <int NT> __device__ __forceinline__ Dual<NT> operator/(const Dual<NT>& a, double b) { return a * (1.0 / b); }
template <int NT> __device__ __forceinline__ Dual<NT> operator/(double a, const Dual<NT>& b) { return dconst<NT>(a) / b; }
template <int NT> __device__ __forceinline__ Dual<NT> exp(const Dual<NT>& a) {
  Dual<NT> r; r.v = ::exp(a.v);
#pragma unroll
  for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] * r.v;
  return r;
}
template <int NT> __device__ __forceinline__ Dual<NT> sqrt(const Dual<NT>& a) {
  Dual<NT> r; r.v = ::sqrt(a.v); const double h = 0.5 / r.v;
#pragma unroll
  for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] * h;
  return r;
}
__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ float val(float x) { return x; }
template <int NT> __device__ __forceinline__ double val(const Dual<NT>& x) { return x.v; }
template <class S> struct Lit { static __device__ __forceinline__ S of(double v) { return S(v); } };
template <int NT> struct Lit<Dual<NT>> { static __device__ __forceinline__ Dual<NT> of(double v) { return dconst<NT>(v); } };

// ------------------------------------------------------------------ Philox ---
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products,
// key bumped by the Weyl constants between rounds.
__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b) {
  return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
}
__host__ __device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = mulhi32(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
    const uint32_t hi1 = mulhi32(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
}
// Uniform of draw i of ray r in pair p: counter (i >> 2, r, p, stream), word i & 3,
// u = ((x >> 9) + 0.5) 2^-23 (exact in fp32 and fp64).
__device__ __forceinline__ double draw_uniform(uint32_t k0, uint32_t k1, uint32_t i, uint32_t r,
                                               uint32_t p, uint32_t stream) {
  uint32_t c[4] = {i >> 2, r, p, stream};
  philox4x32_10(c, k0, k1);
  const uint32_t x = c[i & 3];
  return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

// -------------------------------------------------------------- surfaces ---
struct DevSurf {            // live prescription after lens parameters are applied
  double z, c, k, A4, A6, A8, A10, semi_ap;
  int kind, doe;
  double gh, gw;            // Gaussian-like term gh (exp(-r^2/gw^2) - 1) when gw > 0
};

template <class S> struct Surf { S z, c, k, A4, A6, A8, A10, gh, gw; };

template <class S>
__device__ __forceinline__ Surf<S> surf_of(const DevSurf& s) {
  return {Lit<S>::of(s.z), Lit<S>::of(s.c), Lit<S>::of(s.k), Lit<S>::of(s.A4),
          Lit<S>::of(s.A6), Lit<S>::of(s.A8), Lit<S>::of(s.A10), Lit<S>::of(s.gh),
          Lit<S>::of(s.gw)};
}

// Even-asphere sag and its xy gradient; false where the conic root is imaginary.
template <class S>
__device__ __forceinline__ bool sag_grad(const Surf<S>& s, const S& x, const S& y, S& sag, S& sx,
                                         S& sy) {
  const S rho = x * x + y * y;
  const S arg = Lit<S>::of(1.0) - (Lit<S>::of(1.0) + s.k) * s.c * s.c * rho;
  if (!(val(arg) > 0.0)) return false;
  const S sq = sqrt(arg);
  const S r2 = rho * rho;
  sag = s.c * rho / (Lit<S>::of(1.0) + sq) + s.A4 * r2 + s.A6 * r2 * rho + s.A8 * r2 * r2 +
        s.A10 * r2 * r2 * rho;
  const S ds = s.c / (Lit<S>::of(2.0) * sq) + Lit<S>::of(2.0) * s.A4 * rho +
               Lit<S>::of(3.0) * s.A6 * r2 + Lit<S>::of(4.0) * s.A8 * r2 * rho +
               Lit<S>::of(5.0) * s.A10 * r2 * r2;
  if (val(s.gw) > 0.0) {
    const S iw2 = Lit<S>::of(1.0) / (s.gw * s.gw);
    const S e = exp(-(rho * iw2));
    sag = sag + s.gh * (e - Lit<S>::of(1.0));
    const S dg = -(s.gh * iw2 * e);
    sx = Lit<S>::of(2.0) * x * (ds + dg);
    sy = Lit<S>::of(2.0) * y * (ds + dg);
    return true;
  }
  sx = Lit<S>::of(2.0) * x * ds;
  sy = Lit<S>::of(2.0) * y * ds;
  return true;
}

template <class S> struct Tol;
template <> struct Tol<double> { static constexpr double v = 1e-13; static constexpr int it = 30; };
template <> struct Tol<float> { static constexpr double v = 1e-6; static constexpr int it = 30; };
template <int NT> struct Tol<Dual<NT>> { static constexpr double v = 1e-13; static constexpr int it = 30; };

// Newton's method on f(t) = p_z + t d_z - z_v - sag(p_x + t d_x, p_y + t d_y),
// started on the vertex plane.  Dual inputs carry the implicit derivative.
template <class S>
__device__ __forceinline__ bool intersect(const Surf<S>& s, const S p[3], const S d[3], S& t) {
  t = (s.z - p[2]) / d[2];
  for (int it = 0; it < Tol<S>::it; ++it) {
    const S x = p[0] + t * d[0], y = p[1] + t * d[1];
    S sg, sx, sy;
    if (!sag_grad(s, x, y, sg, sx, sy)) return false;
    const S f = p[2] + t * d[2] - s.z - sg;
    const S fp = d[2] - sx * d[0] - sy * d[1];
    if (val(fp) == 0.0) return false;
    const S step = f / fp;
    t = t - step;
    const double as = val(step) < 0 ? -val(step) : val(step);
    if (as < Tol<S>::v) return true;
  }
  return false;
}

template <class S>
__device__ __forceinline__ void surface_normal(const Surf<S>& s, const S& x, const S& y, S n[3]) {
  S sg, sx, sy;
  sag_grad(s, x, y, sg, sx, sy);
  const S inv = Lit<S>::of(1.0) / sqrt(sx * sx + sy * sy + Lit<S>::of(1.0));
  n[0] = -sx * inv; n[1] = -sy * inv; n[2] = inv;
}

// Smallest principal radius of curvature of the rotationally symmetric surface at
// (x, y): meridional z''/(1 + z'^2)^(3/2), sagittal z'/(r (1 + z'^2)^(1/2));
// infinite for a plane.
__device__ __forceinline__ double local_radius(const Surf<double>& s, double x, double y) {
  const double rho = x * x + y * y, r = sqrt(rho);
  const double arg = 1.0 - (1.0 + s.k) * s.c * s.c * rho;
  const double sq = sqrt(arg > 0.0 ? arg : 1.0);
  double d1 = s.c / (2.0 * sq) + 2.0 * s.A4 * rho + 3.0 * s.A6 * rho * rho +
              4.0 * s.A8 * rho * rho * rho + 5.0 * s.A10 * rho * rho * rho * rho;
  double d2 = s.c * (1.0 + s.k) * s.c * s.c / (4.0 * sq * sq * sq) + 2.0 * s.A4 +
              6.0 * s.A6 * rho + 12.0 * s.A8 * rho * rho + 20.0 * s.A10 * rho * rho * rho;
  if (s.gw > 0.0) {
    const double iw2 = 1.0 / (s.gw * s.gw), e = exp(-rho * iw2);
    d1 += -s.gh * iw2 * e;
    d2 += s.gh * iw2 * iw2 * e;
  }
  const double zp = 2.0 * r * d1, zpp = 2.0 * d1 + 4.0 * rho * d2;
  const double km = fabs(zpp) / pow(1.0 + zp * zp, 1.5);
  const double ks = r > 0.0 ? fabs(2.0 * d1) / sqrt(1.0 + zp * zp) : fabs(zpp);
  const double kmax = km > ks ? km : ks;
  return kmax > 0.0 ? 1.0 / kmax : INFINITY;
}

// Vector Snell law with the normal oriented along the ray; false on TIR.
template <class S>
__device__ __forceinline__ bool refract(S d[3], const S n[3], const S& mu) {
  const S ci = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
  const S rad = Lit<S>::of(1.0) - mu * mu * (Lit<S>::of(1.0) - ci * ci);
  if (!(val(rad) > 0.0)) return false;
  const S g = sqrt(rad) - mu * ci;
#pragma unroll
  for (int i = 0; i < 3; ++i) d[i] = mu * d[i] + g * n[i];
  return true;
}

}  // namespace rw
