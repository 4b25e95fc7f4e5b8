// Run-to-run reproducible spreading of the Eq. 2 records (the plan's
// deterministic mode).
//
// The tiled spreading sums each cell's taps in the order the counting sort
// left the records in their bins, and that order depends on which workgroup
// reserved its range first; the slices of heavy tiles add their tiles with
// float atomics.  Float sums taken in another order round differently, so two
// runs agree only to rounding.
//
// Here every tap is a fixed-point integer: value x kernel factor, scaled by a
// power of two 2^s and rounded to the nearest integer, added with 64-bit
// integer atomics into a per-pair grid of (re, im) integers.  Integer addition
// is exact and associative, so the grid does not depend on the order of the
// adds, and the records need no sort.  The scale comes from an order-free
// bound: every tap is at most A = max |re|, |im| over the group's records
// (the ES kernel is at most 1), a cell holds at most n taps (n = the group's
// record slots), so with 2^s n A <= 2^62 no sum leaves the int64 range.  A tap
// is then rounded to 2^-s <= 2 n A 2^-62: relative to A, n 2^-61 (about 2e-10
// for 2^28 records, below FP32 rounding of the taps themselves).
#pragma once

#include "rw_kernels.h"

namespace rw {

// A = max(|re|, |im|) over the non-empty records, as the bits of a
// non-negative double (whose integer order is its numeric order): atomicMax
// of integers does not depend on the order either.
template <class Tg>
__global__ __launch_bounds__(256) void k_det_absmax(const void* rec_val, size_t n,
                                                    unsigned long long* amax) {
  const C2<Tg>* val = (const C2<Tg>*)rec_val;
  double m = 0.0;
  for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (size_t)gridDim.x * blockDim.x) {
    const C2<Tg> v = val[r];
    if (is_none(v)) continue;
    m = fmax(m, fmax(fabs((double)v.re), fabs((double)v.im)));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0 && m > 0.0)
    atomicMax(amax, (unsigned long long)__double_as_longlong(m));
}

// Exponent s of the fixed-point scale 2^s: n A < 2^e with e from frexp, and
// s = 62 - e.
__device__ __forceinline__ int det_scale_exp(const unsigned long long* amax, size_t n) {
  const double a = __longlong_as_double((long long)*amax);
  int e = 0;
  if (a > 0.0) frexp(a * (double)n, &e);
  return 62 - e;
}

// One thread per record slot of the group: the w x w taps of its ES kernel
// (the same footprint, kernel and periodic wrap as the tiled spreading) added
// to acc[pair][y][x][re, im] as integers.
template <class Tg, int w>
__global__ __launch_bounds__(256) void k_det_spread(const void* rec_pos, const void* rec_val,
                                                    size_t per_pair, int npairs, int nf,
                                                    double beta, size_t n_bound,
                                                    const unsigned long long* amax,
                                                    unsigned long long* acc) {
  using U = typename RecPos<Tg>::T;
  const U* pos = (const U*)rec_pos;
  const C2<Tg>* val = (const C2<Tg>*)rec_val;
  const double sc = ldexp(1.0, det_scale_exp(amax, n_bound));
  const double two_w = 2.0 / w;
  const size_t n = per_pair * (size_t)npairs;
  for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (size_t)gridDim.x * blockDim.x) {
    const C2<Tg> v = val[r];
    if (is_none(v)) continue;
    const size_t pl = r / per_pair;
    const double gx = turns_to_cells(pos[2 * r], nf), gy = turns_to_cells(pos[2 * r + 1], nf);
    const int lx0 = (int)ceil(gx - 0.5 * w), ly0 = (int)ceil(gy - 0.5 * w);
    double kx[w], ky[w];
#pragma unroll
    for (int i = 0; i < w; ++i) {
      kx[i] = es_kernel<double>((double)i - (gx - lx0), two_w, beta);
      ky[i] = es_kernel<double>((double)i - (gy - ly0), two_w, beta);
    }
    const double vr = (double)v.re * sc, vi = (double)v.im * sc;
    unsigned long long* ap = acc + pl * (size_t)nf * nf * 2;
    for (int j = 0; j < w; ++j) {
      const size_t row = (size_t)((ly0 + j) & (nf - 1)) * nf;
#pragma unroll
      for (int i = 0; i < w; ++i) {
        const double kk = kx[i] * ky[j];
        if (kk == 0.0) continue;
        const long long re = llrint(vr * kk), im = llrint(vi * kk);
        unsigned long long* d = ap + (row + ((lx0 + i) & (nf - 1))) * 2;
        if (re) atomicAdd(d, (unsigned long long)re);
        if (im) atomicAdd(d + 1, (unsigned long long)im);
      }
    }
  }
}

// The integer grid back to the spreading grid of pairs pair0 .. pair0 + npairs - 1.
template <class Tg>
__global__ __launch_bounds__(256) void k_det_store(const unsigned long long* acc, size_t ncells,
                                                   size_t n_bound, const unsigned long long* amax,
                                                   C2<Tg>* grid) {
  const double q = ldexp(1.0, -det_scale_exp(amax, n_bound));
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncells;
       i += (size_t)gridDim.x * blockDim.x) {
    const long long re = (long long)acc[2 * i], im = (long long)acc[2 * i + 1];
    grid[i] = {(Tg)((double)re * q), (Tg)((double)im * q)};
  }
}

}  // namespace rw
