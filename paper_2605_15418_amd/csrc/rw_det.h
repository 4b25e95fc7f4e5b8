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
// power of two 2^s and rounded to the nearest integer.  A block adds the taps
// of its sub-tile into LDS with 64-bit integer atomics, then its sub-tile into
// the group's integer grid, again with integer atomics.  Integer addition is
// exact and associative, so neither the order of the binned records nor the
// order of the adds changes a bit of the grid.  The scale comes from an order-free
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

// Sub-tiles of the deterministic spreading: TB x TB bins with TB = min(4, 64 /
// BIN), at most 64 x 64 cells, so that a block's (re, im) int64 accumulator
// takes at most 64 KiB of LDS.  A sub-tile's block scans the (TB + 2)^2 bins
// around it (w / 2 <= BIN: one bin of border holds every record whose kernel
// footprint reaches the sub-tile).
__host__ __device__ __forceinline__ int det_tb(const BinGeom& g) {
  return g.bin >= 64 ? 1 : (64 / g.bin < 4 ? 64 / g.bin : 4);
}
constexpr int kDetSlices = 255;      // most slices of one sub-tile

__device__ __forceinline__ int det_bin_key(const BinGeom& g, int tb, int sy, int sx, int k) {
  const int by = k / (tb + 2) - 1, bx = k % (tb + 2) - 1;
  return bin_key((sy * tb + by + g.nb) % g.nb, (sx * tb + bx + g.nb) % g.nb, g);
}

// Slices per (pair of the group, sub-tile): S = ceil(records scanned / target),
// at most kDetSlices; slices 1 .. S - 1 of a heavy sub-tile go to the list
// (entry: pair * sub-tiles + sub-tile, slice), their count to *n_heavy (zero at
// launch).  The list's order varies between runs; the integer sums do not.
static __global__ __launch_bounds__(256) void k_det_slices(const unsigned long long* offsets,
                                                    BinGeom g, int pair0, int npairs,
                                                    unsigned long long target,
                                                    unsigned char* slices, uint2* heavy,
                                                    unsigned int* n_heavy) {
  const int tb = det_tb(g), nsx = g.nb / tb, ns = nsx * nsx;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)npairs * ns) return;
  const int pl = (int)(i / ns), t = (int)(i % ns);
  const unsigned long long* off = offsets + (size_t)(pair0 + pl) * g.keys;
  unsigned long long n = 0;
  for (int k = 0; k < (tb + 2) * (tb + 2); ++k) {
    const int key = det_bin_key(g, tb, t / nsx, t % nsx, k);
    n += off[key + 1] - off[key];
  }
  const int S = (int)min((unsigned long long)kDetSlices, max(1ull, (n + target - 1) / target));
  slices[i] = (unsigned char)S;
  if (S > 1) {
    const unsigned int b = atomicAdd(n_heavy, (unsigned int)(S - 1));
    for (int k = 1; k < S; ++k) heavy[b + k - 1] = make_uint2((unsigned int)i, (unsigned int)k);
  }
}

// One slice of one sub-tile: each lane takes a record of the scan range, and
// its taps that land in the sub-tile (the same footprint, ES kernel and periodic
// wrap as the tiled spreading) are added to the LDS accumulator as integers;
// the sub-tile is then added to the group's integer grid (nonzero cells only).
template <class Tg, int w>
__device__ __forceinline__ void det_tile(const void* srt_pos, const void* srt_val,
                                         const unsigned long long* offsets, const BinGeom& g,
                                         double beta, int pair0, int pl, int t, int slice, int S,
                                         double sc, unsigned long long* acc) {
  using U = typename RecPos<Tg>::T;
  extern __shared__ unsigned long long s_acc[];
  __shared__ unsigned long long s_beg[36], s_pre[37];
  const int tb = det_tb(g), nsx = g.nb / tb, side = tb * g.bin, nbins = (tb + 2) * (tb + 2);
  const int sy = t / nsx, sx = t % nsx, x0 = sx * side, y0 = sy * side;
  const int nf = g.nf, tid = threadIdx.x;
  const U* pos = (const U*)srt_pos;
  const C2<Tg>* val = (const C2<Tg>*)srt_val;
  const unsigned long long* off = offsets + (size_t)(pair0 + pl) * g.keys;
  __syncthreads();                              // LDS reuse across the entries of a block
  for (int i = tid; i < 2 * side * side; i += blockDim.x) s_acc[i] = 0ull;
  if (tid < nbins) {
    const int key = det_bin_key(g, tb, sy, sx, tid);
    s_beg[tid] = off[key];
    s_pre[tid + 1] = off[key + 1] - off[key];
  }
  __syncthreads();
  if (tid == 0) {
    s_pre[0] = 0;
    for (int i = 1; i <= nbins; ++i) s_pre[i] += s_pre[i - 1];
  }
  __syncthreads();
  const unsigned long long nall = s_pre[nbins];
  const unsigned long long jlo = nall * (unsigned long long)slice / (unsigned long long)S;
  const unsigned long long jhi = nall * (unsigned long long)(slice + 1) / (unsigned long long)S;
  const double two_w = 2.0 / w;
  int b = 0;                                    // bin of record j (j grows per lane)
  for (unsigned long long j = jlo + tid; j < jhi; j += blockDim.x) {
    while (j >= s_pre[b + 1]) ++b;
    const unsigned long long r = s_beg[b] + (j - s_pre[b]);
    const C2<Tg> v = val[r];
    if (is_none(v)) continue;
    const double gx = turns_to_cells(pos[2 * r], nf), gy = turns_to_cells(pos[2 * r + 1], nf);
    const int lx0 = (int)ceil(gx - 0.5 * w), ly0 = (int)ceil(gy - 0.5 * w);
    // first tap relative to the sub-tile origin, in [-w, nf - w) (nf >= side + w)
    const int dx = ((lx0 - x0 + w) & (nf - 1)) - w, dy = ((ly0 - y0 + w) & (nf - 1)) - w;
    if (dx <= -w || dx >= side || dy <= -w || dy >= side) continue;
    double kx[w], ky[w];
#pragma unroll
    for (int i = 0; i < w; ++i) {
      kx[i] = es_kernel<double>((double)i - (gx - lx0), two_w, beta);
      ky[i] = es_kernel<double>((double)i - (gy - ly0), two_w, beta);
    }
    const double vr = (double)v.re * sc, vi = (double)v.im * sc;
    for (int jj = 0; jj < w; ++jj) {
      const int cy = dy + jj;
      if ((unsigned)cy >= (unsigned)side) continue;
#pragma unroll
      for (int i = 0; i < w; ++i) {
        const int cx = dx + i;
        if ((unsigned)cx >= (unsigned)side) continue;
        const double kk = kx[i] * ky[jj];
        const long long re = llrint(vr * kk), im = llrint(vi * kk);
        unsigned long long* d = s_acc + 2 * (cy * side + cx);
        if (re) atomicAdd(d, (unsigned long long)re);
        if (im) atomicAdd(d + 1, (unsigned long long)im);
      }
    }
  }
  __syncthreads();
  unsigned long long* ap = acc + (size_t)pl * nf * nf * 2;
  for (int i = tid; i < side * side; i += blockDim.x) {
    const int cy = i / side, cx = i % side;
    const unsigned long long re = s_acc[2 * i], im = s_acc[2 * i + 1];
    unsigned long long* d = ap + ((size_t)(y0 + cy) * nf + x0 + cx) * 2;
    if (re) atomicAdd(d, re);
    if (im) atomicAdd(d + 1, im);
  }
}

// heavy == null: one block per (sub-tile, pair of the group), slice 0 of the
// sub-tile's S; else the listed further slices, taken in turn by the blocks.
template <class Tg, int w>
__global__ __launch_bounds__(256) void k_det_tiles(const void* srt_pos, const void* srt_val,
                                                   const unsigned long long* offsets, BinGeom g,
                                                   double beta, int pair0, size_t n_bound,
                                                   const unsigned long long* amax,
                                                   unsigned long long* acc,
                                                   const unsigned char* slices,
                                                   const uint2* heavy,
                                                   const unsigned int* n_heavy) {
  const int tb = det_tb(g), ns = (g.nb / tb) * (g.nb / tb);
  const double sc = ldexp(1.0, det_scale_exp(amax, n_bound));
  if (!heavy) {
    det_tile<Tg, w>(srt_pos, srt_val, offsets, g, beta, pair0, blockIdx.y, blockIdx.x, 0,
                    slices[(size_t)blockIdx.y * ns + blockIdx.x], sc, acc);
    return;
  }
  const unsigned int n = *n_heavy;
  for (unsigned int e = blockIdx.x; e < n; e += gridDim.x) {
    const uint2 h = heavy[e];
    det_tile<Tg, w>(srt_pos, srt_val, offsets, g, beta, pair0, (int)(h.x / ns), (int)(h.x % ns),
                    (int)h.y, slices[h.x], sc, acc);
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
