// Batched radix-2 FFTs held in registers, split across a group of L
// consecutive lanes of a wavefront (CDNA4 wave64).  A group computes one
// N = L * E point DFT:
//   input : lane g holds x[n2] = element g + L * n2,          n2 in [0, E)
//   output: lane g holds x[k2] = element E * bitrev_L(g) + k2, k2 in [0, E)
// Stage 1 is an E-point DIT FFT inside each lane, stage 2 multiplies by the
// twiddles W_N^(g k2), stage 3 is an L-point decimation-in-frequency DFT across
// lanes through __shfl_xor.  DIR = -1 is exp(-2 pi i n k / N), DIR = +1 the
// unnormalised inverse.  `tw` points to the table exp(-2 pi i m / N), m < N.
#pragma once
#include "rw_common.h"

namespace rw {

// exp(2 pi i j / 64), j = 0..63 (for the in-lane stages, E <= 64).
__device__ constexpr double kUnit64[64][2] = {
  {1.0, 0.0},
  {9.9518472667219688624e-1, 9.8017140329560601994e-2},
  {9.8078528040323044913e-1, 1.9509032201612826785e-1},
  {9.5694033573220886494e-1, 2.9028467725446236764e-1},
  {9.2387953251128675613e-1, 3.8268343236508977173e-1},
  {8.8192126434835502971e-1, 4.7139673682599764856e-1},
  {8.3146961230254523708e-1, 5.5557023301960222474e-1},
  {7.7301045336273696081e-1, 6.3439328416364549822e-1},
  {7.071067811865475244e-1, 7.071067811865475244e-1},
  {6.3439328416364549822e-1, 7.7301045336273696081e-1},
  {5.5557023301960222474e-1, 8.3146961230254523708e-1},
  {4.7139673682599764856e-1, 8.8192126434835502971e-1},
  {3.8268343236508977173e-1, 9.2387953251128675613e-1},
  {2.9028467725446236764e-1, 9.5694033573220886494e-1},
  {1.9509032201612826785e-1, 9.8078528040323044913e-1},
  {9.8017140329560601994e-2, 9.9518472667219688624e-1},
  {8.478427660368899644e-32, 1.0},
  {-9.8017140329560601994e-2, 9.9518472667219688624e-1},
  {-1.9509032201612826785e-1, 9.8078528040323044913e-1},
  {-2.9028467725446236764e-1, 9.5694033573220886494e-1},
  {-3.8268343236508977173e-1, 9.2387953251128675613e-1},
  {-4.7139673682599764856e-1, 8.8192126434835502971e-1},
  {-5.5557023301960222474e-1, 8.3146961230254523708e-1},
  {-6.3439328416364549822e-1, 7.7301045336273696081e-1},
  {-7.071067811865475244e-1, 7.071067811865475244e-1},
  {-7.7301045336273696081e-1, 6.3439328416364549822e-1},
  {-8.3146961230254523708e-1, 5.5557023301960222474e-1},
  {-8.8192126434835502971e-1, 4.7139673682599764856e-1},
  {-9.2387953251128675613e-1, 3.8268343236508977173e-1},
  {-9.5694033573220886494e-1, 2.9028467725446236764e-1},
  {-9.8078528040323044913e-1, 1.9509032201612826785e-1},
  {-9.9518472667219688624e-1, 9.8017140329560601994e-2},
  {-1.0, 1.6956855320737799288e-31},
  {-9.9518472667219688624e-1, -9.8017140329560601994e-2},
  {-9.8078528040323044913e-1, -1.9509032201612826785e-1},
  {-9.5694033573220886494e-1, -2.9028467725446236764e-1},
  {-9.2387953251128675613e-1, -3.8268343236508977173e-1},
  {-8.8192126434835502971e-1, -4.7139673682599764856e-1},
  {-8.3146961230254523708e-1, -5.5557023301960222474e-1},
  {-7.7301045336273696081e-1, -6.3439328416364549822e-1},
  {-7.071067811865475244e-1, -7.071067811865475244e-1},
  {-6.3439328416364549822e-1, -7.7301045336273696081e-1},
  {-5.5557023301960222474e-1, -8.3146961230254523708e-1},
  {-4.7139673682599764856e-1, -8.8192126434835502971e-1},
  {-3.8268343236508977173e-1, -9.2387953251128675613e-1},
  {-2.9028467725446236764e-1, -9.5694033573220886494e-1},
  {-1.9509032201612826785e-1, -9.8078528040323044913e-1},
  {-9.8017140329560601994e-2, -9.9518472667219688624e-1},
  {-2.5435282981106698932e-31, -1.0},
  {9.8017140329560601994e-2, -9.9518472667219688624e-1},
  {1.9509032201612826785e-1, -9.8078528040323044913e-1},
  {2.9028467725446236764e-1, -9.5694033573220886494e-1},
  {3.8268343236508977173e-1, -9.2387953251128675613e-1},
  {4.7139673682599764856e-1, -8.8192126434835502971e-1},
  {5.5557023301960222474e-1, -8.3146961230254523708e-1},
  {6.3439328416364549822e-1, -7.7301045336273696081e-1},
  {7.071067811865475244e-1, -7.071067811865475244e-1},
  {7.7301045336273696081e-1, -6.3439328416364549822e-1},
  {8.3146961230254523708e-1, -5.5557023301960222474e-1},
  {8.8192126434835502971e-1, -4.7139673682599764856e-1},
  {9.2387953251128675613e-1, -3.8268343236508977173e-1},
  {9.5694033573220886494e-1, -2.9028467725446236764e-1},
  {9.8078528040323044913e-1, -1.9509032201612826785e-1},
  {9.9518472667219688624e-1, -9.8017140329560601994e-2},
};

template <int E> struct Log2 { static constexpr int v = 1 + Log2<E / 2>::v; };
template <> struct Log2<1> { static constexpr int v = 0; };

__host__ __device__ constexpr int bitrev(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
  return r;
}

// In-lane E-point DIT FFT.  HZ: elements E/2 .. E-1 are zero on entry (the
// zero-padded half of the patch), which makes the first stage a copy.
// Twiddles 1 and +-i are applied without multiplications.
template <class T, int E, int DIR, bool HZ = false>
__device__ __forceinline__ void reg_fft(C2<T> (&x)[E]) {
  constexpr int LB = Log2<E>::v;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int j = bitrev(i, LB);
    if (i < j) { C2<T> t = x[i]; x[i] = x[j]; x[j] = t; }
  }
#pragma unroll
  for (int len = 2; len <= E; len <<= 1) {
#pragma unroll
    for (int i = 0; i < E; i += len) {
#pragma unroll
      for (int j = 0; j < len / 2; ++j) {
        const int ti = j * (64 / len);
        const C2<T> u = x[i + j];
        if (HZ && len == 2) {          // the odd (bit-reversed upper) input is zero
          x[i + j + len / 2] = u;
          continue;
        }
        const C2<T> b = x[i + j + len / 2];
        C2<T> v;
        if (ti == 0) {
          v = b;
        } else if (ti == 16) {         // w = DIR * i
          v = DIR > 0 ? C2<T>{-b.im, b.re} : C2<T>{b.im, -b.re};
        } else {
          const C2<T> w = {T(kUnit64[ti][0]), T(DIR * kUnit64[ti][1])};
          v = b * w;
        }
        x[i + j] = u + v;
        x[i + j + len / 2] = u - v;
      }
    }
  }
}

// x ^ MASK lane exchange: DPP quad permutations for masks 1 and 2,
// ds_swizzle (bit mode, within 32 lanes) for 4 .. 16, ds_bpermute for 32.
template <int MASK> __device__ __forceinline__ float xor_lane(float v) {
  const int iv = __float_as_int(v);
  int r;
  if constexpr (MASK == 1)
    r = __builtin_amdgcn_update_dpp(0, iv, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  else if constexpr (MASK == 2)
    r = __builtin_amdgcn_update_dpp(0, iv, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  else if constexpr (MASK < 32)
    r = __builtin_amdgcn_ds_swizzle(iv, 0x1F | (MASK << 10));
  else
    r = __shfl_xor(iv, MASK, 64);
  return __int_as_float(r);
}
template <int MASK> __device__ __forceinline__ double xor_lane(double v) {
  const long long b = __double_as_longlong(v);
  const float lo = xor_lane<MASK>(__int_as_float((int)(b & 0xffffffffll)));
  const float hi = xor_lane<MASK>(__int_as_float((int)(b >> 32)));
  return __longlong_as_double(((long long)__float_as_int(hi) << 32) |
                              (unsigned int)__float_as_int(lo));
}

template <class T> __device__ __forceinline__ C2<T> shfl_xor_c(C2<T> v, int mask, int width) {
  return {__shfl_xor(v.re, mask, width), __shfl_xor(v.im, mask, width)};
}

// Cross-lane DIF stages h = H, H/2, ..., 1 (compile-time recursion).
template <class T, int L, int E, int DIR, int H, class TW>
__device__ __forceinline__ void xlane_stages(C2<T> (&x)[E], int g, const TW* tw) {
  if constexpr (H >= 1) {
    constexpr int N = L * E;
    const bool upper = (g & H) != 0;
    const int a = g & (H - 1);
    C2<T> w = {T(tw[a * (N / (2 * H))].re), T(tw[a * (N / (2 * H))].im)};
    if (DIR > 0) w.im = -w.im;
    // lower lane: x + o; upper lane: (o - x) w
    const T sg = upper ? T(-1) : T(1);
    if (!upper) w = {T(1), T(0)};
#pragma unroll
    for (int k2 = 0; k2 < E; ++k2) {
      const C2<T> o = {xor_lane<H>(x[k2].re), xor_lane<H>(x[k2].im)};
      const C2<T> y = {o.re + sg * x[k2].re, o.im + sg * x[k2].im};
      x[k2] = y * w;
    }
    xlane_stages<T, L, E, DIR, H / 2>(x, g, tw);
  }
}

template <class T, int L, int E, int DIR, bool HZ = false, class TW>
__device__ __forceinline__ void group_fft(C2<T> (&x)[E], int g, const TW* tw) {
  constexpr int N = L * E;
  reg_fft<T, E, DIR, HZ>(x);
  if constexpr (L > 1) {
    // an opaque zero keeps the twiddle reads inside the call: hoisted out of
    // the callers' loops they would pin E + log2 L complex registers for the
    // whole kernel
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    g += z;
#pragma unroll
    for (int k2 = 1; k2 < E; ++k2) {
      const int m = (g * k2) & (N - 1);
      C2<T> w = {T(tw[m].re), T(tw[m].im)};
      if (DIR > 0) w.im = -w.im;
      x[k2] = x[k2] * w;
    }
    xlane_stages<T, L, E, DIR, L / 2>(x, g, tw);
  }
}

}  // namespace rw
