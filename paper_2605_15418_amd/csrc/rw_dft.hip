// Batched 2-D DFT of zero-padded patches with the DOE kernels' LDS transform
// (M <= 64: lane-group FFTs over rows, then columns, in the workgroup's LDS),
// exposed on its own so that the patch transform can be timed and checked
// against other ways of computing it (Formalism: the local angular spectrum of
// a P x P patch zero-padded to M x M).
#include "rw_doe.h"
#include "rw_launch.h"

namespace rw {

template <int M>
__global__ __launch_bounds__(kDoeThreads) void k_patch_dft(const C2<float>* __restrict__ in,
                                                           C2<float>* __restrict__ out, int P,
                                                           long long n) {
  using Gm = DoeGeom<M>;
  constexpr int L = Gm::L, E = Gm::E, G = Gm::G;
  __shared__ C2<float> buf[Gm::SIZE];
  __shared__ C2<float> tw[M];
  const int tid = threadIdx.x;
  for (int m = tid; m < M; m += kDoeThreads) {
    double s, c;
    sincospi(-2.0 * m / M, &s, &c);
    tw[m] = {(float)c, (float)s};
  }
  const int g = tid / L, gl = tid % L, br = bitrev(gl, Gm::LB);
  for (long long p = blockIdx.x; p < n; p += gridDim.x) {
    const C2<float>* src = in + (size_t)p * P * P;
    __syncthreads();
    for (int i = tid; i < P * P; i += kDoeThreads) buf[Gm::at(i / P, i % P)] = src[i];
    __syncthreads();
    for (int row = g; row < P; row += G) {          // rows n < P, inputs m < P
      C2<float> x[E];
#pragma unroll
      for (int n2 = 0; n2 < E; ++n2) {
        const int m = gl + L * n2;
        x[n2] = m < P ? buf[Gm::row(row) + Gm::col_split(gl, L * n2)] : C2<float>{0.f, 0.f};
      }
      group_fft<float, L, E, -1>(x, gl, tw);
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) buf[Gm::row(row) + Gm::col(E * br) + k2] = x[k2];
    }
    __syncthreads();
    C2<float>* dst = out + (size_t)p * M * M;
    for (int col = g; col < M; col += G) {          // columns, inputs n < P
      C2<float> x[E];
#pragma unroll
      for (int n2 = 0; n2 < E; ++n2) {
        const int nn = gl + L * n2;
        x[n2] = nn < P ? buf[Gm::row_split(gl, L * n2) + Gm::col(col)] : C2<float>{0.f, 0.f};
      }
      group_fft<float, L, E, -1>(x, gl, tw);
#pragma unroll
      for (int k2 = 0; k2 < E; ++k2) dst[(size_t)(E * br + k2) * M + col] = x[k2];
    }
  }
}

// Launcher (M in {16, 32, 64}, 1 <= P <= M, checked by the caller).
hipError_t launch_patch_dft(int M, int P, long long n, const void* in, void* out, hipStream_t st) {
  const int blocks = (int)(n < 2048 ? n : 2048);
  const C2<float>* src = (const C2<float>*)in;
  C2<float>* dst = (C2<float>*)out;
  if (M == 16)
    hipLaunchKernelGGL(k_patch_dft<16>, dim3(blocks), dim3(kDoeThreads), 0, st, src, dst, P, n);
  else if (M == 32)
    hipLaunchKernelGGL(k_patch_dft<32>, dim3(blocks), dim3(kDoeThreads), 0, st, src, dst, P, n);
  else
    hipLaunchKernelGGL(k_patch_dft<64>, dim3(blocks), dim3(kDoeThreads), 0, st, src, dst, P, n);
  return hipGetLastError();
}

}  // namespace rw
