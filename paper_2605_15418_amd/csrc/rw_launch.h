// Launchers of the ray-wave interface kernels, one translation unit per
// precision form so that the heavy templates compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include "rw_kernels.h"

namespace rw {
struct RayBlockIter;
// Returns hipSuccess or the launch error; false in *supported when M is not built.
hipError_t launch_doe_fp64(bool fwd, int M, bool lds, const DoeArgs& a, const RayBlockIter& it,
                           long long n_items, int pair0, int blocks, hipStream_t st, bool* supported);
hipError_t launch_doe_mixed(bool fwd, int M, bool lds, const DoeArgs& a, const RayBlockIter& it,
                            long long n_items, int pair0, int blocks, hipStream_t st, bool* supported);
hipError_t launch_doe_fp32(bool fwd, int M, bool lds, const DoeArgs& a, const RayBlockIter& it,
                           long long n_items, int pair0, int blocks, hipStream_t st, bool* supported);
// Batched 2-D DFT of zero-padded P x P patches to M x M (the DOE kernels' transform).
hipError_t launch_patch_dft(int M, int P, long long n, const void* in, void* out, hipStream_t st);
}  // namespace rw
