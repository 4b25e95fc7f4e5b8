// Ray-wave interface kernels of the MIXED form.
#include "rw_doe.h"
#include "rw_launch.h"

namespace rw {

template <int M, bool LDS>
static void go(bool fwd, const DoeArgs& a, const RayBlockIter& it, long long n, int pair0,
               int blocks, hipStream_t st) {
  if (fwd && (a.relay || a.ain)) {
    // the two DOEs of a cascade (built for the patch sizes that stay in LDS)
    if constexpr (LDS) {
      if (a.relay)
        hipLaunchKernelGGL((k_doe_fwd2<PrecMIXED, M, LDS, 1>), dim3(blocks), dim3(kDoeThreads), 0, st,
                           a, it, n, pair0);
      else
        hipLaunchKernelGGL((k_doe_fwd2<PrecMIXED, M, LDS, 2>), dim3(blocks), dim3(kDoeThreads), 0, st,
                           a, it, n, pair0);
    }
  } else if (fwd) {
    hipLaunchKernelGGL((k_doe_fwd2<PrecMIXED, M, LDS>), dim3(blocks), dim3(kDoeThreads), 0, st, a, it,
                       n, pair0);
  } else if (a.gain) {
    // the adjoints of a cascade's two DOEs (patch sizes that stay in LDS)
    if constexpr (LDS) {
      if (a.relay && a.full)
        hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, false, true, true, 1>), dim3(blocks),
                           dim3(kDoeThreads), 0, st, a, it, n, pair0);
      else if (a.relay)
        hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, false, true, false, 1>), dim3(blocks),
                           dim3(kDoeThreads), 0, st, a, it, n, pair0);
      else if (a.full && a.interp)
        hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, false, true, true, 2>), dim3(blocks),
                           dim3(kDoeThreads), 0, st, a, it, n, pair0);
      else if (a.full)
        hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, false, false, true, 2>), dim3(blocks),
                           dim3(kDoeThreads), 0, st, a, it, n, pair0);
      else if (a.interp)
        hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, false, true, false, 2>), dim3(blocks),
                           dim3(kDoeThreads), 0, st, a, it, n, pair0);
      else
        hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, false, false, false, 2>), dim3(blocks),
                           dim3(kDoeThreads), 0, st, a, it, n, pair0);
    }
  } else if (a.full && a.interp)
    hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, false, true, true>), dim3(blocks),
                       dim3(kDoeThreads), 0, st, a, it, n, pair0);
  else if (a.full)
    hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, false, false, true>), dim3(blocks),
                       dim3(kDoeThreads), 0, st, a, it, n, pair0);
  else if (a.g2 && a.interp)
    hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, true, true, false>), dim3(blocks),
                       dim3(kDoeThreads), 0, st, a, it, n, pair0);
  else if (a.g2)
    hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, true, false, false>), dim3(blocks),
                       dim3(kDoeThreads), 0, st, a, it, n, pair0);
  else if (a.interp)
    hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, false, true, false>), dim3(blocks),
                       dim3(kDoeThreads), 0, st, a, it, n, pair0);
  else
    hipLaunchKernelGGL((k_doe_bwd2<PrecMIXED, M, LDS, false, false, false>), dim3(blocks),
                       dim3(kDoeThreads), 0, st, a, it, n, pair0);
}

hipError_t launch_doe_mixed(bool fwd, int M, bool lds, const DoeArgs& a, const RayBlockIter& it,
                          long long n_items, int pair0, int blocks, hipStream_t st,
                          bool* supported) {
  *supported = true;
  switch (M) {
    case 16: go<16, true>(fwd, a, it, n_items, pair0, blocks, st); break;
    case 32: go<32, true>(fwd, a, it, n_items, pair0, blocks, st); break;
    case 64: go<64, true>(fwd, a, it, n_items, pair0, blocks, st); break;
    case 128: go<128, true>(fwd, a, it, n_items, pair0, blocks, st); break;
    case 256: go<256, false>(fwd, a, it, n_items, pair0, blocks, st); break;
    default: *supported = false; return hipSuccess;
  }
  return hipGetLastError();
}

}  // namespace rw
