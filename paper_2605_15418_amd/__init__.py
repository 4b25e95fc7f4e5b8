"""MI355X-native ray-wave hybrid PSF (arXiv 2605.15418): HIP kernels behind a
C ABI (librw.so, include/rw.h) and a thin PyTorch binding."""
from .design import Design  # noqa: F401
from .rw import HybridPSF, Plan, RWError, adam_step, load_library, patch_dft  # noqa: F401
