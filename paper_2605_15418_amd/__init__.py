"""MI355X-native ray-wave hybrid PSF (arXiv 2605.15418): HIP kernels behind a
C ABI (librw.so, include/rw.h) and a thin PyTorch binding."""
from .rw import HybridPSF, Plan, RWError, load_library  # noqa: F401
