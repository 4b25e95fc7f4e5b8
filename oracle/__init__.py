"""FP64 CPU oracle of the ray-wave hybrid PSF -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package; the GPU library never does.
"""
