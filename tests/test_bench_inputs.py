"""bench.py feeds the plan lens parameters it computes itself (it may not call
the oracle outside its CPU baseline); they must be the values the oracle starts
from, rounded to float32, for every workload that has lens parameters (CPU only)."""
import numpy as np
import pytest

import bench
import workloads as W
from oracle import rw_oracle as O


@pytest.mark.parametrize("name", ["asphere_hologram", "two_lens_hybrid"])
def test_bench_lens_values_match_the_oracle(name):
    system, _, _ = W.workload(name)
    got = bench.lens_param_values(system)
    want = O.initial_param_values(system).astype(np.float32)
    assert got.dtype == np.float32 and got.shape == want.shape and want.size > 0
    assert np.array_equal(got, want)
