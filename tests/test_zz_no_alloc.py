"""rw_forward_static, the forward that allocates nothing (its workspace is the
library's static device array), through the C ABI: against rw_forward on the
same plan and inputs, for two calls in a row, the second with a smaller
problem (another plan); sample indices equal, PSF and loss within the
atomics-order bar of the forward (1e-5).  A plan whose forward workspace
exceeds the static array is refused, and no backward may follow."""
import ctypes

import numpy as np
import pytest
import torch

from rwcases import gpu_inputs, rel_l2, small_hologram

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    import paper_2605_15418_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.load_library()
    return pkg


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _static(rw, plan, vals, ph, am, tg):
    psf = torch.full((plan.L, plan.F, plan.Q, plan.Q), float("nan"), device="cuda")
    loss = torch.full((1,), float("nan"), device="cuda")
    idx = torch.full((plan.L * plan.F, plan.cfg["rays_side"] ** 2, plan.N), -7,
                     dtype=torch.int32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = plan.lib.rw_forward_static(plan.handle, _ptr(vals), _ptr(ph), _ptr(am), _ptr(tg),
                                    _ptr(psf), _ptr(loss), None, _ptr(idx), stream)
    return st, psf, loss, idx


def test_static_forward_matches_rw_forward_on_two_calls(rw):
    cases = [small_hologram(sampling="mag", N=32, rays=8),
             small_hologram(sampling="mag", N=32, rays=4, n_lambda=1, n_field_side=1)]
    for k, (system, cfg, maps) in enumerate(cases):
        plan = rw.Plan(system, cfg, precision="mixed")
        assert plan.fwd_bytes <= rw.rw.RW_STATIC_SCRATCH_BYTES, plan.fwd_bytes
        vals, ph, am = gpu_inputs(system, maps)
        tg = torch.tensor(maps["target"], device="cuda")
        psf0, loss0, idx0 = plan.forward(vals, ph, am, target=tg, want_idx=True)
        st, psf, loss, idx = _static(rw, plan, vals, ph, am, tg)
        torch.cuda.synchronize()
        assert st == 0, plan.lib.rw_last_error().decode()
        assert torch.equal(idx, idx0), k
        assert rel_l2(psf.cpu().numpy(), psf0.cpu().numpy()) < 1e-5, k
        assert abs(float(loss) - float(loss0)) <= 1e-5 * abs(float(loss0)), k
        with pytest.raises(rw.RWError, match="RW_ERR_STATE"):
            plan.backward()                     # the static forward leaves no backward state


def test_static_forward_refuses_a_plan_beyond_its_array(rw):
    system, cfg, maps = small_hologram(sampling="mag", N=256, rays=64, P=16, Q=256)
    plan = rw.Plan(system, cfg, precision="mixed")
    assert plan.fwd_bytes > rw.rw.RW_STATIC_SCRATCH_BYTES
    vals, ph, am = gpu_inputs(system, maps)
    st, _, _, _ = _static(rw, plan, vals, ph, am, None)
    assert rw.rw.STATUS[st] == "RW_ERR_UNSUPPORTED"
    assert b"static scratch" in plan.lib.rw_last_error()
