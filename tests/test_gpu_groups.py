"""Launch groups and the fused training step, through the C ABI.

A plan whose secondary-ray records exceed the record budget runs its pairs in
several launch groups; rw_backward then interpolates inside the DOE adjoint
(the records of earlier groups are gone), and rw_forward_backward runs each
group's backward right after its forward with the tiled interpolation.  All
of these must agree with the single-group plan on the same draws (the same
arithmetic up to the order of atomics and of the interpolation sums): PSF,
loss and gradients within 1e-5."""
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


def _case():
    return small_hologram(sampling="mag", N=32, rays=8)     # 27 pairs x 64 rays


def _sep(plan, v, ph, am, tg):
    psf, loss, idx = plan.forward(v, ph, am, target=tg, want_idx=True)
    g = plan.backward()
    torch.cuda.synchronize()
    return psf.cpu().numpy(), float(loss), idx.cpu().numpy(), [x.cpu().numpy() for x in g]


def _close(a, b, tol=1e-5):
    assert rel_l2(a[0], b[0]) < tol
    assert abs(a[1] - b[1]) <= tol * abs(b[1])
    for x, y in zip(a[-1], b[-1]):
        assert rel_l2(x, y) < tol


def test_fused_step_matches_forward_then_backward(rw):
    system, cfg, maps = _case()
    v, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    ref = _sep(rw.Plan(system, cfg, precision="mixed"), v, ph, am, tg)
    plan = rw.Plan(system, cfg, precision="mixed")
    psf, loss, dp, da, dl = plan.step(v, ph, am, tg)
    torch.cuda.synchronize()
    _close((psf.cpu().numpy(), float(loss), [dp.cpu().numpy(), da.cpu().numpy(),
                                              dl.cpu().numpy()]), ref)


@pytest.mark.parametrize("graph", [False, True])
def test_several_launch_groups_match_one(rw, graph):
    system, cfg, maps = _case()
    v, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    ref = _sep(rw.Plan(system, cfg, precision="mixed"), v, ph, am, tg)
    per_pair = cfg["rays_side"] ** 2 * cfg["n_ssr"]
    # five pairs per group: records (3 copies of position + value) and tiled buffers
    cfg_g = dict(cfg, record_budget_bytes=5 * per_pair * (3 * 16 + 40))
    plan = rw.Plan(system, cfg_g, precision="mixed")
    if graph:
        plan.set_graph(True)
    got = _sep(plan, v, ph, am, tg)
    assert np.array_equal(got[2], ref[2])
    _close(got, ref)
    psf = torch.empty((plan.L, plan.F, plan.Q, plan.Q), device="cuda")
    loss = torch.empty(1, device="cuda")
    dp, da, dl = torch.empty_like(ph), torch.empty_like(am), torch.empty_like(v)
    for _ in range(2 if graph else 1):            # with graphs: record, then replay
        out = plan.step(v, ph, am, tg, psf_out=psf, loss_out=loss, d_phase=dp, d_amp=da,
                        d_lens=dl)
        torch.cuda.synchronize()
        _close((out[0].cpu().numpy(), float(out[1]), [x.cpu().numpy() for x in out[2:]]), ref)
