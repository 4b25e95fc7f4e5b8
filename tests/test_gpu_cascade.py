"""GPU two-DOE cascade vs the oracle's cascade (FP64), through the C ABI.

A secondary of the first DOE is traced to the second DOE, where it is an
incident wavelet whose amplitude is its Eq. 1 weight (Formalism, first
paragraph: the construction extends to several DOEs).  Bars as for one DOE:
  * FP64 form: both DOEs' sample indices bit-exact; PSF within 1e-6 (relative
    L2 and element-wise against the peak; float32 output)
  * MIXED form with the oracle's indices replayed, or FULL: PSF within 1e-4
  * both maps' gradients of the Eq. 5 loss: FP64 1e-5, MIXED 1e-3 (relative L2)
Launch grids of 9 x 9 rays (ragged against the 8 x 8 ray blocks), second-DOE
grids of 36 x 36 (48 x 48 under FULL), four (wavelength, field) pairs.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import rw_oracle as O
from rwcases import elementwise_rel, gpu_inputs, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    import paper_2605_15418_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.load_library()
    return pkg


def _case(sampling, rays=9, P=16, N=16, N2=8, **kw):
    return W.two_doe_cascade(rays_side=rays, P=P, pad=2, N=N, N2=N2, Q=32, psf_pitch=0.02,
                             sampling=sampling, lambdas=(W.LAM_D, W.LAM_F),
                             fields=((0.0, 0.0), (0.004, -0.003)), **kw)


def _oracle(system, cfg, maps, replays=None):
    return O.cascade_psf_stack(system, cfg, maps["phase"].astype(np.float64),
                               maps["amp"].astype(np.float64), replays=replays, keep=True)


def _gpu(rw, system, cfg, maps, precision, replay=None):
    plan = rw.Plan(system, cfg, precision=precision)
    _, ph, am = gpu_inputs(system, maps)
    psf, _, idx = plan.forward(None, ph, am, replay=replay, want_idx=cfg["sampling"] != "full")
    torch.cuda.synchronize()
    return plan, psf.cpu().numpy(), idx


@pytest.mark.parametrize("sampling,pitch2", [("mag", 0.02), ("uni", 0.02), ("mag", 0.005)])
def test_fp64_cascade_indices_exact_and_psf(rw, sampling, pitch2):
    # pitch2 = 0.005: the second map (0.32 mm wide) stops part of the relayed rays
    system, cfg, maps = _case(sampling, pitch=(0.004, pitch2))
    print(f"cascade fp64 {sampling} {pitch2}", flush=True)
    plan, psf, idx = _gpu(rw, system, cfg, maps, "fp64")
    ref, aux = _oracle(system, cfg, maps)
    i1, i2 = (x.cpu().numpy() for x in plan.split_idx(idx))
    for pr, a in aux.items():
        assert np.array_equal(i1[pr], a["J1"]), f"first DOE's indices differ (pair {pr})"
        assert np.array_equal(i2[pr], a["J2"]), f"second DOE's indices differ (pair {pr})"
        assert (a["J2"] >= 0).sum() > 0.3 * a["J2"].size
    assert ref.max() > 0
    assert rel_l2(psf, ref) < 1e-6
    assert elementwise_rel(psf, ref) < 1e-6


def test_mixed_cascade_with_oracle_draws(rw):
    system, cfg, maps = _case("mag")
    print("cascade mixed replay", flush=True)
    ref, aux = _oracle(system, cfg, maps)
    plan = rw.Plan(system, cfg, precision="mixed")
    j1 = torch.tensor(np.stack([aux[p]["J1"] for p in sorted(aux)]), dtype=torch.int32)
    j2 = torch.tensor(np.stack([aux[p]["J2"] for p in sorted(aux)]), dtype=torch.int32)
    rep = plan.join_idx(j1, j2).cuda()
    _, ph, am = gpu_inputs(system, maps)
    psf, _, _ = plan.forward(None, ph, am, replay=rep)
    torch.cuda.synchronize()
    psf = psf.cpu().numpy()
    assert rel_l2(psf, ref) < 1e-4
    assert elementwise_rel(psf, ref) < 1e-4


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-6), ("mixed", 1e-4)])
def test_full_cascade(rw, precision, bar):
    # FULL at both DOEs: every propagating bin of every patch; M = 16, so the
    # 3 x 3 launch grid relays to a 48 x 48 second-DOE grid
    system, cfg, maps = _case("full", rays=3, P=8)
    print(f"cascade full {precision}", flush=True)
    _, psf, _ = _gpu(rw, system, cfg, maps, precision)
    ref, _ = _oracle(system, cfg, maps)
    assert ref.max() > 0
    assert rel_l2(psf, ref) < bar
    assert elementwise_rel(psf, ref) < bar


def test_cascade_graph_replays_match_eager(rw):
    system, cfg, maps = _case("mag")
    print("cascade graph", flush=True)
    plan, eager, _ = _gpu(rw, system, cfg, maps, "mixed")
    plan.set_graph(True)
    _, ph, am = gpu_inputs(system, maps)
    out = torch.empty((plan.L, plan.F, plan.Q, plan.Q), dtype=torch.float32, device="cuda")
    for _ in range(3):
        plan.forward(None, ph, am, psf_out=out)
        torch.cuda.synchronize()
        assert rel_l2(out.cpu().numpy(), eager) < 1e-6


def test_cascade_rejections(rw):
    system, cfg, maps = _case("mag", N=12)
    with pytest.raises(rw.RWError, match="RW_ERR_SHAPE"):
        rw.Plan(system, cfg, precision="mixed")
    system, cfg, maps = _case("mag")
    cfg = dict(cfg, patch_classes=[8])
    with pytest.raises(rw.RWError, match="RW_ERR_UNSUPPORTED"):
        rw.Plan(system, cfg, precision="mixed")
    system, cfg, maps = _case("mag", P=64)
    with pytest.raises(rw.RWError, match="RW_ERR_UNSUPPORTED"):
        rw.Plan(system, cfg, precision="fp64")       # M = 128 does not fit LDS in FP64
    system, cfg, maps = _case("mag")
    with pytest.raises(rw.RWError, match="RW_ERR_UNSUPPORTED"):
        rw.Plan(system, dict(cfg, grad="G2"), precision="mixed")


def _target(cfg, seed=3):
    L, F, Q = len(cfg["lambdas"]), len(cfg["fields"]), cfg["psf_q"]
    return np.random.default_rng(seed).uniform(0.0, 1.0, (L, F, Q, Q)).astype(np.float32)


def _grads(rw, system, cfg, maps, precision, target, replay=None):
    plan = rw.Plan(system, cfg, precision=precision)
    _, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(target, device="cuda")
    _, loss, idx = plan.forward(None, ph, am, target=tg, replay=replay,
                                want_idx=cfg["sampling"] != "full")
    dp, da, _ = plan.backward()
    torch.cuda.synchronize()
    return plan, float(loss), dp.cpu().numpy(), da.cpu().numpy(), idx


def _check_grads(L, dp, da, L0, g, bar):
    assert abs(L - L0) <= bar * abs(L0)
    for k in range(2):          # each DOE's maps on their own
        assert np.abs(g["phase"][k]).max() > 0
        assert rel_l2(dp[k], g["phase"][k]) < bar, ("phase", k, rel_l2(dp[k], g["phase"][k]))
        assert rel_l2(da[k], g["amp"][k]) < bar, ("amp", k, rel_l2(da[k], g["amp"][k]))


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-5), ("mixed", 1e-3)])
def test_cascade_map_gradients_full(rw, precision, bar):
    system, cfg, maps = _case("full", rays=2, P=8)
    cfg = dict(cfg, lambdas=cfg["lambdas"][:1], fields=cfg["fields"][:1],
               launch_center=cfg["launch_center"][:1], psf_center=[cfg["psf_center"][0][:1]])
    tgt = _target(cfg)
    print(f"cascade gradients full {precision}", flush=True)
    L0, g, _, _ = O.cascade_loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                          maps["amp"].astype(np.float64), tgt.astype(np.float64))
    _, L, dp, da, _ = _grads(rw, system, cfg, maps, precision, tgt)
    _check_grads(L, dp, da, L0, g, bar)


def test_cascade_map_gradients_fp64_own_draws(rw):
    system, cfg, maps = _case("mag")
    tgt = _target(cfg)
    print("cascade gradients fp64 mag", flush=True)
    plan, L, dp, da, idx = _grads(rw, system, cfg, maps, "fp64", tgt)
    L0, g, _, oidx = O.cascade_loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                             maps["amp"].astype(np.float64),
                                             tgt.astype(np.float64))
    i1, i2 = (x.cpu().numpy() for x in plan.split_idx(idx))
    for pr, (j1, j2) in oidx.items():
        assert np.array_equal(i1[pr], j1) and np.array_equal(i2[pr], j2)
    _check_grads(L, dp, da, L0, g, 1e-5)


@pytest.mark.parametrize("grad", ["G1", "G1_DETACH"])
def test_cascade_map_gradients_mixed_on_oracle_draws(rw, grad):
    system, cfg, maps = _case("mag")
    cfg = dict(cfg, grad=grad)
    tgt = _target(cfg)
    print(f"cascade gradients mixed {grad}", flush=True)
    L0, g, _, oidx = O.cascade_loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                             maps["amp"].astype(np.float64),
                                             tgt.astype(np.float64))
    j1 = torch.tensor(np.stack([oidx[p][0] for p in sorted(oidx)]), dtype=torch.int32)
    j2 = torch.tensor(np.stack([oidx[p][1] for p in sorted(oidx)]), dtype=torch.int32)
    rep = rw.Plan.join_idx(j1, j2).cuda()
    _, L, dp, da, _ = _grads(rw, system, cfg, maps, "mixed", tgt, replay=rep)
    _check_grads(L, dp, da, L0, g, 1e-3)


def test_cascade_backward_graph_replays_match_eager(rw):
    system, cfg, maps = _case("mag")
    tgt = torch.tensor(_target(cfg), device="cuda")
    print("cascade backward graph", flush=True)
    plan = rw.Plan(system, cfg, precision="mixed")
    _, ph, am = gpu_inputs(system, maps)
    plan.forward(None, ph, am, target=tgt)
    dp0, da0, _ = plan.backward()
    torch.cuda.synchronize()
    dp0, da0 = dp0.cpu().numpy(), da0.cpu().numpy()
    plan.set_graph(True)
    psf = torch.empty((plan.L, plan.F, plan.Q, plan.Q), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    dp = torch.empty((2,) + ph.shape[1:], dtype=torch.float32, device="cuda")
    da = torch.empty_like(dp)
    for _ in range(3):
        plan.forward(None, ph, am, target=tgt, psf_out=psf, loss_out=loss)
        plan.backward(d_phase=dp, d_amp=da)
        torch.cuda.synchronize()
        assert rel_l2(dp.cpu().numpy(), dp0) < 1e-5
        assert rel_l2(da.cpu().numpy(), da0) < 1e-5


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-5), ("mixed", 1e-3)])
def test_cascade_on_curved_does(rw, precision, bar):
    """Both DOEs on spheres (R = 5 mm and -8 mm): curved frames and patches at
    each stage, the relay intersecting a curved surface; PSF and both maps'
    gradients on the oracle's draws."""
    system, cfg, maps = _case("mag", curvature=(0.2, -0.125))
    tgt = _target(cfg)
    print(f"cascade curved {precision}", flush=True)
    L0, g, ref, oidx = O.cascade_loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                               maps["amp"].astype(np.float64),
                                               tgt.astype(np.float64))
    j1 = torch.tensor(np.stack([oidx[p][0] for p in sorted(oidx)]), dtype=torch.int32)
    j2 = torch.tensor(np.stack([oidx[p][1] for p in sorted(oidx)]), dtype=torch.int32)
    rep = rw.Plan.join_idx(j1, j2).cuda()
    plan = rw.Plan(system, cfg, precision=precision)
    _, ph, am = gpu_inputs(system, maps)
    psf, loss, _ = plan.forward(None, ph, am, target=torch.tensor(tgt, device="cuda"),
                                replay=rep)
    dp, da, _ = plan.backward()
    torch.cuda.synchronize()
    psf_bar = 1e-6 if precision == "fp64" else 1e-4
    assert rel_l2(psf.cpu().numpy(), ref) < psf_bar
    _check_grads(float(loss), dp.cpu().numpy(), da.cpu().numpy(), L0, g, bar)


def test_cascade_in_several_launch_groups(rw):
    """A record budget of one pair's records splits the four pairs into four
    launch groups (forward and both DOEs' adjoints group by group): same PSF and
    gradients as one group."""
    system, cfg, maps = _case("mag")
    tgt = _target(cfg)
    print("cascade groups", flush=True)
    one = _grads(rw, system, cfg, maps, "fp64", tgt)
    rec = (9 * 4) ** 2 * 8 * 3 * 32          # ~ one pair's records in the FP64 form
    many = _grads(rw, system, dict(cfg, record_budget_bytes=rec), maps, "fp64", tgt)
    assert abs(one[1] - many[1]) <= 1e-9 * abs(one[1])
    assert rel_l2(many[2], one[2]) < 1e-9 and rel_l2(many[3], one[3]) < 1e-9


def test_cascade_uni_gradients_on_oracle_draws(rw):
    system, cfg, maps = _case("uni")
    tgt = _target(cfg)
    print("cascade gradients uni", flush=True)
    L0, g, _, oidx = O.cascade_loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                             maps["amp"].astype(np.float64),
                                             tgt.astype(np.float64))
    j1 = torch.tensor(np.stack([oidx[p][0] for p in sorted(oidx)]), dtype=torch.int32)
    j2 = torch.tensor(np.stack([oidx[p][1] for p in sorted(oidx)]), dtype=torch.int32)
    rep = rw.Plan.join_idx(j1, j2).cuda()
    _, L, dp, da, _ = _grads(rw, system, cfg, maps, "mixed", tgt, replay=rep)
    _check_grads(L, dp, da, L0, g, 1e-3)
