"""The deterministic forward (rw_config.deterministic), through the C ABI.

The Eq. 2 records are spread as 64-bit fixed-point integers with integer
atomics, exact in any order, so forwards on the same inputs give the same PSF
and loss in every bit: two calls of one plan, a second plan, a graph replay,
several launch groups, and a zone plate's focus, where the tiled spreading cuts
heavy tiles into slices added with float atomics.  Against the FP64 oracle the
bars are the tiled spreading's (PSF 1e-4 MIXED, 1e-6 FP64, relative L2 and
element-wise).  Against the tiled spreading the PSF differs only by the FP32
rounding of the taps (MIXED) or by the fixed-point step (FP64).  The backward
entry points refuse such a plan.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import rw_oracle as O
from rwcases import elementwise_rel, gpu_inputs, oracle_psf, rel_l2, small_hologram, worst_pair_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    import paper_2605_15418_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.load_library()
    return pkg


def _fwd(plan, system, maps, target=True, **kw):
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda") if target else None
    psf, loss, _ = plan.forward(vals if plan.n_params else None, ph, am, target=tg, **kw)
    torch.cuda.synchronize()
    return psf.clone(), (loss.clone() if loss is not None else None)


@pytest.mark.parametrize("precision,bar,vs_tiled", [("mixed", 1e-4, 1e-5), ("fp64", 1e-6, 1e-9)])
def test_deterministic_repeats_bitwise_and_matches_oracle(rw, precision, bar, vs_tiled):
    system, cfg, maps = small_hologram(rays=8)           # 27 pairs, FULL
    print(f"deterministic hologram {precision}", flush=True)
    det = dict(cfg, deterministic=True)
    plan = rw.Plan(system, det, precision=precision)
    psf1, loss1 = _fwd(plan, system, maps)
    psf2, loss2 = _fwd(plan, system, maps)
    psf3, loss3 = _fwd(rw.Plan(system, det, precision=precision), system, maps)
    assert torch.equal(psf1, psf2) and torch.equal(psf1, psf3)
    assert torch.equal(loss1, loss2) and torch.equal(loss1, loss3)
    ref, _ = oracle_psf(system, cfg, maps)
    got = psf1.cpu().numpy()
    assert worst_pair_rel(got, ref) < bar
    assert elementwise_rel(got, ref) < bar
    tiled, _ = _fwd(rw.Plan(system, cfg, precision=precision), system, maps)
    assert rel_l2(got, tiled.cpu().numpy()) < vs_tiled


def test_deterministic_graph_replays_and_launch_groups(rw):
    system, cfg, maps = small_hologram(rays=8)
    det = dict(cfg, deterministic=True)
    print("deterministic graph and groups", flush=True)
    eager, loss0 = _fwd(rw.Plan(system, det, precision="mixed"), system, maps)
    plan = rw.Plan(system, det, precision="mixed")
    plan.set_graph(True)
    psf = torch.empty_like(eager)
    loss = torch.empty(1, device="cuda")
    for _ in range(3):                                   # record, then replays
        _fwd(plan, system, maps, psf_out=psf, loss_out=loss)
        assert torch.equal(psf, eager) and torch.equal(loss, loss0)
    # several launch groups: each group takes its own fixed-point scale, so the
    # PSF repeats bitwise per plan and agrees with one group to the step
    per_pair = cfg["rays_side"] ** 2 * (cfg["patch_p"] * cfg["pad"]) ** 2
    cfg_g = dict(det, record_budget_bytes=5 * per_pair * (3 * 16 + 40))
    pg = rw.Plan(system, cfg_g, precision="mixed")
    g1, l1 = _fwd(pg, system, maps)
    g2, l2 = _fwd(pg, system, maps)
    assert torch.equal(g1, g2) and torch.equal(l1, l2)
    assert rel_l2(g1.cpu().numpy(), eager.cpu().numpy()) < 1e-6


def test_deterministic_at_a_focus(rw):
    """A zone plate at its focus: a few tiles hold most of the records (the tiled
    spreading slices them and adds the slices with float atomics)."""
    system, cfg, maps = W.adaptive_zone_plate(rays_side=64, H=256, pitch=0.002, f=5.0, P=16,
                                              classes=(), N=64, Q=32, psf_pitch=0.002,
                                              sampling="mag")
    cfg = dict(cfg, patch_classes=[], bw_periods=0.0, deterministic=True)
    print("deterministic focus mixed", flush=True)
    ref, aux = oracle_psf(system, cfg, maps, keep=True)
    rep = torch.tensor(np.stack([aux[p]["J"] for p in sorted(aux)]), dtype=torch.int32,
                       device="cuda")
    plan = rw.Plan(system, cfg, precision="mixed")
    p1, _ = _fwd(plan, system, maps, target=False, replay=rep)
    p2, _ = _fwd(plan, system, maps, target=False, replay=rep)
    assert torch.equal(p1, p2)
    assert rel_l2(p1.cpu().numpy(), ref) < 1e-4


def test_deterministic_cascade(rw):
    system, cfg, maps = W.two_doe_cascade(rays_side=3, P=8, pad=2, N=16, N2=8, Q=32,
                                          psf_pitch=0.02, sampling="full",
                                          lambdas=(W.LAM_D, W.LAM_F),
                                          fields=((0.0, 0.0), (0.004, -0.003)))
    cfg = dict(cfg, deterministic=True)
    print("deterministic cascade mixed", flush=True)
    plan = rw.Plan(system, cfg, precision="mixed")
    p1, _ = _fwd(plan, system, maps, target=False)
    p2, _ = _fwd(plan, system, maps, target=False)
    assert torch.equal(p1, p2)
    ref, _ = O.cascade_psf_stack(system, cfg, maps["phase"].astype(np.float64),
                                 maps["amp"].astype(np.float64))
    assert rel_l2(p1.cpu().numpy(), ref) < 1e-4
    assert elementwise_rel(p1.cpu().numpy(), ref) < 1e-4


def test_deterministic_refuses_gradients(rw):
    system, cfg, maps = small_hologram(rays=4, n_lambda=1, n_field_side=1)
    plan = rw.Plan(system, dict(cfg, deterministic=True), precision="mixed")
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    plan.forward(vals, ph, am, target=tg)
    with pytest.raises(rw.RWError, match="RW_ERR_UNSUPPORTED"):
        plan.backward()
    with pytest.raises(rw.RWError, match="RW_ERR_UNSUPPORTED"):
        plan.autotune()
    with pytest.raises(rw.RWError, match="RW_ERR_UNSUPPORTED"):
        plan.step(vals, ph, am, tg)
    torch.cuda.synchronize()


def test_deterministic_plain_fp32_per_pair_launches(rw):
    """FP32 everywhere, one launch per pair: the phase drift of the FP32 trace is
    the tiled path's too, so the two PSFs agree to the taps' rounding."""
    system, cfg, maps = small_hologram(rays=8)
    print("deterministic plain fp32", flush=True)
    det = dict(cfg, deterministic=True)
    plan = rw.Plan(system, det, precision="fp32", batched=False)
    p1, l1 = _fwd(plan, system, maps)
    p2, l2 = _fwd(plan, system, maps)
    assert torch.equal(p1, p2) and torch.equal(l1, l2)
    tiled, _ = _fwd(rw.Plan(system, cfg, precision="fp32", batched=False), system, maps)
    assert rel_l2(p1.cpu().numpy(), tiled.cpu().numpy()) < 1e-5


def test_deterministic_class_draws_fp64(rw):
    """Adaptive patch sizing with per-class draw counts: the slots beyond a ray's
    count hold no record.  FP64 draws match the oracle's bit for bit, the PSF
    within 1e-6."""
    system, cfg, maps = W.adaptive_zone_plate(rays_side=16, H=256, pitch=0.002, f=5.0, P=32,
                                              classes=(16, 8), N=32, Q=32, psf_pitch=0.002,
                                              sampling="mag")
    cfg = dict(cfg, class_draws=True, deterministic=True)
    print("deterministic class draws fp64", flush=True)
    plan = rw.Plan(system, cfg, precision="fp64")
    vals, ph, am = gpu_inputs(system, maps)
    psf, _, idx = plan.forward(vals, ph, am, want_idx=True)
    torch.cuda.synchronize()
    p1 = psf.clone()
    p2, _ = _fwd(plan, system, maps, target=False)
    assert torch.equal(p1, p2)
    ref, aux = oracle_psf(system, cfg, maps, keep=True)
    J = aux[0]["J"]
    assert (J < 0).any()                                 # empty slots in play
    assert np.array_equal(idx.cpu().numpy()[0], J)
    assert worst_pair_rel(p1.cpu().numpy(), ref) < 1e-6
