"""Adaptive patch sizing (the smallest patch spanning K local periods of the
phase map, capped by Eq. 4): the GPU against the FP64 oracle, through the C ABI.

A kinoform zone plate's local period falls from the axis outwards, so the
16 x 16 launch grid splits into three classes (patch sides 32, 16 and 8).  The
class decision is taken in FP64 from the float32 phase map on both sides, so
the per-class ray counts must agree exactly; bars otherwise as for fixed
classes (FP64 indices bit-exact and PSF 1e-6; MIXED PSF 1e-4; gradients 1e-3),
also with adaptive ray sampling (N (P / P_0)^2 draws for a ray of side P).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import rw_oracle as O
from rwcases import gpu_inputs, oracle_psf, rel_l2, worst_pair_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    import paper_2605_15418_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.load_library()
    return pkg


def _case(sampling="mag", rays=16, **kw):
    return W.adaptive_zone_plate(rays_side=rays, H=256, pitch=0.002, f=5.0, P=32, classes=(16, 8),
                                 N=32, Q=32, psf_pitch=0.002, sampling=sampling, **kw)


def _forward(rw, system, cfg, maps, precision, **kw):
    plan = rw.Plan(system, cfg, precision=precision)
    vals, ph, am = gpu_inputs(system, maps)
    psf, _, idx = plan.forward(vals, ph, am, **kw)
    torch.cuda.synchronize()
    return plan, psf.cpu().numpy(), idx


def _class_counts(sides):
    return [int((sides == P).sum()) for P in (32, 16, 8)]


def test_adaptive_fp64_classes_indices_and_psf(rw):
    system, cfg, maps = _case()
    print("adaptive fp64 mag", flush=True)
    plan, psf, idx = _forward(rw, system, cfg, maps, "fp64", want_idx=True)
    ref, aux = oracle_psf(system, cfg, maps, keep=True)
    want = _class_counts(aux[0]["sides"])
    assert min(want) > 0                                    # three classes in play
    assert plan.stats()["rays_by_class"][:3] == want
    assert np.array_equal(idx.cpu().numpy()[0], aux[0]["J"])
    assert worst_pair_rel(psf, ref) < 1e-6


def test_adaptive_mixed_full_mode_psf(rw):
    system, cfg, maps = _case(sampling="full", rays=10)
    print("adaptive mixed full", flush=True)
    plan, psf, _ = _forward(rw, system, cfg, maps, "mixed")
    ref, aux = oracle_psf(system, cfg, maps, keep=True)
    assert plan.stats()["rays_by_class"][:3] == _class_counts(aux[0]["sides"])
    assert worst_pair_rel(psf, ref) < 1e-4


def test_adaptive_mixed_gradients_on_oracle_draws(rw):
    system, cfg, maps = _case()
    print("adaptive mixed gradients", flush=True)
    L0, g, _, idx = O.loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                    maps["amp"].astype(np.float64), np.zeros(0),
                                    maps["target"].astype(np.float64))
    rep = torch.tensor(np.stack([idx[p] for p in sorted(idx)]), dtype=torch.int32, device="cuda")
    plan = rw.Plan(system, cfg, precision="mixed")
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    _, loss, _ = plan.forward(vals, ph, am, target=tg, replay=rep)
    dp, da, _ = plan.backward()
    torch.cuda.synchronize()
    assert abs(float(loss) - L0) <= 1e-4 * abs(L0)
    assert rel_l2(dp.cpu().numpy(), g["phase"]) < 1e-3
    assert rel_l2(da.cpu().numpy(), g["amp"]) < 1e-3


def test_adaptive_sizing_rejections(rw):
    system, cfg, maps = _case()
    with pytest.raises(rw.RWError, match="RW_ERR_INVALID_ARG"):
        rw.Plan(system, dict(cfg, patch_classes=[]), precision="mixed")   # no classes to pick
    with pytest.raises(rw.RWError, match="RW_ERR_INVALID_ARG"):
        rw.Plan(system, dict(cfg, bw_periods=-1.0), precision="mixed")
    with pytest.raises(rw.RWError, match="RW_ERR_INVALID_ARG"):
        rw.Plan(system, dict(cfg, class_draws=True, sampling="full"), precision="mixed")


def test_class_draws_fp64_indices_exact_and_psf(rw):
    """Adaptive ray sampling: the 16- and 8-px rays draw 32 (16/32)^2 = 8 and
    32 (8/32)^2 = 2 secondaries; the indices (-1 beyond a ray's count) match the
    oracle's bit for bit, and the PSF within 1e-6."""
    system, cfg, maps = _case()
    cfg = dict(cfg, class_draws=True)
    print("class draws fp64", flush=True)
    plan, psf, idx = _forward(rw, system, cfg, maps, "fp64", want_idx=True)
    ref, aux = oracle_psf(system, cfg, maps, keep=True)
    J = aux[0]["J"]
    sides = aux[0]["sides"]
    assert np.all(J[sides == 16][:, 8:] == -1) and np.all(J[sides == 16][:, :8] >= 0)
    assert np.array_equal(idx.cpu().numpy()[0], J)
    assert plan.stats()["secondaries"] == int((J >= 0).sum())
    assert worst_pair_rel(psf, ref) < 1e-6


def test_class_draws_mixed_gradients_on_oracle_draws(rw):
    system, cfg, maps = _case()
    cfg = dict(cfg, class_draws=True)
    print("class draws mixed gradients", flush=True)
    L0, g, _, idx = O.loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                    maps["amp"].astype(np.float64), np.zeros(0),
                                    maps["target"].astype(np.float64))
    rep = torch.tensor(np.stack([idx[p] for p in sorted(idx)]), dtype=torch.int32, device="cuda")
    plan = rw.Plan(system, cfg, precision="mixed")
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    _, loss, _ = plan.forward(vals, ph, am, target=tg, replay=rep)
    dp, da, _ = plan.backward()
    torch.cuda.synchronize()
    assert abs(float(loss) - L0) <= 1e-4 * abs(L0)
    assert rel_l2(dp.cpu().numpy(), g["phase"]) < 1e-3
    assert rel_l2(da.cpu().numpy(), g["amp"]) < 1e-3


def test_class_draws_g2_fp64_gradients(rw):
    """The Gumbel-softmax straight-through gradient with per-class draw counts:
    each class regenerates the perturbations of its own draws only."""
    system, cfg, maps = _case()
    cfg = dict(cfg, class_draws=True, grad="G2")
    print("class draws g2 fp64", flush=True)
    L0, g, _, _ = O.loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                  maps["amp"].astype(np.float64), np.zeros(0),
                                  maps["target"].astype(np.float64))
    plan = rw.Plan(system, cfg, precision="fp64")
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    _, loss, _ = plan.forward(vals, ph, am, target=tg)
    dp, da, _ = plan.backward()
    torch.cuda.synchronize()
    assert abs(float(loss) - L0) <= 1e-6 * abs(L0)
    assert rel_l2(dp.cpu().numpy(), g["phase"]) < 1e-4
    assert rel_l2(da.cpu().numpy(), g["amp"]) < 1e-4
