"""Patch classes (curvature bound, Eq. 4) on a conformal DOE: the GPU against
the FP64 oracle, through the C ABI.  The conformal workload puts the larger
patch side on the rays near the vertex and the smaller one further out."""
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


def _case(**kw):
    return W.conformal_hologram(**kw)


def _forward(rw, system, cfg, maps, precision, **kw):
    plan = rw.Plan(system, cfg, precision=precision)
    vals, ph, am = gpu_inputs(system, maps)
    psf, _, idx = plan.forward(vals, ph, am, **kw)
    torch.cuda.synchronize()
    return plan, psf.cpu().numpy(), idx


def test_conformal_case_has_two_classes():
    system, cfg, maps = _case()
    _, aux = oracle_psf(system, cfg, maps, keep=True)
    sides = aux[0]["sides"]
    assert set(sides.tolist()) == {16, 32}


def test_classes_fp64_indices_exact_and_psf(rw):
    system, cfg, maps = _case(sampling="mag", n_field_side=2)
    _, psf, idx = _forward(rw, system, cfg, maps, "fp64", want_idx=True)
    ref, aux = oracle_psf(system, cfg, maps, keep=True)
    gi = idx.cpu().numpy()
    for pr, a in aux.items():
        assert np.array_equal(gi[pr], a["J"]), pr
    assert worst_pair_rel(psf, ref) < 1e-6


def test_classes_mixed_full_mode_psf(rw):
    system, cfg, maps = _case(sampling="full", rays_side=6)
    _, psf, _ = _forward(rw, system, cfg, maps, "mixed")
    ref, _ = oracle_psf(system, cfg, maps)
    assert worst_pair_rel(psf, ref) < 1e-4


def test_classes_mixed_map_gradients_on_oracle_draws(rw):
    system, cfg, maps = _case(sampling="mag", n_field_side=2)
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
