"""Lens-parameter gradients through a curved DOE: the end-to-end design shape
(two even-asphere lenses, the DOE on the second lens's rear asphere, which
carries three of the 14 lens parameters; two patch classes by Eq. 4) at test
size, GPU against the FP64 oracle's autograd through the C ABI.  The DOE's
frame moves with the hit point and with the surface parameters, and so do
the patch samples, the incident tangential wavevector and every emitted
direction.  Bars: MIXED 1e-3 per gradient group (FULL mode, and the oracle's
draws replayed), FP64 own draws 1e-5."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import rw_oracle as O
from rwcases import elementwise_rel, gpu_inputs, oracle_param_values, rel_l2, worst_pair_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    import paper_2605_15418_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.load_library()
    return pkg


def _case(sampling):
    return W.two_lens_hybrid(rays_side=8, H=512, pitch=0.004, P=16, classes=(8,), N=32, Q=32,
                             psf_pitch=0.004, n_lambda=2, n_field_side=2, max_deg=5.0,
                             sampling=sampling)


def _oracle(system, cfg, maps):
    return O.loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                           maps["amp"].astype(np.float64), oracle_param_values(system),
                           maps["target"].astype(np.float64))


def _gpu(rw, system, cfg, maps, precision, replay=None):
    plan = rw.Plan(system, cfg, precision=precision)
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    psf, loss, _ = plan.forward(vals, ph, am, target=tg, replay=replay)
    dp, da, dl = plan.backward()
    torch.cuda.synchronize()
    return psf.cpu().numpy(), float(loss), {"phase": dp.cpu().numpy(), "amp": da.cpu().numpy(),
                                            "lens": dl.cpu().numpy()}


def _check(got, ref, tol):
    psf, L, g = got
    L0, gr, psf0, _ = ref
    errs = {k: rel_l2(g[k], gr[k]) for k in g}
    print("psf", worst_pair_rel(psf, psf0), "grads", errs,
          "lens elementwise", elementwise_rel(g["lens"], gr["lens"]))
    assert abs(L - L0) <= max(tol, 1e-6) * abs(L0)
    assert max(errs.values()) < tol, errs


def test_curved_case_has_lens_parameters_on_the_doe_surface_and_two_classes():
    system, cfg, maps = _case("mag")
    assert any(p["surface"] == 3 and p["field"] == "curv" for p in system["params"])
    _, aux = O.psf_stack(system, cfg, maps["phase"].astype(np.float64),
                         maps["amp"].astype(np.float64), keep=True)
    assert set(np.concatenate([a["sides"] for a in aux.values()]).tolist()) == {16, 8}


def test_curved_mixed_full_mode_gradients(rw):
    system, cfg, maps = _case("full")
    _check(_gpu(rw, system, cfg, maps, "mixed"), _oracle(system, cfg, maps), 1e-3)


def test_curved_mixed_gradients_on_oracle_draws(rw):
    system, cfg, maps = _case("mag")
    ref = _oracle(system, cfg, maps)
    idx = ref[3]
    rep = torch.tensor(np.stack([idx[p] for p in sorted(idx)]), dtype=torch.int32, device="cuda")
    _check(_gpu(rw, system, cfg, maps, "mixed", replay=rep), ref, 1e-3)


def test_curved_fp64_gradients_own_draws(rw):
    system, cfg, maps = _case("mag")
    _check(_gpu(rw, system, cfg, maps, "fp64"), _oracle(system, cfg, maps), 1e-5)
