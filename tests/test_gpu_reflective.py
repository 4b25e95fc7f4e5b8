"""The reflective conformal DOE (Fig. 6): a reflective DOE on the Gaussian-like
substrate with the two-phase field exp(i phi1) + exp(i phi2), secondaries
sent back to a sensor in front of the DOE.  GPU against the FP64 oracle
through the C ABI: FP64 draws bit-exact and PSF 1e-6; MIXED PSF 1e-4 (FULL
mode, and the oracle's draws replayed); MIXED gradients w.r.t. both phase
maps 1e-3; the two-focus design on a flat reflective DOE (spots 16 um apart
at NA 0.2) against the oracle's PSF."""
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


def _case(sampling="mag", rays=8):
    return W.reflective_conformal(rays_side=rays, H=121, P=16, N=32, Q=32, psf_pitch=0.001,
                                  sampling=sampling, random_phase=0.5, sep=0.008)


def _fwd(rw, system, cfg, maps, precision, **kw):
    plan = rw.Plan(system, cfg, precision=precision)
    v, ph, am = gpu_inputs(system, maps)
    psf, loss, idx = plan.forward(v, ph, am, **kw)
    torch.cuda.synchronize()
    return plan, psf.cpu().numpy(), idx


def test_reflective_fp64_draws_exact_and_psf(rw):
    system, cfg, maps = _case()
    _, psf, idx = _fwd(rw, system, cfg, maps, "fp64", want_idx=True)
    ref, aux = oracle_psf(system, cfg, maps, keep=True)
    assert np.array_equal(idx.cpu().numpy()[0], aux[0]["J"])
    assert rel_l2(psf, ref) < 1e-6


def test_reflective_mixed_full_mode_psf(rw):
    system, cfg, maps = _case(sampling="full", rays=6)
    _, psf, _ = _fwd(rw, system, cfg, maps, "mixed")
    ref, _ = oracle_psf(system, cfg, maps)
    assert rel_l2(psf, ref) < 1e-4


def test_reflective_two_phase_gradients_on_oracle_draws(rw):
    system, cfg, maps = _case()
    L0, g, ref, idx = O.loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                      maps["amp"].astype(np.float64), np.zeros(0),
                                      maps["target"].astype(np.float64))
    rep = torch.tensor(np.stack([idx[p] for p in sorted(idx)]), dtype=torch.int32, device="cuda")
    plan = rw.Plan(system, cfg, precision="mixed")
    v, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    psf, loss, _ = plan.forward(v, ph, am, target=tg, replay=rep)
    d1, d2, _ = plan.backward()
    torch.cuda.synchronize()
    assert rel_l2(psf.cpu().numpy(), ref) < 1e-4
    assert abs(float(loss) - L0) <= 1e-4 * abs(L0)
    e1, e2 = rel_l2(d1.cpu().numpy(), g["phase"]), rel_l2(d2.cpu().numpy(), g["amp"])
    print("dphi1", e1, "dphi2", e2)
    assert max(e1, e2) < 1e-3


def test_two_focus_design_on_a_flat_reflective_doe(rw):
    system, cfg, maps = W.reflective_conformal(rays_side=24, H=251, P=64, N=64, Q=64,
                                               psf_pitch=0.0005, sampling="full", sep=0.016,
                                               gw=0.0, na=0.2)
    _, psf, _ = _fwd(rw, system, cfg, maps, "mixed")
    ref, _ = oracle_psf(system, cfg, maps)
    assert rel_l2(psf, ref) < 1e-4
    Q = cfg["psf_q"]
    x = (np.arange(Q) - Q // 2) * cfg["psf_pitch"]
    col = psf[0, 0].sum(0)
    assert x[np.argmax(col[:Q // 2])] == -0.008 and x[Q // 2 + np.argmax(col[Q // 2:])] == 0.008
