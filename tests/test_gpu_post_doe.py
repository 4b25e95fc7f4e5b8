"""A refracting surface after the DOE: the conformal DOE on the convex front of
a BK7 plano-convex lens, whose planar rear face every secondary ray crosses
before the sensor (the shape of the conformal workload, at test size: three
patch classes by the Eq. 4 rule).  GPU against the FP64 oracle through the
C ABI: FP64 draws bit-exact and PSF 1e-6; MIXED PSF 1e-4 (FULL mode and the
oracle's draws replayed); MIXED phase / amplitude gradients 1e-3."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import rw_oracle as O
from rwcases import gpu_inputs, oracle_param_values, oracle_psf, rel_l2, worst_pair_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    import paper_2605_15418_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.load_library()
    return pkg


def _case(sampling="mag", rays=8, N=32, n_field_side=2):
    system, cfg, maps = W.conformal_sphere(rays_side=rays, H=512, pitch=0.002, P=32,
                                           classes=(16, 8), N=N, Q=32, psf_pitch=0.004,
                                           n_lambda=2, n_field_side=n_field_side, max_deg=5.0,
                                           sampling=sampling)
    rng = np.random.default_rng(20260204)
    Q = cfg["psf_q"]
    maps["target"] = rng.uniform(size=(2, n_field_side ** 2, Q, Q)).astype(np.float32)
    return system, cfg, maps


def test_post_doe_case_has_a_surface_after_the_doe_and_three_classes():
    system, cfg, maps = _case()
    assert system["surfaces"][0]["doe"] and len(system["surfaces"]) == 2
    _, aux = oracle_psf(system, cfg, maps, keep=True)
    assert set(np.concatenate([a["sides"] for a in aux.values()]).tolist()) == {32, 16, 8}


def test_post_doe_fp64_indices_exact_and_psf(rw):
    system, cfg, maps = _case()
    plan = rw.Plan(system, cfg, precision="fp64")
    vals, ph, am = gpu_inputs(system, maps)
    psf, _, idx = plan.forward(vals, ph, am, want_idx=True)
    torch.cuda.synchronize()
    ref, aux = oracle_psf(system, cfg, maps, keep=True)
    gi = idx.cpu().numpy()
    for pr, a in aux.items():
        assert np.array_equal(gi[pr], a["J"]), pr
    assert worst_pair_rel(psf.cpu().numpy(), ref) < 1e-6


def test_post_doe_mixed_full_mode_psf(rw):
    system, cfg, maps = _case(sampling="full", rays=6)
    plan = rw.Plan(system, cfg, precision="mixed")
    vals, ph, am = gpu_inputs(system, maps)
    psf, _, _ = plan.forward(vals, ph, am)
    torch.cuda.synchronize()
    ref, _ = oracle_psf(system, cfg, maps)
    assert worst_pair_rel(psf.cpu().numpy(), ref) < 1e-4


def test_post_doe_mixed_map_gradients_on_oracle_draws(rw):
    system, cfg, maps = _case()
    L0, g, ref, idx = O.loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                      maps["amp"].astype(np.float64), np.zeros(0),
                                      maps["target"].astype(np.float64))
    rep = torch.tensor(np.stack([idx[p] for p in sorted(idx)]), dtype=torch.int32, device="cuda")
    plan = rw.Plan(system, cfg, precision="mixed")
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    psf, loss, _ = plan.forward(vals, ph, am, target=tg, replay=rep)
    dp, da, _ = plan.backward()
    torch.cuda.synchronize()
    assert worst_pair_rel(psf.cpu().numpy(), ref) < 1e-4
    assert abs(float(loss) - L0) <= 1e-4 * abs(L0)
    assert rel_l2(dp.cpu().numpy(), g["phase"]) < 1e-3
    assert rel_l2(da.cpu().numpy(), g["amp"]) < 1e-3


# ------------------------------- lens-parameter gradients through the surfaces ---
def _grad_case(shape, sampling):
    if shape == "conformal":
        system, cfg, maps = W.conformal_sphere(rays_side=8, H=512, pitch=0.002, P=32,
                                               classes=(16, 8), N=32, Q=32, psf_pitch=0.004,
                                               n_lambda=2, n_field_side=2, max_deg=5.0,
                                               sampling=sampling, with_params=True)
        rng = np.random.default_rng(20260204)
        maps["target"] = rng.uniform(size=(2, 4, 32, 32)).astype(np.float32)
    else:                                  # a DOE before a plano-convex lens
        system, cfg, maps = W.grating_before_lens(rays_side=12, H=256, P=16, N=32, Q=32,
                                                  psf_pitch=0.004, sampling=sampling)
        # a pure blazed grating is constant along y: every k_y != 0 bin of a patch
        # spectrum vanishes, where p_mag's normaliser sum |U~| has no derivative
        # (the kink of |.| at 0); a weak band-limited phase keeps the bins nonzero
        rng = np.random.default_rng(20260206)
        maps["phase"] = (maps["phase"] +
                         0.5 * W.bandlimited_uniform(256, 256, 0.25, rng)).astype(np.float32)
    return system, cfg, maps


def _lens_grads(rw, system, cfg, maps, precision, replay=None):
    plan = rw.Plan(system, cfg, precision=precision)
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    psf, loss, _ = plan.forward(vals, ph, am, target=tg, replay=replay)
    dp, da, dl = plan.backward()
    torch.cuda.synchronize()
    return psf.cpu().numpy(), float(loss), dp.cpu().numpy(), da.cpu().numpy(), dl.cpu().numpy()


@pytest.mark.parametrize("shape", ["conformal", "grating_lens"])
@pytest.mark.parametrize("sampling,precision,tol", [("full", "mixed", 1e-3),
                                                    ("mag", "mixed", 1e-3),
                                                    ("mag", "fp64", 1e-5)])
def test_post_doe_lens_gradients(rw, shape, sampling, precision, tol):
    system, cfg, maps = _grad_case(shape, sampling)
    vals = oracle_param_values(system)
    L0, g, ref, idx = O.loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                      maps["amp"].astype(np.float64), vals,
                                      maps["target"].astype(np.float64))
    rep = None
    if sampling != "full" and precision == "mixed":
        rep = torch.tensor(np.stack([idx[p] for p in sorted(idx)]), dtype=torch.int32,
                           device="cuda")
    psf, L, dp, da, dl = _lens_grads(rw, system, cfg, maps, precision, replay=rep)
    errs = {"psf": worst_pair_rel(psf, ref), "phase": rel_l2(dp, g["phase"]),
            "amp": rel_l2(da, g["amp"]), "lens": rel_l2(dl, g["lens"])}
    print(shape, sampling, precision, errs, dl, g["lens"])
    assert abs(L - L0) <= max(tol, 1e-6) * abs(L0)
    assert max(errs.values()) < tol, errs
