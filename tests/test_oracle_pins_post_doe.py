"""Pins of the oracle when secondary rays cross refracting surfaces after the
DOE: the DOE upstream of a lens (the benchmark's System 1 shape) puts the
first diffraction order of a blazed linear grating where the grating
equation and the lens's focal length place it, and the lens-parameter
gradient through the post-DOE surfaces agrees with central differences on
both post-DOE shapes (a DOE before a plano-convex lens; a conformal DOE on a
lens's convex front with the planar rear face after it)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import rw_oracle as O


def test_grating_before_lens_first_order_centroid():
    """0.7 um light through a 35 x 6.3 um blazed grating 3 mm before an f = 50 mm
    plano-convex: the first order leaves at asin(lambda / period) and focuses at
    EFL tan(theta_1) = 0.160 mm off axis in the back focal plane (the paper's
    System 1 reports a ground-truth centroid of (160.30, 0.35) um for its lens).
    Paraxial tolerance 1%."""
    system, cfg, maps = W.grating_before_lens(rays_side=16, H=128, P=16, N=64, Q=64,
                                              psf_pitch=0.004, sampling="full")
    I, _ = O.psf_stack(system, cfg, maps["phase"].astype(np.float64),
                       maps["amp"].astype(np.float64))
    I = I[0, 0]
    Q = cfg["psf_q"]
    lam, period = cfg["lambdas"][0], 35 * 0.0063
    n = O.cauchy_index(W.BK7[0], W.BK7[1], lam)
    efl = 25.8 / (n - 1)
    x_expect = efl * math.tan(math.asin(lam / period))
    assert abs(x_expect - 0.1603) < 2e-3                  # the paper's 160.30 um, 1.3% apart
    x = (np.arange(Q) - Q // 2) * cfg["psf_pitch"] + cfg["psf_center"][0][0][0]
    y = (np.arange(Q) - Q // 2) * cfg["psf_pitch"] + cfg["psf_center"][0][0][1]
    cx = (I.sum(0) * x).sum() / I.sum()
    cy = (I.sum(1) * y).sum() / I.sum()
    assert abs(cx - x_expect) < 1e-2 * x_expect, (cx, x_expect)
    assert abs(cy) < 2e-3
    # the zeroth and second orders carry little of the blazed grating's light
    assert I.sum() > 0


def _fd_check(system, cfg, maps, h=1e-5):
    vals = O.initial_param_values(system)
    ph = maps["phase"].astype(np.float64)
    am = maps["amp"].astype(np.float64)
    tg = maps["target"].astype(np.float64)
    L0, g, _, idx = O.loss_and_grad(system, cfg, ph, am, vals, tg)
    rep = None if cfg["sampling"] == "full" else idx
    scale = np.abs(g["lens"]).max()
    assert scale > 0
    for k in range(len(vals)):
        vp, vm = vals.copy(), vals.copy()
        vp[k] += h
        vm[k] -= h
        fd = (O.loss_and_grad(system, cfg, ph, am, vp, tg, replays=rep, want_grad=False)[0] -
              O.loss_and_grad(system, cfg, ph, am, vm, tg, replays=rep, want_grad=False)[0]) / (2 * h)
        assert abs(fd - g["lens"][k]) <= 1e-5 * scale + 1e-4 * abs(fd), (k, fd, g["lens"][k])


@pytest.mark.parametrize("sampling", ["full", "mag"])
def test_grating_lens_gradient_matches_central_differences(sampling):
    system, cfg, maps = W.grating_before_lens(rays_side=4, H=64, P=8, N=16, Q=16, psf_pitch=0.008,
                                              sampling=sampling)
    _fd_check(system, cfg, maps)


@pytest.mark.parametrize("sampling", ["full", "mag"])
def test_conformal_lens_gradient_matches_central_differences(sampling):
    system, cfg, maps = W.conformal_sphere(rays_side=4, H=128, pitch=0.008, P=8, classes=(4,),
                                           N=16, Q=16, psf_pitch=0.004, n_lambda=1,
                                           n_field_side=1, sampling=sampling, with_params=True,
                                           curv_eps=0.033)
    rng = np.random.default_rng(20260204)
    maps["target"] = rng.uniform(size=(1, 1, 16, 16))
    _fd_check(system, cfg, maps)
