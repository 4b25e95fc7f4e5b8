"""Pins of the oracle's reflective conformal DOE (the curvilinear-DOE
demonstration, Fig. 6): the Gaussian-like substrate sag against its closed
form and the paper's radius of curvature, the reflective emission at zero
DOE frequency against the law of reflection, the two-phase beam-splitting
field focusing at the two designed spots with the Airy width of its NA, and
the gradient w.r.t. both phase maps against central differences."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import rw_oracle as O


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


def test_gaussian_sag_closed_form_and_radius():
    lam = 1e-3
    system, cfg, maps = W.reflective_conformal(rays_side=8, H=101, P=16, N=16, Q=32)
    surf = O.build_surfaces(system)[0][0]
    gh, gw = float(surf["gh"]), float(surf["gw"])
    rng = np.random.default_rng(12)
    xy = rng.uniform(-0.12, 0.12, (200, 2))
    sag, sx, sy, ok = O.sag_and_grad(surf, _t(xy[:, 0]), _t(xy[:, 1]))
    r2 = (xy ** 2).sum(1)
    e = np.exp(-r2 / gw ** 2)
    assert np.max(np.abs(sag.numpy() - gh * (e - 1))) < 1e-16
    assert np.max(np.abs(sx.numpy() - (-2 * xy[:, 0] * gh / gw ** 2 * e))) < 1e-13
    assert np.max(np.abs(sy.numpy() - (-2 * xy[:, 1] * gh / gw ** 2 * e))) < 1e-13
    # the vertex radius gw^2 / (2 |gh|): the paper's ~506 wavelengths
    R0 = float(O.local_radius(surf, _t([0.0]), _t([0.0]))[0])
    assert abs(R0 - 506 * lam) < 1e-9
    # meridional curvature off axis against a finite difference of the closed form
    r, h = 0.07, 1e-5
    z = lambda rr: gh * (math.exp(-rr * rr / gw ** 2) - 1)
    z1 = (z(r + h) - z(r - h)) / (2 * h)
    z2 = (z(r + h) - 2 * z(r) + z(r - h)) / (h * h)
    km = abs(z2) / (1 + z1 * z1) ** 1.5
    ks = abs(z1) / (r * math.sqrt(1 + z1 * z1))
    R = float(O.local_radius(surf, _t([r]), _t([0.0]))[0])
    assert abs(R - 1 / max(km, ks)) < 1e-6 * R


def test_reflective_zero_frequency_emission_is_specular():
    system, cfg, maps = W.reflective_conformal(rays_side=8, H=101, P=16, N=16, Q=32)
    surf = O.build_surfaces(system)[0][0]
    rng = np.random.default_rng(13)
    k = 50
    xy = rng.uniform(-0.1, 0.1, (k, 2))
    sag = O.sag_and_grad(surf, _t(xy[:, 0]), _t(xy[:, 1]))[0]
    p = torch.stack([_t(xy[:, 0]), _t(xy[:, 1]), sag], 1)
    d = _t(np.c_[rng.uniform(-0.3, 0.3, (k, 2)), np.ones(k)])
    d = d / d.norm(dim=1, keepdim=True)
    u, v, n = O.tangent_frame(surf, p)
    k0 = 2 * math.pi / 1e-3
    ds = O.emit_direction(k0 * (d * u).sum(1), k0 * (d * v).sum(1), u, v, n, k0, -1.0)
    spec = d - 2 * (d * n).sum(1, keepdim=True) * n
    assert torch.max(torch.abs(ds - spec)).item() < 1e-14


def test_two_phase_field_focuses_at_the_two_designed_spots():
    """exp(i phi1) + exp(i phi2) with the point-focus phases of two spots 16 um
    apart, NA 0.2, on a flat reflective DOE (sensor f in front of it, inside one
    period M pitch of the patch spectra): peaks exactly at +-8 um, half the
    energy each, FWHM 0.51 lambda / NA."""
    system, cfg, maps = W.reflective_conformal(rays_side=24, H=251, P=64, N=64, Q=64,
                                               psf_pitch=0.0005, sampling="full", sep=0.016,
                                               gw=0.0, na=0.2)
    assert system["doe"]["reflective"] and system["sensor_z"] < 0
    I, _ = O.psf_stack(system, cfg, maps["phase"].astype(np.float64),
                       maps["amp"].astype(np.float64))
    I = I[0, 0]
    Q = cfg["psf_q"]
    x = (np.arange(Q) - Q // 2) * cfg["psf_pitch"]
    col = I.sum(0)
    assert x[np.argmax(col[:Q // 2])] == -0.008 and x[Q // 2 + np.argmax(col[Q // 2:])] == 0.008
    assert abs(I[:, :Q // 2].sum() / I.sum() - 0.5) < 1e-3
    assert abs((I.sum(1) * x).sum() / I.sum()) < 1e-5
    row = I[Q // 2 + 0, Q // 2:]
    fwhm = (row > row.max() / 2).sum() * cfg["psf_pitch"]
    assert abs(fwhm - 0.51 * 1e-3 / 0.2) <= cfg["psf_pitch"]


@pytest.mark.parametrize("sampling", ["full", "mag"])
def test_two_phase_gradients_match_central_differences(sampling):
    system, cfg, maps = W.reflective_conformal(rays_side=4, H=61, P=16, N=16, Q=16,
                                               psf_pitch=0.001, sampling=sampling,
                                               random_phase=0.5, sep=0.006)
    ph = maps["phase"].astype(np.float64)
    am = maps["amp"].astype(np.float64)
    tg = maps["target"].astype(np.float64)
    L0, g, _, idx = O.loss_and_grad(system, cfg, ph, am, np.zeros(0), tg)
    rep = None if sampling == "full" else idx
    h = 1e-5
    for name, arr in (("phase", ph), ("amp", am)):
        for o in np.argsort(-np.abs(g[name]).ravel())[:3]:
            y, x = np.unravel_index(o, arr.shape)
            ap, an = arr.copy(), arr.copy()
            ap[y, x] += h
            an[y, x] -= h
            args_p = (ap, am) if name == "phase" else (ph, ap)
            args_m = (an, am) if name == "phase" else (ph, an)
            Lp = O.loss_and_grad(system, cfg, *args_p, np.zeros(0), tg, replays=rep,
                                 want_grad=False)[0]
            Lm = O.loss_and_grad(system, cfg, *args_m, np.zeros(0), tg, replays=rep,
                                 want_grad=False)[0]
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[name][y, x]) <= 1e-4 * abs(fd) + 1e-8 * np.abs(g[name]).max(), \
                (name, y, x, fd, g[name][y, x])
