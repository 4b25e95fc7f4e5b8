"""Pins of the oracle's adaptive patch sizing (the paper's future work on
adaptive patch sizing; reading: the smallest candidate patch spanning K local
periods of the phase map, the largest where the map is flatter).

* A linear grating of period Lambda > 2 pixels, wrapped to [0, 2 pi), has
  |grad phi| = 2 pi / (Lambda pitch) exactly (differences of a linear phase,
  with the wrap undone), so the chosen side is the smallest P >= K Lambda (in
  pixels).
* A kinoform zone plate phi = -pi r^2 / (lambda f) mod 2 pi has the local
  frequency r / (lambda f): central differences of a quadratic are exact, so a
  ray whose nearest pixel lies at radius r takes the smallest P with
  P pitch r >= K lambda f -- closed-form class radii.
* Where the curvature bound of Eq. 4 asks for a smaller side, the ray takes it.
* Adaptive ray sampling (a class of side P draws N (P / P_0)^2 secondaries)
  keeps the Monte Carlo field unbiased.
"""
import math

import numpy as np
import torch

import workloads as W
from oracle import rw_oracle as O

CANDS = [64, 32, 16, 8]


def _expected(P_needed):
    """Smallest candidate >= P_needed, else the largest."""
    ok = [P for P in CANDS if P >= P_needed]
    return min(ok) if ok else CANDS[0]


def test_grating_local_period_picks_the_side():
    rng = np.random.default_rng(4)
    pitch = 0.002
    doe = W.doe_desc(128, 128, pitch)
    x = doe["x0"] + np.arange(128) * pitch
    y = doe["y0"] + np.arange(128) * pitch
    K = 2.0
    for period_px in (2.3, 3.3, 5.1, 7.4, 11.0, 19.5, 35.0, 80.0, 1e4):
        for ang in (0.0, 0.7, 2.0):
            kx, ky = math.cos(ang), math.sin(ang)
            phase = np.mod(2 * math.pi * (kx * x[None, :] + ky * y[:, None]) / (period_px * pitch)
                           + 0.3, 2 * math.pi)
            px = rng.uniform(x[2], x[-3], 50)
            py = rng.uniform(y[2], y[-3], 50)
            g2 = O.local_phase_gradient2(phase, doe, px, py)
            want = (2 * math.pi / (period_px * pitch)) ** 2
            assert np.allclose(g2, want, rtol=1e-9), (period_px, ang)
            sides = O.bandwidth_sides(phase, doe, px, py, CANDS, K)
            assert np.all(sides == _expected(K * period_px)), (period_px, ang, sides[:4])


def test_zone_plate_class_radii_in_closed_form():
    pitch, lam, f, K = 0.002, 0.5e-3, 10.0, 2.0
    H = 512
    doe = W.doe_desc(H, H, pitch)
    phase = W.kinoform_zone_plate(doe, f, lam)
    # the wrapped one-pixel difference stays below pi over the whole map
    r_max = math.hypot(H * pitch / 2, H * pitch / 2)
    assert 2 * math.pi * r_max * pitch / (lam * f) < math.pi
    rng = np.random.default_rng(5)
    px = rng.uniform(-0.5, 0.5, 400)
    py = rng.uniform(-0.5, 0.5, 400)
    sides = O.bandwidth_sides(phase, doe, px, py, CANDS, K)
    jx = np.rint((px - doe["x0"]) / pitch)
    jy = np.rint((py - doe["y0"]) / pitch)
    rj = np.hypot(doe["x0"] + jx * pitch, doe["y0"] + jy * pitch)
    # P pitch (2 pi r / (lambda f)) >= 2 pi K  <=>  P >= K lambda f / (r pitch)
    need = K * lam * f / np.maximum(rj * pitch, 1e-300)
    want = np.array([_expected(n) for n in need])
    far = np.abs(need[:, None] - np.array(CANDS)[None, :]).min(1) > 1e-6
    assert far.all()
    assert np.array_equal(sides, want)
    assert len(set(sides.tolist())) >= 3          # the map spans several classes


def test_curvature_bound_wins_where_it_is_smaller():
    # a sphere of radius 2 mm: Eq. 4 at eps = 0.01 allows D <= 2 R sin(0.01) = 0.04 mm,
    # i.e. P <= 20 at 2 um, so the curvature side is 16 wherever the map asks for more
    s = W.surface(0.0, c=1.0 / 2.0, doe=True)
    surfs, _ = O.build_surfaces({"surfaces": [s], "sensor_z": 1.0, "params": []})
    pitch = 0.002
    doe = W.doe_desc(128, 128, pitch)
    flat = np.zeros((128, 128))
    p = torch.tensor([[0.01, -0.02, 0.0], [0.05, 0.03, 0.0]], dtype=torch.float64)
    cfg = {"patch_p": 64, "patch_classes": [32, 16, 8], "curv_eps": 0.01, "bw_periods": 2.0}
    sides = O.ray_patch_sides(surfs[0], p, pitch, cfg, flat, doe)
    assert np.all(sides == 16)
    cfg0 = dict(cfg, curv_eps=1.0)                   # no curvature limit: the flat map's side
    assert np.all(O.ray_patch_sides(surfs[0], p, pitch, cfg0, flat, doe) == 64)


def test_class_draws_keep_the_estimator_unbiased():
    """Adaptive ray sampling: a ray of patch side P draws N (P / P_0)^2 secondaries
    (Eq. 1 divides by that count).  The Monte Carlo field still averages to the
    FULL-mode field of the same classes within its standard error (a weight
    normalised by N instead of the class's count biases the small-patch rays 4x)."""
    s, c, m = W.adaptive_zone_plate(rays_side=6, H=96, pitch=0.002, f=1.0, P=16, classes=(8,),
                                    K=2.0, N=16, Q=16, psf_pitch=0.004, sampling="full")
    tm = O.transmission(O._t(m["phase"].astype(np.float64)), O._t(m["amp"].astype(np.float64)))
    with torch.no_grad():
        r = O.pair_forward(s, c, tm, 0, 0, keep=True, phase_map=m["phase"])
    sides = r["sides"]
    assert set(sides.tolist()) == {16, 8}
    Uf = r["U"].numpy()
    c = dict(c, sampling="mag", class_draws=True)
    S = 400
    Us = []
    with torch.no_grad():
        for k in range(S):
            c["seed"] = 500 + k
            rk = O.pair_forward(s, c, tm, 0, 0, keep=k == 0, phase_map=m["phase"])
            if k == 0:
                # 16 draws for the 16-px rays, 16 (8/16)^2 = 4 for the 8-px ones
                J = rk["J"]
                assert np.all(J[sides == 16] >= 0)
                assert np.all(J[sides == 8][:, :4] >= 0) and np.all(J[sides == 8][:, 4:] == -1)
            Us.append(rk["U"].numpy())
    Us = np.array(Us)
    mean = Us.mean(0)
    var = (np.abs(Us - mean) ** 2).sum(0) / (S - 1)
    T = np.sum(np.abs(mean - Uf) ** 2) / np.sum(var / S)
    assert T < 2.0, T
