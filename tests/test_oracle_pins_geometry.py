"""Pins of the oracle's geometry after the DOE and of its patch and relaxation
helpers, against closed forms and library routines (no GPU):

  * the refracting trace after the DOE (planar exit face): Snell at a plane in
    closed form, and the paraxial back focal length of a plano-convex lens
    whose convex front carries a transparent DOE (thick-lens formula);
  * the emission direction at the zero-frequency bin equals vector Snell;
  * the tangent frame on a sphere: the normal points at the centre, u is the
    projection of the x axis, v = n x u is perpendicular to x;
  * bilinear sampling of the complex map at fractional positions: affine maps
    are reproduced exactly, and any map agrees with scipy's order-1 spline
    with zero padding;
  * the relaxed weights of the straight-through gradient: p_k N w_k is the
    FULL-mode weight U~_k / M^2 of every bin (unbiasedness of Eq. 1).
"""
import math

import numpy as np
import pytest
import torch
from scipy import ndimage

import workloads as W
from oracle import rw_oracle as O

DT = torch.float64


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


# ----------------------------------------------------- trace after the DOE ---
def _plano_convex(lam, R=30.0, ct=4.0, sensor_gap=60.0):
    """BK7 plano-convex: convex front (the DOE surface) at z = 0, planar rear at ct."""
    system = {"surfaces": [W.surface(0.0, c=1 / R, medium=W.BK7, doe=True),
                           W.surface(ct, medium=W.AIR)],
              "sensor_z": ct + sensor_gap, "params": []}
    surfs, sensor_z = O.build_surfaces(system)
    n = O.cauchy_index(W.BK7[0], W.BK7[1], lam)
    return surfs, sensor_z, n


def test_post_doe_plane_refraction_closed_form():
    """A ray in glass crossing a planar exit face: Snell at a plane (tangential
    direction scaled by n1 / n2), straight segments, OPL = n1 t1 + n2 t2."""
    lam = 587.6e-6
    surfs, zs, n1 = _plano_convex(lam)
    rng = np.random.default_rng(11)
    k = 64
    p = np.c_[rng.uniform(-0.3, 0.3, (k, 2)), rng.uniform(0.0, 0.5, k)]
    d = np.c_[rng.uniform(-0.25, 0.25, (k, 2)), np.ones(k)]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    opl0 = rng.uniform(0, 1, k)
    ps, ds, opl, alive, n_s = O.trace_post_doe(surfs, 0, lam, _t(p), _t(d), _t(opl0), zs)
    assert bool(alive.all()) and n_s == 1.0
    zp = 4.0
    t1 = (zp - p[:, 2]) / d[:, 2]
    q = p + t1[:, None] * d
    dxy = n1 * d[:, :2]
    dz = np.sqrt(1 - (dxy ** 2).sum(1))
    t2 = (float(zs) - zp) / dz
    r = q + t2[:, None] * np.c_[dxy, dz]
    assert np.max(np.abs(ds.numpy() - np.c_[dxy, dz])) < 1e-14
    assert np.max(np.abs(ps.numpy() - r)) < 1e-12
    assert np.max(np.abs(opl.numpy() - (opl0 + n1 * t1 + t2))) < 1e-12
    # beyond the critical angle the exit face reflects totally: the ray dies
    dg = np.array([[0.8, 0.0, 0.6]])
    _, _, _, alive, _ = O.trace_post_doe(surfs, 0, lam, _t([[0, 0, 1.0]]), _t(dg), _t([0.0]), zs)
    assert not bool(alive.any())


@pytest.mark.parametrize("lam,bfl", [(400e-6, 53.89), (587.6e-6, 55.41), (700e-6, 55.81)])
def test_plano_convex_back_focus_through_doe_emission(lam, bfl):
    """Collimated paraxial rays on a transparent DOE (t = 1) carried by the R = 30
    convex front of a CT 4 BK7 plano-convex: the zero-frequency secondary of
    each ray is the refracted ray, and after the planar rear face it meets the
    axis at the thick-lens back focal length R / (n - 1) - CT / n."""
    surfs, zs, n = _plano_convex(lam)
    assert abs((30.0 / (n - 1) - 4.0 / n) - bfl) < 5e-3
    h = np.array([2e-3, 4e-3, 8e-3])
    p = _t(np.c_[h, np.zeros(3), -np.ones(3)])
    d = _t(np.tile([0.0, 0.0, 1.0], (3, 1)))
    p, d, opl, alive, s_doe = O.trace_to_doe(surfs, lam, p, d, torch.zeros(3, dtype=DT))
    assert s_doe == 0 and bool(alive.all())
    u, v, nrm = O.tangent_frame(surfs[0], p)
    k0 = 2 * math.pi / lam
    Ku = k0 * (d * u).sum(1)                    # n_in = 1 (air), j = 0: no DOE frequency
    Kv = k0 * (d * v).sum(1)
    ds = O.emit_direction(Ku, Kv, u, v, nrm, k0 * n)
    ps, dout, _, ok, _ = O.trace_post_doe(surfs, 0, lam, p, ds, opl, zs)
    assert bool(ok.all())
    z_cross = ps[:, 2] - ps[:, 0] * dout[:, 2] / dout[:, 0]
    lsa = (4.0 + bfl) - z_cross.numpy()
    assert np.max(np.abs(lsa)) < 5e-3 + 1e-3
    # longitudinal spherical aberration grows as h^2 (marginal focus shorter)
    exact = (4.0 + 30.0 / (n - 1) - 4.0 / n) - z_cross.numpy()
    assert exact[2] > exact[1] > exact[0] > 0
    assert abs(exact[2] / exact[1] - 4) < 0.05


def test_zero_frequency_emission_is_vector_snell():
    """At the zero-frequency bin the emitted direction keeps the incident
    tangential wavevector k0 n_in (d.u, d.v): vector Snell into n_out."""
    lam = 500e-6
    surf = O.build_surfaces({"surfaces": [W.surface(0.0, c=1 / 12.0, A=(0.01, 0, 0, 0),
                                                    medium=W.F2, doe=True)],
                             "sensor_z": 10.0, "params": []})[0][0]
    rng = np.random.default_rng(5)
    k = 40
    xy = rng.uniform(-1.5, 1.5, (k, 2))
    sag = O.sag_and_grad(surf, _t(xy[:, 0]), _t(xy[:, 1]))[0]
    p = torch.stack([_t(xy[:, 0]), _t(xy[:, 1]), sag], 1)
    d = _t(np.c_[rng.uniform(-0.3, 0.3, (k, 2)), np.ones(k)])
    d = d / d.norm(dim=1, keepdim=True)
    u, v, nrm = O.tangent_frame(surf, p)
    n_in, n_out = 1.0, O.cauchy_index(W.F2[0], W.F2[1], lam)
    k0 = 2 * math.pi / lam
    ds = O.emit_direction(k0 * n_in * (d * u).sum(1), k0 * n_in * (d * v).sum(1), u, v, nrm,
                          k0 * n_out)
    ref, ok = O.refract(d, nrm, n_in, n_out)
    assert bool(ok.all())
    assert torch.max(torch.abs(ds - ref)).item() < 1e-14


# ------------------------------------------------------ tangent frame -------
def test_tangent_frame_on_sphere_closed_form():
    R, zv = 30.0, 1.5
    surf = O.build_surfaces({"surfaces": [W.surface(zv, c=1 / R, doe=True)],
                             "sensor_z": 10.0, "params": []})[0][0]
    rng = np.random.default_rng(6)
    xy = np.r_[rng.uniform(-6, 6, (50, 2)), [[0.0, 4.0], [0.0, -3.0], [2.0, 0.0]]]
    z = zv + R - np.sqrt(R * R - (xy ** 2).sum(1))
    p = _t(np.c_[xy, z])
    u, v, n = (x.numpy() for x in O.tangent_frame(surf, p))
    C = np.array([0.0, 0.0, zv + R])
    assert np.max(np.abs(n - (C - p.numpy()) / R)) < 1e-14          # normal points at the centre
    ex = np.array([1.0, 0.0, 0.0])
    u_cf = ex - n[:, :1] * n
    u_cf /= np.linalg.norm(u_cf, axis=1, keepdims=True)
    assert np.max(np.abs(u - u_cf)) < 1e-14                          # projection of x
    v_cf = np.cross(n, ex)
    v_cf /= np.linalg.norm(v_cf, axis=1, keepdims=True)
    assert np.max(np.abs(v - v_cf)) < 1e-14                          # v along n x x
    assert np.max(np.abs(v[:, 0])) < 1e-15
    det = np.einsum("ij,ij->i", np.cross(u, v), n)
    assert np.max(np.abs(det - 1)) < 1e-14                           # right-handed
    on_y = np.abs(xy[:, 0]) == 0
    assert np.all(u[on_y] == ex)


# ------------------------------------------------------ bilinear sampling ---
def test_bilinear_reproduces_affine_maps_at_fractional_points():
    doe = W.doe_desc(40, 50, 0.01, cx=0.03, cy=-0.02)
    x = doe["x0"] + np.arange(50) * 0.01
    y = doe["y0"] + np.arange(40) * 0.01
    a, b, c = 0.3 - 0.2j, 1.7 + 0.4j, -0.9 + 2.1j
    tmap = torch.tensor(a + b * x[None, :] + c * y[:, None])
    rng = np.random.default_rng(8)
    qx = rng.uniform(x[0], x[-1], 500)
    qy = rng.uniform(y[0], y[-1], 500)
    out = O.bilinear_complex(tmap, doe, _t(qx), _t(qy)).numpy()
    assert np.max(np.abs(out - (a + b * qx + c * qy))) < 1e-12


def test_bilinear_matches_library_spline_with_zero_padding():
    doe = W.doe_desc(32, 24, 0.005)
    rng = np.random.default_rng(9)
    m = rng.normal(size=(32, 24)) + 1j * rng.normal(size=(32, 24))
    # fractional points over the whole map and a margin of two pixels beyond it
    fx = rng.uniform(-2.0, 25.0, 2000)
    fy = rng.uniform(-2.0, 33.0, 2000)
    out = O.bilinear_complex(torch.tensor(m), doe, _t(doe["x0"] + fx * 0.005),
                             _t(doe["y0"] + fy * 0.005)).numpy()
    ref = (ndimage.map_coordinates(m.real, [fy, fx], order=1, mode="grid-constant", cval=0.0) +
           1j * ndimage.map_coordinates(m.imag, [fy, fx], order=1, mode="grid-constant", cval=0.0))
    assert np.max(np.abs(out - ref)) < 1e-12


# --------------------------------------------- relaxed straight-through weights ---
@pytest.mark.parametrize("sampling", ["mag", "uni"])
def test_relaxed_weights_are_unbiased_per_bin(sampling):
    """p_k N w_k = U~_k / M^2 on every bin that can be drawn: drawing J ~ p N times
    and weighting by w_J is an unbiased estimate of the FULL field (Eq. 1)."""
    rng = np.random.default_rng(10)
    R, M, Nd = 3, 16, 24
    Ut = torch.tensor(rng.normal(size=(R, M * M)) + 1j * rng.normal(size=(R, M * M)))
    Ut[0, 5] = 0.0                                   # a zero bin cannot be drawn under p_mag
    prop = torch.tensor(rng.uniform(size=(R, M * M)) < 0.7)
    logp, w, live = O.relaxed_weights(Ut, prop, sampling, M, Nd)
    p = torch.exp(logp)
    assert torch.allclose(p.sum(1), torch.ones(R, dtype=DT), atol=1e-14)
    full = torch.where(prop, Ut / (M * M), torch.zeros_like(Ut))
    lhs = torch.where(live, p * Nd * w, torch.zeros_like(w))
    assert torch.max(torch.abs(lhs - torch.where(live, full, torch.zeros_like(full)))).item() < 1e-15
    assert torch.equal(w[~live], torch.zeros_like(w[~live]))
    if sampling == "mag":
        assert not bool(live[0, 5])
        absw = w.abs()[live]
        S = torch.where(prop, Ut.abs(), torch.zeros((), dtype=DT)).sum(1)
        ref = (S[:, None] / (M * M * Nd)).expand(R, M * M)[live]
        assert torch.max(torch.abs(absw - ref)).item() < 1e-15      # |w| = S / (M^2 N)
