"""Pins of the oracle's two-DOE cascade (Formalism, first paragraph: the
construction extends to several DOEs because secondary rays are traced
conventionally).

* A clear second DOE (phase 0, amplitude 1, patch not zero-padded) has one
  nonzero spectrum bin, the zeroth, whose Eq. 1 weights sum to one: the
  cascade must then equal the single-DOE system in which the second DOE's
  surface is an ordinary refracting surface (its emission is Snell's law).
  This pins the first stage's relay: the amplitude and optical path carried to
  the second DOE, the trace between the DOEs and the second DOE's weights.
* A clear first DOE likewise reduces the cascade to the single-DOE system of
  the second DOE, in FULL sampling (the draws' streams differ): this pins the
  second stage on its own.
* With both DOEs nontrivial, the Monte Carlo cascade is unbiased for the
  sensor field: its mean over independent draws is the FULL cascade's field,
  within the standard error (a wrong normalisation of either stage fails).
* The autograd gradient of the Eq. 5 loss with respect to both maps matches
  central differences.
"""
import copy

import numpy as np
import torch

import workloads as W
from oracle import rw_oracle as O


def _tmaps(maps):
    return [O.transmission(O._t(maps["phase"][k].astype(np.float64)),
                           O._t(maps["amp"][k].astype(np.float64))) for k in range(2)]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_clear_second_doe_is_a_refracting_surface():
    s, c, m = W.two_doe_cascade(rays_side=4, P=8, pad=1, N=4, N2=3, sampling="mag",
                                uniform=(False, True), fields=((0.0, 0.0), (0.004, -0.003)))
    I, aux = O.cascade_psf_stack(s, c, m["phase"], m["amp"], keep=True)
    assert all(np.all(np.isin(aux[p]["J2"], (-1, 36))) for p in aux)   # the zeroth bin only
    single = copy.deepcopy(s)
    single["surfaces"][3]["doe"] = False
    single["doe"] = s["does"][0]
    I1, _ = O.psf_stack(single, c, m["phase"][0].astype(np.float64),
                        m["amp"][0].astype(np.float64))
    assert I.max() > 0
    assert _rel(I, I1) < 1e-8


def test_clear_first_doe_reduces_to_the_second():
    s, c, m = W.two_doe_cascade(rays_side=4, P=8, pad=1, N=4, N2=3, sampling="full",
                                uniform=(True, False), lambdas=(W.LAM_D, W.LAM_F))
    I, _ = O.cascade_psf_stack(s, c, m["phase"], m["amp"])
    single = copy.deepcopy(s)
    single["surfaces"][0]["doe"] = False
    single["doe"] = s["does"][1]
    I2, _ = O.psf_stack(single, c, m["phase"][1].astype(np.float64),
                        m["amp"][1].astype(np.float64))
    assert I.max() > 0
    assert _rel(I, I2) < 1e-10


def test_monte_carlo_cascade_is_unbiased():
    s, c, m = W.two_doe_cascade(rays_side=2, P=4, pad=2, N=16, N2=4, Q=16, psf_pitch=0.04,
                                sampling="full", cutoff=0.02, seed=3)
    tm = _tmaps(m)
    with torch.no_grad():
        Uf = O.cascade_pair_forward(s, c, tm, 0, 0)["U"].numpy()
    c = dict(c, sampling="mag")
    S = 400
    Us = []
    with torch.no_grad():
        for k in range(S):
            c["seed"] = 1000 + k
            Us.append(O.cascade_pair_forward(s, c, tm, 0, 0)["U"].numpy())
    Us = np.array(Us)
    mean = Us.mean(0)
    var = (np.abs(Us - mean) ** 2).sum(0) / (S - 1)
    # squared distance of the mean from the FULL field in units of its standard
    # error: about 1 when unbiased; a 20 % scale error of the mean gives about 3
    T = np.sum(np.abs(mean - Uf) ** 2) / np.sum(var / S)
    assert T < 2.0, T


def test_cascade_map_gradients_match_central_differences():
    """Gradient of the Eq. 5 loss with respect to both DOEs' maps (FULL: no draws)
    against central differences of the loss, h = 1e-4 (reading Q18)."""
    s, c, m = W.two_doe_cascade(rays_side=2, P=4, pad=2, N=4, N2=2, Q=16, psf_pitch=0.04,
                                sampling="full", cutoff=0.05, seed=2)
    rng = np.random.default_rng(8)
    target = rng.uniform(0.0, 1.0, (1, 1, 16, 16))
    ph = m["phase"].astype(np.float64)
    am = m["amp"].astype(np.float64)
    L0, g, _, _ = O.cascade_loss_and_grad(s, c, ph, am, target)
    assert np.abs(g["phase"][0]).max() > 0 and np.abs(g["phase"][1]).max() > 0
    h = 1e-4
    for name, arr in (("phase", ph), ("amp", am)):
        for k in range(2):
            # the pixels with the largest gradient of each map
            flat = np.argsort(-np.abs(g[name][k]).ravel())[:3]
            for q in flat:
                iy, ix = divmod(int(q), arr.shape[2])
                hi, lo = arr.copy(), arr.copy()
                hi[k, iy, ix] += h
                lo[k, iy, ix] -= h
                a, b = ((hi, am), (lo, am)) if name == "phase" else ((ph, hi), (ph, lo))
                Lh = O.cascade_loss_and_grad(s, c, a[0], a[1], target, want_grad=False)[0]
                Ll = O.cascade_loss_and_grad(s, c, b[0], b[1], target, want_grad=False)[0]
                fd = (Lh - Ll) / (2 * h)
                assert abs(fd - g[name][k][iy, ix]) <= 1e-5 * max(abs(fd), 1e-3 * abs(L0)), \
                    (name, k, iy, ix, fd, g[name][k][iy, ix])
