"""Pin of the oracle's held-density gradient mode (Eq. 1 with p fixed).

With the drawn bins frozen and the density p_J held constant, one draw's weight
U~_J / (M^2 N p_J) has the derivative dU~_J / (M^2 N p_J); its mean over J ~ p
is the derivative of the FULL-mode weights U~_j / M^2.  For a loss linear in the
sensor field the p-weighted sum of the one-draw gradients over every
propagating bin must therefore equal the FULL-mode gradient exactly (up to
rounding).  The frozen-draw derivative that differentiates p as well (the
default mode) carries an extra term and must not.
"""
import os

import numpy as np
import torch

import workloads as W
from oracle import rw_oracle as O

torch.set_num_threads(min(8, os.cpu_count() or 1))


def _case():
    rng = np.random.default_rng(11)
    H, P = 32, 8
    phase = 2 * np.pi * W.bandlimited_uniform(H, H, 0.2, rng)
    amp = 0.5 + 0.5 * W.bandlimited_uniform(H, H, 0.2, rng)
    system, cfg, maps = W.free_space_doe(phase, amp, 0.002, 1.0, 0.5e-3, 1, P, 16, 0.002,
                                         sampling="mag", N=1)
    return system, cfg, maps


def _linear_loss_grads(system, cfg, maps, c, replay=None):
    ph = torch.tensor(maps["phase"], dtype=torch.float64, requires_grad=True)
    am = torch.tensor(maps["amp"], dtype=torch.float64, requires_grad=True)
    r = O.pair_forward(system, cfg, O.transmission(ph, am), 0, 0, replay=replay)
    loss = (r["U"] * c.conj()).real.sum()
    loss.backward()
    return np.concatenate([ph.grad.numpy().ravel(), am.grad.numpy().ravel()])


def test_held_density_gradient_averages_to_the_full_mode_gradient():
    system, cfg, maps = _case()
    Q = cfg["psf_q"]
    rng = np.random.default_rng(3)
    c = torch.tensor(rng.normal(size=(Q, Q)) + 1j * rng.normal(size=(Q, Q)))
    g_full = _linear_loss_grads(system, dict(cfg, sampling="full"), maps, c)
    # the ray's spectrum and density in the sampler's (j_x-major) bin order
    with torch.no_grad():
        tm = O.transmission(torch.tensor(maps["phase"], dtype=torch.float64),
                            torch.tensor(maps["amp"], dtype=torch.float64))
        r = O.pair_forward(system, cfg, tm, 0, 0, keep=True)
    M = cfg["pad"] * cfg["patch_p"]
    mag = r["spectrum"][0].abs().transpose(0, 1).reshape(-1).numpy()
    prop = r["prop"][0].transpose(0, 1).reshape(-1).numpy()
    p = np.where(prop, mag, 0.0) / mag[prop].sum()
    bins = np.nonzero(p > 0)[0]
    assert len(bins) > 100
    g_det = np.zeros_like(g_full)
    g_dep = np.zeros_like(g_full)
    for j in bins:
        replay = np.array([[j]])
        g_det += p[j] * _linear_loss_grads(system, dict(cfg, grad="G1_DETACH"), maps, c, replay)
        g_dep += p[j] * _linear_loss_grads(system, cfg, maps, c, replay)
    scale = np.linalg.norm(g_full)
    assert np.linalg.norm(g_det - g_full) < 1e-10 * scale
    # differentiating p too is biased: the same average misses the FULL gradient
    assert np.linalg.norm(g_dep - g_full) > 1e-3 * scale
