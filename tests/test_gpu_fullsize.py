"""Parity at the full size of the throughput workload, in the launch
configuration bench.py times (batched MIXED, default launch shape): 27 pairs x
256^2 rays, P = 64 (M = 128), N = 256 draws, Q = 512.

The outputs the oracle can compute ray by ray are checked on a sample of
rays of several pairs: the ray state at the DOE, and the drawn bins (own
draws: the MIXED form's FP32 spectrum may move a CDF edge, so >= 97% equal;
the FP64 form: equal).  The PSF and the gradients, which sum over every ray,
are compared with the FP64 form on its replayed draws.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import rw_oracle as O
from rwcases import gpu_inputs, oracle_param_values

pytestmark = pytest.mark.gpu

SAMPLE_PAIRS = (0, 4, 13, 26)          # (lambda, field) pairs checked
RAYS_PER_PAIR = 6


@pytest.fixture(scope="module")
def rw():
    import paper_2605_15418_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.load_library()
    return pkg


@pytest.fixture(scope="module")
def full():
    system, cfg, maps = W.asphere_hologram()
    return system, cfg, maps


def _sample_rays(cfg, alive_mask, pair, k):
    """k alive rays of one pair, spread over the launch grid (seeded)."""
    R2 = cfg["rays_side"] ** 2
    ids = np.nonzero(alive_mask[pair * R2:(pair + 1) * R2])[0]
    rng = np.random.default_rng(1000 + pair)
    return np.sort(rng.choice(ids, size=min(k, ids.size), replace=False))


def _oracle_pair(system, cfg, maps, pair, subset):
    F = len(cfg["fields"])
    tmap = O.transmission(torch.tensor(maps["phase"].astype(np.float64)),
                          torch.tensor(maps["amp"].astype(np.float64)))
    with torch.no_grad():
        return O.pair_forward(system, cfg, tmap, pair // F, pair % F,
                              torch.tensor(oracle_param_values(system)), keep=True,
                              ray_subset=subset)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_full_size_sampled_rays(rw, full, precision):
    system, cfg, maps = full
    plan = rw.Plan(system, cfg, precision=precision, batched=True)
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    psf, loss, idx = plan.forward(vals, ph, am, target=tg, want_idx=True)
    hits = plan.doe_hits()
    torch.cuda.synchronize()
    assert torch.isfinite(psf).all() and np.isfinite(float(loss))
    R2 = cfg["rays_side"] ** 2
    N = cfg["n_ssr"]
    alive = (hits[:, 7] != 0).cpu().numpy()
    equal, total = 0, 0
    for pair in SAMPLE_PAIRS:
        subset = _sample_rays(cfg, alive, pair, RAYS_PER_PAIR)
        ref = _oracle_pair(system, cfg, maps, pair, subset)
        gid = torch.as_tensor(pair * R2 + subset, device="cuda")
        h = hits[gid].cpu().numpy()
        a = ref["alive"].numpy()
        assert np.array_equal(h[:, 7] != 0, a), pair
        assert np.max(np.abs(h[a, 0:3] - ref["p_doe"].numpy()[a])) < 1e-11
        assert np.max(np.abs(h[a, 3:6] - ref["d_doe"].numpy()[a])) < 1e-13
        assert np.max(np.abs(h[a, 6] - ref["opl_doe"].numpy()[a])) < 1e-11
        gi = idx.view(-1, R2, N)[pair][torch.as_tensor(subset, device="cuda")].cpu().numpy()
        J = ref["J"]
        assert gi.shape == J.shape == (len(subset), N)
        if precision == "fp64":
            assert np.array_equal(gi, J), pair
        equal += int((gi == J).sum())
        total += J.size
    assert equal / total >= 0.97, equal / total


def test_full_size_mixed_against_fp64_form(rw, full):
    """The whole PSF and every gradient at full size: MIXED against the FP64
    form on the FP64 form's own draws replayed (the form is checked against the
    oracle on smaller cases).  Bars: PSF 1e-4 relative L2 per pair, gradients
    1e-3 per group (dphi, dA, dlens)."""
    system, cfg, maps = full
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    p64 = rw.Plan(system, cfg, precision="fp64", batched=True)
    psf64, _, idx = p64.forward(vals, ph, am, target=tg, want_idx=True)
    g64 = [g.double() for g in p64.backward()]
    psf64 = psf64.double()
    del p64
    plan = rw.Plan(system, cfg, precision="mixed", batched=True)
    psf, loss, _ = plan.forward(vals, ph, am, target=tg, replay=idx)
    g = [x.double() for x in plan.backward()]
    torch.cuda.synchronize()
    assert np.isfinite(float(loss))
    d = ((psf.double() - psf64).flatten(2).norm(dim=2) / psf64.flatten(2).norm(dim=2)).max()
    assert float(d) < 1e-4, float(d)
    for name, a, b in zip(("phase", "amp", "lens"), g, g64):
        e = float((a - b).norm() / b.norm())
        assert e < 1e-3, (name, e)
