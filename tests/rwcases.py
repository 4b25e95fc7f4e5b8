"""Shared helpers of the GPU parity tests: small seeded workloads that span
several tiles and ragged tails, and the oracle runs they are compared with."""
import numpy as np
import torch

import workloads as W
from oracle import rw_oracle as O


def small_singlet(sampling="mag", rays=16, P=16, N=64, Q=32, seed=0):
    """Singlet + zone plate (the FP64 workload) at test size."""
    return W.singlet_zoneplate(rays_side=rays, H=128, pitch=0.008, P=P, N=N, Q=Q,
                               psf_pitch=0.004, sampling=sampling, seed=seed)


def small_hologram(sampling="full", rays=8, P=16, N=32, Q=32, n_lambda=3, n_field_side=3,
                   H=256, pitch=0.002, seed=0):
    """Asphere singlet + random complex hologram at test size (all 27 pairs)."""
    s, c, m = W.asphere_hologram(rays_side=rays, H=H, pitch=pitch, P=P, N=N, Q=Q,
                                 psf_pitch=0.004, n_lambda=n_lambda,
                                 n_field_side=n_field_side, sampling=sampling, seed=seed)
    return s, c, m


def oracle_psf(system, cfg, maps, values=None, replays=None, keep=False):
    with torch.no_grad():
        return O.psf_stack(system, cfg, maps["phase"].astype(np.float64),
                           maps["amp"].astype(np.float64), values=values, replays=replays,
                           keep=keep)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def worst_pair_rel(a, b):
    L, F = b.shape[:2]
    return max(rel_l2(a[l, f], b[l, f]) for l in range(L) for f in range(F))


def gpu_inputs(system, maps, device="cuda"):
    vals = torch.tensor(O.initial_param_values(system), dtype=torch.float32, device=device)
    ph = torch.tensor(maps["phase"], device=device)
    am = torch.tensor(maps["amp"], device=device)
    return vals, ph, am


def oracle_param_values(system):
    """The lens parameters as the GPU sees them (rounded to float32)."""
    return O.initial_param_values(system).astype(np.float32).astype(np.float64)


def elementwise_rel(a, b):
    """max |a - b| / max |b|: the worst element against the scale of the reference."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def check_draws_valid(gi, J, spectrum, prop, u, sampling="mag", tol=1e-5):
    """Own draws of a form whose spectrum carries rounding: every index that
    differs from the oracle's must be a CDF edge flip, i.e. the oracle's
    threshold u S lies within tol S of the edge between the two bins (the
    oracle's inclusive CDF at the lower bin), and every bin strictly between
    them has zero weight.  gi, J, u: [rays, N]; spectrum, prop: [rays, M, M]
    in the oracle's (j_y, j_x) shifted layout.  Returns the agreeing fraction."""
    R = J.shape[0]
    mag = spectrum.abs().transpose(1, 2).reshape(R, -1).numpy()
    pr = prop.transpose(1, 2).reshape(R, -1).numpy()
    w = np.where(pr, mag if sampling == "mag" else 1.0, 0.0)
    cdf = np.cumsum(w, axis=1)
    for r, i in zip(*np.nonzero(gi != J)):
        lo, hi = sorted((int(gi[r, i]), int(J[r, i])))
        assert lo >= 0, (r, i, lo, hi)
        assert np.all(w[r, lo + 1:hi] == 0), (r, i, lo, hi)
        S = cdf[r, -1]
        assert abs(u[r, i] * S - cdf[r, lo]) <= tol * S, (r, i, u[r, i] * S, cdf[r, lo], S)
    return float((gi == J).mean())
