"""Philox4x32-10 counter-based generator for the oracle (test infrastructure only).

Written from the published definition (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11, Sec. 3.2): a 4x32-bit counter is
mixed by ten rounds of two 32x32->64 multiplies whose high and low halves are
xor-ed with the other counter words and a 2x32-bit key that is bumped by the
Weyl constants between rounds.

The Monte Carlo draws of the ray-wave method (secondary wavevectors sampled
from p(k_u, k_v), Eq. 1 and Fig. 1c of the paper) take their uniforms from
this stream, so that the CPU oracle and the GPU path see the same numbers.
Counter layout of one draw:   (i >> 2, ray-in-pair, pair, stream), lane i & 3.
Uniform of a 32-bit word x:   u = ((x >> 9) + 0.5) * 2**-23, exact in fp32/fp64.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_LO = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: uint32 array [..., 4]; key: (k0, k1). Returns uint32 [..., 4]."""
    c = np.asarray(ctr, dtype=np.uint32)
    c0, c1, c2, c3 = (c[..., i].astype(np.uint64) for i in range(4))
    k0 = np.uint32(key[0])
    k1 = np.uint32(key[1])
    for rnd in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _LO
        hi1, lo1 = p1 >> np.uint64(32), p1 & _LO
        n0 = hi1 ^ c1 ^ np.uint64(k0)
        n2 = hi0 ^ c3 ^ np.uint64(k1)
        c0, c1, c2, c3 = n0, lo1, n2, lo0
        if rnd != 9:
            k0 = np.uint32((int(k0) + int(_W0)) & 0xFFFFFFFF)
            k1 = np.uint32((int(k1) + int(_W1)) & 0xFFFFFFFF)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def seed_key(seed):
    seed = int(seed)
    return (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def word_to_uniform(x):
    """32-bit word -> uniform in (0, 1) with 23 random bits (exact in fp32)."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(9)).astype(np.float64) + 0.5) * (2.0 ** -23)


def draw_uniforms(seed, pair, ray_ids, n_draws, stream=0):
    """Uniforms u[r, i] for draws i of the rays ray_ids of one (wavelength, field) pair."""
    key = seed_key(seed)
    nblk = (n_draws + 3) // 4
    r = np.asarray(ray_ids, dtype=np.uint32)
    b = np.arange(nblk, dtype=np.uint32)
    ctr = np.zeros((r.shape[0], nblk, 4), dtype=np.uint32)
    ctr[..., 0] = b[None, :]
    ctr[..., 1] = r[:, None]
    ctr[..., 2] = np.uint32(pair)
    ctr[..., 3] = np.uint32(stream)
    out = philox4x32_10(ctr, key).reshape(r.shape[0], nblk * 4)[:, :n_draws]
    return word_to_uniform(out)


# Streams of the Gumbel-softmax straight-through estimator (G2).  Per draw i of
# a ray, the largest perturbed log-probability G*_i takes its uniform from
# counter (i >> 2, ray, pair, 2), word i & 3; the unconditioned Gumbel of bin k
# from counter (k, ray, pair, 0x10000 | (i >> 2)), word i & 3.
STREAM_G2_TOP = 2
STREAM_G2_BIN = 0x10000


def g2_top_uniforms(seed, pair, ray_ids, n_draws):
    """Uniforms u*[r, i] of the top Gumbel of every draw."""
    return draw_uniforms(seed, pair, ray_ids, n_draws, stream=STREAM_G2_TOP)


def g2_bin_uniforms(seed, pair, ray_ids, n_draws, n_bins):
    """Uniforms u[r, i, k] of the per-bin Gumbels of every draw."""
    key = seed_key(seed)
    nblk = (n_draws + 3) // 4
    r = np.asarray(ray_ids, dtype=np.uint32)
    k = np.arange(n_bins, dtype=np.uint32)
    b = np.arange(nblk, dtype=np.uint32)
    ctr = np.zeros((r.shape[0], n_bins, nblk, 4), dtype=np.uint32)
    ctr[..., 0] = k[None, :, None]
    ctr[..., 1] = r[:, None, None]
    ctr[..., 2] = np.uint32(pair)
    ctr[..., 3] = np.uint32(STREAM_G2_BIN) | b[None, None, :]
    out = philox4x32_10(ctr, key).reshape(r.shape[0], n_bins, nblk * 4)[:, :, :n_draws]
    return word_to_uniform(out).transpose(0, 2, 1)
