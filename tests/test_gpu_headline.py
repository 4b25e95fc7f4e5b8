"""The GPU path against the FP64 oracle at the transform and grid sizes of the
throughput workload: the asphere + 1024^2 random hologram system with P = 64
(M = 128), N = 256 draws per ray, Q = 512 (a 1024^2 fine grid of 64 super-bins
per pair and the second sort pass's work list), all 27 (wavelength, field)
pairs in one batched launch, on a 32 x 32 ray grid per pair so that the
oracle finishes in about a minute.  Four pairs are compared, among them both
+-10 degree corners: PSF (Eq. 2) and the G1 gradient of the Eq. 5 loss with
respect to the phase map, the amplitude map and the six lens parameters, by
relative L2 and element by element.

Bars: MIXED on the oracle's draws replayed: PSF 1e-4, gradients 1e-3; its own
draws agree on >= 97% and every disagreement is an FP32 CDF edge flip.
FP64 own draws: indices equal, PSF 1e-6, gradients 1e-5.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import philox
from oracle import rw_oracle as O
from rwcases import check_draws_valid, elementwise_rel, gpu_inputs, oracle_param_values, rel_l2

pytestmark = pytest.mark.gpu

PAIRS = (0, 11, 13, 26)        # (F, -10/-10 deg), (d, +10/-10), (d, on axis), (C, +10/+10)
RAYS = 32


@pytest.fixture(scope="module")
def rw():
    import paper_2605_15418_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.load_library()
    return pkg


@pytest.fixture(scope="module")
def case():
    system, cfg, maps = W.asphere_hologram(rays_side=RAYS)
    assert (cfg["patch_p"], cfg["n_ssr"], cfg["psf_q"], system["doe"]["H"]) == (64, 256, 512, 1024)
    return system, cfg, maps


@pytest.fixture(scope="module")
def oracle(case):
    """Oracle PSF, draws, spectra and the gradient of sum_p <G_p, I_p> with G_p
    the Eq. 5 cogradient 2 a (a I_p - T_p) at the oracle's PSF (a = <I,T>/<I,I>):
    the gradient of the Eq. 5 loss over the compared pairs."""
    system, cfg, maps = case
    F = len(cfg["fields"])
    ph = torch.tensor(maps["phase"].astype(np.float64), requires_grad=True)
    am = torch.tensor(maps["amp"].astype(np.float64), requires_grad=True)
    v = torch.tensor(oracle_param_values(system), requires_grad=True)
    out = {}
    for pr in PAIRS:
        r = O.pair_forward(system, cfg, O.transmission(ph, am), pr // F, pr % F, v, keep=True)
        I = r["psf"]
        T = torch.tensor(maps["target"][pr // F, pr % F].astype(np.float64))
        In = I.detach()
        a = float((In * T).sum() / (In * In).sum())
        G = 2 * a * (a * In - T)
        (G * I).sum().backward()
        out[pr] = dict(psf=In.numpy(), J=r["J"], G=G.numpy(), spectrum=r["spectrum"],
                       prop=r["prop"])
    return out, dict(phase=ph.grad.numpy(), amp=am.grad.numpy(), lens=v.grad.numpy())


def _gpu(rw, case, orc, precision, replay_oracle):
    system, cfg, maps = case
    per_pair, _ = orc
    plan = rw.Plan(system, cfg, precision=precision, batched=True)
    vals, ph, am = gpu_inputs(system, maps)
    _, _, idx = plan.forward(vals, ph, am, want_idx=True)
    rep = None
    if replay_oracle:
        rep = idx.clone()
        for pr in PAIRS:
            rep[pr] = torch.tensor(per_pair[pr]["J"], dtype=torch.int32, device="cuda")
    psf, _, idx2 = plan.forward(vals, ph, am, replay=rep, want_idx=True)
    G = torch.zeros_like(psf)
    L, F = psf.shape[:2]
    for pr in PAIRS:
        G[pr // F, pr % F] = torch.tensor(per_pair[pr]["G"], dtype=torch.float32, device="cuda")
    dp, da, dl = plan.backward(G)
    torch.cuda.synchronize()
    return (psf.cpu().numpy(), idx2.cpu().numpy(),
            dict(phase=dp.cpu().numpy(), amp=da.cpu().numpy(), lens=dl.cpu().numpy()))


def _compare(case, orc, psf, grads, tol_psf, tol_g):
    system, cfg, maps = case
    per_pair, gref = orc
    F = len(cfg["fields"])
    report = {}
    for pr in PAIRS:
        a, b = psf[pr // F, pr % F], per_pair[pr]["psf"]
        report[f"psf{pr}"] = (rel_l2(a, b), elementwise_rel(a, b))
    for k in ("phase", "amp", "lens"):
        report[k] = (rel_l2(grads[k], gref[k]), elementwise_rel(grads[k], gref[k]))
    print(report)
    for name, (l2, el) in report.items():
        tol = tol_psf if name.startswith("psf") else tol_g
        assert l2 < tol and el < tol, (name, l2, el)


def test_headline_mixed_on_oracle_draws(rw, case, oracle):
    psf, _, grads = _gpu(rw, case, oracle, "mixed", replay_oracle=True)
    _compare(case, oracle, psf, grads, 1e-4, 1e-3)


def test_headline_fp64_own_draws(rw, case, oracle):
    psf, idx, grads = _gpu(rw, case, oracle, "fp64", replay_oracle=False)
    for pr in PAIRS:
        assert np.array_equal(idx[pr], oracle[0][pr]["J"]), pr
    _compare(case, oracle, psf, grads, 1e-6, 1e-5)


def test_headline_mixed_own_draws_are_valid(rw, case, oracle):
    system, cfg, maps = case
    plan = rw.Plan(system, cfg, precision="mixed", batched=True)
    vals, ph, am = gpu_inputs(system, maps)
    _, _, idx = plan.forward(vals, ph, am, want_idx=True)
    gi = idx.cpu().numpy()
    agree = []
    for pr in PAIRS:
        o = oracle[0][pr]
        u = philox.draw_uniforms(cfg["seed"], pr, np.arange(RAYS * RAYS), cfg["n_ssr"])
        agree.append(check_draws_valid(gi[pr], o["J"], o["spectrum"], o["prop"], u))
    assert min(agree) >= 0.97, agree
