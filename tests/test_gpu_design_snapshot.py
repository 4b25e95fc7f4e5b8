"""The end-to-end design workload (two even-asphere lenses, 4096^2 complex DOE
at 0.5 um on the second lens's rear asphere, 128 (wavelength, field) pairs,
patch classes 128 / 64 zero-padded to M = 256 / 128, N = 256, Q = 1024) on a
16 x 16 ray grid per pair, in one batched launch, against the FP64 oracle on
two pairs (the shortest wavelength at a +-25 degree corner, and a central
pair): PSF and the G1 gradient of the Eq. 5 loss over those pairs w.r.t. the
phase and amplitude maps and the 14 lens parameters, MIXED on the oracle's
draws.  Bars: PSF 1e-4, gradients 1e-3, relative L2 and element-wise."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import rw_oracle as O
from rwcases import elementwise_rel, gpu_inputs, oracle_param_values, rel_l2

pytestmark = pytest.mark.gpu

RAYS = 16


@pytest.fixture(scope="module")
def rw():
    import paper_2605_15418_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.load_library()
    return pkg


def test_design_snapshot_mixed_against_oracle(rw):
    system, cfg, maps = W.two_lens_hybrid(rays_side=RAYS)
    F = len(cfg["fields"])
    pairs = (0, 4 * F + 6)               # (400 nm, -25/-25 deg), (571 nm, -8/+8 deg)
    ph = torch.tensor(maps["phase"].astype(np.float64), requires_grad=True)
    am = torch.tensor(maps["amp"].astype(np.float64), requires_grad=True)
    v = torch.tensor(oracle_param_values(system), requires_grad=True)
    ref = {}
    classes = set()
    for pr in pairs:
        r = O.pair_forward(system, cfg, O.transmission(ph, am), pr // F, pr % F, v, keep=True)
        I = r["psf"]
        T = torch.tensor(maps["target"][pr // F, pr % F].astype(np.float64))
        In = I.detach()
        a = float((In * T).sum() / (In * In).sum())
        G = 2 * a * (a * In - T)
        (G * I).sum().backward()
        ref[pr] = (In.numpy(), r["J"], G.numpy())
        classes |= set(r["sides"].tolist())
    assert classes == {128, 64}, classes
    plan = rw.Plan(system, cfg, precision="mixed", batched=True)
    vals, gph, gam = gpu_inputs(system, maps)
    _, _, idx = plan.forward(vals, gph, gam, want_idx=True)
    rep = idx.clone()
    for pr in pairs:
        rep[pr] = torch.tensor(ref[pr][1], dtype=torch.int32, device="cuda")
    psf, _, _ = plan.forward(vals, gph, gam, replay=rep)
    Gt = torch.zeros_like(psf)
    for pr in pairs:
        Gt[pr // F, pr % F] = torch.tensor(ref[pr][2], dtype=torch.float32, device="cuda")
    dp, da, dl = plan.backward(Gt)
    torch.cuda.synchronize()
    psf = psf.cpu().numpy()
    report = {}
    for pr in pairs:
        a, b = psf[pr // F, pr % F], ref[pr][0]
        report[f"psf{pr}"] = (rel_l2(a, b), elementwise_rel(a, b))
    for name, got, want in (("phase", dp, ph.grad), ("amp", da, am.grad), ("lens", dl, v.grad)):
        g, w = got.cpu().numpy(), want.numpy()
        report[name] = (rel_l2(g, w), elementwise_rel(g, w))
    print(report)
    for name, (l2, el) in report.items():
        tol = 1e-4 if name.startswith("psf") else 1e-3
        assert l2 < tol and el < tol, (name, l2, el)
