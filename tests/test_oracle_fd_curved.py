"""Finite-difference pin of the oracle's gradient on the shape of the end-to-end
design workload: two even-asphere lenses with the DOE on the rear asphere of
the second (a curved DOE whose surface carries lens parameters), two patch
classes by the Eq. 4 rule, and 14 normalised lens parameters (4 curvatures,
4 A4, 4 A6, 2 centre thicknesses).  Central differences (h = 1e-4, FP64)
against torch autograd of Eq. 5, in FULL mode and with frozen draws.  The step
is h = 1e-5: near-grazing secondaries (|K| close to k_out) make the loss a
square-root function of the geometry there, which h = 1e-4 resolves poorly
on the first lens's curvature (16% off; 1e-5 and 1e-6 agree to 1e-6)."""
import numpy as np
import pytest

import workloads as W
from oracle import rw_oracle as O


@pytest.mark.parametrize("sampling", ["full", "mag"])
def test_curved_doe_lens_gradient_matches_central_differences(sampling):
    system, cfg, maps = W.two_lens_hybrid(rays_side=4, H=128, pitch=0.008, P=8, classes=(4,),
                                          N=16, Q=16, psf_pitch=0.004, n_lambda=1,
                                          n_field_side=1, sampling=sampling)
    assert len(system["params"]) == 14 and system["surfaces"][3]["doe"]
    vals = O.initial_param_values(system)
    phase = maps["phase"].astype(np.float64)
    amp = maps["amp"].astype(np.float64)
    target = maps["target"].astype(np.float64)
    L0, g, psf, idx = O.loss_and_grad(system, cfg, phase, amp, vals, target)
    assert np.abs(g["lens"]).max() > 0
    replays = None if sampling == "full" else idx
    h = 1e-5

    def loss(v):
        return O.loss_and_grad(system, cfg, phase, amp, v, target, replays=replays,
                               want_grad=False)[0]

    scale = np.abs(g["lens"]).max()
    for k in range(len(vals)):
        vp, vm = vals.copy(), vals.copy()
        vp[k] += h
        vm[k] -= h
        fd = (loss(vp) - loss(vm)) / (2 * h)
        assert abs(fd - g["lens"][k]) <= 1e-5 * scale + 1e-4 * abs(fd), (k, fd, g["lens"][k])
