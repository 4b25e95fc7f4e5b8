"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms (lensmaker focus, grating equation,
zone-plate focal length, Parseval, Airy zero), brute-force sums on tiny
inputs, an independent angular-spectrum propagation, the paper's printed
numbers, and finite differences.  None of these needs a GPU.
"""
import math
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import philox
from oracle import rw_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
torch.set_num_threads(min(8, os.cpu_count() or 1))


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- RNG -------
def test_philox_known_answers():
    for row in _golden("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in row]
        out = philox.philox4x32_10(np.array(v[:4], dtype=np.uint32), (v[4], v[5]))
        assert [int(o) for o in out] == v[6:10]


def test_uniform_mapping_exact_and_open():
    u = philox.word_to_uniform(np.array([0, 0xFFFFFFFF, 0x80000000], dtype=np.uint32))
    assert u[0] == 2.0 ** -24 and u[1] == 1 - 2.0 ** -24 and u[2] == 0.5 + 2.0 ** -24
    assert np.all(np.float32(u) == u)       # exactly representable in fp32


# ---------------------------------------------------------------- trace -----
def _sphere(z, R, medium=W.BK7):
    return O.build_surfaces({"surfaces": [W.surface(z, c=1 / R, semi_ap=0, medium=medium)],
                             "sensor_z": z + 10, "params": []})[0][0]


def test_newton_matches_sphere_closed_form():
    rng = np.random.default_rng(1)
    R, zv = 37.0, 2.0
    surf = _sphere(zv, R)
    n = 200
    p = torch.tensor(np.c_[rng.uniform(-4, 4, (n, 2)), np.full(n, -3.0)])
    d = torch.tensor(np.c_[rng.uniform(-0.2, 0.2, (n, 2)), np.ones(n)])
    d = d / d.norm(dim=1, keepdim=True)
    t, ok = O.intersect(surf, p, d)
    assert bool(ok.all())
    # closed form: |p + t d - C|^2 = R^2 with centre C = (0, 0, zv + R), near root
    C = torch.tensor([0.0, 0.0, zv + R], dtype=torch.float64)
    w = p - C
    b = (w * d).sum(1)
    cc = (w * w).sum(1) - R * R
    t_cf = -b - torch.sqrt(b * b - cc)
    assert torch.max(torch.abs(t - t_cf)).item() < 1e-12


def test_snell_invariants():
    rng = np.random.default_rng(2)
    n = 500
    d = torch.tensor(np.c_[rng.uniform(-0.5, 0.5, (n, 2)), np.ones(n)])
    d = d / d.norm(dim=1, keepdim=True)
    N = torch.tensor(np.c_[rng.uniform(-0.3, 0.3, (n, 2)), np.ones(n)])
    N = N / N.norm(dim=1, keepdim=True)
    n1, n2 = 1.0, 1.5168
    dn, ok = O.refract(d, N, n1, n2)
    assert bool(ok.all())
    assert torch.max(torch.abs(dn.norm(dim=1) - 1)).item() < 1e-14
    # tangential momentum: n1 d x N = n2 d' x N
    lhs = n1 * torch.cross(d, N, dim=1)
    rhs = n2 * torch.cross(dn, N, dim=1)
    assert torch.max(torch.abs(lhs - rhs)).item() < 1e-14
    # total internal reflection from glass at grazing incidence is flagged
    dg = torch.tensor([[0.9, 0.0, math.sqrt(1 - 0.81)]], dtype=torch.float64)
    _, ok = O.refract(dg, torch.tensor([[0.0, 0.0, 1.0]], dtype=torch.float64), 1.5168, 1.0)
    assert not bool(ok.any())


def test_singlet_paraxial_focus_matches_lensmaker():
    """Thick-lens focus of the R1 = +50, R2 = -50, CT 5 BK7 singlet
    (lensmaker + principal planes, a textbook closed form, not the tracer)."""
    n = 1.5168
    R1, R2, t = 50.0, -50.0, 5.0
    P = (n - 1) * (1 / R1 - 1 / R2 + (n - 1) * t / (n * R1 * R2))
    efl = 1 / P
    bfl = efl * (1 - (n - 1) * t / (n * R1))
    assert abs(efl - 49.213) < 1e-3 and abs(bfl - 47.536) < 1e-3
    glass = (n, 0.0)       # dispersion-free so that n is exactly 1.5168
    system = {"surfaces": [W.surface(0, c=1 / R1, medium=glass),
                           W.surface(5, c=1 / R2, medium=W.AIR),
                           W.surface(200.0, doe=True)],
              "sensor_z": 300.0, "params": []}
    surfs, _ = O.build_surfaces(system)
    h = torch.tensor([1e-3, 2e-3, 4e-3], dtype=torch.float64)
    p = torch.stack([h, torch.zeros(3), -torch.ones(3)], 1)
    d = torch.tensor([[0.0, 0.0, 1.0]] * 3, dtype=torch.float64)
    p, d, opl, alive, _ = O.trace_to_doe(surfs, 587.6e-6, p, d, torch.zeros(3, dtype=torch.float64))
    z_cross = p[:, 2] - p[:, 0] * d[:, 2] / d[:, 0]      # where each ray meets the axis
    assert torch.max(torch.abs(z_cross - (5 + bfl))).item() < 1e-4
    # spherical aberration grows as h^2 (longitudinal), sign fixed: marginal focus shorter
    lsa = (5 + bfl) - z_cross
    assert lsa[2] > lsa[1] > lsa[0] > 0
    assert abs(lsa[2] / lsa[1] - 4) < 0.05


# --------------------------------------------------------- angular spectrum ---
def test_spectrum_equals_bruteforce_dft():
    rng = np.random.default_rng(3)
    for P, M in ((4, 8), (5, 10), (6, 12)):
        U = torch.tensor(rng.normal(size=(2, P, P)) + 1j * rng.normal(size=(2, P, P)))
        a = O.angular_spectrum(U, M).numpy()
        b = O.angular_spectrum_bruteforce(U, M)
        assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


def test_spectrum_parseval():
    rng = np.random.default_rng(4)
    P, M = 16, 32
    U = torch.tensor(rng.normal(size=(3, P, P)) + 1j * rng.normal(size=(3, P, P)))
    S = O.angular_spectrum(U, M)
    e1 = (U.abs() ** 2).sum((1, 2))
    e2 = (S.abs() ** 2).sum((1, 2)) / M ** 2
    assert torch.max(torch.abs(e1 - e2) / e1).item() < 1e-13


def test_phase_only_patch_energy_conserved_full_mode():
    """Phase-only DOE, every bin propagating: FULL-mode secondary energy
    M^2 sum |w_j|^2 equals the patch energy (Parseval across the ASM step)."""
    rng = np.random.default_rng(5)
    H = 64
    phase = rng.uniform(0, 2 * np.pi, (H, H))
    system, cfg, maps = W.free_space_doe(phase, np.ones((H, H)), 0.002, 5.0, 0.5e-3, 1, 16, 4,
                                         0.002, sampling="full")
    tm = O.transmission(torch.tensor(phase), torch.ones(H, H, dtype=torch.float64))
    r = O.pair_forward(system, cfg, tm, 0, 0, keep=True)
    assert bool(r["prop"].all())
    M = 32
    # w carries U~/M^2 for every bin; energy of the field the secondaries represent
    e_sec = (r["w"].abs() ** 2).sum().item() * M * M
    P = 16
    pitch = 0.002
    pch = O.patch_field(tm, system["doe"], r["p_doe"], r["frame"][0], r["frame"][1], P)
    e_patch = (pch.abs() ** 2).sum().item()
    assert abs(e_sec - e_patch) < 1e-12 * e_patch


# ------------------------------------------------ Eq. 2 == angular spectrum ----
def test_eq2_full_mode_equals_asm_propagation():
    """One incident ray, free space, FULL mode, sensor grid = padded patch
    grid: the Eq. 2 wavelet sum equals ASM propagation with obliquity,
    IFFT(FFT(u) (k_z/k) exp(i k_z z)), computed here with numpy.fft."""
    rng = np.random.default_rng(6)
    H, P, M = 48, 16, 32
    pitch, lam, dz = 0.002, 0.6e-3, 0.4
    phase = 2 * np.pi * W.bandlimited_uniform(H, H, 0.2, rng)
    amp = 0.5 + 0.5 * W.bandlimited_uniform(H, H, 0.2, rng)
    system, cfg, maps = W.free_space_doe(phase, amp, pitch, dz, lam, 1, P, M, pitch,
                                         sampling="full")
    # single ray at the DOE centre (a pixel corner): patch samples at pixel centres
    cfg["launch_center"] = [[0.0, 0.0]]
    # sensor grid point m sits at the padded-grid sample g = m mod M
    cfg["psf_center"] = [[[-(P - 1) / 2 * pitch, -(P - 1) / 2 * pitch]]]
    tm = O.transmission(torch.tensor(phase), torch.tensor(amp))
    r = O.pair_forward(system, cfg, tm, 0, 0, keep=True)
    U = r["U"].numpy()
    u = O.patch_field(tm, system["doe"], r["p_doe"], r["frame"][0], r["frame"][1], P)[0].numpy()
    k0 = 2 * np.pi / lam
    kap = 2 * np.pi * np.fft.fftfreq(M, pitch)
    KX, KY = np.meshgrid(kap, kap)
    kz2 = k0 ** 2 - KX ** 2 - KY ** 2
    kz = np.sqrt(np.maximum(kz2, 0))
    H_asm = np.where(kz2 > 0, (kz / k0) * np.exp(1j * kz * dz), 0)
    up = np.zeros((M, M), complex)
    up[:P, :P] = u
    ref = np.fft.ifft2(np.fft.fft2(up) * H_asm)       # ref[g_y, g_x]
    g = np.arange(M) - M // 2
    ref_on_sensor = ref[np.ix_(np.mod(g, M), np.mod(g, M))]
    # the ray arrives with OPL 0 at z = 0 (launch plane z = -1, OPL_0 = -1)
    err = np.linalg.norm(U - ref_on_sensor) / np.linalg.norm(ref_on_sensor)
    assert err < 1e-12


def test_eq2_matches_bruteforce_huygens_sum():
    """Tiny patch: Eq. 2 (FULL mode) against a brute-force Huygens sum over
    the patch samples.  Eq. 2 weights every plane wave by <n, d> = k_z / k,
    i.e. it propagates (1 / ik) dU/dz; the point-source kernel with that
    angular spectrum is -(1 / (2 pi i k)) d^2/dz^2 (exp(ikR) / R)."""
    lam = 0.5e-3
    pitch = lam / 4
    P, M = 16, 2048
    dz = 0.03
    H = 32
    phase = np.zeros((H, H))
    system, cfg, maps = W.free_space_doe(phase, np.ones((H, H)), pitch, dz, lam, 1, P, 16,
                                         0.001, pad=M // P, sampling="full")
    cfg["launch_center"] = [[0.0, 0.0]]
    tm = O.transmission(torch.tensor(phase), torch.ones(H, H, dtype=torch.float64))
    with torch.no_grad():
        U = O.pair_forward(system, cfg, tm, 0, 0)["U"].numpy()
    k = 2 * np.pi / lam
    s = (np.arange(P) - (P - 1) / 2) * pitch
    sx, sy = np.meshgrid(s, s)
    xs = (np.arange(16) - 8) * 0.001
    X, Y = np.meshgrid(xs, xs)
    R = np.sqrt((X[..., None, None] - sx) ** 2 + (Y[..., None, None] - sy) ** 2 + dz ** 2)
    e = np.exp(1j * k * R)
    f1 = e * (1j * k / R - 1 / R ** 2)
    f2 = e * (-k * k / R - 2j * k / R ** 2 + 2 / R ** 3)
    d2 = f2 * dz ** 2 / R ** 2 + f1 * (1 / R - dz ** 2 / R ** 3)
    Uh = (-(1 / (2j * np.pi * k)) * d2).sum((-1, -2)) * pitch ** 2
    err = np.linalg.norm(U - Uh) / np.linalg.norm(Uh)
    assert err < 1e-2, err


# ------------------------------------------------------------ grating --------
@pytest.mark.parametrize("theta_deg", [0.0, 7.0])
def test_grating_equation(theta_deg):
    """Linear-phase grating phi = 2 pi x / Lg with Lg = M pitch / j0: the
    strongest bin is j0 and the emitted direction obeys the grating equation
    sin(theta_out) = sin(theta_in) + lam / Lg; the FULL-mode PSF centroid in
    free space lands at z tan(theta_out)."""
    P, M, j0 = 16, 32, 5
    pitch, lam, dz = 0.002, 0.55e-3, 1.0
    Lg = M * pitch / j0
    H = 128
    x = (np.arange(H) - (H - 1) / 2) * pitch
    phase = np.mod(2 * np.pi * x[None, :] / Lg, 2 * np.pi) * np.ones((H, 1))
    tan_in = math.tan(math.radians(theta_deg))
    sin_in = tan_in / math.sqrt(1 + tan_in ** 2)
    sin_out = sin_in + lam / Lg
    tan_out = sin_out / math.sqrt(1 - sin_out ** 2)
    Q, sp = 64, 0.004
    system, cfg, maps = W.free_space_doe(phase, np.ones((H, H)), pitch, dz, lam, 8, P, Q, sp,
                                         sampling="full", field=(tan_in, 0.0),
                                         launch_half=0.05, psf_center=(dz * tan_out, 0.0))
    cfg["launch_center"] = [[0.0, 0.0]]
    tm = O.transmission(torch.tensor(phase), torch.ones(H, H, dtype=torch.float64))
    r = O.pair_forward(system, cfg, tm, 0, 0, keep=True)
    spec = r["spectrum"][0].abs().numpy()
    jy, jx = np.unravel_index(np.argmax(spec), spec.shape)
    assert (jy - M // 2, jx - M // 2) == (0, j0)
    k0 = 2 * np.pi / lam
    kin = r["k_in_t"][0, 0].item()
    dx = (kin + 2 * np.pi * j0 / (M * pitch)) / k0
    assert abs(dx - sin_out) < 1e-12
    I = r["psf"].numpy()
    c = (np.arange(Q) - Q // 2) * sp
    cx = (I.sum(0) * c).sum() / I.sum()
    # the beam is centred on the launch centre (0) at the DOE: centroid offset
    # relative to dz tan(theta_out) stays within a pixel
    assert abs(cx) < sp


# ---------------------------------------------------------- zone plate -------
def _zp_center_intensity(lam, dz, f0=10.0, lam0=0.5e-3):
    H, pitch = 256, 0.004
    doe = W.doe_desc(H, H, pitch)
    phase = W.kinoform_zone_plate(doe, f0, lam0)
    system, cfg, maps = W.free_space_doe(phase, np.ones((H, H)), pitch, dz, lam, 8, 32, 2, 0.001,
                                         sampling="full", psf_center=(0.0005, 0.0005))
    tm = O.transmission(torch.tensor(phase), torch.ones(H, H, dtype=torch.float64))
    with torch.no_grad():
        r = O.pair_forward(system, cfg, tm, 0, 0)
    return r["psf"][1, 1].item()   # pixel (0, 0) at the optical axis


def test_zone_plate_focal_length_scales_with_wavelength():
    """Kinoform zone plate designed for f0 at lam0 focuses at f0 lam0 / lam.
    The finite-aperture focal shift (a fixed fraction of f at a fixed
    Fresnel number, which f0 lam0 / lam keeps constant) cancels in the ratio."""
    from scipy.optimize import minimize_scalar
    zs = {}
    for lam in (0.5e-3, 0.6e-3):
        f_expect = 10.0 * 0.5e-3 / lam
        res = minimize_scalar(lambda z: -_zp_center_intensity(lam, z),
                              bounds=(0.9 * f_expect, 1.1 * f_expect), method="bounded",
                              options={"xatol": 1e-4})
        dof = lam / (0.456 / f_expect) ** 2
        assert abs(res.x - f_expect) < 0.25 * dof, (lam, res.x, f_expect)
        zs[lam] = res.x
    assert abs(zs[0.5e-3] / zs[0.6e-3] - 0.6 / 0.5) < 2e-3, zs


# -------------------------------------------------------- Monte Carlo --------
def _one_ray_spectrum(seed=7, H=64, P=16):
    rng = np.random.default_rng(seed)
    phase = 2 * np.pi * W.bandlimited_uniform(H, H, 0.15, rng)
    system, cfg, maps = W.free_space_doe(phase, np.ones((H, H)), 0.002, 1.0, 0.5e-3, 1, P, 16,
                                         0.002, sampling="mag", N=64)
    return system, cfg, maps


def test_mag_weights_have_constant_modulus_and_sampler_chi2():
    system, cfg, maps = _one_ray_spectrum()
    N = 20000
    cfg["n_ssr"] = N
    tm = O.transmission(torch.tensor(maps["phase"], dtype=torch.float64),
                        torch.tensor(maps["amp"], dtype=torch.float64))
    r = O.pair_forward(system, cfg, tm, 0, 0, keep=True)
    M = 32
    # bins flattened in the sampler's order: j_x major
    mag = r["spectrum"][0].abs().transpose(0, 1).reshape(-1).numpy()
    prop = r["prop"][0].transpose(0, 1).reshape(-1).numpy()
    S = mag[prop].sum()
    w = r["w"].numpy()
    assert np.max(np.abs(np.abs(w) - S / (M * M * N))) < 1e-12 * S / (M * M * N)
    # chi-square goodness of fit on the bins holding 90% of the mass
    counts = np.bincount(r["J"][0], minlength=M * M)
    p = np.where(prop, mag, 0) / S
    order = np.argsort(-p)
    keep = order[: np.searchsorted(np.cumsum(p[order]), 0.9) + 1]
    exp_ = N * p[keep]
    obs = counts[keep]
    rest_e = N - exp_.sum()
    rest_o = N - obs.sum()
    chi2 = ((obs - exp_) ** 2 / exp_).sum() + (rest_o - rest_e) ** 2 / rest_e
    from scipy.stats import chi2 as C2
    assert C2.sf(chi2, len(keep)) > 1e-3


def test_inverse_cdf_equals_literal_gumbel_max_in_distribution():
    """Fig. 1c: replicate p N times, add Gumbel noise, take the max score.
    The oracle's inverse-CDF draws follow the same law (two-sample chi2)."""
    rng = np.random.default_rng(8)
    K = 12
    p = rng.uniform(0.1, 1.0, K)
    p /= p.sum()
    N = 40000
    u = philox.draw_uniforms(11, 0, [0], N)[0]
    J, _ = O.draw_bins(p[None, :], np.ones((1, K), bool), u[None, :], "mag")
    g = -np.log(-np.log(rng.uniform(size=(N, K))))
    Jg = np.argmax(np.log(p)[None, :] + g, axis=1)
    c1 = np.bincount(J[0], minlength=K)
    c2 = np.bincount(Jg, minlength=K)
    chi2 = ((c1 - c2) ** 2 / (c1 + c2)).sum()
    from scipy.stats import chi2 as C2
    assert C2.sf(chi2, K - 1) > 1e-3
    assert np.max(np.abs(c1 / N - p)) < 0.01


def test_mc_mean_converges_to_full_field_at_inverse_sqrt_n():
    system, cfg, maps = _one_ray_spectrum(seed=9)
    tm = O.transmission(torch.tensor(maps["phase"], dtype=torch.float64),
                        torch.tensor(maps["amp"], dtype=torch.float64))
    cfg_full = dict(cfg, sampling="full")
    with torch.no_grad():
        Uf = O.pair_forward(system, cfg_full, tm, 0, 0)["U"].numpy()
        errs = {}
        for N in (64, 1024):
            e = []
            for seed in range(12):
                c = dict(cfg, n_ssr=N, seed=seed)
                U = O.pair_forward(system, c, tm, 0, 0)["U"].numpy()
                e.append(np.linalg.norm(U - Uf) ** 2 / np.linalg.norm(Uf) ** 2)
            errs[N] = math.sqrt(np.mean(e))
    ratio = errs[64] / errs[1024]
    assert 2.5 < ratio < 6.5, errs     # sqrt(16) = 4


# ------------------------------------------------------- loss and metrics ----
def test_eq5_closed_form_alpha_is_optimal_and_envelope_gradient():
    rng = np.random.default_rng(10)
    I = torch.tensor(rng.uniform(size=(8, 8)), requires_grad=True)
    T = torch.tensor(rng.uniform(size=(8, 8)))
    from scipy.optimize import minimize_scalar
    f = lambda a: float(((a * I.detach() - T) ** 2).sum())
    a_num = minimize_scalar(f).x
    L = O.eq5_loss(I, T)
    assert abs(L.item() - f(a_num)) < 1e-10
    L.backward()
    a = (I * T).sum().item() / (I * I).sum().item()
    g_detached = 2 * a * (a * I.detach() - T)
    assert torch.max(torch.abs(I.grad - g_detached)).item() < 1e-12


def test_ncc_and_mse():
    rng = np.random.default_rng(12)
    I = rng.uniform(size=(10, 10))
    assert abs(O.ncc(I, I) - 1) < 1e-15
    assert abs(O.ncc(3.7 * I, I) - 1) < 1e-15
    assert O.ncc(I, rng.uniform(size=(10, 10))) < 1
    assert O.mse(I, I) == 0


def test_paper_printed_numbers():
    g = {row[0]: float(row[1]) for row in _golden("paper_numbers.txt")}
    lam = 1.0
    eps = O.curvature_error_bound(100 * lam, 506 * lam)
    assert round(eps, 4) == g["curvature_bound_rad"]
    assert eps <= g["curvature_threshold_rad"]
    assert O.largest_patch([50, 100, 150, 200], lam, 506 * lam, 0.1) == 100
    assert round(40 * 6.3) == g["patch_40px_um"] and round(100 * 6.3) == g["patch_100px_um"]
    # Airy first-zero diameter of the target generator: 1.22 lam / NA
    Q, pitch = 512, 0.01e-3
    I = W.airy_target(Q, pitch, 1e-3, 0.5, (0.0, 0.0), (0.0, 0.0))
    row = I[Q // 2, Q // 2:]
    r = np.arange(row.size) * pitch
    first_min = r[1 + np.argmax(np.diff(row) > 0)]         # first local minimum
    assert abs(2 * first_min * 1e3 - g["airy_diameter_um"]) <= 2 * pitch * 1e3 + 1e-9


# --------------------------------------------------------- gradients ---------
def _tiny_lens_system(sampling):
    system, cfg, maps = W.asphere_hologram(rays_side=4, H=48, pitch=0.004, P=8, N=16, Q=16,
                                           psf_pitch=0.004, n_lambda=1, n_field_side=1,
                                           sampling=sampling)
    cfg["fields"] = [[0.03, -0.02]]
    cfg["launch_center"] = [[-0.18, 0.12]]
    cfg["psf_center"] = [[[0.68, -0.45]]]
    return system, cfg, maps


@pytest.mark.parametrize("sampling", ["full", "mag"])
def test_autograd_gradient_matches_central_differences(sampling):
    system, cfg, maps = _tiny_lens_system(sampling)
    vals = O.initial_param_values(system)
    phase = maps["phase"].astype(np.float64)
    amp = maps["amp"].astype(np.float64)
    target = maps["target"].astype(np.float64)
    L0, g, psf, idx = O.loss_and_grad(system, cfg, phase, amp, vals, target)
    replays = None if sampling == "full" else idx
    h = 1e-4

    def loss(ph=phase, am=amp, v=vals):
        return O.loss_and_grad(system, cfg, ph, am, v, target, replays=replays,
                               want_grad=False)[0]

    for k in range(len(vals)):
        vp, vm = vals.copy(), vals.copy()
        vp[k] += h
        vm[k] -= h
        fd = (loss(v=vp) - loss(v=vm)) / (2 * h)
        assert abs(fd - g["lens"][k]) <= 1e-5 * max(1e-8, np.abs(g["lens"]).max()) + \
            2e-4 * abs(fd), (k, fd, g["lens"][k])
    rng = np.random.default_rng(0)
    iy, ix = np.unravel_index(np.argsort(-np.abs(g["phase"]).ravel())[:3], phase.shape)
    for y, x in list(zip(iy, ix)) + [tuple(rng.integers(10, 38, 2))]:
        for name, arr in (("phase", phase), ("amp", amp)):
            ap, am_ = arr.copy(), arr.copy()
            ap[y, x] += h
            am_[y, x] -= h
            if name == "phase":
                fd = (loss(ph=ap) - loss(ph=am_)) / (2 * h)
            else:
                fd = (loss(am=ap) - loss(am=am_)) / (2 * h)
            ref = g[name][y, x]
            assert abs(fd - ref) <= 1e-6 * np.abs(g[name]).max() + 1e-4 * abs(fd), \
                (name, y, x, fd, ref)


# ----------------------------------------------- G2 (straight-through) ------
def test_conditional_gumbels_have_argmax_j_and_iid_gumbel_marginals():
    """Top-down conditional Gumbels (Maddison, Tarlow & Minka 2014): with J drawn
    from p, (J, phi) has the law of (argmax, values) of log p plus iid Gumbel(0)
    noise, so every phi_k - log p_k is Gumbel(0) and the argmax is J."""
    from scipy import stats
    rng = np.random.default_rng(21)
    K, N = 10, 20000
    p = rng.uniform(0.05, 1.0, K)
    p /= p.sum()
    logp = np.log(p)[None, :]
    u = philox.draw_uniforms(5, 3, [7], N)[0]
    J, _ = O.draw_bins(p[None, :], np.ones((1, K), bool), u[None, :], "mag")
    ut = philox.g2_top_uniforms(5, 3, [7], N)
    ub = philox.g2_bin_uniforms(5, 3, [7], N, K)
    phi = O.conditional_gumbels(logp, J, ut, ub)
    assert np.array_equal(np.argmax(phi, axis=2), J)
    noise = (phi - logp[:, None, :])[0]
    for k in range(K):
        ks = stats.kstest(noise[:, k], stats.gumbel_r.cdf)
        assert ks.pvalue > 1e-3, (k, ks)
    assert abs(noise.mean() - np.euler_gamma) < 0.02
    assert abs(noise.var() - math.pi ** 2 / 6) < 0.05


def test_straight_through_gradient_is_the_softmax_jacobian_of_the_scores():
    """y = y_hard - stopgrad(y_soft) + y_soft keeps y_hard in value and passes
    dL/dlog p_k = (1/tau) y_k (g_k - <y, g>) with g = dL/dy."""
    rng = np.random.default_rng(4)
    K, tau = 9, 0.7
    logp = torch.tensor(np.log(rng.dirichlet(np.ones(K))), requires_grad=True)
    z = torch.tensor(-np.log(-np.log(rng.uniform(size=K))))
    c = torch.tensor(rng.normal(size=K))
    ys = torch.softmax((logp + z) / tau, dim=0)
    yh = torch.zeros(K, dtype=torch.float64)
    yh[int(torch.argmax(logp + z))] = 1.0
    y = yh - ys.detach() + ys
    assert torch.equal(y.detach(), yh) or float((y.detach() - yh).abs().max()) < 1e-15
    (c * y).sum().backward()
    yv = ys.detach().numpy()
    expect = (1.0 / tau) * yv * (c.numpy() - (yv * c.numpy()).sum())
    assert np.allclose(logp.grad.numpy(), expect, rtol=1e-12, atol=1e-15)


def _g2_case(sampling, grad, tau=1.0):
    from rwcases import oracle_param_values, small_hologram
    system, cfg, maps = small_hologram(sampling=sampling, rays=6, N=16, n_lambda=1,
                                       n_field_side=1)
    cfg = dict(cfg, grad=grad, tau=tau)
    return O.loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                           maps["amp"].astype(np.float64), oracle_param_values(system),
                           maps["target"].astype(np.float64))


def test_g2_equals_g1_for_uniform_sampling_and_tends_to_it_as_tau_vanishes():
    """p_uni does not depend on the DOE, so the softmax path carries nothing;
    as tau -> 0 the soft sample tends to the hard one-hot and its Jacobian
    vanishes.  Both limits of the relaxed estimator reduce to frozen draws."""
    L1, g1, _, _ = _g2_case("uni", "G1")
    L2, g2, _, _ = _g2_case("uni", "G2")
    assert L1 == L2
    for k in g1:
        assert np.array_equal(g1[k], g2[k]), k
    L1, g1, _, _ = _g2_case("mag", "G1")
    L3, g3, _, _ = _g2_case("mag", "G2", tau=1e-6)
    for k in g1:
        assert np.linalg.norm(g3[k] - g1[k]) <= 1e-9 * np.linalg.norm(g1[k]), k
    _, g4, _, _ = _g2_case("mag", "G2")
    assert np.linalg.norm(g4["phase"] - g1["phase"]) > 1e-3 * np.linalg.norm(g1["phase"])


# ---------------------------------------------------- patch classes (Eq. 4) --
def test_local_radius_sphere_and_asphere_against_sag_derivatives():
    """Sphere: R_loc = R everywhere.  Even asphere: the closed-form principal
    curvatures against autograd derivatives of the sag itself."""
    sph = {"c": 1 / 30.0, "k": 0.0, "A": [0.0, 0.0, 0.0, 0.0]}
    x = torch.tensor([0.0, 1.0, 3.0, -4.0], dtype=torch.float64)
    y = torch.tensor([0.0, 2.0, -1.0, 5.0], dtype=torch.float64)
    assert torch.allclose(O.local_radius(sph, x, y), torch.full_like(x, 30.0), rtol=1e-12)
    asp = {"c": 1 / 40.0, "k": -0.7, "A": [2e-5, -3e-7, 1e-9, 0.0]}
    for r0 in (0.0, 0.8, 2.5, 6.0):
        r = torch.tensor(r0, dtype=torch.float64, requires_grad=True)
        z = O.sag_and_grad(asp, r, torch.zeros((), dtype=torch.float64))[0]
        (zp,) = torch.autograd.grad(z, r, create_graph=True)
        (zpp,) = torch.autograd.grad(zp, r)
        km = abs(float(zpp)) / (1 + float(zp) ** 2) ** 1.5
        ks = abs(float(zp)) / (r0 * math.sqrt(1 + float(zp) ** 2)) if r0 > 0 else abs(float(zpp))
        R = float(O.local_radius(asp, torch.tensor([r0], dtype=torch.float64),
                                 torch.zeros(1, dtype=torch.float64))[0])
        assert abs(R - 1.0 / max(km, ks)) <= 1e-10 * R, (r0, R)
    plane = {"c": 0.0, "k": 0.0, "A": [0.0, 0.0, 0.0, 0.0]}
    assert torch.isinf(O.local_radius(plane, x, y)).all()


def test_patch_class_rule_follows_the_curvature_bound():
    """Largest candidate P with arcsin(P pitch / 2R) <= eps (Eq. 4)."""
    pitch, eps = 0.5e-3, 0.1
    cfg = {"patch_p": 128, "patch_classes": [64, 32], "curv_eps": eps}
    p = torch.zeros((3, 3), dtype=torch.float64)
    for R, expect in ((1e9, 128), (0.5, 128), (0.2, 64), (0.1, 32), (0.05, 32)):
        surf = {"c": 1.0 / R, "k": 0.0, "A": [0.0, 0.0, 0.0, 0.0]}
        sides = O.ray_patch_sides(surf, p, pitch, cfg)
        assert (sides == expect).all(), (R, sides)
        P = int(sides[0])
        fits = P * pitch <= 2 * R and math.asin(P * pitch / (2 * R)) <= eps
        assert fits or P == 32                     # the smallest side when none fits
        if P < 128:                                # the next larger side violates the bound
            D = 2 * P * pitch
            assert D > 2 * R or math.asin(D / (2 * R)) > eps
