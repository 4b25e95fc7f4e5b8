"""Seeded synthetic inputs for the ray-wave hybrid PSF: optical prescriptions,
DOE maps, launch grids, sensor windows and targets.

This module holds none of the method's arithmetic: it only lays out inputs
(shapes, sizes, value distributions) shaped like the systems of the paper's
benchmark and design demonstrations.  Both the GPU library's tests/benchmark
and the CPU oracle consume its output; neither is imported here.

A workload is (system, cfg, maps):
  system: {"surfaces": [...], "sensor_z", "doe": {...}, "params": [...]}
  cfg:    wavelengths, field tangents, launch grid, patch / sampling / PSF
          settings, seed
  maps:   {"phase": float32 [H, W], "amp": float32 [H, W], "target": float32
          [L, F, Q, Q] or None}
Lengths are mm; wavelengths are mm.
"""
import math

import numpy as np
from scipy import special

# Two-term Cauchy coefficients (A, B[um^2]) fitted to (n_d, V_d) of the
# catalogue glasses -- stand-ins, since catalogue dispersion data is not at hand.
BK7 = (1.504586, 0.0042172)    # n_d 1.5168, V_d 64.17
F2 = (1.594154, 0.0089237)     # n_d 1.6200, V_d 36.37
AIR = (1.0, 0.0)

LAM_D = 587.6e-6
LAM_F = 486.1e-6
LAM_C = 656.3e-6

PARAM_FIELDS = ("curv", "conic", "A4", "A6", "A8", "A10", "gap")


def surface(z, c=0.0, k=0.0, A=(0.0, 0.0, 0.0, 0.0), semi_ap=0.0, medium=AIR, doe=False,
            gh=0.0, gw=0.0):
    """Even asphere (plane when c = 0 and no A); gh, gw > 0 add the Gaussian-like
    term gh (exp(-r^2 / gw^2) - 1) to the sag."""
    kind = "gauss" if gw > 0 else ("plane" if (c == 0.0 and not any(A)) else "asphere")
    return {"kind": kind, "z": float(z), "c": float(c), "k": float(k), "A": [float(a) for a in A],
            "semi_ap": float(semi_ap), "nA": float(medium[0]), "nB": float(medium[1]),
            "doe": bool(doe), "gh": float(gh), "gw": float(gw)}


def doe_desc(H, W, pitch, cx=0.0, cy=0.0):
    """Map of H x W pixels at `pitch`, centred on (cx, cy); pixel (iy, ix)
    has its centre at (x0 + ix pitch, y0 + iy pitch)."""
    return {"H": int(H), "W": int(W), "pitch": float(pitch),
            "x0": float(cx - (W - 1) / 2.0 * pitch), "y0": float(cy - (H - 1) / 2.0 * pitch)}


def bandlimited_uniform(H, W, cutoff, rng):
    """White Gaussian field -> radial low-pass at `cutoff` cycles/pixel ->
    standardise -> normal CDF: a band-limited field with uniform marginals."""
    g = rng.standard_normal((H, W))
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    lp = (fx * fx + fy * fy) <= cutoff * cutoff
    f = np.real(np.fft.ifft2(np.fft.fft2(g) * lp))
    f = (f - f.mean()) / max(f.std(), 1e-30)
    return special.ndtr(f)


def kinoform_zone_plate(doe, f, lam0):
    """phi = mod(-pi r^2 / (lam0 f), 2 pi) on the pixel centres."""
    x = doe["x0"] + np.arange(doe["W"]) * doe["pitch"]
    y = doe["y0"] + np.arange(doe["H"]) * doe["pitch"]
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    return np.mod(-math.pi * r2 / (lam0 * f), 2 * math.pi)


def airy_target(Q, pitch, lam, NA, center_px, rng_off):
    """Airy intensity (2 J1(v)/v)^2, v = 2 pi NA r / lam, unit sum."""
    c = np.arange(Q) - Q // 2
    X = (c[None, :] - center_px[0] - rng_off[0]) * pitch
    Y = (c[:, None] - center_px[1] - rng_off[1]) * pitch
    v = 2 * math.pi * NA * np.sqrt(X * X + Y * Y) / lam
    vs = np.where(v == 0, 1.0, v)
    I = np.where(v == 0, 1.0, (2 * special.j1(vs) / vs) ** 2)
    return I / I.sum()


def field_grid(max_deg, n):
    a = np.tan(np.deg2rad(np.linspace(-max_deg, max_deg, n))) if n > 1 else np.zeros(1)
    return [[float(tx), float(ty)] for ty in a for tx in a]


def _launch_centres(fields, z_aim, z_launch):
    """Launch-grid centres whose central ray heads for (0, 0, z_aim)."""
    return [[-tx * (z_aim - z_launch), -ty * (z_aim - z_launch)] for tx, ty in fields]


def singlet_entrance_pupil(n, R1, R2, ct, z_front, z_stop):
    """Paraxial entrance pupil (position, magnification) of a stop behind a
    thick singlet: the stop imaged back through the lens (thick-lens focal
    length and principal planes).  Used only to aim the launch grid."""
    P = (n - 1) * (1 / R1 - 1 / R2 + (n - 1) * ct / (n * R1 * R2))
    f = 1 / P
    zH = z_front - f * (n - 1) * ct / (n * R2)          # front principal plane
    zH2 = z_front + ct - f * (n - 1) * ct / (n * R1)    # rear principal plane
    so = z_stop - zH2
    si = 1 / (1 / f - 1 / so)
    return zH - si, -si / so


def _psf_centres(lambdas, fields, dz):
    return [[[tx * dz, ty * dz] for tx, ty in fields] for _ in lambdas]


def _cfg(lambdas, fields, z_aim, z_launch, launch_half, rays_side, Q, psf_pitch, dz_sensor,
         P, N, sampling="mag", pad=2, seed=0):
    return {"lambdas": [float(l) for l in lambdas], "fields": fields,
            "launch_center": _launch_centres(fields, z_aim, z_launch),
            "launch_z": float(z_launch), "launch_half": float(launch_half),
            "rays_side": int(rays_side), "psf_q": int(Q), "psf_pitch": float(psf_pitch),
            "psf_center": _psf_centres(lambdas, fields, dz_sensor),
            "patch_p": int(P), "pad": int(pad), "n_ssr": int(N), "sampling": sampling,
            "seed": int(seed)}


# ----------------------------------------------------------------------------
# Workload 1: BK7 singlet (R1 = +50, R2 = -50, CT 5, semi-aperture 5) followed
# 1 mm behind its rear vertex by a planar 256 x 256 kinoform zone plate
# (f = 100 mm at 587.6 nm, 4 um pitch) that is also the stop; 64 x 64 rays,
# 32 x 32 patches, 128 x 128 PSF at 2 um, one wavelength on axis.
# Sensor 31.758 mm after the DOE (paraxial focus of lens + zone plate).
# ----------------------------------------------------------------------------
def singlet_zoneplate(rays_side=64, H=256, pitch=0.004, P=32, N=256, Q=128, psf_pitch=0.002,
                      sampling="mag", seed=0):
    z_doe = 6.0
    surfs = [surface(0.0, c=1 / 50.0, semi_ap=5.0, medium=BK7),
             surface(5.0, c=-1 / 50.0, semi_ap=5.0, medium=AIR),
             surface(z_doe, doe=True)]
    dz = 31.758
    system = {"surfaces": surfs, "sensor_z": z_doe + dz, "doe": doe_desc(H, H, pitch),
              "params": [{"surface": 0, "field": "curv", "scale": 1 / 50.0},
                         {"surface": 1, "field": "curv", "scale": 1 / 50.0}]}
    z_ep, mag = singlet_entrance_pupil(1.5168, 50.0, -50.0, 5.0, 0.0, z_doe)
    half = 0.95 * mag * 0.5 * H * pitch
    cfg = _cfg([LAM_D], [[0.0, 0.0]], z_ep, -1.0, half, rays_side, Q, psf_pitch, dz, P, N,
               sampling, seed=seed)
    phase = kinoform_zone_plate(system["doe"], 100.0, LAM_D)
    maps = {"phase": phase.astype(np.float32), "amp": np.ones_like(phase, dtype=np.float32),
            "target": None}
    return system, cfg, maps


# ----------------------------------------------------------------------------
# Workloads 2 and 3: equiconvex BK7 even asphere (R = +-25.14, CT 4, EFL 25)
# with A4, A6 ~ N(0, 1e-6) per surface, then a planar 1024 x 1024 random
# holographic complex DOE at 1 um pitch 1 mm behind the rear vertex (the
# stop).  Phase uniform on [0, 2 pi), amplitude uniform on [0.5, 1], both
# band-limited to 0.25 cycles/pixel.  3 wavelengths (F, d, C lines), 3 x 3
# fields up to +-10 deg, 256 x 256 rays per field, 64 x 64 patches, 512 x 512
# PSF at 1 um.  Workload 3 adds Airy targets for Eq. 5 and six lens
# parameters (2 curvatures, 4 asphere coefficients).
# ----------------------------------------------------------------------------
def asphere_hologram(rays_side=256, H=1024, pitch=0.001, P=64, N=256, Q=512, psf_pitch=0.001,
                     n_lambda=3, n_field_side=3, max_deg=10.0, sampling="mag", seed=0,
                     with_target=True, cfg_id=2):
    rng_a = np.random.default_rng(20260100 + cfg_id)
    A1 = rng_a.normal(0.0, 1e-6, 2)
    A2 = rng_a.normal(0.0, 1e-6, 2)
    R = 25.140
    z_doe = 5.0
    surfs = [surface(0.0, c=1 / R, A=(A1[0], A1[1], 0, 0), semi_ap=5.0, medium=BK7),
             surface(4.0, c=-1 / R, A=(A2[0], A2[1], 0, 0), semi_ap=5.0, medium=AIR),
             surface(z_doe, doe=True)]
    # keep the surfaces aspheric in the description even if coefficients are small
    surfs[0]["kind"] = surfs[1]["kind"] = "asphere"
    dz = 22.645
    r_fp = 0.55
    s4 = LAM_D / r_fp ** 4
    s6 = LAM_D / r_fp ** 6
    system = {"surfaces": surfs, "sensor_z": z_doe + dz, "doe": doe_desc(H, H, pitch),
              "params": [{"surface": 0, "field": "curv", "scale": 1 / R},
                         {"surface": 1, "field": "curv", "scale": 1 / R},
                         {"surface": 0, "field": "A4", "scale": s4},
                         {"surface": 0, "field": "A6", "scale": s6},
                         {"surface": 1, "field": "A4", "scale": s4},
                         {"surface": 1, "field": "A6", "scale": s6}]}
    lambdas = [LAM_F, LAM_D, LAM_C][:n_lambda] if n_lambda <= 3 else \
        list(np.linspace(400e-6, 700e-6, n_lambda))
    fields = field_grid(max_deg, n_field_side)
    z_ep, mag = singlet_entrance_pupil(1.5168, R, -R, 4.0, 0.0, z_doe)
    half = 0.9 * mag * 0.5 * H * pitch
    cfg = _cfg(lambdas, fields, z_ep, -1.0, half, rays_side, Q, psf_pitch, dz, P, N, sampling,
               seed=seed)
    rng = np.random.default_rng(20260000 + cfg_id)
    phase = 2 * math.pi * bandlimited_uniform(H, H, 0.25, rng)
    amp = 0.5 + 0.5 * bandlimited_uniform(H, H, 0.25, rng)
    target = None
    if with_target:
        rng_t = np.random.default_rng(20260200 + cfg_id)
        NA = (H * pitch / 2) / dz
        L, F = len(lambdas), len(fields)
        target = np.zeros((L, F, Q, Q), dtype=np.float32)
        for l in range(L):
            for f in range(F):
                off = rng_t.uniform(-8, 8, 2)
                target[l, f] = airy_target(Q, psf_pitch, lambdas[l], NA, (0.0, 0.0), off)
    maps = {"phase": phase.astype(np.float32), "amp": amp.astype(np.float32),
            "target": target}
    return system, cfg, maps


# ----------------------------------------------------------------------------
# Free-space DOE (no refractive surface) for the closed-form pins: a planar
# DOE at z = 0 under a collimated beam, sensor at `dz`.
# ----------------------------------------------------------------------------
def free_space_doe(phase, amp, pitch, dz, lam, rays_side, P, Q, psf_pitch, N=256, pad=2,
                   sampling="full", field=(0.0, 0.0), launch_half=None, seed=0,
                   psf_center=(0.0, 0.0)):
    H, W = phase.shape
    surfs = [surface(0.0, doe=True)]
    system = {"surfaces": surfs, "sensor_z": float(dz), "doe": doe_desc(H, W, pitch),
              "params": []}
    if launch_half is None:
        launch_half = 0.5 * W * pitch * (1 - 1.0 / rays_side)
    cfg = _cfg([lam], [list(field)], 0.0, -1.0, launch_half, rays_side, Q, psf_pitch, dz, P, N,
               sampling, pad=pad, seed=seed)
    cfg["psf_center"] = [[list(psf_center)]]
    maps = {"phase": np.asarray(phase, np.float32), "amp": np.asarray(amp, np.float32),
            "target": None}
    return system, cfg, maps


# ----------------------------------------------------------------------------
# Conformal DOE: a random complex hologram on an even-asphere surface in air
# (R = 10 mm at the vertex, A4 = 0.42 mm^-3, so the smallest principal radius
# falls to ~2.4 mm at the map edge) under collimated light; the patch-class
# rule (Eq. 4) gives patch side P near the axis and the smaller class further
# out.  Sensor 5 mm behind the vertex.
# ----------------------------------------------------------------------------
def conformal_hologram(rays_side=8, H=256, pitch=0.002, P=32, classes=(16,), N=32, Q=32,
                       psf_pitch=0.004, sampling="mag", curv_eps=0.006, n_field_side=1,
                       max_deg=2.0, seed=0, cfg_id=7):
    surfs = [surface(0.0, c=0.1, A=(0.42, 0.0, 0.0, 0.0), medium=AIR, doe=True)]
    dz = 5.0
    system = {"surfaces": surfs, "sensor_z": dz, "doe": doe_desc(H, H, pitch), "params": []}
    fields = field_grid(max_deg, n_field_side)
    half = 0.45 * H * pitch
    cfg = _cfg([LAM_D], fields, 0.0, -1.0, half, rays_side, Q, psf_pitch, dz, P, N, sampling,
               seed=seed)
    cfg["patch_classes"] = [int(q) for q in classes]
    cfg["curv_eps"] = float(curv_eps)
    rng = np.random.default_rng(20260000 + cfg_id)
    phase = 2 * math.pi * bandlimited_uniform(H, H, 0.25, rng)
    amp = 0.5 + 0.5 * bandlimited_uniform(H, H, 0.25, rng)
    rng_t = np.random.default_rng(20260200 + cfg_id)
    NA = (H * pitch / 2) / dz
    target = np.zeros((1, len(fields), Q, Q), dtype=np.float32)
    for f in range(len(fields)):
        target[0, f] = airy_target(Q, psf_pitch, LAM_D, NA, (0.0, 0.0), rng_t.uniform(-2, 2, 2))
    maps = {"phase": phase.astype(np.float32), "amp": amp.astype(np.float32), "target": target}
    return system, cfg, maps


def paraxial_pupil(surfs, z_stop, lam):
    """Paraxial entrance pupil of a stop at z_stop behind the given surfaces
    (first-order ray transfer, nu' = nu - y c (n' - n)): returns (z_ep, m), the
    pupil position and the ratio of stop height to pupil height.  Used only to
    aim the launch grids."""
    def trace(y, u, z):
        n = 1.0
        for sf in surfs:
            if sf["z"] >= z_stop:
                break
            y += u * (sf["z"] - z)
            z = sf["z"]
            na = sf["nA"] + sf["nB"] / (lam * 1e3) ** 2
            u = (n * u - y * sf["c"] * (na - n)) / na
            n = na
        return y + u * (z_stop - z)
    z0 = surfs[0]["z"] - 1.0
    m = trace(1.0, 0.0, z0)                     # a collimated ray's height at the stop
    y_a = trace(0.0, 1e-3, z0)                  # a ray crossing the axis at z0 ...
    y_b = trace(-1e-3, 1e-3, z0)                # ... and one crossing it at z0 + 1
    z_ep = z0 + y_a / (y_a - y_b)               # the axis point whose ray meets the stop centre
    return z_ep, m


# ----------------------------------------------------------------------------
# Workload 4: conformal DOE on the convex R = 30 front of a BK7 plano-convex
# (CT 4, planar rear face after the DOE), 2048 x 2048 random phase at 0.5 um
# on the xy projection (band-limited to 0.4 cycles/pixel, A = 1), 31
# wavelengths 400-700 nm x 25 fields (5 x 5 up to +-20 deg), 128 x 128 rays per
# field, N = 256, 256 x 256 PSF at 1 um at the 587.6 nm back focus.  Patch
# classes 128 / 64 / 32 by the curvature bound (Eq. 4): the front is the
# R = 30 sphere plus an A4 term that lowers the local radius across the DOE,
# so that the bound splits the rays into three concentric zones.
# ----------------------------------------------------------------------------
def conformal_sphere(rays_side=128, H=2048, pitch=0.0005, P=128, classes=(64, 32), N=256,
                     Q=256, psf_pitch=0.001, n_lambda=31, n_field_side=5, max_deg=20.0,
                     sampling="mag", curv_eps=0.0082, A4=0.2, seed=0, with_params=False,
                     cfg_id=4):
    R, ct = 30.0, 4.0
    surfs = [surface(0.0, c=1 / R, A=(A4, 0.0, 0.0, 0.0), semi_ap=6.0, medium=BK7, doe=True),
             surface(ct, medium=AIR)]
    surfs[0]["kind"] = "asphere"
    n_d = BK7[0] + BK7[1] / (LAM_D * 1e3) ** 2
    bfl = R / (n_d - 1) - ct / n_d
    params = []
    if with_params:        # the DOE surface's shape, the rear face's curvature, both gaps
        r_fp = 0.5 * H * pitch
        params = [{"surface": 0, "field": "curv", "scale": 1 / R},
                  {"surface": 0, "field": "A4", "scale": LAM_D / r_fp ** 4},
                  {"surface": 1, "field": "curv", "scale": 1 / R},
                  {"surface": 0, "field": "gap", "scale": 1.0},
                  {"surface": 1, "field": "gap", "scale": 1.0}]
    system = {"surfaces": surfs, "sensor_z": ct + bfl, "doe": doe_desc(H, H, pitch),
              "params": params}
    lambdas = list(np.linspace(400e-6, 700e-6, n_lambda)) if n_lambda > 1 else [LAM_D]
    fields = field_grid(max_deg, n_field_side)
    half = 0.5 * H * pitch * (1 - 1.0 / rays_side)
    cfg = _cfg(lambdas, fields, 0.0, -1.0, half, rays_side, Q, psf_pitch, 0.0, P, N, sampling,
               seed=seed)
    # sensor window on each chief ray (paraxial: through the DOE centre, n_d inside the lens)
    cfg["psf_center"] = [[[tx * (ct / n_d + bfl), ty * (ct / n_d + bfl)] for tx, ty in fields]
                         for _ in lambdas]
    cfg["patch_classes"] = [int(q) for q in classes]
    cfg["curv_eps"] = float(curv_eps)
    rng = np.random.default_rng(20260000 + cfg_id)
    phase = 2 * math.pi * bandlimited_uniform(H, H, 0.4, rng)
    maps = {"phase": phase.astype(np.float32), "amp": np.ones((H, H), dtype=np.float32),
            "target": None}
    return system, cfg, maps


# ----------------------------------------------------------------------------
# Workload 5: end-to-end hybrid design.  L1 (BK7, R +40 / -60, CT 5) and L2
# (F2, R +30 / -200, CT 3), semi-apertures 7.5, even-asphere terms A4, A6 on
# every surface (seeded, small, plus a fixed A4 on the DOE surface so that its
# local radius varies), a 4096 x 4096 complex DOE at 0.5 um on L2's rear
# surface (F2 -> air), the stop.  8 wavelengths 400-700 nm x 16 fields (4 x 4
# up to +-25 deg), 512 x 512 rays per field, patch classes 128 / 64 by Eq. 4,
# N = 256, 1024 x 1024 PSF at 1 um at the paraxial focus, Airy targets;
# 14 lens parameters: 4 curvatures, 4 A4, 4 A6, 2 centre thicknesses.
# ----------------------------------------------------------------------------
def two_lens_hybrid(rays_side=512, H=4096, pitch=0.0005, P=128, classes=(64,), N=256, Q=1024,
                    psf_pitch=0.001, n_lambda=8, n_field_side=4, max_deg=25.0, sampling="mag",
                    curv_eps=2.5e-4, A4_doe=2e-3, seed=0, with_target=True, cfg_id=5):
    rng_a = np.random.default_rng(20260100 + cfg_id)
    Rs = (40.0, -60.0, 30.0, -200.0)
    zs = (0.0, 5.0, 7.0, 10.0)
    meds = (BK7, AIR, F2, AIR)
    A = rng_a.normal(0.0, 1e-6, (4, 2))
    A[3, 0] += A4_doe
    surfs = [surface(zs[i], c=1 / Rs[i], A=(A[i, 0], A[i, 1], 0.0, 0.0), semi_ap=7.5,
                     medium=meds[i], doe=(i == 3)) for i in range(4)]
    for sf in surfs:
        sf["kind"] = "asphere"
    # paraxial focus of the d line behind the DOE surface
    y, u, n, z = 1.0, 0.0, 1.0, zs[0]
    for sf in surfs:
        y += u * (sf["z"] - z)
        z = sf["z"]
        na = sf["nA"] + sf["nB"] / (LAM_D * 1e3) ** 2
        u = (n * u - y * sf["c"] * (na - n)) / na
        n = na
    dz = -y / u
    r_fp = 0.5 * H * pitch
    system = {"surfaces": surfs, "sensor_z": zs[3] + dz, "doe": doe_desc(H, H, pitch),
              "params": []}
    for s_i in range(4):
        system["params"].append({"surface": s_i, "field": "curv", "scale": 1 / abs(Rs[s_i])})
    for s_i in range(4):
        system["params"].append({"surface": s_i, "field": "A4", "scale": LAM_D / r_fp ** 4})
    for s_i in range(4):
        system["params"].append({"surface": s_i, "field": "A6", "scale": LAM_D / r_fp ** 6})
    system["params"].append({"surface": 0, "field": "gap", "scale": 1.0})
    system["params"].append({"surface": 2, "field": "gap", "scale": 1.0})
    lambdas = list(np.linspace(400e-6, 700e-6, n_lambda)) if n_lambda > 1 else [LAM_D]
    fields = field_grid(max_deg, n_field_side)
    z_ep, m = paraxial_pupil(surfs, zs[3], LAM_D)
    half = 0.5 * H * pitch * (1 - 1.0 / rays_side) / abs(m)
    cfg = _cfg(lambdas, fields, z_ep, -1.0, half, rays_side, Q, psf_pitch, dz, P, N, sampling,
               seed=seed)
    cfg["patch_classes"] = [int(q) for q in classes]
    cfg["curv_eps"] = float(curv_eps)
    rng = np.random.default_rng(20260000 + cfg_id)
    phase = 2 * math.pi * bandlimited_uniform(H, H, 0.25, rng)
    amp = 0.5 + 0.5 * bandlimited_uniform(H, H, 0.25, rng)
    target = None
    if with_target:
        rng_t = np.random.default_rng(20260200 + cfg_id)
        NA = r_fp / dz
        L, F = len(lambdas), len(fields)
        target = np.zeros((L, F, Q, Q), dtype=np.float32)
        for l in range(L):
            for f in range(F):
                target[l, f] = airy_target(Q, psf_pitch, lambdas[l], NA, (0.0, 0.0),
                                           rng_t.uniform(-8, 8, 2))
    maps = {"phase": phase.astype(np.float32), "amp": amp.astype(np.float32), "target": target}
    return system, cfg, maps


# ----------------------------------------------------------------------------
# DOE upstream of refractive optics (the benchmark's System 1 shape): a planar
# blazed linear grating of period `period_px` pixels at 6.3 um pitch, the stop,
# 3 mm before a BK7 plano-convex of f = 50 mm (R 25.8 convex side first, CT
# 5.3, the catalogue LA1131 shape), sensor at the back focus; 0.7 um light,
# collimated on axis.  Every secondary ray crosses both lens surfaces.
# Lens parameters: the front curvature, the DOE-lens gap, CT and back distance.
# ----------------------------------------------------------------------------
def grating_before_lens(rays_side=64, H=512, pitch=0.0063, period_px=35, lam=700e-6, P=32, N=256,
                        Q=128, psf_pitch=0.002, sampling="mag", field_deg=0.0, seed=0,
                        with_target=True, cfg_id=6):
    R, ct, gap = 25.8, 5.3, 3.0
    surfs = [surface(0.0, doe=True),
             surface(gap, c=1 / R, semi_ap=12.7, medium=BK7),
             surface(gap + ct, semi_ap=12.7, medium=AIR)]
    n = BK7[0] + BK7[1] / (lam * 1e3) ** 2
    bfl = R / (n - 1) - ct / n
    system = {"surfaces": surfs, "sensor_z": gap + ct + bfl, "doe": doe_desc(H, H, pitch),
              "params": [{"surface": 1, "field": "curv", "scale": 1 / R},
                         {"surface": 0, "field": "gap", "scale": 1.0},
                         {"surface": 1, "field": "gap", "scale": 1.0},
                         {"surface": 2, "field": "gap", "scale": 1.0}]}
    t = math.tan(math.radians(field_deg))
    fields = [[t, 0.0]]
    half = 0.5 * H * pitch * (1 - 1.0 / rays_side)
    efl = R / (n - 1)
    cfg = _cfg([lam], fields, 0.0, -1.0, half, rays_side, Q, psf_pitch, 0.0, P, N, sampling,
               seed=seed)
    # sensor window on the first diffraction order (the blaze puts the light there)
    cfg["psf_center"] = [[[efl * math.tan(math.asin(lam / (period_px * pitch)) + math.atan(t)),
                           0.0]]]
    x = system["doe"]["x0"] + np.arange(H) * pitch
    phase = np.mod(2 * math.pi * x / (period_px * pitch), 2 * math.pi)
    phase = np.broadcast_to(phase[None, :], (H, H)).astype(np.float32).copy()
    target = None
    if with_target:
        rng_t = np.random.default_rng(20260200 + cfg_id)
        target = airy_target(Q, psf_pitch, lam, 0.5 * H * pitch / bfl, (0.0, 0.0),
                             rng_t.uniform(-4, 4, 2))[None, None].astype(np.float32)
    maps = {"phase": phase, "amp": np.ones((H, H), dtype=np.float32), "target": target}
    return system, cfg, maps


# ----------------------------------------------------------------------------
# Reflective conformal DOE (the curvilinear-DOE demonstration, Fig. 6): a
# reflective DOE on a Gaussian-like substrate sag gh (exp(-r^2/gw^2) - 1) whose
# smallest radius of curvature, gw^2 / (2 |gh|) at the vertex, is about 506
# wavelengths; a circular aperture of 501 pixels at lambda / 2 pitch, 1 um
# light, NA 0.5 (sensor before the DOE at the aperture radius / tan(asin 0.5)),
# collimated along the axis.  The field is exp(i phi1) + exp(i phi2) (the
# beam-splitting design; the amplitude map holds phi2); the maps are the
# point-focus phases of two spots 0.1 mm apart on the sensor (for a flat DOE:
# the substrate's sag is left for the design to compensate).
# Patch side 128 (64 lambda, curvature bound 0.063 rad), N = 2048 draws.
# ----------------------------------------------------------------------------
def reflective_conformal(rays_side=64, H=501, lam=1e-3, P=128, N=2048, Q=512, psf_pitch=0.0005,
                         sampling="mag", classes=(), curv_eps=0.1, r_min_waves=506.0,
                         gw=0.15, sep=0.1, random_phase=0.0, na=0.5, seed=0, with_target=True,
                         cfg_id=8):
    pitch = lam / 2
    r_ap = 0.5 * H * pitch
    gh = -gw * gw / (2 * r_min_waves * lam) if gw > 0 else 0.0   # concave towards the light
    f = r_ap / math.tan(math.asin(na))
    surfs = [surface(0.0, semi_ap=r_ap, medium=AIR, doe=True, gh=gh, gw=gw)]
    doe = doe_desc(H, H, pitch)
    doe["reflective"] = True
    doe["field"] = "two_phase"
    system = {"surfaces": surfs, "sensor_z": -f, "doe": doe, "params": []}
    cfg = _cfg([lam], [[0.0, 0.0]], 0.0, -2.0 * f, r_ap * (1 - 1.0 / rays_side), rays_side, Q,
               psf_pitch, 0.0, P, N, sampling, seed=seed)
    cfg["psf_center"] = [[[0.0, 0.0]]]
    cfg["patch_classes"] = [int(q) for q in classes]
    cfg["curv_eps"] = float(curv_eps)
    x = doe["x0"] + np.arange(H) * pitch
    y = doe["y0"] + np.arange(H) * pitch
    # point-focus phases of the two spots (x = +-sep/2 on the sensor plane, a
    # distance f in front of a flat DOE): -k0 |(x, y, 0) - (xs, 0, -f)|
    k0 = 2 * math.pi / lam
    phi1 = np.mod(-k0 * np.sqrt((x[None, :] - 0.5 * sep) ** 2 + y[:, None] ** 2 + f * f), 2 * math.pi)
    phi2 = np.mod(-k0 * np.sqrt((x[None, :] + 0.5 * sep) ** 2 + y[:, None] ** 2 + f * f), 2 * math.pi)
    if random_phase > 0:
        rng = np.random.default_rng(20260000 + cfg_id)
        phi1 = phi1 + random_phase * bandlimited_uniform(H, H, 0.25, rng)
        phi2 = phi2 + random_phase * bandlimited_uniform(H, H, 0.25, rng)
    target = None
    if with_target:
        NA = na
        target = (airy_target(Q, psf_pitch, lam, NA, (sep / 2 / psf_pitch, 0.0), (0.0, 0.0)) +
                  airy_target(Q, psf_pitch, lam, NA, (-sep / 2 / psf_pitch, 0.0), (0.0, 0.0)))
        target = (target / target.sum())[None, None].astype(np.float32)
    maps = {"phase": phi1.astype(np.float32), "amp": phi2.astype(np.float32), "target": target}
    return system, cfg, maps


# ----------------------------------------------------------------------------
# Adaptive patch sizing: a kinoform zone plate (focal length f at lam) on a
# planar DOE in air under collimated light, with a band-limited amplitude in
# [0.5, 1]; its local period lam f / r falls from the axis outwards, so the
# K-period rule gives the largest patch near the axis and smaller ones further
# out.  Sensor at the focus; Airy target of the aperture's NA with a seeded
# offset of up to 2 px.
# ----------------------------------------------------------------------------
def adaptive_zone_plate(rays_side=256, H=1024, pitch=0.001, lam=0.5e-3, f=10.0, P=64,
                        classes=(32, 16), K=2.0, N=256, Q=128, psf_pitch=0.001, sampling="mag",
                        seed=0):
    rng = np.random.default_rng(20260007 + seed)
    doe = doe_desc(H, H, pitch)
    phase = kinoform_zone_plate(doe, f, lam).astype(np.float32)
    amp = (0.5 + 0.5 * bandlimited_uniform(H, H, 0.05, rng)).astype(np.float32)
    system, cfg, maps = free_space_doe(phase, amp, pitch, f, lam, rays_side, P, Q, psf_pitch,
                                       N=N, pad=2, sampling=sampling, seed=seed)
    cfg["patch_classes"] = [int(c) for c in classes]
    cfg["bw_periods"] = float(K)
    NA = 0.5 * H * pitch / f
    tgt = airy_target(Q, psf_pitch, lam, NA, (0.0, 0.0), rng.uniform(-2, 2, 2))
    maps["target"] = tgt[None, None].astype(np.float32)
    return system, cfg, maps


# ----------------------------------------------------------------------------
# Two DOEs in sequence: DOE 1 on a plane in air 1 mm before a BK7 plano-convex
# (curved face R = 20 mm first, CT 1.5 mm), DOE 2 on the front face of a 1 mm
# BK7 plate 1.5 mm behind the lens; sensor near the paraxial focus.  Both maps
# are band-limited random holograms (phase uniform in [0, 2 pi), amplitude in
# [0.5, 1]) on their own pitch, or, where `uniform` says so, a clear aperture
# (phase 0, amplitude 1).  N draws per launched ray at DOE 1 (a square), N2 per
# arriving secondary at DOE 2.
# ----------------------------------------------------------------------------
def two_doe_cascade(rays_side=8, H=64, pitch=(0.004, 0.02), P=16, pad=2, N=16, N2=8, Q=32,
                    psf_pitch=0.02, sampling="mag", lambdas=(LAM_D,), fields=((0.0, 0.0),),
                    cutoff=0.05, uniform=(False, False), curvature=(0.0, 0.0), seed=0):
    """curvature: of the two DOE surfaces (0: planar)."""
    rng = np.random.default_rng(seed)
    z_doe2 = 4.0
    surfs = [surface(0.0, c=curvature[0], doe=True),
             surface(1.0, c=1.0 / 20.0, medium=BK7),
             surface(2.5),
             surface(z_doe2, c=curvature[1], medium=BK7, doe=True),
             surface(5.0)]
    does = [dict(doe_desc(H, H, pitch[k]), field="amp_phase") for k in range(2)]
    phase = np.zeros((2, H, H), np.float32)
    amp = np.ones((2, H, H), np.float32)
    for k in range(2):
        if not uniform[k]:
            phase[k] = 2 * math.pi * bandlimited_uniform(H, H, cutoff, rng)
            amp[k] = 0.5 + 0.5 * bandlimited_uniform(H, H, cutoff, rng)
    system = {"surfaces": surfs, "sensor_z": 40.5, "does": does, "doe": does[0], "params": []}
    fields = [list(f) for f in fields]
    cfg = _cfg(lambdas, fields, 0.0, -1.0, 0.1, rays_side, Q, psf_pitch, 38.7, P, N,
               sampling, pad=pad, seed=seed)
    cfg["n_ssr2"] = int(N2)
    maps = {"phase": phase, "amp": amp, "target": None}
    return system, cfg, maps


def workload(name):
    """Named full-size workloads."""
    if name == "singlet_zoneplate":
        return singlet_zoneplate()
    if name == "asphere_hologram":
        return asphere_hologram()
    if name == "conformal_sphere":
        return conformal_sphere()
    if name == "two_lens_hybrid":
        return two_lens_hybrid()
    if name == "grating_before_lens":
        return grating_before_lens()
    if name == "reflective_conformal":
        return reflective_conformal()
    if name == "adaptive_zone_plate":
        return adaptive_zone_plate()
    if name == "two_doe_cascade":
        # 3 wavelengths x 128^2 launched rays, 16 relayed secondaries each (a
        # 512^2 second-DOE grid), 16 draws per arriving ray: 4.2e6 records a pair
        return two_doe_cascade(rays_side=128, H=256, pitch=(0.001, 0.02), P=32, pad=2, N=16,
                               N2=16, Q=256, psf_pitch=0.01, sampling="mag",
                               lambdas=(LAM_F, LAM_D, LAM_C))
    raise KeyError(name)
