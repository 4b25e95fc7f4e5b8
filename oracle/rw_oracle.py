"""Plain FP64 CPU oracle of the differentiable ray-wave hybrid PSF.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this module: it exists so that tests, the smoke check and the CPU
baseline of the benchmark can compare the GPU library against a slow,
obviously correct implementation written directly from the paper
(arXiv 2605.15418, "A general differentiable ray-wave framework for hybrid
refractive-diffractive system modeling and optimization").

Everything is float64 / complex128 (NumPy for integer work, PyTorch CPU for
the differentiable arithmetic so that torch.autograd supplies the oracle's
gradients).  Each function names the passage of the paper it follows.
Readings of passages that the paper leaves open are marked READING and are
listed together in the design notes of the repository.

Units: lengths in mm, wavelengths in mm, k0 = 2*pi/lambda in rad/mm.

Pipeline for one (wavelength, field) pair  -- Results, "Ray-Wave Simulator
Formalism", Fig. 1b/c, Eqs. 1, 2 and 5:
  launch -> conventional refractive trace to the DOE -> tangent frame ->
  square patch of the complex transmission -> zero-padded FFT (angular
  spectrum) -> propagating-mode cut -> sampling density p -> N secondary
  wavevectors -> weights a = U~/p (Eq. 1) -> conventional trace to the sensor
  -> coherent wavelet sum (Eq. 2) -> |U|^2 -> normalised least squares (Eq. 5).
"""
import math

import numpy as np
import torch

from .philox import draw_uniforms, g2_bin_uniforms, g2_top_uniforms

DT = torch.float64
CT = torch.complex128
TWO_PI = 2.0 * math.pi


def _t(x):
    return torch.as_tensor(x, dtype=DT)


# ----------------------------------------------------------------------------
# Materials.  READING: the paper gives catalogue glasses only (N-BK7,
# Benchmark section); a two-term Cauchy law n = A + B / lambda_um^2 stands in.
# ----------------------------------------------------------------------------
def cauchy_index(nA, nB, lam_mm):
    lam_um = lam_mm * 1e3
    return nA + nB / (lam_um * lam_um)


# ----------------------------------------------------------------------------
# System description with differentiable lens parameters.
# A lens parameter value v maps to the physical quantity scale * v.  Fields:
#   curv -> surface curvature c;  conic -> conic constant;
#   A4..A10 -> even asphere coefficients;  gap -> axial distance from the
#   surface to the next surface (or to the sensor after the last surface).
# ----------------------------------------------------------------------------
_FIELDS = ("curv", "conic", "A4", "A6", "A8", "A10", "gap")


def build_surfaces(system, values=None):
    surfs = system["surfaces"]
    S = len(surfs)
    c = [_t(s["c"]) for s in surfs]
    kk = [_t(s["k"]) for s in surfs]
    A = [[_t(a) for a in s["A"]] for s in surfs]
    gaps = [_t(surfs[i + 1]["z"] - surfs[i]["z"]) for i in range(S - 1)]
    gaps.append(_t(system["sensor_z"] - surfs[-1]["z"]))
    if values is not None:
        for ref, v in zip(system["params"], values):
            s, f = ref["surface"], ref["field"]
            phys = ref["scale"] * v
            if f == "curv":
                c[s] = phys
            elif f == "conic":
                kk[s] = phys
            elif f in ("A4", "A6", "A8", "A10"):
                A[s][("A4", "A6", "A8", "A10").index(f)] = phys
            elif f == "gap":
                gaps[s] = phys
            else:
                raise ValueError(f)
    z = [_t(surfs[0]["z"])]
    for i in range(S - 1):
        z.append(z[-1] + gaps[i])
    sensor_z = z[-1] + gaps[-1]
    out = []
    for i, s in enumerate(surfs):
        out.append(dict(kind=s["kind"], z=z[i], c=c[i], k=kk[i], A=A[i],
                        gh=_t(s.get("gh", 0.0)), gw=_t(s.get("gw", 0.0)),
                        semi_ap=s["semi_ap"], nA=s["nA"], nB=s["nB"],
                        doe=bool(s.get("doe", False))))
    return out, sensor_z


def initial_param_values(system):
    """Normalised values reproducing the nominal prescription."""
    surfs = system["surfaces"]
    vals = []
    for ref in system["params"]:
        s, f = ref["surface"], ref["field"]
        if f == "curv":
            phys = surfs[s]["c"]
        elif f == "conic":
            phys = surfs[s]["k"]
        elif f in ("A4", "A6", "A8", "A10"):
            phys = surfs[s]["A"][("A4", "A6", "A8", "A10").index(f)]
        else:
            znext = surfs[s + 1]["z"] if s + 1 < len(surfs) else system["sensor_z"]
            phys = znext - surfs[s]["z"]
        vals.append(phys / ref["scale"])
    return np.array(vals, dtype=np.float64)


# ----------------------------------------------------------------------------
# Even-asphere sag z(r) = c r^2 / (1 + sqrt(1 - (1+k) c^2 r^2)) + A4 r^4 + ...
# plus, for the Gaussian-like substrate of the conformal DOE demonstration
# (Fig. 6b), gh (exp(-r^2 / gw^2) - 1) when gw > 0 (zero at the vertex).
# Conventional ray tracing of refractive surfaces (Formalism, first paragraph;
# Benchmark section, "propagated ... via conventional ray tracing").
# ----------------------------------------------------------------------------
def _gauss_terms(surf, rho):
    """The Gaussian term g(rho) and its first two rho-derivatives (zeros if gw = 0)."""
    gh, gw = surf.get("gh", 0.0), surf.get("gw", 0.0)
    if not (float(gw) > 0):
        z = torch.zeros_like(rho)
        return z, z, z
    e = torch.exp(-rho / (gw * gw))
    return gh * (e - 1.0), -gh / (gw * gw) * e, gh / (gw ** 4) * e


def sag_and_grad(surf, x, y):
    """Returns (sag, dsag/dx, dsag/dy, valid)."""
    rho = x * x + y * y
    c, k = surf["c"], surf["k"]
    A4, A6, A8, A10 = surf["A"]
    arg = 1.0 - (1.0 + k) * c * c * rho
    valid = arg > 0
    arg_s = torch.where(valid, arg, torch.ones_like(arg))
    sq = torch.sqrt(arg_s)
    g0, g1, _ = _gauss_terms(surf, rho)
    sag = c * rho / (1.0 + sq) + A4 * rho ** 2 + A6 * rho ** 3 + A8 * rho ** 4 + A10 * rho ** 5 \
        + g0
    dsdrho = c / (2.0 * sq) + 2.0 * A4 * rho + 3.0 * A6 * rho ** 2 + 4.0 * A8 * rho ** 3 \
        + 5.0 * A10 * rho ** 4 + g1
    return sag, 2.0 * x * dsdrho, 2.0 * y * dsdrho, valid


def intersect(surf, p, d, tol=1e-13, max_iter=30):
    """Ray-sag intersection by Newton's method on f(t) = p_z + t d_z - z_v - sag(x(t), y(t)).

    The iteration starts at the vertex plane and runs without autograd; one
    final Newton step with autograd gives the exact first-order derivative of
    the root (implicit function theorem).  Returns (t, valid).
    """
    zv = surf["z"]
    with torch.no_grad():
        pd, dd, zvd = p.detach(), d.detach(), zv.detach() if torch.is_tensor(zv) else zv
        sd = {kk: (v.detach() if torch.is_tensor(v) else v) for kk, v in surf.items() if kk != "A"}
        sd["A"] = [a.detach() for a in surf["A"]]
        t = (zvd - pd[:, 2]) / dd[:, 2]
        ok = torch.ones_like(t, dtype=torch.bool)
        conv = torch.zeros_like(ok)
        for _ in range(max_iter):
            x = pd[:, 0] + t * dd[:, 0]
            y = pd[:, 1] + t * dd[:, 1]
            s, sx, sy, v = sag_and_grad(sd, x, y)
            f = pd[:, 2] + t * dd[:, 2] - zvd - s
            fp = dd[:, 2] - sx * dd[:, 0] - sy * dd[:, 1]
            ok = ok & v & (fp.abs() > 1e-300)
            step = torch.where(ok, f / torch.where(ok, fp, torch.ones_like(fp)), torch.zeros_like(f))
            t = t - step
            conv = step.abs() < tol
            if bool(torch.all(conv | ~ok)):
                break
        ok = ok & conv
    t0 = t
    x = p[:, 0] + t0 * d[:, 0]
    y = p[:, 1] + t0 * d[:, 1]
    s, sx, sy, v = sag_and_grad(surf, x, y)
    f = p[:, 2] + t0 * d[:, 2] - zv - s
    fp = d[:, 2] - sx * d[:, 0] - sy * d[:, 1]
    fp = torch.where(ok, fp, torch.ones_like(fp))
    t = t0 - torch.where(ok, f, torch.zeros_like(f)) / fp
    return t, ok & v


def surface_normal(surf, x, y):
    """Unit normal (-s_x, -s_y, 1)/|.|, oriented along +z (propagation side)."""
    _, sx, sy, _ = sag_and_grad(surf, x, y)
    n = torch.stack([-sx, -sy, torch.ones_like(sx)], dim=-1)
    return n / torch.linalg.norm(n, dim=-1, keepdim=True)


def refract(d, nrm, n1, n2):
    """Vector Snell law, normal oriented with the ray: d' = mu d + (cos_t - mu cos_i) N."""
    mu = n1 / n2
    cos_i = (d * nrm).sum(-1)
    rad = 1.0 - mu * mu * (1.0 - cos_i * cos_i)
    ok = rad > 0
    cos_t = torch.sqrt(torch.where(ok, rad, torch.ones_like(rad)))
    dn = mu * d + (cos_t - mu * cos_i)[:, None] * nrm
    return dn, ok


def medium_index(surfs, s, lam):
    """Index of the medium after surface s (s = -1: the object-side air)."""
    if s < 0:
        return 1.0
    return cauchy_index(surfs[s]["nA"], surfs[s]["nB"], lam)


# ----------------------------------------------------------------------------
# Launch.  READING: rays uniformly sampled over the entrance pupil (Benchmark
# section, Systems 1 and 3 and the conformal DOE) as an R x R grid on the
# launch plane; a flat incident wavefront, OPL_0 = d . P_0.
# ----------------------------------------------------------------------------
def launch(cfg, f_idx):
    R = cfg["rays_side"]
    tx, ty = cfg["fields"][f_idx]
    cx, cy = cfg["launch_center"][f_idx]
    h = cfg["launch_half"]
    g = (np.arange(R) + 0.5) / R * 2.0 - 1.0
    X = cx + g[None, :] * h
    Y = cy + g[:, None] * h
    P0 = np.stack([np.broadcast_to(X, (R, R)), np.broadcast_to(Y, (R, R)),
                   np.full((R, R), cfg["launch_z"])], axis=-1).reshape(-1, 3)
    d = np.array([tx, ty, 1.0])
    d = d / np.linalg.norm(d)
    D = np.broadcast_to(d, P0.shape).copy()
    opl = P0 @ d
    return _t(P0), _t(D), _t(opl)


def trace_to_doe(surfs, lam, p, d, opl):
    """Sequential trace through the surfaces before the DOE, then the DOE hit.

    Each refractive surface: Newton intersection, aperture clip, OPL += n t,
    vector Snell.  The DOE surface: intersection and OPL only (its refraction
    is part of the emission of secondary rays).  Returns p, d, opl, alive,
    index of the DOE surface.
    """
    alive = torch.ones(p.shape[0], dtype=torch.bool)
    n_before = 1.0
    for s, surf in enumerate(surfs):
        t, ok = intersect(surf, p, d)
        alive = alive & ok
        t = torch.where(alive, t, torch.zeros_like(t))
        p = p + t[:, None] * d
        opl = opl + n_before * t
        if surf["semi_ap"] > 0:
            alive = alive & ((p[:, 0] ** 2 + p[:, 1] ** 2) <= surf["semi_ap"] ** 2)
        if surf["doe"]:
            return p, d, opl, alive, s
        n_after = medium_index(surfs, s, lam)
        nrm = surface_normal(surf, p[:, 0], p[:, 1])
        dn, ok = refract(d, nrm, n_before, n_after)
        alive = alive & ok
        d = torch.where(alive[:, None], dn, d)
        n_before = n_after
    raise ValueError("system has no DOE surface")


# ----------------------------------------------------------------------------
# Tangent frame at the ray-DOE intersection (Formalism, second paragraph).
# READING: u = normalised projection of the global x axis on the tangent
# plane, v = n x u; a planar DOE gives u = x, v = y, n = z.
# ----------------------------------------------------------------------------
def tangent_frame(surf, p):
    n = surface_normal(surf, p[:, 0], p[:, 1])
    ex = torch.zeros_like(n)
    ex[:, 0] = 1.0
    u = ex - (ex * n).sum(-1, keepdim=True) * n
    u = u / torch.linalg.norm(u, dim=-1, keepdim=True)
    v = torch.cross(n, u, dim=-1)
    return u, v, n


# ----------------------------------------------------------------------------
# DOE patch (Formalism, second paragraph; conformal DOE defined "as projected
# to a flat xy-plane", last demonstration).  READING: P x P samples at the DOE
# pitch centred on the hit, s_m = (m - (P-1)/2) pitch; bilinear interpolation
# of the complex transmission t = A exp(i phi) at the xy projection of each
# sample point; t = 0 outside the map.
# ----------------------------------------------------------------------------
def cis(x):
    """exp(i x) for real x, differentiable."""
    return torch.complex(torch.cos(x), torch.sin(x))


def transmission(phase, amp, field="amp_phase"):
    """Complex transmission of the DOE map: A exp(i phi) (Formalism, second
    paragraph), or the two-phase field exp(i phi1) + exp(i phi2) of the
    beam-splitting demonstration (the second map then holds phi2)."""
    if field == "two_phase":
        return torch.complex(torch.cos(phase) + torch.cos(amp), torch.sin(phase) + torch.sin(amp))
    return torch.complex(amp * torch.cos(phase), amp * torch.sin(phase))


def bilinear_complex(tmap, doe, qx, qy):
    H, W = tmap.shape
    fx = (qx - doe["x0"]) / doe["pitch"]
    fy = (qy - doe["y0"]) / doe["pitch"]
    ix = torch.floor(fx.detach())
    iy = torch.floor(fy.detach())
    wx = fx - ix
    wy = fy - iy
    ix = ix.long()
    iy = iy.long()
    out = torch.zeros(qx.shape, dtype=CT)
    for dy, wyv in ((0, 1.0 - wy), (1, wy)):
        for dx, wxv in ((0, 1.0 - wx), (1, wx)):
            jx = ix + dx
            jy = iy + dy
            inside = (jx >= 0) & (jx < W) & (jy >= 0) & (jy < H)
            val = tmap[jy.clamp(0, H - 1), jx.clamp(0, W - 1)]
            val = torch.where(inside, val, torch.zeros_like(val))
            out = out + (wxv * wyv) * val
    return out


def patch_field(tmap, doe, p, u, v, P):
    """U[r, n, m] = t(xy(p + s_m u + s_n v)) -- rows along v, columns along u."""
    pitch = doe["pitch"]
    s = (torch.arange(P, dtype=DT) - (P - 1) / 2.0) * pitch
    q = p[:, None, None, :] + s[None, None, :, None] * u[:, None, None, :] \
        + s[None, :, None, None] * v[:, None, None, :]
    return bilinear_complex(tmap, doe, q[..., 0], q[..., 1])


# ----------------------------------------------------------------------------
# Local angular spectrum (Formalism, second paragraph; zero padding in the
# patch-size study and System 3).  Plain definition:
#   U~[j] = sum_{m,n} U[n,m] exp(-i kappa_j . (s_m, s_n)),
#   kappa_j = 2 pi j / (M pitch), j in [-M/2, M/2)^2, M = pad * P.
# Evaluated as a zero-padded FFT times the phase of the patch-centre reference.
# Output is in shifted order: index (j_y + M/2, j_x + M/2).
# ----------------------------------------------------------------------------
def angular_spectrum(U, M):
    R, P, _ = U.shape
    X = torch.fft.fft2(U, s=(M, M))
    j = torch.arange(M) - M // 2
    idx = torch.remainder(j, M)
    X = X[:, idx][:, :, idx]
    ph = math.pi * (P - 1) / M * j.to(DT)
    ref = cis(ph[:, None] + ph[None, :])
    return X * ref[None]


def angular_spectrum_bruteforce(U, M, pitch=1.0):
    """The explicit double sum of the definition, for tiny inputs only."""
    R, P, _ = U.shape
    s = (np.arange(P) - (P - 1) / 2.0) * pitch
    kap = 2 * np.pi * (np.arange(M) - M // 2) / (M * pitch)
    E = np.exp(-1j * kap[:, None] * s[None, :])   # [j, m]
    Un = U.detach().numpy()
    # out[r, j_y, j_x] = sum_{n, m} U[r, n, m] E[j_x, m] E[j_y, n]
    return np.einsum("rnm,am,bn->rba", Un, E, E)


def wavevectors(k_in_t, M, pitch):
    """K_j = k_in,t + kappa_j  (tilt as a continuous shift; READING)."""
    kap = TWO_PI * (torch.arange(M, dtype=DT) - M // 2) / (M * pitch)
    Ku = k_in_t[:, 0, None, None] + kap[None, None, :]
    Kv = k_in_t[:, 1, None, None] + kap[None, :, None]
    return Ku.expand(-1, M, M), Kv.expand(-1, M, M)


# ----------------------------------------------------------------------------
# Sampling of secondary wavevectors and their weights (Formalism, Eq. 1, the
# reparameterised sampling of Fig. 1c, and the sampling-density study).
#   MAG : p_j = |U~_j| / S over propagating bins, S = sum |U~|
#   UNI : p_j = 1 / |Pi|
#   FULL: every propagating bin once, weight U~_j / M^2 (the deterministic
#         limit that the Monte Carlo estimate converges to).
# Draw by inverse CDF in shifted column-major bin order, linear bin index
# J = (j_x + M/2) M + (j_y + M/2), J = min{j : C_j > u S},
# distributionally identical to the arg-max of N Gumbel-perturbed replicas of
# log p (Gumbel-max theorem).  READING: weight = U~_J / (M^2 N p_J): the
# Monte Carlo mean of Eq. 1 with the 1/N and 1/M^2 normalisations.
# ----------------------------------------------------------------------------
def draw_bins(mag, prop, u, sampling):
    """mag, prop: [R, M*M] (numpy, shifted column-major bin order); u: [R, N].
    Returns J [R, N] (int64, -1 where the ray has no propagating weight) and S [R]."""
    w = np.where(prop, mag if sampling == "mag" else 1.0, 0.0)
    cdf = np.cumsum(w, axis=1)
    S = cdf[:, -1]
    J = np.full(u.shape, -1, dtype=np.int64)
    for r in range(u.shape[0]):
        if S[r] > 0:
            last = int(np.nonzero(w[r] > 0)[0][-1])
            J[r] = np.minimum(np.searchsorted(cdf[r], u[r] * S[r], side="right"), last)
    return J, S


# ----------------------------------------------------------------------------
# Conventional trace of secondary rays to the sensor and the coherent sensor
# field of Eq. 2:  U(x, y) = sum_i a_i exp[i k (OPL_i + dr_i(x, y))] <n, d_i>,
# READING: dr = n_s d . (X - r_s) (plane-wave tilt across the sensor),
# <n, d> = |d_z|, point samples at pixel centres X = X_c + (m, n) pitch.
# ----------------------------------------------------------------------------
def trace_post_doe(surfs, s_doe, lam, p, d, opl, sensor_z, reflective=False):
    """Secondaries from the DOE hit through the surfaces after it to the sensor;
    after a reflective DOE they travel back through the incident medium (no
    surface between the DOE and the sensor)."""
    alive = torch.ones(p.shape[0], dtype=torch.bool)
    n_before = medium_index(surfs, s_doe - 1 if reflective else s_doe, lam)
    if reflective:
        t = (sensor_z - p[:, 2]) / d[:, 2]
        alive = alive & (t > 0)
        return p + t[:, None] * d, d, opl + n_before * t, alive, n_before
    for s in range(s_doe + 1, len(surfs)):
        surf = surfs[s]
        t, ok = intersect(surf, p, d)
        alive = alive & ok
        t = torch.where(alive, t, torch.zeros_like(t))
        p = p + t[:, None] * d
        opl = opl + n_before * t
        if surf["semi_ap"] > 0:
            alive = alive & ((p[:, 0] ** 2 + p[:, 1] ** 2) <= surf["semi_ap"] ** 2)
        n_after = medium_index(surfs, s, lam)
        nrm = surface_normal(surf, p[:, 0], p[:, 1])
        dn, ok = refract(d, nrm, n_before, n_after)
        alive = alive & ok
        d = torch.where(alive[:, None], dn, d)
        n_before = n_after
    t = (sensor_z - p[:, 2]) / d[:, 2]
    alive = alive & (t > 0)
    p = p + t[:, None] * d
    opl = opl + n_before * t
    return p, d, opl, alive, n_before


def sensor_field(amp, phi0, wx, wy, Q, chunk=1 << 15):
    """Direct Eq. 2 on the Q x Q pixel grid as separable complex128 products:
    U[n, m] = sum_s c_s exp(i wx_s m) exp(i wy_s n), m, n in [-Q/2, Q/2)."""
    m = torch.arange(Q, dtype=DT) - Q // 2
    U = torch.zeros(Q, Q, dtype=CT)
    Ns = amp.shape[0]
    for a in range(0, Ns, chunk):
        b = min(Ns, a + chunk)
        c = amp[a:b] * cis(phi0[a:b])
        Ex = cis(wx[a:b, None] * m[None, :])
        Ey = cis(wy[a:b, None] * m[None, :])
        U = U + Ey.transpose(0, 1) @ (c[:, None] * Ex)
    return U


# ----------------------------------------------------------------------------
# One (wavelength, field) pair, end to end.
# ----------------------------------------------------------------------------
def local_radius(surf, x, y):
    """Smallest principal radius of curvature of a rotationally symmetric surface
    z(r) at (x, y): meridional z'' / (1 + z'^2)^(3/2), sagittal z' / (r (1 + z'^2)^(1/2))
    (-> z''(0) on axis); infinite for a plane."""
    rho = x * x + y * y
    r = torch.sqrt(rho)
    c, k = surf["c"], surf["k"]
    A4, A6, A8, A10 = surf["A"]
    arg = 1.0 - (1.0 + k) * c * c * rho
    sq = torch.sqrt(torch.where(arg > 0, arg, torch.ones_like(arg)))
    _, g1, g2 = _gauss_terms(surf, rho)
    d1 = c / (2.0 * sq) + 2.0 * A4 * rho + 3.0 * A6 * rho ** 2 + 4.0 * A8 * rho ** 3 \
        + 5.0 * A10 * rho ** 4 + g1                                # dz/d(rho)
    d2 = c * (1.0 + k) * c * c / (4.0 * sq ** 3) + 2.0 * A4 + 6.0 * A6 * rho \
        + 12.0 * A8 * rho ** 2 + 20.0 * A10 * rho ** 3 + g2        # d2z/d(rho)2
    zp = 2.0 * r * d1
    zpp = 2.0 * d1 + 4.0 * rho * d2
    km = zpp / (1.0 + zp * zp) ** 1.5
    ks = torch.where(r > 0, 2.0 * d1 / torch.sqrt(1.0 + zp * zp), zpp)
    kmax = torch.maximum(km.abs(), ks.abs())
    return torch.where(kmax > 0, 1.0 / torch.where(kmax > 0, kmax, torch.ones_like(kmax)),
                       torch.full_like(kmax, math.inf))


def patch_classes(cfg):
    """Candidate patch sides, largest first: patch_p and cfg["patch_classes"]."""
    return sorted({int(cfg["patch_p"])} | {int(q) for q in cfg.get("patch_classes", [])},
                  reverse=True)


# ----------------------------------------------------------------------------
# Adaptive patch sizing (Conclusion: future work on adaptive patch sizing that
# balances local diffraction accuracy against propagation cost).  READING Q31:
# a patch resolves the diffraction orders of a locally periodic map when it
# spans K local periods; the ray takes the smallest candidate side with
# P pitch >= K Lambda_loc, Lambda_loc = 2 pi / |grad phi| at the map pixel
# nearest the hit, and the largest side where the map is flatter than that.
# The gradient is the mean of the two one-pixel differences of the phase, each
# wrapped to [-pi, pi] (exact for linear and quadratic phases, valid for local
# periods above two pixels, the map's Nyquist limit); the pixel is clamped one
# away from the map edge.  Combined with Eq. 4, the ray takes the smaller side.
# ----------------------------------------------------------------------------
def wrap_phase(a):
    """a - 2 pi round(a / 2 pi): the phase difference in [-pi, pi]."""
    return a - TWO_PI * np.rint(a / TWO_PI)


def local_phase_gradient2(phase, doe, x, y):
    """|grad phi|^2 (rad^2/mm^2) at the map pixel nearest each (x, y)."""
    H, W = phase.shape
    pitch = doe["pitch"]
    jx = np.clip(np.rint((x - doe["x0"]) / pitch), 1, W - 2).astype(np.int64)
    jy = np.clip(np.rint((y - doe["y0"]) / pitch), 1, H - 2).astype(np.int64)
    c = phase[jy, jx]
    gx = (wrap_phase(phase[jy, jx + 1] - c) + wrap_phase(c - phase[jy, jx - 1])) / (2.0 * pitch)
    gy = (wrap_phase(phase[jy + 1, jx] - c) + wrap_phase(c - phase[jy - 1, jx])) / (2.0 * pitch)
    return gx * gx + gy * gy


def bandwidth_sides(phase, doe, x, y, cands, K):
    """Smallest candidate side spanning K local periods ((P pitch)^2 |grad phi|^2
    >= (2 pi K)^2), else the largest; cands sorted largest first."""
    g2 = local_phase_gradient2(phase, doe, x, y)
    out = np.full(x.shape[0], cands[0], dtype=np.int64)
    lim = (TWO_PI * K) * (TWO_PI * K)
    for i in range(x.shape[0]):
        for P in reversed(cands):
            D = P * doe["pitch"]
            if D * D * g2[i] >= lim:
                out[i] = P
                break
    return out


def ray_patch_sides(surf, p, pitch, cfg, phase_map=None, doe=None):
    """Per-ray patch side by the curvature bound of Eq. 4: the largest candidate
    P with arcsin(P pitch / 2 R_loc) <= eps (READING: R_loc the smallest principal
    radius at the hit); the smallest candidate when none qualifies.  With
    cfg["bw_periods"] = K > 0, the smaller of that side and the bandwidth side
    (adaptive patch sizing, READING Q31) of the phase map."""
    cands = patch_classes(cfg)
    if len(cands) == 1:
        return np.full(p.shape[0], cands[0], dtype=np.int64)
    K = float(cfg.get("bw_periods", 0.0))
    if K > 0:
        if phase_map is None:
            raise ValueError("adaptive patch sizing needs the phase map")
        xy = p[:, :2].detach().numpy()
        bw = bandwidth_sides(np.asarray(phase_map, dtype=np.float64), doe, xy[:, 0], xy[:, 1],
                             cands, K)
        return np.minimum(ray_patch_sides(surf, p, pitch, dict(cfg, bw_periods=0.0)), bw)
    eps = float(cfg.get("curv_eps", 0.1))
    R = local_radius(surf, p[:, 0].detach(), p[:, 1].detach()).detach().numpy()
    out = np.full(p.shape[0], cands[-1], dtype=np.int64)
    for i, Rl in enumerate(R):
        for P in cands:
            D = P * pitch
            if math.isinf(Rl) or (D <= 2.0 * Rl and math.asin(D / (2.0 * Rl)) <= eps):
                out[i] = P
                break
    return out


def class_draws(cfg, P):
    """Draws per ray of patch side P.  Adaptive ray sampling (READING Q32):
    with cfg["class_draws"], N (P / P_0)^2 rounded down (at least one), the Monte
    Carlo budget per spectrum bin kept across classes; else N."""
    N = int(cfg["n_ssr"])
    if not cfg.get("class_draws", False):
        return N
    P0 = patch_classes(cfg)[0]
    return max(1, (N * P * P) // (P0 * P0))


def detach_pdf(cfg):
    """Gradient mode with the sampling density held constant (the unbiased variant
    of the frozen-draw derivative of Eq. 1)."""
    return bool(cfg.get("detach_pdf", False)) or cfg.get("grad", "G1") == "G1_DETACH"


def pair_forward(system, cfg, tmap, lam_idx, f_idx, values=None, replay=None,
                 keep=False, ray_subset=None, phase_map=None):
    """Returns dict with field U [Q, Q] (complex, differentiable), PSF, and
    (if keep) intermediate quantities for stage-level comparison.  phase_map:
    the phase map (numpy), for adaptive patch sizing."""
    surfs, sensor_z = build_surfaces(system, values)
    doe = system["doe"]
    lam = cfg["lambdas"][lam_idx]
    k0 = TWO_PI / lam
    Nd = cfg["n_ssr"]
    Q = cfg["psf_q"]
    F = len(cfg["fields"])
    pair = lam_idx * F + f_idx
    sampling = cfg["sampling"]

    p, d, opl = launch(cfg, f_idx)
    ray_ids = np.arange(p.shape[0])
    if ray_subset is not None:
        ray_ids = np.asarray(ray_subset)
        p, d, opl = p[ray_ids], d[ray_ids], opl[ray_ids]
    p, d, opl, alive, s_doe = trace_to_doe(surfs, lam, p, d, opl)
    # The DOE is the stop: rays outside the map are terminated (READING).
    H, W = tmap.shape
    fx = (p[:, 0] - doe["x0"]) / doe["pitch"]
    fy = (p[:, 1] - doe["y0"]) / doe["pitch"]
    alive = alive & (fx >= -0.5) & (fx <= W - 0.5) & (fy >= -0.5) & (fy <= H - 0.5)
    out = {}
    if keep:
        out.update(p_doe=p.detach().clone(), d_doe=d.detach().clone(),
                   opl_doe=opl.detach().clone(), alive=alive.clone(), ray_ids=ray_ids)
    surf_doe = surfs[s_doe]
    reflective = bool(doe.get("reflective", False))
    n_in = medium_index(surfs, s_doe - 1, lam)
    # READING: a reflective DOE sends its secondaries back into the incident medium
    n_out = n_in if reflective else medium_index(surfs, s_doe, lam)
    k_out = k0 * n_out
    u, v, nrm = tangent_frame(surf_doe, p)
    k_in_t = k0 * n_in * torch.stack([(d * u).sum(-1), (d * v).sum(-1)], dim=-1)

    # patch classes (Eq. 4); one class unless cfg lists several candidate sides
    sides = ray_patch_sides(surf_doe, p, doe["pitch"], cfg, phase_map, doe)
    # READING: unit amplitude per live ray, times (P_0 / P)^2 for a ray whose
    # patch side P is below the largest candidate P_0: the rays' patches cover
    # the DOE uniformly (Formalism), so on one ray grid every part of the DOE
    # counts equally whatever the side of the patches that cover it
    P0 = patch_classes(cfg)[0]
    amp_in = alive.to(DT) * torch.as_tensor((P0 / sides.astype(np.float64)) ** 2)
    R = p.shape[0]
    J_all = np.full((R, Nd), -1, dtype=np.int64) if sampling != "full" else None
    parts = []
    for P in sorted(set(sides.tolist()), reverse=True):
        sel = np.nonzero(sides == P)[0]
        rsel = torch.as_tensor(sel)
        Nk = class_draws(cfg, P) if sampling != "full" else Nd
        rep = None
        if replay is not None:
            rep = np.asarray(replay, dtype=np.int64).reshape(R, Nd)[sel][:, :Nk]
        part = _class_secondaries(cfg, tmap, doe, pair, ray_ids[sel], P, p[rsel], opl[rsel],
                                  amp_in[rsel], u[rsel], v[rsel], nrm[rsel], k_in_t[rsel],
                                  alive[rsel], k_out, rep, sampling, Nk)
        if J_all is not None:
            J_all[sel, :Nk] = part["J"]
        parts.append((sel, part))
        if keep and len(parts) == 1 and len(set(sides.tolist())) == 1:
            out.update(spectrum=part["Ut"].detach(), prop=part["prop"])
    rr = torch.cat([torch.as_tensor(sel)[part["rr"]] for sel, part in parts])
    w = torch.cat([part["w"] for _, part in parts])
    Kus = torch.cat([part["Kus"] for _, part in parts])
    Kvs = torch.cat([part["Kvs"] for _, part in parts])
    ds = emit_direction(Kus, Kvs, u[rr], v[rr], nrm[rr], k_out, -1.0 if reflective else 1.0)
    a_s = amp_in[rr] * w
    ps, dsn, opls, ok2, n_s = trace_post_doe(surfs, s_doe, lam, p[rr], ds, opl[rr], sensor_z,
                                             reflective)
    a_s = torch.where(ok2, a_s, torch.zeros_like(a_s))
    lc = cfg["psf_center"][lam_idx][f_idx]
    Xc = torch.stack([_t(lc[0]), _t(lc[1]), sensor_z * torch.ones((), dtype=DT)])
    phi0 = k0 * (opls + n_s * (dsn * (Xc[None, :] - ps)).sum(-1))
    wx = k0 * n_s * cfg["psf_pitch"] * dsn[:, 0]
    wy = k0 * n_s * cfg["psf_pitch"] * dsn[:, 1]
    amp = a_s * dsn[:, 2].abs()
    U = sensor_field(amp, phi0, wx, wy, Q)
    out["U"] = U
    out["psf"] = (U.real ** 2 + U.imag ** 2)
    if keep:
        out.update(k_in_t=k_in_t.detach(), J=J_all, sides=sides, amp=amp.detach(),
                   phi0=phi0.detach(), wx=wx.detach(), wy=wy.detach(), w=w.detach(),
                   frame=(u.detach(), v.detach(), nrm.detach()))
    return out


def emit_direction(Ku, Kv, u, v, nrm, k_out, sign=1.0):
    """Unit direction of the plane wave with tangential wavevector (Ku, Kv) in
    the frame (u, v, n) leaving the DOE into the medium of wavenumber k_out
    (Formalism, second paragraph): (Ku u + Kv v + sign sqrt(k_out^2 - |K|^2) n) / k_out,
    the forward-going root (sign +1) for a transmissive DOE, the backward one
    (sign -1, the normal component flipped) for a reflective DOE."""
    kz2 = k_out * k_out - Ku * Ku - Kv * Kv
    kz = torch.sqrt(torch.where(kz2 > 0, kz2, torch.ones_like(kz2)))
    return (Ku[:, None] * u + Kv[:, None] * v + sign * kz[:, None] * nrm) / k_out


def _class_secondaries(cfg, tmap, doe, pair, ray_ids, P, p, opl, amp_in, u, v, nrm, k_in_t,
                       alive, k_out, replay, sampling, Nd):
    """Patch spectra, evanescent cut, draws (or FULL) and Eq. 1 weights of the
    rays of one patch class (side P, M = pad P).  Returns the secondary rays as
    (parent index rr into the class's rays, weight w, tangential wavevector)."""
    M = cfg["pad"] * P
    Upatch = patch_field(tmap, doe, p, u, v, P)
    Ut = angular_spectrum(Upatch, M)                        # [R, M, M]
    Ku, Kv = wavevectors(k_in_t, M, doe["pitch"])
    K2 = Ku * Ku + Kv * Kv
    prop = (K2 < k_out * k_out) & alive[:, None, None]
    R = p.shape[0]
    # flatten j_x-major: linear bin index J = (j_x + M/2) M + (j_y + M/2)
    Utf = Ut.transpose(1, 2).reshape(R, M * M)
    propf = prop.transpose(1, 2).reshape(R, M * M)
    J = None
    if sampling == "full":
        rr, jj = torch.nonzero(propf, as_tuple=True)
        w = Utf[rr, jj] / (M * M)
    else:
        mag = Utf.detach().abs().numpy()
        pn = propf.numpy()
        if replay is not None:
            J = np.asarray(replay, dtype=np.int64).reshape(R, Nd)
        else:
            uu = draw_uniforms(cfg["seed"], pair, ray_ids, Nd, stream=cfg.get("draw_stream", 0))
            J, _ = draw_bins(mag, pn, uu, sampling)
        rr = torch.arange(R).repeat_interleave(Nd)
        jj = torch.as_tensor(np.maximum(J, 0).reshape(-1))
        UJ = Utf[rr, jj]
        valid = torch.as_tensor((J >= 0).reshape(-1)) & propf[rr, jj]
        zero = torch.zeros_like(UJ)
        if sampling == "mag":
            Sg = torch.where(propf, Utf.abs(), torch.zeros((), dtype=DT)).sum(1)
            magJ = UJ.abs()
            ok = valid & (magJ > 0)
            magJ = torch.where(ok, magJ, torch.ones_like(magJ))
            scale = Sg[rr] / (M * M * Nd * magJ)             # 1 / (M^2 N p_J)
            if detach_pdf(cfg):
                # READING: the density p_J = |U~_J| / S enters as a constant; the
                # gradient then flows through U~_J alone, and its mean over the
                # draws is the FULL-mode gradient of any loss linear in the field
                scale = scale.detach()
            w = torch.where(ok, UJ * scale, zero)
        else:
            nprop = propf.sum(1).to(DT)
            w = torch.where(valid, UJ * (nprop[rr] / (M * M * Nd)), zero)
    # Emission: direction from the tangential wavevector (Formalism; READING Q1).
    jx = jj // M
    jy = jj % M
    Kus = Ku[rr, jy, jx]
    Kvs = Kv[rr, jy, jx]
    if sampling != "full" and cfg.get("grad", "G1") == "G2":
        w, Kus, Kvs = _straight_through(cfg, pair, ray_ids, J, Utf, propf, Ku, Kv, w, Kus, Kvs,
                                        rr, valid, sampling, M, Nd)
    return dict(rr=rr, jj=jj, w=w, Kus=Kus, Kvs=Kvs, J=J, Ut=Ut, prop=prop)


# ----------------------------------------------------------------------------
# Gumbel-softmax straight-through relaxation of the draws (reparameterised
# sampling, Fig. 1c; G2).  Per draw i the hard one-hot y_hard(J_i) is kept in
# value while the gradient flows through
#     y_soft = softmax((log p + z_i) / tau),
# z_i the Gumbel perturbations of the replica of p that draw i came from,
# generated conditioned on argmax = J_i: the maximum G*_i = log sum p + Gumbel
# (from its own uniform) sits at J_i, every other bin takes an unconditioned
# Gumbel g_k = log p_k + Gumbel truncated below G*_i,
#     g_k = -log(exp(-G*_i) + exp(-(log p_k + Gumbel))),
# (the top-down construction of Maddison, Tarlow & Minka, "A* sampling", 2014),
# and z = g - log p is held fixed (noise).  The relaxed weight and wavevector
# of the draw are sum_k y_k w_k and sum_k y_k K_k with
#     y = y_hard - stopgrad(y_soft) + y_soft.
# READING: tau = 1 unless cfg["tau"] says otherwise; both the amplitude and the
# wavevector are relaxed (the paper's softmax carries "the full scattering
# wavevector distribution").  Parity unpinned beyond this construction (a
# surrogate gradient has no finite-difference truth); pinned limits: G2 == G1
# for uniform sampling, and G2 -> G1 as tau -> 0.
# ----------------------------------------------------------------------------
def conditional_gumbels(logp, J, u_top, u_bin):
    """Perturbed log-probabilities phi[r, i, k] whose maximum over k is at J[r, i]:
    logp [R, K] (-inf where p = 0), J [R, N], uniforms u_top [R, N], u_bin [R, N, K]."""
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        lse = np.log(np.sum(np.exp(logp), axis=1))                       # log sum p
        gstar = lse[:, None] - np.log(-np.log(u_top))                    # [R, N]
        ghat = logp[:, None, :] - np.log(-np.log(u_bin))                 # [R, N, K]
        phi = -np.logaddexp(-gstar[:, :, None], -ghat)
    np.put_along_axis(phi, J[:, :, None], gstar[:, :, None], axis=2)
    return phi


def relaxed_weights(Utf, propf, sampling, M, Nd):
    """Per bin k of every ray: log p_k, and the Eq. 1 weight w_k = U~_k / (M^2 N p_k)
    that draw i would carry had it landed on k (the quantities the softmax
    relaxation mixes); -inf / 0 on bins that cannot be drawn.  Returns
    (logp, w_all, live), each [R, M*M]."""
    absU = Utf.abs()
    live = propf & (absU > 0) if sampling == "mag" else propf
    if sampling == "mag":
        S = torch.where(propf, absU, torch.zeros((), dtype=DT)).sum(1)
        logp = torch.log(torch.where(live, absU, torch.ones_like(absU))) - torch.log(
            torch.where(S > 0, S, torch.ones_like(S)))[:, None]
        w_all = Utf * (S[:, None] / (M * M * Nd * torch.where(live, absU, torch.ones_like(absU))))
    else:
        nprop = propf.sum(1).to(DT)
        logp = -torch.log(torch.where(nprop > 0, nprop, torch.ones_like(nprop)))[:, None] * \
            torch.ones_like(absU)
        w_all = Utf * (nprop[:, None] / (M * M * Nd))
    w_all = torch.where(live, w_all, torch.zeros_like(w_all))
    neg_inf = torch.full((), -math.inf, dtype=DT)
    logp = torch.where(live, logp, neg_inf)
    return logp, w_all, live


def _straight_through(cfg, pair, ray_ids, J, Utf, propf, Ku, Kv, w_hard, Kus, Kvs, rr, valid,
                      sampling, M, Nd):
    R = Utf.shape[0]
    tau = float(cfg.get("tau", 1.0))
    Kuf = Ku.transpose(1, 2).reshape(R, M * M)
    Kvf = Kv.transpose(1, 2).reshape(R, M * M)
    logp, w_all, live = relaxed_weights(Utf, propf, sampling, M, Nd)
    # Gumbel perturbations conditioned on argmax = J (numbers: no gradient)
    ut = g2_top_uniforms(cfg["seed"], pair, ray_ids, Nd)                 # [R, N]
    ub = g2_bin_uniforms(cfg["seed"], pair, ray_ids, Nd, M * M)          # [R, N, K]
    lp = logp.detach().numpy()
    Jc = np.maximum(J, 0)
    phi = conditional_gumbels(lp, Jc, ut, ub)
    with np.errstate(invalid="ignore"):
        z = np.where(np.isfinite(lp)[:, None, :], phi - lp[:, None, :], 0.0)
    zt = torch.as_tensor(z)
    y_soft = torch.softmax((logp[:, None, :] + zt) / tau, dim=2)         # [R, N, K]
    y_hard = torch.zeros_like(y_soft)
    y_hard.scatter_(2, torch.as_tensor(Jc)[:, :, None], 1.0)
    y = y_hard - y_soft.detach() + y_soft
    a = (y * w_all[:, None, :]).sum(2).reshape(-1)
    Kr = (y * Kuf[:, None, :]).sum(2).reshape(-1)
    Kv_r = (y * Kvf[:, None, :]).sum(2).reshape(-1)
    ok = valid & (w_hard != 0)
    a = torch.where(ok, a, torch.zeros_like(a))
    Kr = torch.where(ok, Kr, Kus)
    Kv_r = torch.where(ok, Kv_r, Kvs)
    return a, Kr, Kv_r


# ----------------------------------------------------------------------------
# Whole stack, loss (Eq. 5) and gradients.
# ----------------------------------------------------------------------------
def eq5_loss(I, T):
    """Normalised least squares of Eq. 5 with the closed-form optimal alpha
    (READING: alpha* = <I,T>/<I,I> per PSF)."""
    ii = (I * I).sum()
    it = (I * T).sum()
    alpha = it / ii
    return ((alpha * I - T) ** 2).sum()


def psf_stack(system, cfg, phase, amp, values=None, replays=None, pairs=None, keep=False):
    """PSF stack [L, F, Q, Q] (numpy) plus per-pair aux dicts."""
    L = len(cfg["lambdas"])
    F = len(cfg["fields"])
    Q = cfg["psf_q"]
    tmap = transmission(_t(phase), _t(amp), system["doe"].get("field", "amp_phase"))
    vals = None if values is None else _t(values)
    out = np.zeros((L, F, Q, Q))
    aux = {}
    with torch.no_grad():
        for l in range(L):
            for f in range(F):
                pr = l * F + f
                if pairs is not None and pr not in pairs:
                    continue
                rep = None if replays is None else replays.get(pr)
                r = pair_forward(system, cfg, tmap, l, f, vals, rep, keep=keep,
                                 phase_map=phase)
                out[l, f] = r["psf"].numpy()
                aux[pr] = r
    return out, aux


def loss_and_grad(system, cfg, phase, amp, values, target, replays=None, want_grad=True):
    """Eq. 5 summed over all pairs and its gradient w.r.t. the DOE phase map,
    the amplitude map and the normalised lens parameters (torch autograd in
    float64; frozen draws, i.e. the a.e. derivative with the index set fixed)."""
    L = len(cfg["lambdas"])
    F = len(cfg["fields"])
    ph = _t(phase).clone().requires_grad_(want_grad)
    am = _t(amp).clone().requires_grad_(want_grad)
    vals = _t(values).clone().requires_grad_(want_grad)
    total = 0.0
    psfs = np.zeros((L, F, cfg["psf_q"], cfg["psf_q"]))
    idx = {}
    for l in range(L):
        for f in range(F):
            pr = l * F + f
            tmap = transmission(ph, am, system["doe"].get("field", "amp_phase"))
            rep = None if replays is None else replays.get(pr)
            r = pair_forward(system, cfg, tmap, l, f, vals, rep, keep=True,
                             phase_map=phase)
            Lp = eq5_loss(r["psf"], _t(target[l, f]))
            if want_grad:
                Lp.backward()
            total += float(Lp.detach())
            psfs[l, f] = r["psf"].detach().numpy()
            idx[pr] = r["J"]
    g = None
    if want_grad:
        g = dict(phase=ph.grad.numpy().copy(), amp=am.grad.numpy().copy(),
                 lens=(vals.grad.numpy().copy() if vals.grad is not None
                       else np.zeros(vals.shape)))
    return total, g, psfs, idx


# ----------------------------------------------------------------------------
# Two DOEs in sequence (Formalism, first paragraph: the construction extends to
# systems with more than one DOE, since every secondary ray is propagated by
# conventional ray tracing).  READING (cascade):
# * a secondary of the first DOE is traced through the surfaces between the
#   DOEs to the second DOE's surface, where it is an incident ray: a plane-wave
#   wavelet whose complex amplitude is the Eq. 1 weight it left the first DOE
#   with and whose phase is its optical path; the second map is the stop of
#   these rays as the first map is of the launched ones;
# * the second DOE applies the same patch, spectrum, draws and Eq. 1 weights
#   to it, with n_ssr2 draws (MAG, UNI) or every propagating bin (FULL): the
#   fan-out N1 N2 per launched ray is bounded by the choice of n_ssr2, and the
#   nested estimator stays unbiased for any n_ssr2 >= 1;
# * one patch side, pad factor and sampling mode for both DOEs;
# * the secondaries of the first DOE form a grid of side R n1 (n1^2 = N1,
#   n1 = M under FULL): secondary i of launched ray (iy, ix) is grid ray
#   (iy n1 + i div n1, ix n1 + i mod n1), i the draw (MAG, UNI) or the linear
#   bin index J (FULL); the second DOE's draws take that grid ray's id and
#   Philox stream 1.
# ----------------------------------------------------------------------------
def trace_between(surfs, s_from, s_to, lam, p, d, opl):
    """From the hit on surface s_from to the hit on surface s_to: the surfaces
    in between refract (intersection, aperture clip, OPL += n t, vector Snell);
    s_to is intersected and clipped only."""
    alive = torch.ones(p.shape[0], dtype=torch.bool)
    n_before = medium_index(surfs, s_from, lam)
    for s in range(s_from + 1, s_to + 1):
        surf = surfs[s]
        t, ok = intersect(surf, p, d)
        alive = alive & ok
        t = torch.where(alive, t, torch.zeros_like(t))
        p = p + t[:, None] * d
        opl = opl + n_before * t
        if surf["semi_ap"] > 0:
            alive = alive & ((p[:, 0] ** 2 + p[:, 1] ** 2) <= surf["semi_ap"] ** 2)
        if s == s_to:
            break
        n_after = medium_index(surfs, s, lam)
        nrm = surface_normal(surf, p[:, 0], p[:, 1])
        dn, ok = refract(d, nrm, n_before, n_after)
        alive = alive & ok
        d = torch.where(alive[:, None], dn, d)
        n_before = n_after
    return p, d, opl, alive


def inside_map(p, doe, H, W):
    """Hit inside the map (the stop): pixel coordinate within [-1/2, side - 1/2]."""
    fx = (p[:, 0] - doe["x0"]) / doe["pitch"]
    fy = (p[:, 1] - doe["y0"]) / doe["pitch"]
    return (fx >= -0.5) & (fx <= W - 0.5) & (fy >= -0.5) & (fy <= H - 0.5)


def cascade_side(cfg):
    """n1: side of the block of grid rays that one launched ray's first-DOE
    secondaries occupy."""
    if cfg["sampling"] == "full":
        return cfg["pad"] * cfg["patch_p"]
    n1 = int(round(math.sqrt(cfg["n_ssr"])))
    if n1 * n1 != cfg["n_ssr"]:
        raise ValueError("a cascade needs n_ssr = n1^2")
    return n1


def _doe_stage(cfg, surfs, s_doe, doe, tmap, lam, pair, ray_ids, p, d, opl, alive, Nd, replay):
    """Frame, spectrum, draws and Eq. 1 weights of the rays incident on one DOE
    (one patch class), and the directions of their secondaries."""
    k0 = TWO_PI / lam
    n_in = medium_index(surfs, s_doe - 1, lam)
    k_out = k0 * medium_index(surfs, s_doe, lam)
    u, v, nrm = tangent_frame(surfs[s_doe], p)
    k_in_t = k0 * n_in * torch.stack([(d * u).sum(-1), (d * v).sum(-1)], dim=-1)
    part = _class_secondaries(cfg, tmap, doe, pair, ray_ids, cfg["patch_p"], p, opl,
                              alive.to(DT), u, v, nrm, k_in_t, alive, k_out, replay,
                              cfg["sampling"], Nd)
    rr = part["rr"]
    ds = emit_direction(part["Kus"], part["Kvs"], u[rr], v[rr], nrm[rr], k_out)
    return part, ds


def cascade_pair_forward(system, cfg, tmaps, lam_idx, f_idx, values=None, replays=(None, None),
                         keep=False):
    """One (wavelength, field) pair through two DOEs: system["does"] describes the
    two maps (the surfaces flagged doe, in order), tmaps their transmissions,
    cfg["n_ssr2"] the draws per ray at the second DOE.  replays: the first DOE's
    indices [R^2, N1] and the second's [(R n1)^2, N2], or None."""
    surfs, sensor_z = build_surfaces(system, values)
    does = system["does"]
    s1, s2 = [i for i, s in enumerate(surfs) if s["doe"]]
    lam = cfg["lambdas"][lam_idx]
    k0 = TWO_PI / lam
    F = len(cfg["fields"])
    pair = lam_idx * F + f_idx
    R = cfg["rays_side"]
    n1 = cascade_side(cfg)
    Rg = R * n1
    N1, N2 = cfg["n_ssr"], cfg["n_ssr2"]
    H, W = tmaps[0].shape
    # first DOE: the single-DOE steps up to the emission
    p, d, opl = launch(cfg, f_idx)
    p, d, opl, alive, s = trace_to_doe(surfs, lam, p, d, opl)
    assert s == s1
    alive = alive & inside_map(p, does[0], H, W)
    part1, ds1 = _doe_stage(cfg, surfs, s1, does[0], tmaps[0], lam, pair, np.arange(R * R),
                            p, d, opl, alive, N1, replays[0])
    rr = part1["rr"]
    slot = part1["jj"] if cfg["sampling"] == "full" else torch.arange(rr.shape[0]) % N1
    # conventional trace to the second DOE, which is the stop of these rays
    p2, d2, opl2, ok = trace_between(surfs, s1, s2, lam, p[rr], ds1, opl[rr])
    ok = ok & inside_map(p2, does[1], H, W)
    a2 = torch.where(ok, part1["w"], torch.zeros_like(part1["w"]))
    # the second DOE's incident rays on the grid of side R n1
    iy = torch.div(rr, R, rounding_mode="floor")
    ix = rr % R
    g = (iy * n1 + torch.div(slot, n1, rounding_mode="floor")) * Rg + ix * n1 + slot % n1
    n2 = Rg * Rg
    P2 = torch.zeros(n2, 3, dtype=DT).index_put((g,), p2)
    D2 = torch.zeros(n2, 3, dtype=DT)
    D2[:, 2] = 1.0
    D2 = D2.index_put((g,), d2)
    O2 = torch.zeros(n2, dtype=DT).index_put((g,), opl2)
    A2 = torch.zeros(n2, dtype=CT).index_put((g,), a2)
    alive2 = torch.zeros(n2, dtype=torch.bool).index_put((g,), ok)
    # second DOE, then the conventional trace to the sensor and Eq. 2
    cfg2 = dict(cfg, n_ssr=N2, draw_stream=1)
    part2, ds2 = _doe_stage(cfg2, surfs, s2, does[1], tmaps[1], lam, pair, np.arange(n2),
                            P2, D2, O2, alive2, N2, replays[1])
    rr2 = part2["rr"]
    a_s = A2[rr2] * part2["w"]
    ps, dsn, opls, ok2, n_s = trace_post_doe(surfs, s2, lam, P2[rr2], ds2, O2[rr2], sensor_z)
    a_s = torch.where(ok2, a_s, torch.zeros_like(a_s))
    lc = cfg["psf_center"][lam_idx][f_idx]
    Xc = torch.stack([_t(lc[0]), _t(lc[1]), sensor_z * torch.ones((), dtype=DT)])
    phi0 = k0 * (opls + n_s * (dsn * (Xc[None, :] - ps)).sum(-1))
    wx = k0 * n_s * cfg["psf_pitch"] * dsn[:, 0]
    wy = k0 * n_s * cfg["psf_pitch"] * dsn[:, 1]
    amp = a_s * dsn[:, 2].abs()
    U = sensor_field(amp, phi0, wx, wy, cfg["psf_q"])
    out = {"U": U, "psf": U.real ** 2 + U.imag ** 2}
    if keep:
        out.update(J1=part1["J"], J2=part2["J"], alive2=alive2, p2=P2.detach(),
                   d2=D2.detach(), opl2=O2.detach(), a2=A2.detach())
    return out


def cascade_psf_stack(system, cfg, phases, amps, values=None, replays=None, keep=False):
    """PSF stack [L, F, Q, Q] of a two-DOE system (maps [2, H, W]) plus per-pair
    aux dicts; replays: {pair: (first DOE's indices, second DOE's)}."""
    L = len(cfg["lambdas"])
    F = len(cfg["fields"])
    Q = cfg["psf_q"]
    tmaps = [transmission(_t(phases[k]), _t(amps[k]), system["does"][k].get("field", "amp_phase"))
             for k in range(2)]
    vals = None if values is None else _t(values)
    out = np.zeros((L, F, Q, Q))
    aux = {}
    with torch.no_grad():
        for l in range(L):
            for f in range(F):
                pr = l * F + f
                rep = (None, None) if replays is None else replays[pr]
                r = cascade_pair_forward(system, cfg, tmaps, l, f, vals, rep, keep=keep)
                out[l, f] = r["psf"].numpy()
                aux[pr] = r
    return out, aux


def cascade_loss_and_grad(system, cfg, phases, amps, target, replays=None, want_grad=True):
    """Eq. 5 summed over the pairs of a two-DOE system and its gradient with
    respect to both DOEs' maps (torch autograd in float64, frozen draws): the
    relayed rays' positions and directions follow from the drawn bins alone, so
    the maps act through the amplitudes.  Returns (loss, {"phase", "amp"} [2, H, W],
    psfs, {pair: (J1, J2)})."""
    L = len(cfg["lambdas"])
    F = len(cfg["fields"])
    ph = _t(np.asarray(phases)).clone().requires_grad_(want_grad)
    am = _t(np.asarray(amps)).clone().requires_grad_(want_grad)
    total = 0.0
    psfs = np.zeros((L, F, cfg["psf_q"], cfg["psf_q"]))
    idx = {}
    for l in range(L):
        for f in range(F):
            pr = l * F + f
            tmaps = [transmission(ph[k], am[k], system["does"][k].get("field", "amp_phase"))
                     for k in range(2)]
            rep = (None, None) if replays is None else replays[pr]
            r = cascade_pair_forward(system, cfg, tmaps, l, f, None, rep, keep=True)
            Lp = eq5_loss(r["psf"], _t(target[l, f]))
            if want_grad:
                Lp.backward()
            total += float(Lp.detach())
            psfs[l, f] = r["psf"].detach().numpy()
            idx[pr] = (r["J1"], r["J2"])
    g = None
    if want_grad:
        g = dict(phase=ph.grad.numpy().copy(), amp=am.grad.numpy().copy())
    return total, g, psfs, idx


# ----------------------------------------------------------------------------
# Figures of merit (patch-size study).
# ----------------------------------------------------------------------------
def ncc(I, Igt):
    """Normalised cross-correlation of Eq. 3 (patch-size study)."""
    I = np.asarray(I, dtype=np.float64)
    Igt = np.asarray(Igt, dtype=np.float64)
    return float((Igt * I).sum() / math.sqrt((Igt ** 2).sum() * (I ** 2).sum()))


def mse(I, Igt):
    return float(np.mean((np.asarray(I) - np.asarray(Igt)) ** 2))


def curvature_error_bound(D, R):
    """Upper bound of the curvature-induced angular-spectrum error for a flat
    patch of side D on a surface of radius R (Eq. 4): eps <= arcsin(D / 2R)."""
    return math.asin(D / (2.0 * R))


def largest_patch(candidates_p, pitch, R_loc, eps):
    """Largest patch side (in samples) whose curvature bound stays below eps."""
    best = None
    for P in sorted(candidates_p):
        if P * pitch <= 2 * R_loc and curvature_error_bound(P * pitch, R_loc) <= eps:
            best = P
    return best
