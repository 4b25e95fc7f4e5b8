"""Thin Python binding of librw.so (the C ABI declared in include/rw.h).

Argument marshalling only: every step of the ray-wave path runs in the HIP
kernels behind the C ABI.  PyTorch supplies device memory and the current
HIP stream.  There is no CPU fallback: if the library is missing, or no GPU
is present, the calls raise.
"""
import ctypes
import hashlib
import json
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librw.so")

RW_SURF_ASPHERE, RW_SURF_PLANE, RW_SURF_GAUSS = 0, 1, 2
FIELDS = {"amp_phase": 0, "two_phase": 1}
PARAM_FIELDS = {"curv": 0, "conic": 1, "A4": 2, "A6": 3, "A8": 4, "A10": 5, "gap": 6}
SAMPLING = {"mag": 0, "uni": 1, "full": 2}
PRECISION = {"fp64": 0, "mixed": 1, "fp32": 2}
GRAD = {"G1": 0, "G2": 1, "G1_DETACH": 2}
RW_STATIC_SCRATCH_BYTES = 256 << 20   # workspace of rw_forward_static (include/rw.h)
AUTOTUNE_CACHE = os.path.join(_HERE, "autotune_cache.json")   # launch shapes by arch + geometry
STATUS = {0: "RW_OK", 1: "RW_ERR_INVALID_ARG", 2: "RW_ERR_SHAPE", 3: "RW_ERR_STATE",
          4: "RW_ERR_NONFINITE", 5: "RW_ERR_OOM", 6: "RW_ERR_HIP", 7: "RW_ERR_UNSUPPORTED"}

EXPORTED = ("rw_plan_create", "rw_plan_create_cascade", "rw_plan_workspace_bytes", "rw_forward", "rw_forward_static",
            "rw_backward", "rw_forward_backward", "rw_set_launch_shape",
            "rw_get_stats", "rw_export_doe_hits", "rw_plan_destroy", "rw_status_string",
            "rw_last_error", "rw_set_profiling", "rw_get_profile", "rw_set_graph",
            "rw_autotune", "rw_adam_step", "rw_patch_dft")
STAGES = ("trace", "doe_fwd", "bin", "spread", "grid_fwd", "grid_bwd", "doe_bwd", "trace_bwd",
          "interp")


class rw_surface(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("carries_doe", ctypes.c_int),
                ("z_vertex", ctypes.c_double), ("curvature", ctypes.c_double),
                ("conic", ctypes.c_double), ("asph", ctypes.c_double * 4),
                ("semi_aperture", ctypes.c_double), ("n_A", ctypes.c_double),
                ("n_B", ctypes.c_double), ("gauss_height", ctypes.c_double),
                ("gauss_width", ctypes.c_double)]


class rw_doe_desc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int), ("pitch", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("reflective", ctypes.c_int),
                ("field", ctypes.c_int)]


class rw_param_ref(ctypes.Structure):
    _fields_ = [("surface", ctypes.c_int), ("field", ctypes.c_int), ("scale", ctypes.c_double)]


class rw_config(ctypes.Structure):
    _fields_ = [("n_lambda", ctypes.c_int), ("lambda_host", ctypes.POINTER(ctypes.c_double)),
                ("n_field", ctypes.c_int), ("field_tan_host", ctypes.POINTER(ctypes.c_double)),
                ("launch_center_host", ctypes.POINTER(ctypes.c_double)),
                ("launch_z", ctypes.c_double), ("launch_half", ctypes.c_double),
                ("rays_side", ctypes.c_int), ("sensor_z", ctypes.c_double),
                ("psf_q", ctypes.c_int), ("psf_pitch", ctypes.c_double),
                ("psf_center_host", ctypes.POINTER(ctypes.c_double)),
                ("patch_p", ctypes.c_int), ("pad_factor", ctypes.c_int), ("n_ssr", ctypes.c_int),
                ("sampling", ctypes.c_int), ("precision", ctypes.c_int), ("batched", ctypes.c_int),
                ("spread_width", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("grad", ctypes.c_int), ("tau", ctypes.c_double),
                ("n_patch_class", ctypes.c_int), ("patch_class_p", ctypes.c_int * 3),
                ("curv_eps", ctypes.c_double), ("check_finite", ctypes.c_int),
                ("record_budget_bytes", ctypes.c_uint64),
                ("bandwidth_periods", ctypes.c_double), ("class_draws", ctypes.c_int),
                ("deterministic", ctypes.c_int)]


class rw_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(STAGES)), ("launches", ctypes.c_uint64 * len(STAGES))]


STATS = ("rays_total", "rays_alive", "secondaries", "killed_no_hit", "killed_aperture",
         "killed_tir", "killed_outside_doe", "secondaries_lost", "evanescent_bins",
         "spectrum_bins")


class rw_stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in STATS] + \
        [("rays_by_class", ctypes.c_uint64 * 4)]


_lib = None
_lib_id = None     # content hash of the loaded library (part of the autotune key)


def load_library(path=LIB_PATH):
    """Load librw.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.rw_plan_create.argtypes = [ctypes.POINTER(rw_surface), ctypes.c_int,
                                   ctypes.POINTER(rw_doe_desc), ctypes.POINTER(rw_param_ref),
                                   ctypes.c_int, ctypes.POINTER(rw_config), ctypes.POINTER(vp)]
    lib.rw_plan_create_cascade.argtypes = [ctypes.POINTER(rw_surface), ctypes.c_int,
                                           ctypes.POINTER(rw_doe_desc),
                                           ctypes.POINTER(rw_doe_desc), ctypes.c_int,
                                           ctypes.POINTER(rw_param_ref), ctypes.c_int,
                                           ctypes.POINTER(rw_config), ctypes.POINTER(vp)]
    lib.rw_plan_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.rw_forward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp, vp, vp]
    lib.rw_forward_static.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.rw_backward.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    lib.rw_forward_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.rw_get_stats.argtypes = [vp, ctypes.POINTER(rw_stats)]
    lib.rw_export_doe_hits.argtypes = [vp, vp, vp, vp]
    lib.rw_plan_destroy.argtypes = [vp]
    lib.rw_set_profiling.argtypes = [vp, ctypes.c_int]
    lib.rw_get_profile.argtypes = [vp, ctypes.POINTER(rw_profile)]
    lib.rw_set_graph.argtypes = [vp, ctypes.c_int]
    lib.rw_autotune.argtypes = [vp, vp, sz, ctypes.POINTER(ctypes.c_int), vp]
    lib.rw_set_launch_shape.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    f32 = ctypes.c_float
    lib.rw_adam_step.argtypes = [vp, vp, vp, vp, sz, f32, f32, f32, f32, ctypes.c_int, f32, f32, vp]
    lib.rw_patch_dft.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_longlong, vp, vp, vp]
    lib.rw_status_string.argtypes = [ctypes.c_int]
    lib.rw_status_string.restype = ctypes.c_char_p
    lib.rw_last_error.restype = ctypes.c_char_p
    for name in ("rw_plan_create", "rw_plan_create_cascade", "rw_plan_workspace_bytes",
                 "rw_forward", "rw_forward_static",
                 "rw_backward", "rw_forward_backward",
                 "rw_get_stats", "rw_export_doe_hits", "rw_plan_destroy", "rw_set_profiling",
                 "rw_get_profile", "rw_set_graph", "rw_autotune", "rw_set_launch_shape",
                 "rw_adam_step", "rw_patch_dft"):
        getattr(lib, name).restype = ctypes.c_int
    global _lib_id
    with open(path, "rb") as f:
        _lib_id = hashlib.sha256(f.read()).hexdigest()[:12]
    _lib = lib
    return lib


class RWError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(lib, st):
    if st != 0:
        raise RWError(st, lib.rw_last_error().decode())


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, bounds=None):
    """rw_adam_step on float32 device tensors of one shape (params, m, v updated in
    place on the current stream); bounds = (lo, hi) clamps the parameters."""
    lib = load_library()
    for x in (params, grads, m, v):
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("adam_step takes contiguous float32 device tensors")
        if x.numel() != params.numel():
            raise ValueError("adam_step: shapes differ")
    lo, hi = bounds if bounds is not None else (1.0, 0.0)
    st = torch.cuda.current_stream(params.device).cuda_stream
    _check(lib, lib.rw_adam_step(_dptr(params), _dptr(grads), _dptr(m), _dptr(v), params.numel(),
                                 float(lr), float(beta1), float(beta2), float(eps), int(t),
                                 float(lo), float(hi), ctypes.c_void_p(st)))


def patch_dft(patches, M, out=None):
    """rw_patch_dft: the DOE kernels' M x M transform of zero-padded patches
    (complex64 device tensor [n, P, P] -> [n, M, M], natural frequency order)."""
    lib = load_library()
    if patches.dtype != torch.complex64 or not patches.is_cuda or not patches.is_contiguous():
        raise ValueError("patch_dft takes a contiguous complex64 device tensor")
    n, P = patches.shape[0], patches.shape[1]
    if out is None:
        out = torch.empty((n, M, M), dtype=torch.complex64, device=patches.device)
    st = torch.cuda.current_stream(patches.device).cuda_stream
    _check(lib, lib.rw_patch_dft(int(M), int(P), int(n), _dptr(patches), _dptr(out),
                                 ctypes.c_void_p(st)))
    return out


def _dbl_array(vals):
    a = np.ascontiguousarray(np.asarray(vals, dtype=np.float64).ravel())
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Plan:
    """A plan of the library for one system description and configuration.

    system / cfg are the dictionaries produced by the workload generators:
    system = {"surfaces", "sensor_z", "doe", "params"}, cfg = {"lambdas",
    "fields", "launch_center", "launch_z", "launch_half", "rays_side", "psf_q",
    "psf_pitch", "psf_center", "patch_p", "pad", "n_ssr", "sampling", "seed"}.
    A system with "does" (two map descriptions, for the two surfaces flagged
    "doe") and a cfg with "n_ssr2" make a two-DOE cascade plan (forward only):
    its maps are [2, H, W] and its sample indices the first DOE's followed by
    the second's (split_idx separates them).
    """

    def __init__(self, system, cfg, precision="mixed", batched=True, spread_width=0,
                 device="cuda", check_finite=False):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the ray-wave library runs on the GPU only")
        self.device = torch.device(device)
        self.system, self.cfg = system, cfg
        surfs = system["surfaces"]
        arr = (rw_surface * len(surfs))()
        for i, s in enumerate(surfs):
            arr[i].kind = {"plane": RW_SURF_PLANE, "gauss": RW_SURF_GAUSS}.get(s["kind"],
                                                                             RW_SURF_ASPHERE)
            arr[i].gauss_height = s.get("gh", 0.0)
            arr[i].gauss_width = s.get("gw", 0.0)
            arr[i].carries_doe = int(bool(s.get("doe", False)))
            arr[i].z_vertex = s["z"]
            arr[i].curvature = s["c"]
            arr[i].conic = s["k"]
            for j in range(4):
                arr[i].asph[j] = s["A"][j]
            arr[i].semi_aperture = s["semi_ap"]
            arr[i].n_A = s["nA"]
            arr[i].n_B = s["nB"]
        def desc(d):
            return rw_doe_desc(d["H"], d["W"], d["pitch"], d["x0"], d["y0"],
                               int(bool(d.get("reflective", False))),
                               FIELDS[d.get("field", "amp_phase")])
        self.cascade = "does" in system
        doe = desc(system["does"][1] if self.cascade else system["doe"])
        prm = system.get("params", [])
        parr = (rw_param_ref * max(1, len(prm)))()
        for i, p in enumerate(prm):
            parr[i].surface = p["surface"]
            parr[i].field = PARAM_FIELDS[p["field"]]
            parr[i].scale = p["scale"]
        self._keep = []
        lam, lam_p = _dbl_array(cfg["lambdas"])
        ft, ft_p = _dbl_array(cfg["fields"])
        lc, lc_p = _dbl_array(cfg["launch_center"])
        pc, pc_p = _dbl_array(cfg["psf_center"])
        self._keep += [lam, ft, lc, pc]
        c = rw_config()
        c.n_lambda = len(cfg["lambdas"])
        c.lambda_host = lam_p
        c.n_field = len(cfg["fields"])
        c.field_tan_host = ft_p
        c.launch_center_host = lc_p
        c.launch_z = cfg["launch_z"]
        c.launch_half = cfg["launch_half"]
        c.rays_side = cfg["rays_side"]
        c.sensor_z = system["sensor_z"]
        c.psf_q = cfg["psf_q"]
        c.psf_pitch = cfg["psf_pitch"]
        c.psf_center_host = pc_p
        c.patch_p = cfg["patch_p"]
        c.pad_factor = cfg["pad"]
        c.n_ssr = cfg["n_ssr"]
        c.sampling = SAMPLING[cfg["sampling"]]
        c.precision = PRECISION[precision]
        c.batched = int(bool(batched))
        c.spread_width = int(spread_width)
        c.seed = int(cfg["seed"])
        c.grad = GRAD[cfg.get("grad", "G1")]
        c.tau = float(cfg.get("tau", 1.0))
        extra = sorted({int(q) for q in cfg.get("patch_classes", [])} - {int(cfg["patch_p"])},
                       reverse=True)
        if len(extra) > 3:
            raise ValueError("at most three patch classes besides patch_p")
        c.n_patch_class = len(extra)
        for i, q in enumerate(extra):
            c.patch_class_p[i] = q
        c.curv_eps = float(cfg.get("curv_eps", 0.1))
        c.check_finite = int(bool(check_finite))
        c.record_budget_bytes = int(cfg.get("record_budget_bytes", 0))
        c.bandwidth_periods = float(cfg.get("bw_periods", 0.0))
        c.class_draws = int(bool(cfg.get("class_draws", False)))
        c.deterministic = int(bool(cfg.get("deterministic", False)))
        h = ctypes.c_void_p()
        if self.cascade:
            doe1 = desc(system["does"][0])
            _check(self.lib, self.lib.rw_plan_create_cascade(
                arr, len(surfs), ctypes.byref(doe1), ctypes.byref(doe), int(cfg["n_ssr2"]), parr,
                len(prm), ctypes.byref(c), ctypes.byref(h)))
        else:
            _check(self.lib, self.lib.rw_plan_create(arr, len(surfs), ctypes.byref(doe), parr,
                                                     len(prm), ctypes.byref(c),
                                                     ctypes.byref(h)))
        self.handle = h
        nf, nx = ctypes.c_size_t(), ctypes.c_size_t()
        _check(self.lib, self.lib.rw_plan_workspace_bytes(h, ctypes.byref(nf), ctypes.byref(nx)))
        self.fwd_bytes = nf.value
        self.ws_bytes = nf.value + nx.value
        self._ws_raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws_raw.data_ptr()) % 256
        self.ws = self._ws_raw[off:off + self.ws_bytes]
        self.L = len(cfg["lambdas"])
        self.F = len(cfg["fields"])
        self.Q = cfg["psf_q"]
        self.n_params = len(prm)
        self.n_rays = self.L * self.F * cfg["rays_side"] ** 2
        self.N = cfg["n_ssr"]
        self.M = cfg["patch_p"] * cfg["pad"]
        if self.cascade:
            # the second DOE's ray grid: side rays_side n1, n_ssr2 draws per ray
            n1 = self.M if cfg["sampling"] == "full" else int(round(self.N ** 0.5))
            self.casc_shape = ((self.L * self.F, cfg["rays_side"] ** 2, self.N),
                               (self.L * self.F, (cfg["rays_side"] * n1) ** 2, cfg["n_ssr2"]))
        self.precision = precision
        self.generation = 0        # forwards run on this plan (HybridPSF checks it)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.rw_plan_destroy(h)
            self.handle = None

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def forward(self, lens_params, phase, amp, target=None, replay=None, want_idx=False,
                psf_out=None, loss_out=None, idx_out=None):
        """Returns (psf [L,F,Q,Q] float32, loss (tensor [1]) or None, idx or None)."""
        dev = self.device
        psf = psf_out if psf_out is not None else torch.empty(
            (self.L, self.F, self.Q, self.Q), dtype=torch.float32, device=dev)
        loss = None
        if target is not None:
            loss = loss_out if loss_out is not None else torch.empty(1, dtype=torch.float32,
                                                                     device=dev)
        idx = idx_out
        if want_idx and idx is None:
            if self.cascade:
                idx = torch.empty(sum(int(np.prod(s)) for s in self.casc_shape),
                                  dtype=torch.int32, device=dev)
            else:
                idx = torch.empty((self.L * self.F, self.cfg["rays_side"] ** 2, self.N),
                                  dtype=torch.int32, device=dev)
        self._fwd_keep = (lens_params, phase, amp, target, replay)
        self.generation += 1
        st = self.lib.rw_forward(self.handle, _dptr(lens_params), _dptr(phase), _dptr(amp),
                                 _dptr(target), _dptr(psf), _dptr(loss), _dptr(self.ws),
                                 self.ws_bytes, _dptr(replay), _dptr(idx), self._stream())
        _check(self.lib, st)
        return psf, loss, idx

    def split_idx(self, idx):
        """A cascade's sample indices as (first DOE [pairs, R^2, N1], second DOE
        [pairs, (R n1)^2, N2]); join_idx is the inverse."""
        n = int(np.prod(self.casc_shape[0]))
        return idx[:n].reshape(self.casc_shape[0]), idx[n:].reshape(self.casc_shape[1])

    @staticmethod
    def join_idx(idx1, idx2):
        return torch.cat([idx1.reshape(-1), idx2.reshape(-1)]).contiguous()

    def backward(self, dL_dpsf=None, d_phase=None, d_amp=None, d_lens=None):
        """Map (and lens) gradients of the preceding forward; a cascade's map
        gradients are [2, H, W] (first DOE, then second)."""
        d = self.system["doe"]
        dev = self.device
        shape = (2, d["H"], d["W"]) if self.cascade else (d["H"], d["W"])
        dp = d_phase if d_phase is not None else torch.empty(shape, dtype=torch.float32,
                                                             device=dev)
        da = d_amp if d_amp is not None else torch.empty_like(dp)
        dl = d_lens
        if dl is None and self.n_params:
            dl = torch.empty(self.n_params, dtype=torch.float32, device=dev)
        st = self.lib.rw_backward(self.handle, _dptr(dL_dpsf), _dptr(dp), _dptr(da), _dptr(dl),
                                  _dptr(self.ws), self.ws_bytes, self._stream())
        _check(self.lib, st)
        return dp, da, dl

    def step(self, lens_params, phase, amp, target, psf_out=None, loss_out=None, d_phase=None,
             d_amp=None, d_lens=None):
        """One fused forward + backward on the Eq. 5 loss (rw_forward_backward):
        returns (psf, loss, d_phase, d_amp, d_lens)."""
        d = self.system["doe"]
        dev = self.device
        psf = psf_out if psf_out is not None else torch.empty(
            (self.L, self.F, self.Q, self.Q), dtype=torch.float32, device=dev)
        loss = loss_out if loss_out is not None else torch.empty(1, dtype=torch.float32, device=dev)
        dp = d_phase if d_phase is not None else torch.empty((d["H"], d["W"]), dtype=torch.float32,
                                                             device=dev)
        da = d_amp if d_amp is not None else torch.empty_like(dp)
        dl = d_lens
        if dl is None and self.n_params:
            dl = torch.empty(self.n_params, dtype=torch.float32, device=dev)
        self._fwd_keep = (lens_params, phase, amp, target, None)
        self.generation += 1
        st = self.lib.rw_forward_backward(self.handle, _dptr(lens_params), _dptr(phase), _dptr(amp),
                                          _dptr(target), _dptr(psf), _dptr(loss), _dptr(dp),
                                          _dptr(da), _dptr(dl), _dptr(self.ws), self.ws_bytes,
                                          self._stream())
        _check(self.lib, st)
        return psf, loss, dp, da, dl

    def stats(self):
        s = rw_stats()
        _check(self.lib, self.lib.rw_get_stats(self.handle, ctypes.byref(s)))
        out = {name: getattr(s, name) for name in STATS}
        out["rays_by_class"] = list(s.rays_by_class)
        return out

    def tune_key(self):
        """What a launch shape depends on: the library build, the GPU architecture
        and the plan's geometry (precision, patch classes, draws, PSF, rays per
        pair, pairs)."""
        c = self.cfg
        arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        classes = sorted({int(c["patch_p"])} | {int(q) for q in c.get("patch_classes", [])})
        return "|".join(str(x) for x in (_lib_id, arch, self.precision, c["pad"], classes,
                                         c["sampling"],
                                         self.N, self.Q, c["rays_side"], self.L * self.F))

    def autotune(self, cache=None):
        """Fastest launch shape of the DOE kernels, returned as (fwd workgroups, fwd
        ray block, bwd workgroups, bwd ray block).  With `cache` (a JSON file path) a
        shape stored there under tune_key() is applied without timing; otherwise
        rw_autotune times the candidates on the inputs of the last forward (run the
        forward again before a backward) and the result is stored in the cache."""
        key = self.tune_key()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                self.set_launch_shape(table[key])
                return tuple(table[key])
        shape = (ctypes.c_int * 4)()
        _check(self.lib, self.lib.rw_autotune(self.handle, _dptr(self.ws), self.ws_bytes, shape,
                                              self._stream()))
        if cache:
            # entries of other library builds are dropped
            table = {k: v for k, v in table.items() if k.startswith(f"{_lib_id}|")}
            table[key] = list(shape)
            try:
                with open(cache, "w") as f:
                    json.dump(table, f, indent=1, sort_keys=True)
            except OSError:
                pass
        return tuple(shape)

    def set_launch_shape(self, shape):
        arr = (ctypes.c_int * 4)(*[int(x) for x in shape])
        _check(self.lib, self.lib.rw_set_launch_shape(self.handle, arr))

    def set_graph(self, enable=True):
        """Record the forward / backward launch sequences as HIP graphs and replay them."""
        _check(self.lib, self.lib.rw_set_graph(self.handle, int(bool(enable))))

    def set_profiling(self, enable=True):
        _check(self.lib, self.lib.rw_set_profiling(self.handle, int(bool(enable))))

    def profile(self):
        """Summed kernel milliseconds and launch counts per stage (HIP events)."""
        p = rw_profile()
        _check(self.lib, self.lib.rw_get_profile(self.handle, ctypes.byref(p)))
        return {name: (p.ms[i], p.launches[i]) for i, name in enumerate(STAGES)}

    def doe_hits(self):
        out = torch.empty((self.n_rays, 8), dtype=torch.float64, device=self.device)
        _check(self.lib, self.lib.rw_export_doe_hits(self.handle, _dptr(self.ws), _dptr(out),
                                                     self._stream()))
        return out


class HybridPSF(torch.autograd.Function):
    """torch.autograd.Function over rw_forward / rw_backward (the plan's gradient mode).

    The backward reads the state the forward left in the plan's workspace, so a
    plan serves one pending backward at a time: if another forward ran on the
    same plan in between, the backward raises (RW_ERR_STATE) instead of
    returning the gradient of the later forward."""

    @staticmethod
    def forward(ctx, plan, lens_params, phase, amp):
        psf, _, _ = plan.forward(lens_params, phase, amp)
        ctx.plan = plan
        ctx.generation = plan.generation
        return psf

    @staticmethod
    def backward(ctx, g):
        if ctx.plan.generation != ctx.generation:
            raise RWError(3, "the plan ran another forward after the one being differentiated")
        dp, da, dl = ctx.plan.backward(g.contiguous())
        return None, dl, dp, da
