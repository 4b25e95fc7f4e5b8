#!/usr/bin/env python3
"""Throughput of the forward + backward ray-wave hybrid PSF on one MI355X.

Headline workload (synthetic, seeded; the largest configuration of the
benchmark set, end-to-end hybrid design): BK7 and F2 even-asphere lenses with
a 4096 x 4096 complex DOE at 0.5 um on the second lens's rear asphere (the
stop); 8 wavelengths x 16 field angles (4 x 4 up to +-25 deg) x 512 x 512
incident rays per pair; patch classes 128 / 64 by the curvature bound (Eq. 4),
zero-padded to 256 / 128; 256 secondary rays per incident ray (p ~ |U~|);
1024 x 1024 PSF per pair; Eq. 5 loss against seeded Airy targets; gradients
w.r.t. the phase and amplitude maps and 14 lens parameters.

One step = one iteration of the design loop: rw_forward_backward (forward,
Eq. 5 loss and backward, fused per launch group of pairs) over all 128 pairs,
then the Adam update (rw_adam_step) of the phase and amplitude maps and the lens
parameters; inputs resident in HBM, batched MIXED form (persistent launches,
launch shapes from the autotuner, the fused sequence replayed as a HIP graph).
value = incident rays traced per second (128 x 512^2 per step).

Beside it, on the asphere-singlet + 1024^2 hologram system (27 pairs x 256^2
rays, P 64, N 256, Q 512): the same step with the per-kernel rooflines, the
plain FP32 comparator (same kernels, FP32 everywhere, one launch per pair),
the error of the measured form against the FP64 form on the same draws, the
Gumbel-softmax straight-through gradient, and forward-only rates of the
other workloads.  The FP64 CPU oracle is timed on bounded samples of the
headline and of the singlet system on the host cores.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "traced rays/s fwd+bwd to PSF, batched vs plain FP32, at ≤1e-4 PSF err vs FP64"
PEAK_FP32_VECTOR_TFLOPS = 157.3
CSRC = os.path.join(ROOT, "paper_2605_15418_amd", "csrc")
# sources compiled into the MIXED DOE kernels
DOE_SOURCES = ("rw_common.h", "rw_fft.h", "rw_kernels.h", "rw_backward.h", "rw_doe.h",
               "rw_doe_mixed.hip")
PROFILES = os.path.join(ROOT, "profiles")


def doe_source_hash():
    h = hashlib.sha256()
    for name in DOE_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (profiles/<kernel>_traffic_<workload>.md, already scaled
    by the copy-kernel calibration) if it was taken on the current kernel
    sources; else None."""
    path = os.path.join(PROFILES, f"{kernel}_traffic_{workload}.md")
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    m_src = re.search(r"kernel sources sha256\[:16\]: `([0-9a-f]+)`", text)
    m_b = re.search(r"HBM bytes per launch \(calibrated\): `([0-9.eE+]+)`", text)
    if not (m_src and m_b) or m_src.group(1) != doe_source_hash():
        return None
    return float(m_b.group(1))


def copy_calibration(nbytes):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE
    counters (run under rocprofv3 --pmc)."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}),
          flush=True)


# ----------------------------------------------------- algorithmic work ---
# Per incident ray, the forward's algorithmic flops F of the hot-path model:
#   5 M^2 log2 M^2 (patch FFT) + 14 P^2 (bilinear gather) + 8 M^2 (|U~|, cut,
#   CDF) + N (40 + log2 M^2) (draws) + 120 N (emission, FP64 phase, free-space
#   step) + N (8 w^2 + 20 w) (ES-kernel spreading);
# the backward is 1.1 F (inverse FFT, type-2 interpolation, bilinear scatter).
# Kernels: the forward DOE kernel does F without the spreading, the spreading
# kernel 8 w^2 + 20 w per record, the tiled interpolation the same per record
# (the backward's share of the type-2 NUFFT), and the DOE adjoint 1.1 F minus
# that interpolation share.  Recomputations (the adjoint redoes the forward
# transform) are not the method's work and are not counted.
def spread_flops(w):
    return 8 * w * w + 20 * w


def forward_flops_per_ray(P, M, N, w):
    return (5 * M * M * math.log2(M * M) + 14 * P * P + 8 * M * M
            + N * (40 + math.log2(M * M)) + 120 * N + N * spread_flops(w))


def kernel_flops(stats, classes, pad, N, w):
    """Algorithmic flops per launch of the DOE forward, DOE adjoint, spreading and
    interpolation kernels, summed over the patch classes (alive rays per class)."""
    fwd = bwd = 0.0
    for c, P in enumerate(classes):
        n = stats["rays_by_class"][c]
        F = forward_flops_per_ray(P, pad * P, N, w)
        fwd += n * (F - N * spread_flops(w))
        bwd += n * (1.1 * F - N * spread_flops(w))
    rec = stats["secondaries"]
    return {"doe_fwd": fwd, "doe_bwd": bwd, "spread": rec * spread_flops(w),
            "interp": rec * spread_flops(w)}


def rooflines(prof, steps, flops):
    """Achieved algorithmic TFLOP/s of each kernel over its mean launch time (HIP
    events on the plan's stream) against the FP32 vector peak."""
    out = {}
    for k, f in flops.items():
        ms, n = prof[k]
        if n == 0 or ms <= 0:
            continue
        per_launch_ms = ms / n
        launches_per_step = n / steps
        ach = f / launches_per_step / (per_launch_ms * 1e-3) / 1e12
        out[k] = {"launch_ms": round(per_launch_ms, 3), "achieved": round(ach, 3),
                  "frac": round(ach / PEAK_FP32_VECTOR_TFLOPS, 4),
                  "algorithmic_flop_per_launch": f / launches_per_step}
    return out


def dft_compare(n_patches):
    """The patch transform (M <= 64) three ways on the same batch of zero-padded
    P = M / 2 patches: the DOE kernels' LDS FFT (rw_patch_dft), and the DFT as two
    dense GEMMs per patch batch on the matrix cores through the library GEMMs
    (FP32 and BF16 operands, real block form [Re | Im] x [[C, S], [-S, C]]).
    Prints one JSON line: time per patch, achieved rate and accuracy against a
    complex128 FFT of the first patches."""
    import numpy as np
    import torch
    import paper_2605_15418_amd as rw
    dev = torch.device("cuda:0")
    out = {"metric": "patch DFT time per patch", "n_patches": n_patches, "results": {}}
    for M in (32, 64):
        P = M // 2
        g = torch.Generator(device="cpu").manual_seed(M)
        x = torch.complex(torch.randn((n_patches, P, P), generator=g),
                          torch.randn((n_patches, P, P), generator=g)).to(dev)
        ref = np.fft.fft2(np.pad(x[:64].cpu().numpy().astype(np.complex128),
                                 ((0, 0), (0, M - P), (0, M - P))))
        k = torch.arange(M, dtype=torch.float64)
        j = torch.arange(P, dtype=torch.float64)
        ang = -2 * np.pi * torch.outer(j, k) / M                  # [P, M]: x index j -> bin k
        C, S = torch.cos(ang), torch.sin(ang)
        res = {}

        def timed(fn, reps=5):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                y = fn()
            e1.record()
            torch.cuda.synchronize()
            return y, e0.elapsed_time(e1) / reps

        y, ms = timed(lambda: rw.patch_dft(x, M))
        e = float(np.linalg.norm(y[:64].cpu().numpy() - ref) / np.linalg.norm(ref))
        res["lds_fft"] = {"ms": ms, "ns_per_patch": ms * 1e6 / n_patches, "rel_err": e,
                          "flop_per_patch_fft": 5 * M * M * math.log2(M * M)}
        for dt in (torch.float32, torch.bfloat16):
            B1 = torch.cat([torch.cat([C, S], 1), torch.cat([-S, C], 1)], 0).to(dev, dt)   # [2P, 2M]
            Ck, Sk = torch.cos(-2 * np.pi * torch.outer(k, k) / M), torch.sin(-2 * np.pi * torch.outer(k, k) / M)
            B2 = torch.cat([torch.cat([Ck[:P], Sk[:P]], 1), torch.cat([-Sk[:P], Ck[:P]], 1)], 0).to(dev, dt)
            xr = torch.cat([x.real, x.imag], 2).to(dt).reshape(n_patches * P, 2 * P)

            def gemm_dft():
                y1 = (xr @ B1).reshape(n_patches, P, 2 * M)          # rows: [Re | Im] over kx
                y1 = torch.cat([y1[:, :, :M], y1[:, :, M:]], 1)      # [n, 2P, M]: Re rows, Im rows
                y1 = y1.transpose(1, 2).reshape(n_patches * M, 2 * P)
                y2 = (y1 @ B2).reshape(n_patches, M, 2 * M)          # [n, kx, (Re|Im) over ky]
                return torch.complex(y2[:, :, :M].float(), y2[:, :, M:].float()).transpose(1, 2)

            y, ms = timed(gemm_dft)
            e = float(np.linalg.norm(y[:64].cpu().numpy() - ref) / np.linalg.norm(ref))
            fl = 2 * (2 * P) * (2 * M) * P + 2 * (2 * P) * (2 * M) * M   # per patch, both GEMMs
            name = "gemm_fp32" if dt == torch.float32 else "gemm_bf16"
            res[name] = {"ms": ms, "ns_per_patch": ms * 1e6 / n_patches, "rel_err": e,
                         "flop_per_patch": fl,
                         "tflops": fl * n_patches / (ms * 1e-3) / 1e12}
        out["results"][f"M{M}"] = res
    print(json.dumps(out), flush=True)


def next_rows(iters=3):
    """Forward + backward of the two-DOE cascade and of adaptive patch sizing with
    class draw budgets (MIXED, batched), `iters` times each; one JSON line of the
    last iteration's times."""
    import numpy as np
    import torch
    import paper_2605_15418_amd as rw
    import workloads as W
    dev = torch.device("cuda:0")
    out = {}
    rng = np.random.default_rng(20260300)
    for name, tweak in (("two_doe_cascade", {}), ("adaptive_zone_plate", {"class_draws": True})):
        s, c, m = W.workload(name)
        c = dict(c, **tweak)
        L, F, Q = len(c["lambdas"]), len(c["fields"]), c["psf_q"]
        tg = m["target"] if m["target"] is not None else rng.uniform(0, 1, (L, F, Q, Q))
        tg = torch.tensor(tg, dtype=torch.float32, device=dev)
        plan = rw.Plan(s, c, precision="mixed", batched=True)
        ph = torch.tensor(m["phase"], device=dev)
        am = torch.tensor(m["amp"], device=dev)
        v = torch.zeros(0, device=dev)
        for _ in range(iters):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.forward(v, ph, am, target=tg)
            plan.backward()
            torch.cuda.synchronize()
            out[name] = (time.perf_counter() - t0) * 1e3
        del plan
        torch.cuda.empty_cache()
    print(json.dumps({"ms_fwd_bwd": out}), flush=True)


def lens_param_values(system):
    """The system's lens parameters in the plan's normalised units (float32)."""
    import numpy as np
    vals = []
    for ref in system["params"]:
        s, f = ref["surface"], ref["field"]
        surf = system["surfaces"][s]
        if f == "curv":
            phys = surf["c"]
        elif f == "gap":
            znext = (system["surfaces"][s + 1]["z"] if s + 1 < len(system["surfaces"])
                     else system["sensor_z"])
            phys = znext - surf["z"]
        else:
            phys = surf["A"][("A4", "A6", "A8", "A10").index(f)]
        vals.append(phys / ref["scale"])
    return np.array(vals, dtype=np.float32)


def deterministic_forward(iters=4):
    """Forward of the asphere-hologram workload (MIXED, batched) with the tiled
    spreading and with the deterministic fixed-point spreading, `iters` timed
    forwards each after one untimed: wall time per forward, the binning and
    spreading stages (HIP events), whether the timed forwards repeat bit for bit,
    and the relative L2 distance of the two PSFs.  One JSON line."""
    import numpy as np
    import torch
    import paper_2605_15418_amd as rw
    import workloads as W
    dev = torch.device("cuda:0")
    s, c, m = W.asphere_hologram()
    v = torch.tensor(lens_param_values(s), device=dev)
    ph = torch.tensor(m["phase"], device=dev)
    am = torch.tensor(m["amp"], device=dev)
    out, psfs = {}, {}
    for name, det in (("tiled", False), ("deterministic", True)):
        plan = rw.Plan(s, dict(c, deterministic=det), precision="mixed", batched=True)
        psf = torch.empty((plan.L, plan.F, plan.Q, plan.Q), device=dev)
        plan.forward(v, ph, am, psf_out=psf)
        torch.cuda.synchronize()
        plan.set_profiling(True)
        ms, first, same = [], None, True
        for _ in range(iters):
            t0 = time.perf_counter()
            plan.forward(v, ph, am, psf_out=psf)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
            if first is None:
                first = psf.clone()
            else:
                same = same and torch.equal(psf, first)
        prof = plan.profile()
        out[name] = {"ms_forward": round(min(ms), 2), "repeats_bitwise": bool(same),
                     **{f"ms_{k}": round(prof[k][0] / iters, 2) for k in ("bin", "spread")}}
        psfs[name] = first.cpu().numpy().astype(np.float64)
        del plan
        torch.cuda.empty_cache()
    a, b = psfs["deterministic"], psfs["tiled"]
    out["rel_l2_deterministic_vs_tiled"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print(json.dumps({"workload": "asphere_hologram", "forward": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed steps of the headline")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="two_lens_hybrid",
                    choices=("two_lens_hybrid", "asphere_hologram"))
    ap.add_argument("--side-steps", type=int, default=3, help="timed steps of the side system")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--g2-steps", type=int, default=1,
                    help="fwd+bwd steps timed with the Gumbel-softmax straight-through gradient")
    ap.add_argument("--no-side", action="store_true", help="headline only")
    ap.add_argument("--no-check", action="store_true", help="skip the FP64 error check")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-forward-only", action="store_true",
                    help="skip the forward-only rates of the other workloads")
    ap.add_argument("--no-graph", action="store_true", help="eager launches (no HIP graphs)")
    ap.add_argument("--dft-compare", type=int, default=0,
                    help="only compare patch-transform methods on this many patches")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    ap.add_argument("--next-rows", action="store_true",
                    help="only the forward + backward of the two-DOE cascade and of adaptive "
                         "patch sizing with class draw budgets, three times each (for traces)")
    ap.add_argument("--deterministic", action="store_true",
                    help="only the forward of the asphere hologram with the tiled and with the "
                         "deterministic spreading")
    args = ap.parse_args()
    if args.deterministic:
        deterministic_forward()
        return
    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
        return
    if args.next_rows:
        next_rows()
        return
    if args.dft_compare:
        dft_compare(args.dft_compare)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the single-GPU share is the measured unit); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2605_15418_amd as rw
    import workloads as W

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")

    def inputs(system, maps):
        v = torch.tensor(lens_param_values(system), device=dev)
        ph = torch.tensor(maps["phase"], device=dev)
        am = torch.tensor(maps["amp"], device=dev)
        tg = None if maps["target"] is None else torch.tensor(maps["target"], device=dev)
        return v, ph, am, tg

    def classes_of(cfg):
        return sorted({int(cfg["patch_p"])} | {int(q) for q in cfg.get("patch_classes", [])},
                      reverse=True)

    def measured_step(name, system, cfg, maps, steps, warmup):
        """Batched MIXED fwd+bwd: autotuned launch shapes (cached per arch and
        geometry), one eager profiled warm-up step (per-stage HIP events), then
        the timed steps replayed as HIP graphs."""
        v, ph, am, tg = inputs(system, maps)
        L, F = len(cfg["lambdas"]), len(cfg["fields"])
        n_rays = L * F * cfg["rays_side"] ** 2
        plan = rw.Plan(system, cfg, precision="mixed", batched=True)
        log(f"{name}: workspace {plan.ws_bytes / 2**30:.1f} GiB; autotune")
        plan.forward(v, ph, am, target=tg)
        shape = plan.autotune(cache=rw.rw.AUTOTUNE_CACHE)
        # one design-loop iteration: rw_forward_backward, then rw_adam_step
        des = rw.Design(plan, v, ph, am, tg, lr=(1e-2, 1e-2, 1e-2))

        def step():
            des.step()

        torch.cuda.synchronize()
        plan.set_profiling(True)
        t0 = time.perf_counter()
        step()                                     # eager, profiled: the per-kernel times
        torch.cuda.synchronize()
        eager_ms = (time.perf_counter() - t0) * 1e3
        prof = plan.profile()
        plan.set_profiling(False)
        stats = plan.stats()
        if not args.no_graph:
            plan.set_graph(True)
        for _ in range(max(0, warmup - 1) + (0 if args.no_graph else 1)):
            step()                                 # records the graphs, then replays
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms = (t1 - t0) * 1e3 / steps
        value = n_rays * steps / (t1 - t0)
        w = 7
        cls = classes_of(cfg)
        flops = kernel_flops(stats, cls, cfg["pad"], cfg["n_ssr"], w)
        roof = rooflines(prof, 1, flops)
        log(f"{name}: {ms:.1f} ms/step ({value:.3e} rays/s), eager profiled step {eager_ms:.1f} ms")
        rec = {"value": value, "unit": "rays/s", "ms_per_step": ms, "steps": steps,
               "eager_profiled_ms_per_step": eager_ms, "launch_shape": list(shape),
               "incident_rays_per_step": n_rays, "secondary_rays_per_step": stats["secondaries"],
               "secondary_rays_per_s": stats["secondaries"] / (ms * 1e-3),
               "stages_ms_per_step": {k: round(v_[0], 3) for k, v_ in prof.items()},
               "kernel_rooflines": roof, "stats": stats}
        return plan, rec, (v, ph, am, tg)

    # ----------------------------------------------------------- headline
    log(f"building the {args.workload} workload")
    system, cfg, maps = W.workload(args.workload)
    plan, head, head_in = measured_step(args.workload, system, cfg, maps, args.steps,
                                        args.warmup)
    roof = head["kernel_rooflines"]
    dom = max(roof, key=lambda k: roof[k]["launch_ms"])
    roofline = {"bound": "alu", "kernel": dom, "achieved": roof[dom]["achieved"],
                "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s", "frac": roof[dom]["frac"],
                "traffic": measured_traffic(dom, args.workload),
                "kernel_sources": doe_source_hash(), "launch_ms": roof[dom]["launch_ms"],
                "algorithmic_flop_per_launch": roof[dom]["algorithmic_flop_per_launch"],
                "per_kernel": {k: {"frac": r["frac"], "achieved": r["achieved"],
                                   "launch_ms": r["launch_ms"]} for k, r in roof.items()},
                "launch_ms_from": "HIP events on the plan's stream, eager profiled step"}
    del plan
    torch.cuda.empty_cache()
    if args.plain_steps > 0 and not args.no_side:
        # the plain FP32 comparator on the headline workload: the same kernels in
        # FP32 everywhere, one launch per pair, no graph, default launch shapes
        log(f"{args.workload}: plain FP32 form (one launch per pair)")
        v, ph, am, tg = head_in
        plain = rw.Plan(system, cfg, precision="fp32", batched=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            plain.forward(v, ph, am, target=tg)
            plain.backward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pv = head["incident_rays_per_step"] * args.plain_steps / (t1 - t0)
        head["plain_fp32"] = {"value": pv, "unit": "rays/s",
                              "ms_per_step": (t1 - t0) * 1e3 / args.plain_steps,
                              "speedup_batched_mixed": head["value"] / pv,
                              "note": "forward + backward on the same inputs; no Adam update"}
        log(f"{args.workload}: plain FP32 {(t1 - t0) * 1e3 / args.plain_steps:.1f} ms/step")
        del plain
        torch.cuda.empty_cache()

    # ------------------------------------------ the asphere-hologram system
    side = None
    if not args.no_side and args.workload != "asphere_hologram":
        s3, c3, m3 = W.asphere_hologram()
        p3, side, (v3, ph3, am3, tg3) = measured_step("asphere_hologram", s3, c3, m3,
                                                      args.side_steps, 1)
        side["workload"] = ("asphere singlet f=25 mm + 1024^2 random complex DOE @1 um; "
                            "3 lambda x 3x3 fields (+-10 deg) x 256^2 rays; P=64 (M=128), "
                            "N=256 (p_mag), Q=512; Eq. 5 loss; fwd+bwd (G1)")
        n3 = len(c3["lambdas"]) * len(c3["fields"]) * c3["rays_side"] ** 2

        def step(pl, replay=None):
            pl.forward(v3, ph3, am3, target=tg3, replay=replay)
            return pl.backward()

        if args.plain_steps > 0:
            log("plain FP32 form (one launch per pair)")
            plain = rw.Plan(s3, c3, precision="fp32", batched=False)
            step(plain)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.plain_steps):
                step(plain)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            pv = n3 * args.plain_steps / (t1 - t0)
            side["plain_fp32"] = {"value": pv, "ms_per_step": (t1 - t0) * 1e3 / args.plain_steps,
                                  "speedup_batched_mixed": side["value"] / pv}
        else:
            plain = None
        if not args.no_check:
            log("FP64 reference form on the same workload")
            p64 = rw.Plan(s3, c3, precision="fp64", batched=True)
            psf64, _, idx = p64.forward(v3, ph3, am3, target=tg3, want_idx=True)
            g64 = [g.double() for g in p64.backward()]
            psf64 = psf64.double()

            def errs(pl):
                psf, _, _ = pl.forward(v3, ph3, am3, target=tg3, replay=idx)
                g = pl.backward()
                d = (psf.double() - psf64).flatten(2).norm(dim=2) / psf64.flatten(2).norm(dim=2)
                ge = [float((a.double() - b).norm() / b.norm()) for a, b in zip(g, g64)]
                return {"psf_rel_l2_worst_pair": float(d.max()),
                        "grad_rel_l2": {"phase": ge[0], "amp": ge[1], "lens": ge[2]}}

            p3.set_graph(False)
            side["error_vs_fp64"] = {
                "mixed": errs(p3), "plain_fp32": errs(plain) if plain else None,
                "note": "same sample indices (FP64 draws replayed); relative L2 per pair / group"}
            del p64
        del plain
        if args.g2_steps > 0:
            log("G2 (Gumbel-softmax straight-through) backward, batched MIXED")
            p2 = rw.Plan(s3, dict(c3, grad="G2", tau=1.0), precision="mixed", batched=True)
            p2.set_profiling(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.g2_steps):
                step(p2)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            pr2 = p2.profile()
            side["g2_straight_through"] = {
                "value": n3 * args.g2_steps / (t1 - t0), "unit": "rays/s",
                "ms_per_step": (t1 - t0) * 1e3 / args.g2_steps, "steps": args.g2_steps,
                "tau": 1.0, "doe_bwd_ms_per_step": round(pr2["doe_bwd"][0] / args.g2_steps, 1)}
            del p2
        # forward only (the benchmark's holographic forward configuration)
        p3.set_graph(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.side_steps):
            p3.forward(v3, ph3, am3)
        torch.cuda.synchronize()
        side["forward_only"] = {"value": n3 * args.side_steps / (time.perf_counter() - t0),
                                "unit": "rays/s"}
        del p3
        torch.cuda.empty_cache()

    # ---------------------------------------- forward-only other workloads
    fwd_only = None
    if not args.no_forward_only:
        fwd_only = {}
        for name, prec in (("conformal_sphere", "mixed"), ("singlet_zoneplate", "fp64"),
                           ("two_doe_cascade", "mixed")):
            s_, c_, m_ = W.workload(name)
            v_, ph_, am_, _ = inputs(s_, m_)
            pl = rw.Plan(s_, c_, precision=prec, batched=True)
            pl.forward(v_, ph_, am_)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pl.forward(v_, ph_, am_)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            n_ = len(c_["lambdas"]) * len(c_["fields"]) * c_["rays_side"] ** 2
            st = pl.stats()
            fwd_only[name] = {"value": n_ / dt, "unit": "rays/s", "ms": dt * 1e3,
                              "precision": prec, "incident_rays": n_,
                              "secondaries": st["secondaries"], "rays_by_class":
                              st["rays_by_class"][:len(classes_of(c_))]}
            log(f"{name} forward ({prec}): {dt * 1e3:.1f} ms")
            del pl
            torch.cuda.empty_cache()

        # the cascade's forward + backward (both maps' gradients of Eq. 5)
        s_, c_, m_ = W.workload("two_doe_cascade")
        v_, ph_, am_, _ = inputs(s_, m_)
        Lc, Fc, Qc = len(c_["lambdas"]), len(c_["fields"]), c_["psf_q"]
        tg_ = torch.tensor(np.random.default_rng(20260300).uniform(0, 1, (Lc, Fc, Qc, Qc)),
                           dtype=torch.float32, device=dev)
        pl = rw.Plan(s_, c_, precision="mixed", batched=True)
        pl.forward(v_, ph_, am_, target=tg_)
        pl.backward()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pl.forward(v_, ph_, am_, target=tg_)
        pl.backward()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        fwd_only["two_doe_cascade"]["ms_fwd_bwd"] = dt * 1e3
        log(f"two_doe_cascade forward + backward (mixed): {dt * 1e3:.1f} ms")
        del pl
        torch.cuda.empty_cache()

    # ------------------------------------- adaptive patch sizing (K local periods)
    adaptive = None
    if not args.no_forward_only:
        adaptive = {}
        s_, c_, m_ = W.workload("adaptive_zone_plate")
        v_, ph_, am_, tg_ = inputs(s_, m_)
        big = max(classes_of(c_))
        forms = (("adaptive", c_), ("adaptive_class_draws", dict(c_, class_draws=True)),
                 (f"fixed_P{big}", dict(c_, patch_classes=[], bw_periods=0.0)))
        for tag, cc in forms:
            # fwd + bwd (MAG, G1) at full size
            pl = rw.Plan(s_, cc, precision="mixed", batched=True)
            pl.step(v_, ph_, am_, tg_)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pl.step(v_, ph_, am_, tg_)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            adaptive[tag] = {"ms_fwd_bwd": dt * 1e3,
                             "rays_by_class": pl.stats()["rays_by_class"][:len(classes_of(cc))]}
            del pl
            torch.cuda.empty_cache()
        # accuracy of the rule: FULL-mode PSFs on a 64^2 sub-grid of rays, against
        # every ray at the largest patch
        cf = dict(c_, sampling="full", rays_side=64,
                  launch_half=c_["launch_half"] * (1 - 1 / 64) / (1 - 1 / c_["rays_side"]))
        psfs = {}
        for tag, cc in (("adaptive", cf), (f"P{big}", dict(cf, patch_classes=[], bw_periods=0.0)),
                        ("adaptive_class_draws_mag", dict(cf, sampling="mag", class_draws=True)),
                        (f"P{big}_mag", dict(cf, sampling="mag", patch_classes=[], bw_periods=0.0)),
                        *[(f"P{q}", dict(cf, patch_p=q, patch_classes=[], bw_periods=0.0))
                          for q in classes_of(c_)[1:]]):
            pl = rw.Plan(s_, cc, precision="mixed", batched=True)
            psf_, _, _ = pl.forward(v_, ph_, am_)
            torch.cuda.synchronize()
            psfs[tag] = psf_.double().cpu().numpy()
            del pl
            torch.cuda.empty_cache()
        # agreement with every ray at the largest patch by the normalised cross-
        # correlation of Eq. 3 (scale-free: one patch side on its own changes the
        # overall scale through the patches' overlap)
        def ncc(a, b_):
            a, b_ = a - a.mean(), b_ - b_.mean()
            return float((a * b_).sum() / np.sqrt((a * a).sum() * (b_ * b_).sum()))
        ref_ = psfs[f"P{big}"]
        adaptive["ncc_vs_all_largest"] = {t: ncc(v, ref_) for t, v in psfs.items()
                                          if t != f"P{big}"}
        adaptive["speedup"] = {t: adaptive[f"fixed_P{big}"]["ms_fwd_bwd"] / adaptive[t]["ms_fwd_bwd"]
                               for t in ("adaptive", "adaptive_class_draws")}
        log(f"adaptive_zone_plate: fwd+bwd {adaptive['adaptive']['ms_fwd_bwd']:.1f} ms adaptive, "
            f"{adaptive['adaptive_class_draws']['ms_fwd_bwd']:.1f} ms with class draws, "
            f"{adaptive[f'fixed_P{big}']['ms_fwd_bwd']:.1f} ms at P = {big}; "
            f"NCC with all-P{big}: {adaptive['ncc_vs_all_largest']}")

    # -------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu:
        from oracle import rw_oracle as O
        nthreads = torch.get_num_threads()
        R = cfg["rays_side"]
        side_n = 32
        c0 = R // 2 - side_n // 2
        subset = [(c0 + iy) * R + (c0 + ix) for iy in range(side_n) for ix in range(side_n)]
        F = len(cfg["fields"])
        pr = F * (len(cfg["lambdas"]) // 2) + F // 2
        l_idx, f_idx = pr // F, pr % F
        vals = head_in[0].cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        phd = torch.tensor(maps["phase"].astype(np.float64), requires_grad=True)
        amd = torch.tensor(maps["amp"].astype(np.float64), requires_grad=True)
        vd = torch.tensor(vals, requires_grad=True)
        r = O.pair_forward(system, cfg, O.transmission(phd, amd), l_idx, f_idx, vd,
                           ray_subset=subset)
        loss = O.eq5_loss(r["psf"], torch.tensor(maps["target"][l_idx, f_idx],
                                                 dtype=torch.float64))
        loss.backward()
        t1 = time.perf_counter()
        cpu = {"value": len(subset) / (t1 - t0), "unit": "rays/s", "cores": nthreads,
               "kind": "oracle",
               "sample": f"1 pair (lambda {cfg['lambdas'][l_idx] * 1e6:.0f} nm, field {f_idx}) x "
                         f"{len(subset)} central rays of {R * R}, full map, classes, N and Q, "
                         f"forward + Eq. 5 loss + autograd backward, {t1 - t0:.1f} s"}
        log(f"CPU oracle: {cpu['value']:.2f} rays/s on {nthreads} threads")

    desc = {"two_lens_hybrid": "two even-asphere lenses (BK7, F2) + 4096^2 complex DOE @0.5 um on "
                               "L2's rear asphere; 8 lambda x 4x4 fields (+-25 deg) x 512^2 rays; "
                               "patch classes P=128/64 (M=256/128, Eq. 4), N=256 (p_mag), Q=1024; "
                               "Eq. 5 loss; fwd+bwd (G1) w.r.t. phase, amplitude, 14 lens params",
            "asphere_hologram": side["workload"] if side else
            "asphere singlet + 1024^2 random complex DOE; 27 pairs x 256^2 rays; P=64, N=256, "
            "Q=512; Eq. 5 loss; fwd+bwd (G1)"}
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc[args.workload],
                   "form": "batched MIXED (FP32 patch FFTs, spectra and grids; FP64 trace, "
                           "OPL and phases), autotuned launch shapes, HIP-graph replays",
                   "incident_rays_per_step": head["incident_rays_per_step"],
                   "secondary_rays_per_step": head["secondary_rays_per_step"],
                   "secondary_rays_per_s": head["secondary_rays_per_s"]},
        "headline": head,
        "asphere_hologram": side,
        "forward_only": fwd_only,
        "adaptive_patch_sizing": adaptive,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
