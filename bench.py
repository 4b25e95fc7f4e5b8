#!/usr/bin/env python3
"""Throughput of the forward + backward ray-wave hybrid PSF on one MI355X.

Workload (synthetic, seeded): equiconvex BK7 even-asphere singlet (f = 25 mm,
random A4/A6) followed by a planar 1024 x 1024 random holographic complex DOE
at 1 um pitch; 3 wavelengths x 3 x 3 field angles (+-10 deg) x 256 x 256
incident rays per pair; 64 x 64 DOE patches zero-padded to 128 x 128; 256
secondary rays per incident ray (p ~ |U~|); 512 x 512 PSF per pair; Eq. 5
loss against seeded Airy targets; gradients w.r.t. the 1024 x 1024 phase and
amplitude maps and 6 lens parameters.

One step = rw_forward (with the loss) + rw_backward over all 27 pairs, inputs
resident in HBM.  value = incident rays traced per second (27 x 65536 per step).

Also reported: the plain FP32 form (same kernels, FP32 everywhere, one launch
per pair), the PSF / gradient error of the measured form against the FP64 form
on the same sample indices, per-stage kernel time from HIP events, the
roofline of the dominant kernel, and the FP64 CPU oracle timed on a bounded
sample of the same workload on the host cores.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "doe_bwd_traffic_asphere_hologram.md")


def doe_source_hash():
    h = hashlib.sha256()
    for name in DOE_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes (already scaled by the copy-kernel calibration), if they
    were taken on the current kernel sources; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            text = f.read()
    except OSError:
        return None
    m_src = re.search(r"kernel sources sha256\[:16\]: `([0-9a-f]+)`", text)
    m_k = re.search(r"kernel: `([a-z_]+)`", text)
    m_b = re.search(r"HBM bytes per launch \(calibrated\): `([0-9.eE+]+)`", text)
    if not (m_src and m_k and m_b) or m_k.group(1) != kernel or m_src.group(1) != doe_source_hash():
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


def doe_fwd_flops_per_ray(P, M, N):
    """Algorithmic flops of the ray-wave interface for one incident ray: the
    zero-padded 2-D FFT, bilinear patch gather, |U~| / cut / CDF, N draws,
    N emissions with their FP64 phase and free-space step."""
    return (5 * M * M * math.log2(M * M) + 14 * P * P + 8 * M * M
            + N * (40 + math.log2(M * M)) + 120 * N)


def doe_bwd_flops_per_ray(P, M, N, w):
    """Recomputed forward FFT (the draws and their normaliser are the
    forward's, not recomputed), the inverse FFT of the spectrum cogradient,
    bilinear adjoint, and per draw the type-2 interpolation of the value and
    its two frequency derivatives."""
    return (2 * 5 * M * M * math.log2(M * M) + 2 * 14 * P * P
            + 240 * N + N * 3 * 8 * w * w)


def spread_flops_per_record(w):
    return 8 * w * w + 20 * w


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-check", action="store_true", help="skip the FP64 error check")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--g2-steps", type=int, default=1,
                    help="fwd+bwd steps timed with the Gumbel-softmax straight-through gradient")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
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
    system, cfg, maps = W.asphere_hologram()
    L, F = len(cfg["lambdas"]), len(cfg["fields"])
    n_rays = L * F * cfg["rays_side"] ** 2
    P, M, N, Q = cfg["patch_p"], cfg["patch_p"] * cfg["pad"], cfg["n_ssr"], cfg["psf_q"]
    from_params = []
    for ref in system["params"]:
        s, f = ref["surface"], ref["field"]
        surf = system["surfaces"][s]
        phys = surf["c"] if f == "curv" else surf["A"][("A4", "A6", "A8", "A10").index(f)]
        from_params.append(phys / ref["scale"])
    vals = torch.tensor(np.array(from_params, dtype=np.float32), device=dev)
    ph = torch.tensor(maps["phase"], device=dev)
    am = torch.tensor(maps["amp"], device=dev)
    tg = torch.tensor(maps["target"], device=dev)

    def step(plan, replay=None):
        plan.forward(vals, ph, am, target=tg, replay=replay)
        return plan.backward()

    # ---------------------------------------------------------------- batched
    log("building the batched MIXED plan")
    plan = rw.Plan(system, cfg, precision="mixed", batched=True)
    for _ in range(args.warmup):
        step(plan)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(plan)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile()
    plan.set_profiling(False)
    stats = plan.stats()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n_rays * args.steps / (t1 - t0)
    log(f"batched MIXED: {ms_per_step:.1f} ms/step, {value:.3e} rays/s")

    # roofline of the dominant kernel (algorithmic flops / measured kernel time)
    w = 7
    alive = stats["rays_alive"]
    records = stats["secondaries"]
    flops = {
        "doe_fwd": alive * doe_fwd_flops_per_ray(P, M, N),
        "doe_bwd": alive * doe_bwd_flops_per_ray(P, M, N, w),
        "spread": records * spread_flops_per_record(w),
    }
    per_launch_ms = {k: prof[k][0] / max(prof[k][1], 1) for k in prof}
    dom = max(flops, key=lambda k: per_launch_ms[k])
    achieved = flops[dom] / (per_launch_ms[dom] * 1e-3) / 1e12
    traffic = measured_traffic(dom)
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3),
                "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": traffic,
                "kernel_sources": doe_source_hash(),
                "launch_ms": round(per_launch_ms[dom], 3),
                "algorithmic_flop_per_launch": flops[dom]}

    # ------------------------------------------------------------ plain FP32
    plain, plain_rec = None, None
    if args.plain_steps > 0:
        log("plain FP32 form (one launch per pair)")
        plain = rw.Plan(system, cfg, precision="fp32", batched=False)
        step(plain)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            step(plain)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain_value = n_rays * args.plain_steps / (t1 - t0)
        plain_rec = {"value": plain_value, "ms_per_step": (t1 - t0) * 1e3 / args.plain_steps,
                     "speedup_batched_mixed": value / plain_value}
        log(f"plain FP32: {plain_rec['ms_per_step']:.1f} ms/step")

    # ------------------------------------------------ G2 (straight-through)
    g2_rec = None
    if args.g2_steps > 0:
        log("G2 (Gumbel-softmax straight-through) backward, batched MIXED")
        p2 = rw.Plan(system, dict(cfg, grad="G2", tau=1.0), precision="mixed", batched=True)
        p2.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.g2_steps):
            step(p2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pr2 = p2.profile()
        g2_rec = {"value": n_rays * args.g2_steps / (t1 - t0), "unit": "rays/s",
                  "ms_per_step": (t1 - t0) * 1e3 / args.g2_steps, "steps": args.g2_steps,
                  "tau": 1.0,
                  "doe_bwd_ms_per_step": round(pr2["doe_bwd"][0] / args.g2_steps, 1)}
        del p2
        log(f"G2: {g2_rec['ms_per_step']:.0f} ms/step")

    # ---------------------------------------------- error against FP64 form
    check = None
    if not args.no_check:
        log("FP64 reference form on the same workload")
        p64 = rw.Plan(system, cfg, precision="fp64", batched=True)
        psf64, _, idx = p64.forward(vals, ph, am, target=tg, want_idx=True)
        g64 = p64.backward()
        psf64 = psf64.double()
        g64 = [g.double() for g in g64]

        def errs(pl):
            psf, _, _ = pl.forward(vals, ph, am, target=tg, replay=idx)
            g = pl.backward()
            d = (psf.double() - psf64).flatten(2).norm(dim=2) / psf64.flatten(2).norm(dim=2)
            ge = [float((a.double() - b).norm() / b.norm()) for a, b in zip(g, g64)]
            return {"psf_rel_l2_worst_pair": float(d.max()), "grad_rel_l2":
                    {"phase": ge[0], "amp": ge[1], "lens": ge[2]}}

        check = {"mixed": errs(plan), "plain_fp32": errs(plain) if plain else None,
                 "note": "same sample indices (FP64 draws replayed); relative L2 per pair / per group"}
        del p64
        log(f"errors vs FP64: {json.dumps(check)}")

    # -------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu:
        from oracle import rw_oracle as O
        nthreads = torch.get_num_threads()
        R = cfg["rays_side"]
        side = 48
        c0 = R // 2 - side // 2
        subset = [(c0 + iy) * R + (c0 + ix) for iy in range(side) for ix in range(side)]
        l_idx, f_idx = 1, F // 2
        t0 = time.perf_counter()
        phd = torch.tensor(maps["phase"].astype(np.float64), requires_grad=True)
        amd = torch.tensor(maps["amp"].astype(np.float64), requires_grad=True)
        vd = torch.tensor(vals.cpu().numpy().astype(np.float64), requires_grad=True)
        r = O.pair_forward(system, cfg, O.transmission(phd, amd), l_idx, f_idx, vd,
                           ray_subset=subset)
        loss = O.eq5_loss(r["psf"], torch.tensor(maps["target"][l_idx, f_idx], dtype=torch.float64))
        loss.backward()
        t1 = time.perf_counter()
        cpu = {"value": len(subset) / (t1 - t0), "unit": "rays/s", "cores": nthreads,
               "kind": "oracle",
               "sample": f"1 pair (587.6 nm, on axis) x {len(subset)} central rays of {R * R}, "
                         f"full P/M/N/Q, forward + Eq. 5 loss + autograd backward, "
                         f"{t1 - t0:.1f} s"}
        log(f"CPU oracle: {cpu['value']:.2f} rays/s on {nthreads} threads")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "asphere singlet f=25 mm + 1024^2 random complex DOE @1 um; "
                               "3 lambda x 3x3 fields (+-10 deg) x 256^2 rays; P=64 (M=128), "
                               "N=256 (p_mag), Q=512; Eq. 5 loss; fwd+bwd (G1)",
                   "form": "batched MIXED (FP32 FFT/grids, FP64 trace and phases)",
                   "incident_rays_per_step": n_rays,
                   "secondary_rays_per_step": records,
                   "secondary_rays_per_s": records * args.steps / (ms_per_step * args.steps / 1e3)},
        "plain_fp32": plain_rec,
        "g2_straight_through": g2_rec,
        "error_vs_fp64": check,
        "stages_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in prof.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
