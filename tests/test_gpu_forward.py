"""GPU forward path vs the FP64 oracle, through the C ABI.

Bars (written here, derived in the design notes):
  * FP64 form: sample indices bit-exact; PSF within 1e-6 (float32 output)
  * MIXED form (FP32 FFT / grids, FP64 trace and phases): PSF within 1e-4 of
    the oracle with the same sample indices (FULL mode, or the oracle's own
    indices replayed on the GPU); own draws agree on >= 97% of indices and
    every disagreement sits on a CDF edge the FP32 spectrum can move
  * plain FP32 form: shows the phase drift of FP32 optical path (P12)
"""
import numpy as np
import pytest
import torch

from oracle import philox
from oracle import rw_oracle as O
from rwcases import (check_draws_valid, gpu_inputs, oracle_param_values, oracle_psf, rel_l2,
                     small_hologram, small_singlet, worst_pair_rel)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    import paper_2605_15418_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.load_library()
    return pkg


def _run(rw, system, cfg, maps, precision, **kw):
    plan = rw.Plan(system, cfg, precision=precision, batched=kw.pop("batched", True),
                   spread_width=kw.pop("spread_width", 0))
    vals, ph, am = gpu_inputs(system, maps)
    psf, loss, idx = plan.forward(vals, ph, am, **kw)
    torch.cuda.synchronize()
    return plan, psf.cpu().numpy(), idx


@pytest.mark.parametrize("case", ["singlet", "hologram"])
def test_trace_state_at_doe(rw, case):
    system, cfg, maps = small_singlet() if case == "singlet" else small_hologram(rays=12)
    plan, _, _ = _run(rw, system, cfg, maps, "fp64" if case == "singlet" else "mixed")
    hits = plan.doe_hits().cpu().numpy()
    vals = oracle_param_values(system)
    surfs, _ = O.build_surfaces(system, torch.tensor(vals))
    R2 = cfg["rays_side"] ** 2
    F = len(cfg["fields"])
    for l in range(len(cfg["lambdas"])):
        for f in range(F):
            p, d, opl = O.launch(cfg, f)
            p, d, opl, alive, _ = O.trace_to_doe(surfs, cfg["lambdas"][l], p, d, opl)
            doe = system["doe"]
            fx = (p[:, 0] - doe["x0"]) / doe["pitch"]
            fy = (p[:, 1] - doe["y0"]) / doe["pitch"]
            alive = alive & (fx >= -0.5) & (fx <= doe["W"] - 0.5) & (fy >= -0.5) & \
                (fy <= doe["H"] - 0.5)
            g = hits[(l * F + f) * R2:(l * F + f + 1) * R2]
            a = alive.numpy()
            assert np.array_equal(g[:, 7] != 0, a)
            assert np.max(np.abs(g[a, 0:3] - p.numpy()[a])) < 1e-11
            assert np.max(np.abs(g[a, 3:6] - d.numpy()[a])) < 1e-13
            assert np.max(np.abs(g[a, 6] - opl.numpy()[a])) < 1e-11


def test_fp64_mc_indices_exact_and_psf(rw):
    system, cfg, maps = small_singlet(sampling="mag")
    plan, psf, idx = _run(rw, system, cfg, maps, "fp64", want_idx=True)
    ref, aux = oracle_psf(system, cfg, maps, values=oracle_param_values(system), keep=True)
    gi = idx.cpu().numpy()
    for pr, a in aux.items():
        assert np.array_equal(gi[pr], a["J"]), "sample indices differ"
    assert rel_l2(psf, ref) < 1e-6
    st = plan.stats()
    assert st["rays_total"] == cfg["rays_side"] ** 2
    assert st["secondaries"] == int(sum((a["J"] >= 0).sum() for a in aux.values()))


@pytest.mark.parametrize("sampling", ["full", "uni"])
def test_fp64_other_samplings(rw, sampling):
    system, cfg, maps = small_singlet(sampling=sampling, rays=8)
    plan, psf, idx = _run(rw, system, cfg, maps, "fp64", want_idx=(sampling != "full"))
    ref, aux = oracle_psf(system, cfg, maps, values=oracle_param_values(system), keep=True)
    if sampling != "full":
        assert np.array_equal(idx.cpu().numpy()[0], aux[0]["J"])
    assert rel_l2(psf, ref) < 1e-6


def test_mixed_full_mode_psf_within_1e4(rw):
    system, cfg, maps = small_hologram(sampling="full")
    plan, psf, _ = _run(rw, system, cfg, maps, "mixed")
    ref, _ = oracle_psf(system, cfg, maps, values=oracle_param_values(system))
    assert worst_pair_rel(psf, ref) < 1e-4


def test_mixed_mc_replayed_oracle_indices_within_1e4(rw):
    system, cfg, maps = small_hologram(sampling="mag", N=48)
    ref, aux = oracle_psf(system, cfg, maps, values=oracle_param_values(system), keep=True)
    rep = torch.tensor(np.stack([aux[p]["J"] for p in sorted(aux)]), dtype=torch.int32,
                       device="cuda")
    plan, psf, _ = _run(rw, system, cfg, maps, "mixed", replay=rep)
    assert worst_pair_rel(psf, ref) < 1e-4


def test_mixed_mc_own_draws_agree_and_are_valid(rw):
    system, cfg, maps = small_hologram(sampling="mag", N=48)
    plan, psf, idx = _run(rw, system, cfg, maps, "mixed", want_idx=True)
    ref, aux = oracle_psf(system, cfg, maps, values=oracle_param_values(system), keep=True)
    gi = idx.cpu().numpy()
    agree = []
    for pr, a in aux.items():
        u = philox.draw_uniforms(cfg["seed"], pr, np.arange(a["J"].shape[0]), cfg["n_ssr"])
        agree.append(check_draws_valid(gi[pr], a["J"], a["spectrum"], a["prop"], u))
    assert np.mean(agree) >= 0.97, agree


def test_batched_equals_per_pair_launches(rw):
    system, cfg, maps = small_hologram(sampling="mag", N=32, rays=8)
    _, a, ia = _run(rw, system, cfg, maps, "mixed", want_idx=True)
    _, b, ib = _run(rw, system, cfg, maps, "mixed", want_idx=True, batched=False)
    assert torch.equal(ia, ib)
    assert rel_l2(a, b) < 1e-5


def test_plain_fp32_shows_phase_drift(rw):
    system, cfg, maps = small_hologram(sampling="full", rays=6, n_lambda=1, n_field_side=1)
    ref, _ = oracle_psf(system, cfg, maps, values=oracle_param_values(system))
    _, mixed, _ = _run(rw, system, cfg, maps, "mixed")
    _, fp32, _ = _run(rw, system, cfg, maps, "fp32", batched=False)
    e_mixed, e_fp32 = rel_l2(mixed, ref), rel_l2(fp32, ref)
    assert e_mixed < 1e-4
    assert e_fp32 > 10 * e_mixed


def test_edge_cases_dead_rays_and_single_ray(rw):
    # launch grid entirely outside the DOE: every ray dies, PSF is zero
    system, cfg, maps = small_singlet(sampling="mag", rays=4)
    cfg["launch_center"] = [[3.0, 3.0]]
    plan, psf, idx = _run(rw, system, cfg, maps, "fp64", want_idx=True)
    assert np.all(psf == 0) and np.all(idx.cpu().numpy() == -1)
    assert plan.stats()["rays_alive"] == 0
    # one ray
    system, cfg, maps = small_singlet(sampling="mag", rays=1)
    plan, psf, idx = _run(rw, system, cfg, maps, "fp64", want_idx=True)
    ref, aux = oracle_psf(system, cfg, maps, values=oracle_param_values(system), keep=True)
    assert np.array_equal(idx.cpu().numpy()[0], aux[0]["J"])
    assert rel_l2(psf, ref) < 1e-6


def test_invalid_shapes_are_rejected(rw):
    system, cfg, maps = small_singlet()
    bad = dict(cfg, psf_q=48)
    with pytest.raises(rw.RWError, match="RW_ERR_SHAPE"):
        rw.Plan(system, bad, precision="fp64")
    bad = dict(cfg, patch_p=12)
    with pytest.raises(rw.RWError, match="RW_ERR_SHAPE"):
        rw.Plan(system, bad, precision="fp64")


def test_graph_replays_match_eager(rw):
    """Recorded launch sequences (HIP graphs): several forward + backward replays,
    with eager work and synchronisations between them, against the eager run;
    changing an argument pointer records anew."""
    system, cfg, maps = small_hologram(sampling="mag", N=32, rays=8)
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    eager = rw.Plan(system, cfg, precision="mixed")
    psf0, loss0, idx0 = eager.forward(vals, ph, am, target=tg, want_idx=True)
    g0 = eager.backward()
    torch.cuda.synchronize()
    plan = rw.Plan(system, cfg, precision="mixed")
    plan.set_graph(True)
    psf = torch.empty_like(psf0)
    loss = torch.empty_like(loss0)
    idx = torch.empty_like(idx0)
    dp, da, dl = (torch.empty_like(x) for x in g0)
    for rep in range(3):                                     # same pointers: replays
        plan.forward(vals, ph, am, target=tg, psf_out=psf, loss_out=loss, idx_out=idx)
        plan.backward(d_phase=dp, d_amp=da, d_lens=dl)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(idx, idx0), rep
        assert rel_l2(psf.cpu().numpy(), psf0.cpu().numpy()) < 1e-5, rep
        assert abs(float(loss) - float(loss0)) <= 1e-5 * abs(float(loss0)), rep
        for a, b in zip((dp, da, dl), g0):
            assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-5, rep
        psf.zero_()
        dp.zero_()
    ph2 = ph.clone()                                         # new pointer: records again
    psf2, _, _ = plan.forward(vals, ph2, am, target=tg)
    torch.cuda.synchronize()
    assert rel_l2(psf2.cpu().numpy(), psf0.cpu().numpy()) < 1e-5


def test_graph_backward_follows_the_psf_buffer_of_each_forward(rw):
    """A training loop with graphs on, fixed gradient buffers and a fresh PSF
    tensor per step (two buffers in turn): the backward of the Eq. 5 loss reads
    the PSF of the forward it follows, so its replay must match eager every step."""
    system, cfg, maps = small_hologram(sampling="mag", N=32, rays=8)
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    eager = rw.Plan(system, cfg, precision="mixed")
    plan = rw.Plan(system, cfg, precision="mixed")
    plan.set_graph(True)
    psf_bufs = [torch.empty((plan.L, plan.F, plan.Q, plan.Q), device="cuda") for _ in range(2)]
    loss = torch.empty(1, device="cuda")
    dp = torch.empty_like(ph)
    da = torch.empty_like(am)
    dl = torch.empty_like(vals)
    for step in range(4):
        v = vals * (1.0 + 1e-3 * step)                   # the parameters move every step
        vk = torch.empty_like(vals)
        vk.copy_(v)
        eager.forward(vk, ph, am, target=tg)
        g0 = eager.backward()
        psf_bufs[step % 2].fill_(float("nan"))           # stale contents must never be read
        plan.forward(vk, ph, am, target=tg, psf_out=psf_bufs[step % 2], loss_out=loss)
        plan.backward(d_phase=dp, d_amp=da, d_lens=dl)
        torch.cuda.synchronize()
        for a, b in zip((dp, da, dl), g0):
            assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-5, step


def test_hybrid_psf_autograd_matches_oracle_and_guards_the_workspace(rw):
    """torch.autograd through HybridPSF: the gradient of a scalar loss of the PSF
    against the oracle's; a backward whose forward was followed by another
    forward on the same plan raises instead of differentiating the later one."""
    system, cfg, maps = small_hologram(sampling="full", rays=6, n_lambda=1, n_field_side=1)
    Q = cfg["psf_q"]
    Wt = np.random.default_rng(4).uniform(size=(1, 1, Q, Q))
    vals = oracle_param_values(system)
    ph64 = torch.tensor(maps["phase"].astype(np.float64), requires_grad=True)
    am64 = torch.tensor(maps["amp"].astype(np.float64), requires_grad=True)
    v64 = torch.tensor(vals, requires_grad=True)
    r = O.pair_forward(system, cfg, O.transmission(ph64, am64), 0, 0, v64)
    (r["psf"] * torch.tensor(Wt[0, 0])).sum().backward()
    plan = rw.Plan(system, cfg, precision="mixed")
    gv, gph, gam = gpu_inputs(system, maps)
    gv.requires_grad_(True)
    gph.requires_grad_(True)
    gam.requires_grad_(True)
    psf = rw.HybridPSF.apply(plan, gv, gph, gam)
    (psf * torch.tensor(Wt, dtype=torch.float32, device="cuda")).sum().backward()
    torch.cuda.synchronize()
    assert rel_l2(gph.grad.cpu().numpy(), ph64.grad.numpy()) < 1e-3
    assert rel_l2(gam.grad.cpu().numpy(), am64.grad.numpy()) < 1e-3
    assert rel_l2(gv.grad.cpu().numpy(), v64.grad.numpy()) < 1e-3
    psf1 = rw.HybridPSF.apply(plan, gv, gph, gam)
    psf2 = rw.HybridPSF.apply(plan, gv, gph, gam)          # overwrites the workspace
    with pytest.raises(RuntimeError, match="RW_ERR_STATE"):
        psf1.sum().backward()
    psf2.sum().backward()                                   # the latest forward is fine
    torch.cuda.synchronize()


def test_forward_only_workspace(rw):
    """A workspace of fwd_bytes runs a forward without the backward's state: the
    same PSF and draws as with the whole workspace, and rw_backward refuses."""
    import ctypes
    system, cfg, maps = small_hologram(sampling="mag", N=32, rays=8)
    plan = rw.Plan(system, cfg, precision="mixed")
    assert 0 < plan.fwd_bytes < plan.ws_bytes
    vals, ph, am = gpu_inputs(system, maps)
    psf0, _, idx0 = plan.forward(vals, ph, am, want_idx=True)
    psf = torch.empty_like(psf0)
    idx = torch.empty_like(idx0)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    st = plan.lib.rw_forward(plan.handle, p(vals), p(ph), p(am), None, p(psf), None, p(plan.ws),
                             plan.fwd_bytes, None, p(idx),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == 0
    assert torch.equal(idx, idx0)
    assert rel_l2(psf.cpu().numpy(), psf0.cpu().numpy()) < 1e-5
    with pytest.raises(rw.RWError, match="RW_ERR_STATE"):
        plan.backward(torch.ones_like(psf))
    st = plan.lib.rw_forward(plan.handle, p(vals), p(ph), p(am), None, p(psf), None, p(plan.ws),
                             plan.fwd_bytes - 256, None, None,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rw.rw.STATUS[st] == "RW_ERR_STATE"


def test_autotune_keeps_results(rw):
    """The launch shape chosen by rw_autotune changes nothing but speed."""
    system, cfg, maps = small_hologram(sampling="mag", N=32, rays=8)
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    ref = rw.Plan(system, cfg, precision="mixed")
    p0, l0, i0 = ref.forward(vals, ph, am, target=tg, want_idx=True)
    g0 = ref.backward()
    plan = rw.Plan(system, cfg, precision="mixed")
    plan.forward(vals, ph, am, target=tg)
    shape = plan.autotune()
    assert shape[0] in (256, 512, 1024, 2048) and shape[1] in (4, 8, 16)
    assert shape[2] in (256, 512, 1024, 2048) and shape[3] in (4, 8, 16)
    with pytest.raises(rw.RWError, match="RW_ERR_STATE"):
        plan.backward()                          # autotune invalidated the forward state
    p1, l1, i1 = plan.forward(vals, ph, am, target=tg, want_idx=True)
    g1 = plan.backward()
    torch.cuda.synchronize()
    assert torch.equal(i0, i1)
    assert rel_l2(p1.cpu().numpy(), p0.cpu().numpy()) < 1e-6
    for a, b in zip(g1, g0):
        assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-5


# ------------------------------------------- the headline FFT size, M = 128 --
def _p64_case(sampling, N=64):
    """Patch side 64 (M = 128, the transform size of the throughput workload),
    one wavelength and field, 4 x 4 rays."""
    return small_hologram(sampling=sampling, P=64, N=N, rays=4, n_lambda=1, n_field_side=1)


def test_mixed_p64_full_mode_psf_within_1e4(rw):
    system, cfg, maps = _p64_case("full")
    plan, psf, _ = _run(rw, system, cfg, maps, "mixed")
    ref, _ = oracle_psf(system, cfg, maps, values=oracle_param_values(system))
    assert worst_pair_rel(psf, ref) < 1e-4


def test_mixed_p64_mc_replayed_oracle_indices_within_1e4(rw):
    system, cfg, maps = _p64_case("mag")
    ref, aux = oracle_psf(system, cfg, maps, values=oracle_param_values(system), keep=True)
    rep = torch.tensor(np.stack([aux[p]["J"] for p in sorted(aux)]), dtype=torch.int32,
                       device="cuda")
    plan, psf, _ = _run(rw, system, cfg, maps, "mixed", replay=rep)
    assert worst_pair_rel(psf, ref) < 1e-4


def test_mixed_p64_own_draws_agree(rw):
    system, cfg, maps = _p64_case("mag")
    plan, psf, idx = _run(rw, system, cfg, maps, "mixed", want_idx=True)
    ref, aux = oracle_psf(system, cfg, maps, values=oracle_param_values(system), keep=True)
    gi = idx.cpu().numpy()
    J = np.stack([aux[p]["J"] for p in sorted(aux)])
    assert (gi == J).mean() >= 0.97


# ----------------------------------------------------- counters and checks ---
def test_stats_count_ended_rays_by_cause_and_evanescent_bins(rw):
    """Rays launched past the lens aperture and past the DOE map end by those
    causes; the other counters against the oracle: alive rays equal, and the
    evanescent bins of the alive rays' spectra equal the oracle's count (FP64
    form: its propagation test is the same FP64 comparison)."""
    system, cfg, maps = small_singlet(sampling="full", rays=32, P=8)
    cfg["launch_half"] *= 10.0                 # well past the map, corners past the lens rim
    plan, psf, _ = _run(rw, system, cfg, maps, "fp64")
    st = plan.stats()
    ref, aux = oracle_psf(system, cfg, maps, values=oracle_param_values(system), keep=True)
    alive = aux[0]["alive"].numpy()
    prop = aux[0]["prop"].numpy()
    print(st)
    assert st["rays_alive"] == int(alive.sum())
    assert st["killed_aperture"] > 0 and st["killed_outside_doe"] > 0
    assert st["rays_total"] == (st["rays_alive"] + st["killed_no_hit"] + st["killed_aperture"] +
                                st["killed_tir"] + st["killed_outside_doe"])
    M = cfg["patch_p"] * cfg["pad"]
    assert st["spectrum_bins"] == int(alive.sum()) * M * M
    assert st["evanescent_bins"] == int(alive.sum()) * M * M - int(prop.sum())
    # FULL mode: every propagating bin becomes a secondary or is lost on the way
    assert st["secondaries"] + st["secondaries_lost"] == int(prop.sum())


def test_check_finite_refuses_nan_inputs(rw):
    system, cfg, maps = small_singlet(rays=4)
    plan = rw.Plan(system, cfg, precision="fp64", check_finite=True)
    vals, ph, am = gpu_inputs(system, maps)
    plan.forward(vals, ph, am)                                   # clean inputs pass
    bad = ph.clone()
    bad[3, 5] = float("nan")
    with pytest.raises(rw.RWError, match="RW_ERR_NONFINITE"):
        plan.forward(vals, bad, am)
    am2 = am.clone()
    am2[0, 0] = float("inf")
    with pytest.raises(rw.RWError, match="RW_ERR_NONFINITE"):
        plan.forward(vals, ph, am2)
    with pytest.raises(rw.RWError, match="RW_ERR_STATE"):
        plan.backward(torch.ones((1, 1, plan.Q, plan.Q), device="cuda"))


def _busiest_tile_records(aux, cfg):
    """Records of the busiest spreading tile (fine grid of 2Q cells, tiles of 4
    bins) computed from the oracle's wavelet frequencies."""
    Q = cfg["psf_q"]
    nf = max(2 * Q, 64)
    tile = 4 * (nf // min(64, nf // 8))
    out = 0
    for a in aux.values():
        t = [(w.numpy() / (2 * np.pi)) % 1.0 * nf // tile for w in (a["wx"], a["wy"])]
        ids = t[1].astype(np.int64) * (nf // tile) + t[0].astype(np.int64)
        out = max(out, int(np.bincount(ids).max()))
    return out


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-6), ("mixed", 1e-4)])
def test_focused_records_split_heavy_tiles(rw, precision, bar):
    """A zone plate at its focus sends a million records into four tiles: the
    spreading cuts each into slices (slice 0 stored, the rest added) and must
    still give the oracle's PSF."""
    import workloads as W
    system, cfg, maps = W.adaptive_zone_plate(rays_side=64, H=256, pitch=0.002, f=5.0, P=16,
                                              classes=(), N=256, Q=32, psf_pitch=0.002,
                                              sampling="mag")
    cfg = dict(cfg, patch_classes=[], bw_periods=0.0)
    print(f"heavy tiles {precision}", flush=True)
    ref, aux = oracle_psf(system, cfg, maps, keep=True)
    assert _busiest_tile_records(aux, cfg) > 4 * 65536
    rep = torch.tensor(np.stack([aux[p]["J"] for p in sorted(aux)]), dtype=torch.int32,
                       device="cuda")
    _, psf, _ = _run(rw, system, cfg, maps, precision, replay=rep)
    assert rel_l2(psf, ref) < bar


def test_focused_records_gradients_split_interpolation(rw):
    """At a zone plate's focus the tiled interpolation's few busy blocks are cut
    into slices as well; the map gradients on the oracle's draws still match."""
    import workloads as W
    system, cfg, maps = W.adaptive_zone_plate(rays_side=64, H=256, pitch=0.002, f=5.0, P=16,
                                              classes=(), N=64, Q=32, psf_pitch=0.002,
                                              sampling="mag")
    cfg = dict(cfg, patch_classes=[], bw_periods=0.0)
    print("heavy interpolation gradients", flush=True)
    L0, g, _, idx = O.loss_and_grad(system, cfg, maps["phase"].astype(np.float64),
                                    maps["amp"].astype(np.float64), np.zeros(0),
                                    maps["target"].astype(np.float64))
    rep = torch.tensor(np.stack([idx[p] for p in sorted(idx)]), dtype=torch.int32, device="cuda")
    plan = rw.Plan(system, cfg, precision="mixed")
    vals, ph, am = gpu_inputs(system, maps)
    tg = torch.tensor(maps["target"], device="cuda")
    _, loss, _ = plan.forward(vals, ph, am, target=tg, replay=rep)
    dp, da, _ = plan.backward()
    torch.cuda.synchronize()
    assert abs(float(loss) - L0) <= 1e-4 * abs(L0)
    assert rel_l2(dp.cpu().numpy(), g["phase"]) < 1e-3
    assert rel_l2(da.cpu().numpy(), g["amp"]) < 1e-3
