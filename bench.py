"""Benchmark: one IEWPF data-assimilation cycle per step on the paper-scale ensemble.

Workload (synthetic, shaped like the paper's 500x300 identical-twin experiments): 500x300
periodic grid, dx = dy = 5 km, H = 230 m, 100 particles (float32 state), model error on a
125x75 coarse grid, 225 moored buoys (15x15) observing (hu, hv).  One step = one 5-minute
cycle: 10 model steps of 30 s (2 scheme steps each, model error after each model step but
the last) followed by one two-stage IEWPF analysis.  Truth run and its observations are
synthesised before the timed region (inputs resident when timing starts).

value = particle-cell-scheme-steps per second over the whole cycle (forecast + analysis):
  n_particles * nx * ny * 20 * K / elapsed.

Prints one JSON line.  `--gpus N` with N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
N_CU, CLOCK_GHZ = 256, 2.4
# VALU wave-instructions issued per clock per CU (at the nominal 2.4 GHz) by a probe of
# eight independent non-packed FP32 multiply-add chains per wave at 8 waves per SIMD: the
# attainable issue rate of a kernel built without packed FP32 (0.91 at 5 waves per SIMD;
# square roots and reciprocals issue at about half that rate)
VALU_ISSUE_CEILING = 0.94
# Algorithmic work of one scheme step (both SSP-RK2 stages) per cell: read eta, hu, hv
# once and write them once (float32) ...
BYTES_PER_CELL_STEP = 24.0
# ... and the scheme's arithmetic, counted from its definition (each +, -, x, /, sqrt, min,
# max one flop): per stage 3 (primitives) + 2 x 54 (x and y reconstructions) + 2 x 55 (one
# x and one y face flux) + 25 (update) = 246; two stages and the RK2 average: 498.
FLOPS_PER_CELL_STEP = 498.0
# Network forward: 2 x (27 x 48 + 4 x 432 x 48 + 432 x 3) multiply-adds per pixel.
SURROGATE_FLOPS_PER_PIXEL = 171_072
# Counters of one launch of the plain scheme step on this workload (rocprofv3 --pmc):
# HBM bytes = FETCH_SIZE x 2 + WRITE_SIZE x 1 KiB (the scale factors a plain device copy of
# known size reads) and SQ_INSTS_VALU, with the SHA-256 of the kernel source they were taken
# on: reported only while the source is unchanged.
MEASURED_COUNTERS = {"hbm_bytes": (2 * 104328 + 175832) * 1024,
                     "valu_insts": 76.388e6,
                     "source_sha256": "17c9fc28aa1ea2a9ae13d941514ed9d49029c55e44fe90d5e4f5875e84af0da1"}


def _kernel_source_hash():
    """SHA-256 over the scheme kernels' source, the headers their code depends on and the
    build flags."""
    import hashlib
    h = hashlib.sha256()
    for rel in (("csrc", "swe_kernels.hip"), ("csrc", "swe_const.hpp"), ("csrc", "buffer_dev.hpp"),
                ("build.py",)):
        with open(os.path.join(ROOT, "paper_1910_01031_amd", *rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def gpu_state(torch):
    """Clock, power and temperature of cuda:0 from the driver's metrics table (amdsmi).

    The device is matched by PCI domain and bus.  Fields the table leaves out are null; any
    failure is reported as {"error": ...} and never stops the benchmark.
    """
    try:
        import amdsmi
    except ImportError as e:
        return {"error": f"amdsmi not importable: {e}"}
    keep = ("current_gfxclk", "average_gfxclk_frequency", "current_uclk", "current_socket_power",
            "average_socket_power", "temperature_hotspot", "temperature_mem")
    try:
        amdsmi.amdsmi_init()
        try:
            prop = torch.cuda.get_device_properties(0)
            want = (prop.pci_domain_id, prop.pci_bus_id)
            for h in amdsmi.amdsmi_get_processor_handles():
                dom, bus = amdsmi.amdsmi_get_gpu_device_bdf(h).split(":")[:2]
                if (int(dom, 16), int(bus, 16)) == want:
                    m = amdsmi.amdsmi_get_gpu_metrics_info(h)
                    return {k: m.get(k) for k in keep}
            return {"error": "no amdsmi device on the PCI bus of cuda:0"}
        finally:
            amdsmi.amdsmi_shut_down()
    except Exception as e:  # noqa: BLE001 - reported, not raised
        return {"error": f"{type(e).__name__}: {e}"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--particles", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-large-ensemble", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched leg (3 graph replays), e.g. under a profiler")
    ap.add_argument("--surrogate-train-steps", type=int, default=1000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 360 MB device copy (counter calibration)")
    return ap.parse_args()


def _oracle_forecast_task(args):
    """Oracle model steps of one particle of the paper-scale ensemble (one process)."""
    cfg, particle, n_steps = args
    from threadpoolctl import threadpool_limits

    from oracle import ensemble as oens
    with threadpool_limits(1):
        psi = oens.init_member(cfg, W.jet_state(cfg), 0, particle)
        t0 = time.perf_counter()
        oens.step_member(psi, cfg, particle, 0, n_steps, noise_on_last=False)
        return time.perf_counter() - t0


def _oracle_analysis_task(args):
    """Oracle analysis of the paper-scale ensemble with the 225 buoys, the state update
    (stage 6) restricted to `particles` (stages 1-5 always cover the whole ensemble)."""
    cfg, cells, particles = args
    from threadpoolctl import threadpool_limits

    from oracle import ensemble as oens
    from oracle import iewpf as oiewpf
    from oracle import observe as oobs
    from oracle import philox as ophil
    with threadpool_limits(1):
        jet = W.jet_state(cfg)
        ens = np.stack([oens.init_member(cfg, jet, 0, i) for i in range(cfg.n_particles)])
        truth = oens.init_member(cfg.replace(ensemble_id=0x7FFF), jet, 1, 0)
        noise = ophil.normals(2 * len(cells), cfg.seed, 0, ophil.TAG_OBS, 0x7FFF, 0).reshape(-1, 2)
        y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, noise)
        consts = oiewpf.AnalysisConstants(cfg)
        t0 = time.perf_counter()
        oiewpf.analysis(ens, cells, y, cfg, 0, consts=consts, particles=list(particles))
        return time.perf_counter() - t0


def _oracle_tiny_end_to_end():
    """The tiny drifter-observing run on the oracle: 32x32, 10 particles, 4 drifters, 12
    cycles of 10 model steps and one analysis (truth and observations included)."""
    from oracle import drifters as odr
    from oracle import ensemble as oens
    from oracle import iewpf as oiewpf
    from oracle import observe as oobs
    from oracle import philox as ophil
    cfg = W.tiny()
    steps = cfg.obs_every
    t0 = time.perf_counter()
    base = oens.init_member(cfg, None, 0, 999)
    small = cfg.replace(init_std=0.003)
    ens = np.stack([oens.init_member(small, base, 1, i) for i in range(cfg.n_particles)])
    truth = oens.init_member(small.replace(ensemble_id=77), base, 1, 0)
    tcfg = cfg.replace(ensemble_id=77)
    pos = W.drifter_lattice(cfg, 2, 2)
    consts = oiewpf.AnalysisConstants(cfg)
    for c in range(12):
        prev = pos.copy()
        for s in range(steps):
            nxt = oens.step_member(truth, tcfg, 0, c * steps + s, 1, noise_on_last=True)
            pos = odr.heun_step(pos, truth, nxt, cfg, cfg.dt)
            truth = nxt
        noise = ophil.normals(2 * len(pos), cfg.seed, c, ophil.TAG_OBS, 77, 1).reshape(-1, 2)
        y = oobs.drifter_obs(pos, prev, steps * cfg.dt, cfg.H, cfg.obs_sigma, noise)
        cells = oobs.obs_cell(pos, cfg.dx, cfg.dy, cfg.nx, cfg.ny)
        fc = np.stack([oens.step_member(ens[i], cfg, i, c * steps, steps, noise_on_last=False)
                       for i in range(cfg.n_particles)])
        ens, _ = oiewpf.analysis(fc, cells, y, cfg, c, consts=consts)
    return time.perf_counter() - t0


def cpu_baseline(cfg, cells):
    """The FP64 oracle on a bounded sample of the paper-scale cycle, on the host's cores.

    N = the cores this process may run on (at most 16, the host share of one GPU), one
    single-threaded process each.  Measured: 4 model steps of one particle alone and of N
    particles at once (one per process); the analysis's whole-ensemble stages 1-5 alone; the
    state update of one particle alone and of N particles at once.  The cycle of all 100
    particles (10 model steps + one analysis) is extrapolated from them: per particle the
    model steps scale linearly, and the updates run in ceil(100 / N) rounds of N.  The tiny
    drifter-observing run (12 cycles) is timed whole on one core."""
    import multiprocessing as mp
    n_cores = max(1, min(16, len(os.sched_getaffinity(0))))
    ne = cfg.n_particles
    steps = 4
    fc1 = _oracle_forecast_task((cfg, 0, steps))
    an0 = _oracle_analysis_task((cfg, cells, []))
    an1 = _oracle_analysis_task((cfg, cells, [0])) - an0
    with mp.get_context("fork").Pool(n_cores) as pool:
        t0 = time.perf_counter()
        pool.map(_oracle_forecast_task, [(cfg, i, steps) for i in range(n_cores)])
        fcn = time.perf_counter() - t0
        t0 = time.perf_counter()
        times = pool.map(_oracle_analysis_task, [(cfg, cells, [i]) for i in range(n_cores)])
        ann = max(times) - an0  # each process ran stages 1-5 once before its update
    tiny_s = _oracle_tiny_end_to_end()
    rounds = -(-ne // n_cores)
    per_model_step = 10 / steps
    cycle_1 = ne * fc1 * per_model_step + an0 + ne * an1
    cycle_n = rounds * fcn * per_model_step + an0 + rounds * ann
    work = ne * cfg.nx * cfg.ny * cfg.n_sub * 10
    return {"value": work / cycle_n, "unit": "particle-cell-steps/s", "cores": n_cores,
            "kind": "oracle", "value_per_core": work / cycle_1,
            "cycle_s_extrapolated": {"1_core": cycle_1, f"{n_cores}_cores": cycle_n},
            "analysis_s_extrapolated": {"1_core": an0 + ne * an1,
                                        f"{n_cores}_cores": an0 + rounds * ann},
            "tiny_drifter_run_s_1_core": tiny_s,
            "sample": (f"paper-scale cycle ({ne} particles, 500x300, 225 buoys) extrapolated "
                       f"from: {steps} model steps of 1 particle ({fc1:.2f} s) and of "
                       f"{n_cores} particles on {n_cores} processes ({fcn:.2f} s); analysis "
                       f"stages 1-5 ({an0:.2f} s) and the state update of 1 particle "
                       f"({an1:.2f} s) and of {n_cores} on {n_cores} processes "
                       f"({ann:.2f} s); the tiny drifter run (12 cycles, 10 particles) "
                       f"timed whole ({tiny_s:.2f} s)")}


def batched_leg(torch, dev, steps: int):
    """Eight ensembles of uneven grids and sizes (500x300 x2, 400x400, ... 128x512; 50-200
    particles; 30-225 buoys), strips autotuned per ensemble, one cycle = one hipGraph replay
    (10 model steps + one analysis per ensemble)."""
    from paper_1910_01031_amd import Batch, Context
    ctxs, states, cells, ys, strips, work = [], [], [], [], [], 0
    for cfg, (nbx, nby) in W.batched():
        cl = W.buoy_cells(cfg.nx, cfg.ny, nbx, nby)
        ctx = Context(cfg, max_obs=len(cl))
        base = torch.from_numpy(W.as_f32(W.jet_state(cfg))).to(dev)
        st = torch.empty((cfg.n_particles, 3, cfg.ny, cfg.nx), dtype=torch.float32, device=dev)
        ctx.init_ensemble(st, base, stream_index=0)
        tctx = Context(cfg.replace(n_particles=1, ensemble_id=0x7000 + cfg.ensemble_id),
                       max_obs=len(cl))
        truth = torch.empty((1, 3, cfg.ny, cfg.nx), dtype=torch.float32, device=dev)
        tctx.init_ensemble(truth, base, stream_index=1)
        ys.append(tctx.observe_moorings(truth, cl, analysis_index=0))
        tctx.close()
        strips.append(ctx.autotune(st))
        ctxs.append(ctx)
        states.append(st)
        cells.append(cl)
        work += cfg.n_particles * cfg.nx * cfg.ny * cfg.n_sub * 10
    b = Batch(ctxs, states)
    for e, cl in enumerate(cells):
        b.set_cells(e, cl)
    b.cycle(10, 0, 0, ys, use_graph=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for c in range(1, steps + 1):
        b.cycle(10, 10 * c, c, ys, use_graph=True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    finite = all(bool(torch.isfinite(st).all().item()) for st in states)
    out = {"workload": "8 uneven ensembles (850 particles, 945 buoys), one graph per cycle",
           "ms_per_cycle": ms, "value": work / (ms / 1e3), "unit": "particle-cell-steps/s",
           "autotuned_strip_rows": strips,
           "state_finite": finite}
    b.close()
    for c in ctxs:
        c.close()
    return out


def full_covariance_leg(torch, ctx, ens, cells, obs, n_cycles):
    """The analysis with the full innovation covariance (450x450 over the 225 buoys): the
    first call builds and inverts S (float64 Cholesky on the device), later calls reuse it."""
    ctx.set_full_innovation(True)
    saved = ens.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.assimilate(ens, cells, None, analysis_index=n_cycles, want_stats=True, obs=obs[-1])
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record()
    for r in range(reps):
        ctx.assimilate(ens, cells, None, analysis_index=n_cycles + 1 + r, want_stats=False,
                       obs=obs[-1])
    e1.record()
    torch.cuda.synchronize()
    ctx.set_full_innovation(False)
    ens.copy_(saved)
    return {"n_y": 2 * int(len(cells)), "first_analysis_ms_with_factorisation": first_ms,
            "analysis_ms": e0.elapsed_time(e1) / reps}


def side_legs(torch, dev, ctx, ens, cfg):
    """Drifter forecast (64 drifters per particle, 10 model steps) and SIR residual
    resampling on the paper-scale ensemble."""
    pos0 = np.stack([W.drifter_lattice(cfg, 8, 8) for _ in range(cfg.n_particles)])
    pos = torch.from_numpy(pos0).to(dev)
    traj = torch.zeros((11,) + pos.shape, dtype=torch.float64, device=dev)
    logw = torch.from_numpy(np.random.default_rng(0).normal(size=cfg.n_particles)).to(dev)
    par = torch.zeros(cfg.n_particles, dtype=torch.int32, device=dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e2 = torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.forecast_drifters(ens, pos, 10, first_step=100000, traj=traj)
    e1.record()
    ctx.resample(ens, logw, analysis_index=100000, parents=par)
    e2.record()
    torch.cuda.synchronize()
    return {"drifter_forecast_ms_per_model_step": e0.elapsed_time(e1) / 10,
            "drifters": int(pos.shape[0] * pos.shape[1]),
            "resample_ms": e1.elapsed_time(e2)}


def drifter_comparison(torch, dev, ctx, net, start, cfg, windows: int = 12):
    """One hour (12 windows of 10 model steps) of drifter forecast, 64 drifters per particle
    on an 8x8 lattice, from the same ensemble: plain model (two runs with different
    model-error streams) and surrogate (plain re-step above a mass drift of 1e-4, one
    model-error draw scaled by 3 per window).  Position RMSE between paired drifters
    (minimum-image distances): surrogate vs plain, and plain vs plain (what the model error
    alone makes two forecasts differ by); the ensemble spread of the plain forecast."""
    from paper_1910_01031_amd import forecast_drifters_surrogate
    lx, ly = cfg.nx * cfg.dx, cfg.ny * cfg.dy
    pos0 = torch.from_numpy(np.stack([W.drifter_lattice(cfg, 8, 8)
                                      for _ in range(cfg.n_particles)])).to(dev)
    n_steps = 10 * windows
    runs = {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    for k, (name, first) in enumerate((("plain_a", 700_000), ("plain_b", 800_000),
                                       ("surrogate", 700_000))):
        st = start.clone()
        pos = pos0.clone()
        ev[2 * k].record()
        if name == "surrogate":
            nf = forecast_drifters_surrogate(ctx, net, st, pos, windows, 10, first, 1e-4, 3.0)
        else:
            ctx.forecast_drifters(st, pos, n_steps, first_step=first)
            nf = None
        ev[2 * k + 1].record()
        runs[name] = (pos, nf)
    torch.cuda.synchronize()
    ms = {name: ev[2 * k].elapsed_time(ev[2 * k + 1]) for k, name in
          enumerate(("plain_a", "plain_b", "surrogate"))}

    def min_image(d):
        L = torch.tensor([lx, ly], dtype=torch.float64, device=dev)
        return torch.remainder(d + 0.5 * L, L) - 0.5 * L

    def rmse(a, b):
        return float(min_image(a - b).pow(2).sum(dim=-1).mean().sqrt())

    pa = runs["plain_a"][0]
    centre = pa[0:1] + min_image(pa - pa[0:1]).mean(dim=0, keepdim=True)
    spread = float(min_image(pa - centre).pow(2).sum(dim=-1).mean().sqrt())
    return {"drifters": int(pos0.shape[0] * pos0.shape[1]), "hours": windows / 12.0,
            "ms_plain": ms["plain_a"], "ms_surrogate": ms["surrogate"],
            "speedup": ms["plain_a"] / ms["surrogate"],
            "rmse_surrogate_vs_plain_m": rmse(runs["surrogate"][0], pa),
            "rmse_plain_vs_plain_m": rmse(runs["plain_b"][0], pa),
            "spread_plain_m": spread, "surrogate_fallbacks": runs["surrogate"][1]}


def large_ensemble_leg(torch, net):
    """The large-ensemble drift forecast at reduced duration: 1000 particles on the 500x300
    grid through 2 h of IEWPF on the 225 moorings (24 analyses), then a 1 h forecast of 64
    drifters per particle with the plain model and with the surrogate (the network of the
    surrogate leg), side by side: E(t), RMSE(t) per hour, throughput."""
    from paper_1910_01031_amd import experiments as ex
    r = ex.drift_forecast(torch, n_particles=1000, da_hours=2.0, forecast_hours=1.0,
                          n_drifters=64, net=net)
    r["workload"] = ("1000 particles, 500x300, 2 h of IEWPF on 225 moorings, then 1 h of "
                     "64 drifters per particle, plain and surrogate")
    return r


def surrogate_leg(torch, dev, ctx, ens, cfg, train_steps: int, keep_net: bool = False):
    """Learned surrogate of the 5-minute window on the paper-scale ensemble.  Training pairs
    (psi, ten deterministic model steps of psi) come from the same workload's own forecast:
    four windows of a 100-particle ensemble drawn around the jet with its own random
    streams (400 states of 500x300, 60 M cells); held-out pairs from one window of another
    ensemble.  Reports the training time, held-out RMSE against the plain forecast (and
    persistence for scale), the time of the network forward alone and of the guarded window
    against ten plain model steps, and the fallbacks."""
    from paper_1910_01031_amd import Net, surrogate_window
    from paper_1910_01031_amd import surrogate as sur
    base = W.jet_state(cfg)
    t0 = time.perf_counter()
    pairs = sur.make_pairs(torch, cfg, 400, base, group=cfg.n_particles, spinup_steps=10,
                           windows_per_group=4, stream_base=100)
    held = sur.make_pairs(torch, cfg, 100, base, group=cfg.n_particles, spinup_steps=30,
                          windows_per_group=1, stream_base=900)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    net = Net(cfg.n_particles * cfg.n_cells)
    net.set_params(sur.init_params(0))
    t0 = time.perf_counter()
    hist = sur.train(net, pairs, train_steps, batch=1, log_every=max(1, train_steps // 5))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    held.mu, held.sigma, held.scale = pairs.mu, pairs.sigma, pairs.scale
    rmse, persist = sur.evaluate(torch, net, held, batch=25)
    del pairs, held

    start = ens.clone()
    out = torch.empty_like(ens)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    reps = 10
    for _ in range(2):
        net.forward(start, out)
    e[0].record()
    for r in range(reps):
        net.forward(start, out)
    e[1].record()
    plain = ens.clone()
    e[2].record()
    for r in range(reps):
        ctx.step_ensemble(plain, 10, first_step=500_000 + 10 * r, noise_on_last=True)
    e[3].record()
    sst = start.clone()
    nfs = []
    e[4].record()
    for r in range(reps):
        nf, _ = surrogate_window(ctx, net, sst, 10, 500_000 + 10 * r, drift_tol=1e-4,
                                 noise_scale=3.0)
        nfs.append(nf)
    e[5].record()
    torch.cuda.synchronize()
    fwd_ms = e[0].elapsed_time(e[1]) / reps
    plain_ms = e[2].elapsed_time(e[3]) / reps
    sur_ms = e[4].elapsed_time(e[5]) / reps
    # accuracy on the benchmark ensemble: one deterministic window from the same states
    pdet = start.clone()
    for k in range(10):
        ctx.step_ensemble(pdet, 1, first_step=600_000 + k, noise_on_last=False)
    sdet = start.clone()
    nf_det, drift_w = surrogate_window(ctx, net, sdet, 10, 600_000, drift_tol=1e-4,
                                       noise_scale=0.0)
    net.forward(start, out)
    torch.cuda.synchronize()
    d = (out - pdet).double()
    inc = (pdet - start).double()
    rm = [float(d[:, c].pow(2).mean().sqrt()) for c in range(3)]
    ri = [float(inc[:, c].pow(2).mean().sqrt()) for c in range(3)]
    eta_drift = float(((out[:, 0] - start[:, 0]).double().mean(dim=(1, 2)).abs()).max() / cfg.H)
    drift = drifter_comparison(torch, dev, ctx, net, start, cfg)
    ens.copy_(start)
    if not keep_net:
        net.close()
    flop = SURROGATE_FLOPS_PER_PIXEL * cfg.n_particles * cfg.n_cells
    res = {"train_states": 400, "train_cells": 400 * cfg.n_cells, "train_steps": train_steps,
            "batch_states": 1, "pair_generation_s": gen_s, "train_s": train_s,
            "loss_history": hist,
            "heldout_rmse_eta_hu_hv": rmse.tolist(),
            "heldout_persistence_rmse": persist.tolist(),
            "forward_ms": fwd_ms, "forward_tflops": flop / (fwd_ms / 1e3) / 1e12,
            "forward_mfma_frac": flop / (fwd_ms / 1e3) / 1e12 / BF16_MFMA_PEAK_TFLOPS,
            "window_ms_plain": plain_ms, "window_ms_surrogate": sur_ms,
            "speedup": plain_ms / sur_ms, "fallbacks_per_window": nfs,
            "rmse_vs_plain_eta_hu_hv": rm,
            "window_increment_rms_eta_hu_hv": ri,
            "fallbacks_deterministic": nf_det,
            "max_mass_drift": float(np.max(drift_w)), "max_mean_eta_drift_over_H": eta_drift,
            "drifters_1h": drift}
    return (res, net) if keep_net else res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    cfg = W.paper_scale(args.particles)
    cells = W.buoy_cells(cfg.nx, cfg.ny, 15, 15)
    # the oracle's worker processes are forked before anything touches the GPU
    cpu = None if (args.no_cpu_baseline or args.batched_only) else cpu_baseline(cfg, cells)
    import torch
    from paper_1910_01031_amd import Context, abi

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.batched_only:
        print(json.dumps({"batched": batched_leg(torch, dev, 10)}), flush=True)
        return
    n_cycles = args.warmup + args.steps
    steps_per_cycle = 10

    ctx = Context(cfg, max_obs=len(cells))
    tcfg = cfg.replace(n_particles=1, ensemble_id=0x7FFF)
    tctx = Context(tcfg, max_obs=len(cells))
    base = torch.from_numpy(W.as_f32(W.jet_state(cfg))).to(dev)
    truth = torch.empty((1, 3, cfg.ny, cfg.nx), dtype=torch.float32, device=dev)
    ens = torch.empty((cfg.n_particles, 3, cfg.ny, cfg.nx), dtype=torch.float32, device=dev)
    tctx.init_ensemble(truth, base, stream_index=1)
    ctx.init_ensemble(ens, base, stream_index=0)
    obs = []
    for c in range(n_cycles):
        tctx.step_ensemble(truth, steps_per_cycle, first_step=c * steps_per_cycle, noise_on_last=True)
        y = tctx.observe_moorings(truth, cells, analysis_index=c)
        obs.append(abi.obs_array(cells, y))
    torch.cuda.synchronize()

    def cycle(c, stats=False):
        ctx.step_ensemble(ens, steps_per_cycle, first_step=c * steps_per_cycle, noise_on_last=False)
        return ctx.assimilate(ens, cells, None, analysis_index=c, want_stats=stats, obs=obs[c])

    for c in range(args.warmup):
        cycle(c)
    torch.cuda.synchronize()
    state_idle = gpu_state(torch)

    # timed region: K whole cycles
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps - 1)]
    e0.record()
    for i, c in enumerate(range(args.warmup, n_cycles - 1)):
        cycle(c)
        marks[i].record()
    last = cycle(n_cycles - 1, stats=True)
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    bounds = [e0] + marks + [e1]
    per_cycle = sorted(bounds[i].elapsed_time(bounds[i + 1]) for i in range(args.steps))
    ms_per_step = ms_total / args.steps
    work = cfg.n_particles * cfg.nx * cfg.ny * cfg.n_sub * steps_per_cycle
    value = work * args.steps / (ms_total / 1e3)
    finite = bool(torch.isfinite(ens).all().item())

    # per-kernel durations: the same cycles again with an event pair around every launch
    # (the clock and power state is read half-way, outside the timed region)
    ctx.set_trace(True)
    mid = torch.cuda.Event()
    state_during, busy = None, None
    for c in range(args.warmup, n_cycles):
        cycle(c)
        if c == args.warmup + args.steps // 2:
            mid.record()
            busy = not mid.query()
            state_during = gpu_state(torch)
    torch.cuda.synchronize()
    tr = ctx.trace_read()
    ctx.set_trace(False)
    stage_sum_ms = sum(tr[k][0] for k in ("innovation", "rand_dots", "beta_alpha",
                                          "posterior_coarse", "analysis_update")) / args.steps
    stage_sum_ms += tr["soar"][0] / max(tr["soar"][1], 1)  # one of the SOAR launches per cycle
    # ms per analysis: one event pair around consecutive whole analyses (observation upload
    # included, no per-stage events between the kernels), repeated on the last forecast
    saved = ens.clone()
    reps = 10
    a0 = torch.cuda.Event(enable_timing=True)
    a1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a0.record()
    for r in range(reps):
        ctx.assimilate(ens, cells, None, analysis_index=n_cycles + r, want_stats=False,
                       obs=obs[-1])
    a1.record()
    torch.cuda.synchronize()
    analysis_ms = a0.elapsed_time(a1) / reps
    ens.copy_(saved)
    del saved
    plain_ms = tr["scheme_step"][0] / max(tr["scheme_step"][1], 1)
    launch_cells = cfg.n_particles * cfg.nx * cfg.ny
    bytes_per_launch = BYTES_PER_CELL_STEP * launch_cells
    flops_per_launch = FLOPS_PER_CELL_STEP * launch_cells
    achieved_tflops = flops_per_launch / (plain_ms / 1e3) / 1e12
    achieved_gbs = bytes_per_launch / (plain_ms / 1e3) / 1e9
    counters_current = MEASURED_COUNTERS["source_sha256"] == _kernel_source_hash()
    traffic = MEASURED_COUNTERS["hbm_bytes"] if counters_current else None
    valu = MEASURED_COUNTERS["valu_insts"] if counters_current else None
    issue = valu / (plain_ms * 1e-3 * CLOCK_GHZ * 1e9 * N_CU) if valu is not None else None

    if args.copy_calibration:
        a = torch.empty(90_000_000, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    out = {
        "metric": "particle-cell-steps/s",
        "value": value,
        "unit": "particle-cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "cycle_ms": {"min": per_cycle[0], "median": per_cycle[len(per_cycle) // 2],
                     "max": per_cycle[-1]},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 state, f64 weights/alpha/Cholesky",
        "data": "synthetic",
        "config": {"workload": "paper-scale IEWPF cycle: 500x300 grid, dx 5 km, 100 particles, "
                               "225 moored buoys, 10 model steps x 2 scheme steps + 1 analysis",
                   "nx": cfg.nx, "ny": cfg.ny, "particles": cfg.n_particles,
                   "buoys": int(len(cells)), "scheme_steps_per_cycle": cfg.n_sub * steps_per_cycle},
        "iewpf_ms_per_analysis": analysis_ms,
        "analysis_stage_event_sum_ms": stage_sum_ms,
        "analysis_stats_last": {"beta": last["beta"], "cbar": last["cbar"],
                                "alpha_min": last["alpha_min"], "alpha_max": last["alpha_max"]},
        "state_finite": finite,
        "kernel_ms": {k: (v[0] / v[1] if v[1] else None) for k, v in tr.items()},
        "gpu_state": {"before_timed_region": state_idle, "during_same_cycles_traced": state_during,
                      "gpu_busy_when_read": busy},
        # the stencil's bound: HBM, 24 B per cell and scheme step (one read and one write of
        # eta, hu, hv); the instruction-issue figure beside it
        "roofline": {"bound": "hbm",
                     "kernel": "swe_row_kernel<false, 512, false> (scheme step, full-row form)",
                     "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_ms": plain_ms,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     # measured HBM bytes (counters) per launch over the same duration
                     "traffic_gbs": (traffic / (plain_ms / 1e3) / 1e9
                                     if traffic is not None else None),
                     "alu": {"valu_insts_per_launch": valu,
                             "valu_issue_per_clk_per_cu": issue,
                             "issue_ceiling_measured": VALU_ISSUE_CEILING,
                             "issue_frac": (issue / VALU_ISSUE_CEILING
                                            if issue is not None else None),
                             "algorithmic_flops_per_launch": flops_per_launch,
                             "achieved_tflops": achieved_tflops,
                             "fp32_vector_peak_tflops": FP32_VECTOR_PEAK_TFLOPS},
                     "avg_launch_ms_with_model_error": (tr["scheme_step_noise"][0] /
                                                        max(tr["scheme_step_noise"][1], 1))},
    }
    out["full_covariance"] = full_covariance_leg(torch, ctx, ens, cells, obs, n_cycles)
    out["side"] = side_legs(torch, dev, ctx, ens, cfg)
    if not args.no_batched:
        out["batched"] = batched_leg(torch, dev, 10)
    if not args.no_surrogate:
        out["surrogate"], net = surrogate_leg(torch, dev, ctx, ens, cfg, args.surrogate_train_steps,
                                              keep_net=True)
        ctx.close()
        tctx.close()
        del ens, truth
        if not args.no_large_ensemble:
            out["large_ensemble"] = large_ensemble_leg(torch, net)
        net.close()
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
