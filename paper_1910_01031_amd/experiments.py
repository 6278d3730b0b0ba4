"""Statistical checks of the filter on the GPU (Section "Rank histograms for IEWPF" and Section
"Collapse of the standard particle filter"), at reduced scale.

rank_histograms: independent data-assimilation experiments, each with its own truth drawn
  from the same prior as its ensemble.  Moorings in the western half of the domain are
  assimilated every 5 minutes, then a 1-hour forecast follows.  For hu and hv at six cells
  at least 80 cells apart, the rank of the observed truth (truth + observation error)
  among the ensemble values (member + observation error) is recorded.  A correct filter
  gives flat histograms.  Experiments run 16 at a time as one batch (one hipGraph replay
  per cycle).

sir_collapse: an ensemble assimilates drifter observations with the IEWPF, runs to the
  next observation time, and the standard particle filter's normalised weights (depending on
  the innovations and R only, computed by the library) are taken for random subsets of the
  drifters.  For each subset size, the mean number of particles whose weight exceeds 1/N_e
  (those residual resampling is guaranteed to keep) is reported, for R and for 10 R.

drift_forecast: the large-ensemble drift forecast (1000 particles, 24 h of analyses on the
  225 moorings, then 12 h of drifter forecast with the plain model and the surrogate side by
  side): forecast error and spread per hour, throughput.

Every model step, analysis, observation and weight runs in the library's kernels; the
ranks and the counts of weights above 1/N_e are taken here from a handful of values read
back.
Run as `python -m paper_1910_01031_amd.experiments` from the repository root (it uses the
seeded workload recipes in `workloads/`).
"""
from __future__ import annotations

import math

import numpy as np

from . import abi


def _workloads():
    import workloads
    return workloads


def rank_histograms(torch, n_experiments: int = 128, n_particles: int = 40, da_hours: float = 6.0,
                    forecast_hours: float = 1.0, spinup_hours: float = 1.0, batch: int = 16,
                    seed: int = 0, probe=None):
    """Returns dict(hist=[2][6][N_e+1] int (hu, hv x cells), accumulated=[2][N_e+1],
    chi2 / p-value of each accumulated histogram against the uniform one)."""
    W = _workloads()
    from scipy.stats import chi2 as chi2_dist
    dev = torch.device("cuda")
    cfg0 = W.paper_scale(n_particles)
    cells = W.buoy_cells(cfg0.nx // 2, cfg0.ny, 8, 15)  # 120 moorings, western half
    if probe is None:  # six cells at least 80 cells apart, inside and east of the moorings
        probe = [(40, 20), (120, 120), (200, 220), (60, 270), (180, 50), (300, 170)]
    base = torch.from_numpy(W.as_f32(W.jet_state(cfg0))).to(dev)
    steps = 10                                          # model steps per 5-minute cycle
    n_spin = int(round(spinup_hours * 12)) * steps
    n_cyc = int(round(da_hours * 12))
    n_fc = int(round(forecast_hours * 12)) * steps
    rng = np.random.default_rng(seed)
    sig = cfg0.obs_sigma
    hist = np.zeros((2, len(probe), n_particles + 1), dtype=np.int64)
    for b0 in range(0, n_experiments, batch):
        ne_b = min(batch, n_experiments - b0)
        ctxs, ens, tctxs, truths = [], [], [], []
        for e in range(b0, b0 + ne_b):
            c = abi.Context(cfg0.replace(ensemble_id=1000 + e, seed=cfg0.seed + seed),
                            max_obs=len(cells))
            st = torch.empty((n_particles, 3, cfg0.ny, cfg0.nx), device=dev)
            c.init_ensemble(st, base, stream_index=e)
            c.step_ensemble(st, n_spin, first_step=0, noise_on_last=True)
            t = abi.Context(cfg0.replace(n_particles=1, ensemble_id=100000 + e,
                                         seed=cfg0.seed + seed), max_obs=len(cells))
            tr = torch.empty((1, 3, cfg0.ny, cfg0.nx), device=dev)
            t.init_ensemble(tr, base, stream_index=e)   # same prior, own random stream
            t.step_ensemble(tr, n_spin, first_step=0, noise_on_last=True)
            ctxs.append(c)
            ens.append(st)
            tctxs.append(t)
            truths.append(tr)
        bt = abi.Batch(ctxs, ens)
        for e in range(ne_b):
            bt.set_cells(e, cells)
        for cyc in range(n_cyc):
            first = n_spin + cyc * steps
            ys = []
            for t, tr in zip(tctxs, truths):
                t.step_ensemble(tr, steps, first_step=first, noise_on_last=True)
                ys.append(t.observe_moorings(tr, cells, analysis_index=cyc))
            bt.cycle(steps, first, cyc, ys, use_graph=True)
        first = n_spin + n_cyc * steps
        for e in range(ne_b):
            ctxs[e].step_ensemble(ens[e], n_fc, first_step=first, noise_on_last=True)
            tctxs[e].step_ensemble(truths[e], n_fc, first_step=first, noise_on_last=True)
        torch.cuda.synchronize()
        for e in range(ne_b):
            for p, (j, k) in enumerate(probe):
                vals = ens[e][:, 1:3, k, j].double().cpu().numpy()      # [N_e][hu, hv]
                tv = truths[e][0, 1:3, k, j].double().cpu().numpy()
                for v in range(2):
                    member = vals[:, v] + sig * rng.standard_normal(n_particles)
                    observed = tv[v] + sig * rng.standard_normal()
                    hist[v, p, int(np.sum(member < observed))] += 1
        bt.close()
        for c in ctxs + tctxs:
            c.close()
    acc = hist.sum(axis=1)
    out = {"n_experiments": n_experiments, "n_particles": n_particles, "da_hours": da_hours,
           "forecast_hours": forecast_hours, "cells": probe, "hist": hist.tolist(),
           "accumulated": acc.tolist()}
    for v, name in enumerate(("hu", "hv")):
        expect = acc[v].sum() / (n_particles + 1)
        chi2 = float(((acc[v] - expect) ** 2 / expect).sum())
        out[f"chi2_{name}"] = chi2
        out[f"p_{name}"] = float(chi2_dist.sf(chi2, n_particles))
    return out


def sir_collapse(torch, n_particles: int = 100, da_hours: float = 6.0, n_drifters: int = 64,
                 max_observed: int = 10, subsets: int = 50, seed: int = 0):
    """Mean number of particles with standard-particle-filter weight > 1/N_e for 1..max_observed
    observed drifters (random subsets), with R and with 10 R.

    The truth's drifters observe the current (eq. drifterObservation, observations every
    5 minutes from the displacement over the interval); the ensemble assimilates all of
    them with the IEWPF for da_hours and runs to the next observation time, where the
    library computes the standard filter's normalised weights (eq.
    standardParticleFilterWeight) from the eta-compensated innovations of each subset."""
    W = _workloads()
    dev = torch.device("cuda")
    cfg = W.paper_scale(n_particles)
    base = torch.from_numpy(W.as_f32(W.jet_state(cfg))).to(dev)
    ctx = abi.Context(cfg, max_obs=n_drifters)
    ens = torch.empty((n_particles, 3, cfg.ny, cfg.nx), device=dev)
    ctx.init_ensemble(ens, base, stream_index=0)
    tctx = abi.Context(cfg.replace(n_particles=1, ensemble_id=0x7FFF), max_obs=n_drifters)
    truth = torch.empty((1, 3, cfg.ny, cfg.nx), device=dev)
    tctx.init_ensemble(truth, base, stream_index=1)
    side = int(round(math.sqrt(n_drifters)))
    pos = torch.from_numpy(W.drifter_lattice(cfg, side, side)[None]).to(dev)
    steps = cfg.obs_every

    n_cyc = int(round(da_hours * 12))
    for cyc in range(n_cyc + 1):
        prev = pos.clone()
        tctx.forecast_drifters(truth, pos, steps, first_step=cyc * steps)  # truth and drifters
        cells, y = tctx.observe_drifters(pos[0], prev[0], steps * cfg.dt, analysis_index=cyc)
        ctx.step_ensemble(ens, steps, first_step=cyc * steps, noise_on_last=False)
        if cyc < n_cyc:
            ctx.assimilate(ens, cells, y, analysis_index=cyc, want_stats=False)
    rng = np.random.default_rng(seed)
    lw = torch.zeros(n_particles, dtype=torch.float64, device=dev)
    w = torch.zeros_like(lw)
    out = {"n_particles": n_particles, "da_hours": da_hours, "n_drifters": n_drifters,
           "observed": list(range(1, max_observed + 1)), "observation": "drifters"}
    for label, r_scale in (("R", 1.0), ("10R", 10.0)):
        means = []
        for m in range(1, max_observed + 1):
            kept = []
            for _ in range(subsets):
                sub = np.sort(rng.choice(n_drifters, size=m, replace=False))
                ctx.sir_log_weights(ens, cells[sub], y[sub], lw, w, r_scale=r_scale)
                kept.append(int(np.sum(w.cpu().numpy() > 1.0 / n_particles)))
            means.append(float(np.mean(kept)))
        out[f"kept_{label}"] = means
    ctx.close()
    tctx.close()
    return out


def _errors(torch, pos, truth_pos, lx, ly):
    """E(t) (eq. errorNorm: RMS distance of every member's drifter from the true drifter)
    and RMSE(t) (the same about the ensemble mean), minimum-image distances, metres."""
    L = torch.tensor([lx, ly], dtype=torch.float64, device=pos.device)

    def mi(d):
        return torch.remainder(d + 0.5 * L, L) - 0.5 * L

    err = float(mi(pos - truth_pos[None]).pow(2).sum(dim=-1).mean().sqrt())
    centre = pos[0:1] + mi(pos - pos[0:1]).mean(dim=0, keepdim=True)
    rmse = float(mi(pos - centre).pow(2).sum(dim=-1).mean().sqrt())
    return err, rmse


def drift_forecast(torch, n_particles: int = 1000, da_hours: float = 24.0,
                   forecast_hours: float = 12.0, n_drifters: int = 64, train_steps: int = 1000,
                   net_particles: int = 100, net=None, keep_positions: bool = False):
    """The large-ensemble drift forecast: n_particles through da_hours of two-stage IEWPF on
    the 225 moorings, then a forecast of n_drifters drifters per particle (bilinear velocity,
    Heun, dt = 30 s) with the plain model and with the surrogate (trained first on the
    workload's own forecast windows unless a trained `net` is given, plain re-step above a
    mass drift of 1e-4, one model-error draw scaled by 3 per window).  Reports, per forecast
    hour, the forecast error E(t) against the true drifters and the spread RMSE(t) for both
    (eq. errorPerEnsembleDrifter, eq. errorNorm; minimum-image distances), and the
    throughput.  keep_positions: also return the positions of every hour (float64 arrays:
    truth [hours][n_drifters][2], each form [hours][n_particles][n_drifters][2])."""
    import time
    W = _workloads()
    from . import surrogate as sur
    dev = torch.device("cuda")
    cfg = W.large_ensemble().replace(n_particles=n_particles)
    cells = W.buoy_cells(cfg.nx, cfg.ny, 15, 15)
    lx, ly = cfg.nx * cfg.dx, cfg.ny * cfg.dy
    base = torch.from_numpy(W.as_f32(W.jet_state(cfg))).to(dev)
    ctx = abi.Context(cfg, max_obs=len(cells))
    ens = torch.empty((n_particles, 3, cfg.ny, cfg.nx), device=dev)
    ctx.init_ensemble(ens, base, stream_index=0)
    tctx = abi.Context(cfg.replace(n_particles=1, ensemble_id=0x7FFF), max_obs=len(cells))
    truth = torch.empty((1, 3, cfg.ny, cfg.nx), device=dev)
    tctx.init_ensemble(truth, base, stream_index=1)
    steps = 10
    n_cyc = int(round(da_hours * 12))
    obs = []
    for cyc in range(n_cyc):  # the truth run and its observations, before timing
        tctx.step_ensemble(truth, steps, first_step=cyc * steps, noise_on_last=True)
        obs.append(abi.obs_array(cells, tctx.observe_moorings(truth, cells, analysis_index=cyc)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for cyc in range(n_cyc):
        ctx.step_ensemble(ens, steps, first_step=cyc * steps, noise_on_last=False)
        ctx.assimilate(ens, cells, None, analysis_index=cyc, want_stats=False, obs=obs[cyc])
    torch.cuda.synchronize()
    da_s = time.perf_counter() - t0
    # surrogate trained on the workload's own windows (a 100-particle ensemble of this grid)
    pairs = None
    if net is None:
        pairs = sur.make_pairs(torch, cfg.replace(n_particles=net_particles), 4 * net_particles,
                               W.jet_state(cfg), group=net_particles, spinup_steps=10,
                               windows_per_group=4, stream_base=100)
    own_net = net is None
    if own_net:
        net = abi.Net(net_particles * cfg.n_cells)
        net.set_params(sur.init_params(0))
        sur.train(net, pairs, train_steps, batch=1)
    del pairs
    side = int(round(math.sqrt(n_drifters)))
    lattice = torch.from_numpy(W.drifter_lattice(cfg, side, side)).to(dev)
    pos_t = lattice[None].clone()
    runs = {"plain": [ens.clone(), lattice[None].repeat(n_particles, 1, 1).contiguous()],
            "surrogate": [ens.clone(), lattice[None].repeat(n_particles, 1, 1).contiguous()]}
    del ens
    hours = int(round(forecast_hours))
    first = n_cyc * steps
    out = {"n_particles": n_particles, "da_hours": da_hours, "forecast_hours": hours,
           "n_drifters": n_drifters, "da_seconds": da_s,
           "da_particle_cell_steps_per_s": n_particles * cfg.n_cells * cfg.n_sub * steps * n_cyc / da_s,
           "hour": list(range(1, hours + 1)), "plain": {"E": [], "RMSE": [], "seconds": 0.0},
           "surrogate": {"E": [], "RMSE": [], "seconds": 0.0, "fallbacks": 0}}
    kept = {"truth": [], "plain": [], "surrogate": []}
    for h in range(hours):
        f0 = first + h * 12 * steps
        tctx.forecast_drifters(truth, pos_t, 12 * steps, first_step=f0)
        for name, (st, pos) in runs.items():
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if name == "plain":
                ctx.forecast_drifters(st, pos, 12 * steps, first_step=f0)
            else:
                out[name]["fallbacks"] += abi.forecast_drifters_surrogate(
                    ctx, net, st, pos, 12, steps, f0, 1e-4, 3.0)
            torch.cuda.synchronize()
            out[name]["seconds"] += time.perf_counter() - t1
            e, r = _errors(torch, pos, pos_t[0], lx, ly)
            out[name]["E"].append(e)
            out[name]["RMSE"].append(r)
            if keep_positions:
                kept[name].append(pos.cpu().numpy())
        if keep_positions:
            kept["truth"].append(pos_t[0].cpu().numpy())
    cells_steps = n_particles * cfg.n_cells * cfg.n_sub * steps * 12 * hours
    for name in runs:
        out[name]["particle_cell_steps_per_s"] = cells_steps / out[name]["seconds"]
    out["speedup"] = out["plain"]["seconds"] / out["surrogate"]["seconds"]
    if own_net:
        net.close()
    ctx.close()
    tctx.close()
    if keep_positions:
        out["positions"] = {k: np.stack(v) for k, v in kept.items()}
    return out


if __name__ == "__main__":
    import argparse
    import json
    import sys
    import time

    import torch

    ap = argparse.ArgumentParser(description="rank histograms and SIR collapse (reduced scale)")
    ap.add_argument("--experiments", type=int, default=128)
    ap.add_argument("--da-hours", type=float, default=6.0)
    ap.add_argument("--skip-rank", action="store_true")
    ap.add_argument("--skip-sir", action="store_true")
    ap.add_argument("--drift", action="store_true", help="also the large-ensemble drift forecast")
    ap.add_argument("--drift-particles", type=int, default=1000)
    a = ap.parse_args()
    res = {}
    if not a.skip_rank:
        t0 = time.perf_counter()
        res["rank_histograms"] = rank_histograms(torch, n_experiments=a.experiments,
                                                 da_hours=a.da_hours)
        res["rank_histograms"]["seconds"] = time.perf_counter() - t0
        print("rank histograms done", file=sys.stderr, flush=True)
    if not a.skip_sir:
        t0 = time.perf_counter()
        res["sir_collapse"] = sir_collapse(torch, da_hours=a.da_hours)
        res["sir_collapse"]["seconds"] = time.perf_counter() - t0
    if a.drift:
        t0 = time.perf_counter()
        res["drift_forecast"] = drift_forecast(torch, n_particles=a.drift_particles)
        res["drift_forecast"]["seconds"] = time.perf_counter() - t0
    print(json.dumps(res), flush=True)
