"""Drifter observations (eq. drifterObservation), the standard particle filter's weights
and resampling (Section "Standard particle filter", eq. standardParticleFilterWeight), and
the tiny drifter-observing data-assimilation run end to end, against the FP64 oracle,
through the C ABI.

Tolerances: float64 observation synthesis and log-weights 1e-12 relative; integer cells and
parents bit-exact (the oracle's resampling takes the GPU's float64 log-weights, so both
sides decide the integers from the same values); float32 state 1e-5 relative per field.

The end-to-end run (32x32 grid, 10 particles, 4 drifters observing every 5 minutes for one
hour, 12 analyses): the truth run and its drifters are the oracle's (float64, own random
stream, model error after every step), so no input comes from the GPU path.  Every cycle
the GPU forecasts the oracle's analysed ensemble (rounded to float32) and the oracle
forecasts the same input; the GPU then analyses its own forecast and the oracle analyses
that same forecast (beta moves ~1e-8 relative per 1e-7 change of the forecast, so both sides
start from one input), and the weights the GPU realises are equal to the target.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import drifters as odr
from oracle import ensemble as oens
from oracle import iewpf as oiewpf
from oracle import observe as oobs
from oracle import philox as ophil
from oracle import resample as ores

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1910_01031_amd import load
    load()
    return torch, torch.device("cuda:0")


def _near_ensemble(cfg, spread=0.003):
    base = oens.init_member(cfg, None, 0, 999)
    small = cfg.replace(init_std=spread)
    ens = W.as_f32(np.stack([oens.init_member(small, base, 1, i)
                             for i in range(cfg.n_particles)]))
    truth = oens.init_member(small.replace(ensemble_id=77), base, 1, 0)
    return base, ens, truth


def test_observe_drifters_parity(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    cfg = W.tiny().replace(ensemble_id=77)
    rng = np.random.default_rng(21)
    lx, ly = cfg.nx * cfg.dx, cfg.ny * cfg.dy
    n = 13  # ragged: more than one Philox block of four normals, not a multiple of four
    prev = np.stack([rng.uniform(-lx, 2 * lx, n), rng.uniform(-ly, 2 * ly, n)], axis=1)
    prev[0] = [lx - 10.0, 0.5 * ly]           # crosses x = L_x during the interval
    now = prev + rng.normal(scale=300.0, size=(n, 2))
    now[0] = [lx + 250.0, 0.5 * ly + 20.0]
    ctx = Context(cfg, max_obs=16)
    pn, pp = torch.from_numpy(now).to(dev), torch.from_numpy(prev).to(dev)
    for aidx in (0, 7):
        cells, y = ctx.observe_drifters(pn, pp, 300.0, analysis_index=aidx)
        noise = ophil.normals(2 * n, cfg.seed, aidx, ophil.TAG_OBS, 77, 1).reshape(n, 2)
        ref = oobs.drifter_obs(now, prev, 300.0, cfg.H, cfg.obs_sigma, noise)
        assert np.array_equal(cells, oobs.obs_cell(now, cfg.dx, cfg.dy, cfg.nx, cfg.ny))
        assert np.abs(y - ref).max() < 1e-12 * np.abs(ref).max()
    assert cells[0, 0] == 0  # the unwrapped position lx + 250 m lies in cell 0
    ctx.close()


def test_sir_log_weights_parity(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    cfg = W.tiny()
    _, ens, truth = _near_ensemble(cfg, spread=0.02)
    cells = np.array([[3, 5], [17, 30], [17, 30], [31, 0], [12, 12], [0, 31]], dtype=np.int32)
    noise = ophil.normals(12, cfg.seed, 2, ophil.TAG_OBS, 77, 0).reshape(6, 2)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, noise)
    ctx = Context(cfg, max_obs=8)
    st = torch.from_numpy(ens).to(dev)
    lw = torch.zeros(cfg.n_particles, dtype=torch.float64, device=dev)
    w = torch.zeros_like(lw)
    d = np.stack([oobs.innovations(ens[i].astype(np.float64), cells, y, cfg.H)
                  for i in range(cfg.n_particles)])
    for r_scale in (1.0, 10.0):
        ctx.sir_log_weights(st, cells, y, lw, w, r_scale=r_scale)
        got = lw.cpu().numpy()
        ref = ores.sir_log_weights(d, cfg.obs_sigma * np.sqrt(r_scale))
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max(), r_scale
        e = np.exp(ref - ref.max())
        assert np.abs(w.cpu().numpy() - e / e.sum()).max() < 1e-12
    ctx.close()


def test_sir_analysis_parents_and_states_bit_exact(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    cfg = W.tiny().replace(n_particles=37)
    _, ens, truth = _near_ensemble(cfg, spread=0.01)
    cells = np.array([[8, 8], [24, 8], [8, 24], [24, 24]], dtype=np.int32)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, np.zeros((4, 2)))
    ctx = Context(cfg, max_obs=8)
    ctx.set_scheme(2)
    lw = torch.zeros(cfg.n_particles, dtype=torch.float64, device=dev)
    for aidx in range(3):
        st = torch.from_numpy(ens.copy()).to(dev)
        ctx.sir_log_weights(st, cells, y, lw)
        glw = lw.cpu().numpy()
        stats = ctx.assimilate(st, cells, y, analysis_index=aidx)
        par = ctx.sir_parents()
        u = ores.resample_uniforms(cfg.n_particles, cfg.seed, aidx, cfg.ensemble_id)
        ref, _ = ores.residual_resample(glw, u)
        assert np.array_equal(par, ref)
        assert np.array_equal(st.cpu().numpy(), ens[ref])
        assert stats["c_min"] == -2.0 * glw.max() and stats["c_max"] == -2.0 * glw.min()
        assert stats["argmin_beta"] == int(np.argmax(glw))
    # identical particles: equal weights, exact multiples, no residual draw
    same = np.repeat(ens[:1], cfg.n_particles, axis=0)
    st = torch.from_numpy(same.copy()).to(dev)
    ctx.assimilate(st, cells, y, analysis_index=9)
    assert np.array_equal(ctx.sir_parents(), np.arange(cfg.n_particles))
    ctx.close()


def test_sir_nonfinite_weight_leaves_the_state_untouched(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context, IewpfError, abi
    cfg = W.tiny()
    _, ens, truth = _near_ensemble(cfg)
    cells = np.array([[8, 8], [24, 24]], dtype=np.int32)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, np.zeros((2, 2)))
    ens[5, 2, 24, 24] = np.inf
    ctx = Context(cfg, max_obs=4)
    ctx.set_scheme(2)
    st = torch.from_numpy(ens.copy()).to(dev)
    with pytest.raises(IewpfError) as e:
        ctx.assimilate(st, cells, y, analysis_index=0, want_stats=False)
    assert e.value.code == abi.IEWPF_E_NONFINITE and "particle 5" in str(e.value)
    assert np.array_equal(st.cpu().numpy().view(np.int32), ens.view(np.int32))
    ctx.close()


def _truth_run(cfg, truth0, pos0, n_cycles, steps):
    """Oracle truth (float64) with its drifters: model error after every model step, Heun
    drifters; per cycle the drifter observations and their cells."""
    tcfg = cfg.replace(ensemble_id=77)
    psi = truth0.copy()
    pos = pos0.copy()
    out = []
    for c in range(n_cycles):
        prev = pos.copy()
        for s in range(steps):
            nxt = oens.step_member(psi, tcfg, 0, c * steps + s, 1, noise_on_last=True)
            pos = odr.heun_step(pos, psi, nxt, cfg, cfg.dt)
            psi = nxt
        noise = ophil.normals(2 * len(pos), cfg.seed, c, ophil.TAG_OBS, 77, 1).reshape(-1, 2)
        y = oobs.drifter_obs(pos, prev, steps * cfg.dt, cfg.H, cfg.obs_sigma, noise)
        out.append((oobs.obs_cell(pos, cfg.dx, cfg.dy, cfg.nx, cfg.ny), y))
    return out


def test_tiny_drifter_assimilation_end_to_end(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    cfg = W.tiny()
    steps, n_cycles = cfg.obs_every, 12
    base, ens, truth0 = _near_ensemble(cfg)
    pos0 = W.drifter_lattice(cfg, 2, 2)
    obs = _truth_run(cfg, truth0, pos0, n_cycles, steps)
    ctx = Context(cfg, max_obs=4)
    consts = oiewpf.AnalysisConstants(cfg)
    start = ens
    for c, (cells, y) in enumerate(obs):
        st = torch.from_numpy(start.copy()).to(dev)
        ctx.step_ensemble(st, steps, first_step=c * steps, noise_on_last=False)
        fc = st.cpu().numpy().astype(np.float64)
        ref_f = np.stack([oens.step_member(start[i], cfg, i, c * steps, steps, noise_on_last=False)
                          for i in range(cfg.n_particles)])
        for f in range(3):
            err = np.abs(fc[:, f] - ref_f[:, f]).max() / np.abs(ref_f[:, f]).max()
            assert err < TOL, (c, "forecast", f, err)
        stats = ctx.assimilate(st, cells, y, analysis_index=c)
        got = st.cpu().numpy().astype(np.float64)
        sc = ctx.particle_scalars()
        ref, info = oiewpf.analysis(fc, cells, y, cfg, c, consts=consts)
        for f in range(3):
            err = np.abs(got[:, f] - ref[:, f]).max() / np.abs(ref[:, f]).max()
            assert err < TOL, (c, "analysis", f, err)
        # beta = (cbar - c_i)/zeta_i + 1 at its argmin; zeta_i is a sum of squares of the
        # normals, which the GPU rounds to float32 (relative 2^-24 each), so |d zeta / zeta|
        # <= 2^-23 and |d beta| <= 2^-23 |beta - 1| (twice that as the bound) plus float64
        # rounding
        tol_beta = 2.0 ** -22 * abs(info["beta"] - 1.0) + 1e-12
        assert abs(stats["beta"] - info["beta"]) < tol_beta, (c, stats["beta"], info["beta"])
        w = oiewpf.realized_weight(sc[:, 3], sc[:, 1], sc[:, 2], stats["beta"], sc[:, 0],
                                   cfg.n_psi)
        assert np.abs(w - stats["cbar"]).max() < 1e-9 * cfg.n_psi, c
        _say(f"cycle {c}: cells {cells.tolist()} beta {stats['beta']:.6f}")
        start = W.as_f32(ref)
    ctx.close()
