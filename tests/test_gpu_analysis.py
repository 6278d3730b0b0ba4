"""GPU parity of the IEWPF analysis (and its host precompute), observation synthesis,
drifters and residual resampling against the FP64 oracle, through the C ABI.

Tolerances: float64 host precompute 1e-12 relative; float64 per-particle scalars
(c_i, gamma, zeta, alpha, beta) 1e-9 relative (the only float32 inputs are the state
values and the normals, both identical on the two sides up to the float32 rounding of
the normals); float32 state 1e-5 relative per field; integers bit-exact."""
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


def _ensemble_near(cfg, ne, spread, seed_stream=1, base_state=None):
    base = oens.init_member(cfg, None, 0, 999) if base_state is None else base_state
    small = cfg.replace(init_std=spread)
    ens = np.stack([oens.init_member(small, base, seed_stream, i) for i in range(ne)])
    truth = oens.init_member(small.replace(ensemble_id=77), base, seed_stream, 0)
    return W.as_f32(ens), truth


def test_precompute_matches_oracle(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    for cfg in (W.tiny(), W.paper_scale(2), W.Config(nx=70, ny=56, dx=5e3, dy=4e3, c_omega=7),
                W.Config(nx=45, ny=45, dx=5e3, dy=5e3, c_omega=5)):
        _say(f"precompute {cfg.nx}x{cfg.ny} c={cfg.c_omega}")
        ctx = Context(cfg, max_obs=4)
        consts = oiewpf.AnalysisConstants(cfg)
        S = ctx.read_buffer(3, (2, 2), np.float64)
        Sc = ctx.read_buffer(4, (2, 2), np.float64)
        Ah = ctx.read_buffer(5, (49, 49), np.float64)
        w = ctx.read_buffer(8, (5, 5), np.float64)
        assert np.abs(w - consts.w).max() < 1e-13 * np.abs(w).max()
        assert np.abs(S - consts.S).max() < 1e-11 * np.abs(S).max()
        assert np.abs(Sc - consts.Sc).max() < 1e-11 * np.abs(Sc).max()
        assert np.abs(Ah - consts.Ahalf).max() < 1e-10
        # pull windows = the literal per-observation chain of the oracle
        wx, wy = ctx.window_size()
        win = ctx.read_buffer(6, (2, 3, wy, wx), np.float32).astype(np.float64)
        jo, ko = 11, 13
        for b, (su, sv) in enumerate(((1.0, 0.0), (0.0, 1.0))):
            ref = oiewpf.pull_one(su, sv, jo, ko, cfg, consts.w)
            rx = (wx - 1) // 2 if wx < cfg.nx else None
            ry = (wy - 1) // 2 if wy < cfg.ny else None
            got = np.zeros_like(ref)
            for iy in range(wy):
                k = (ko + (iy - ry if ry is not None else iy)) % cfg.ny
                for ix in range(wx):
                    j = (jo + (ix - rx if rx is not None else ix)) % cfg.nx
                    got[:, k, j] += win[b, :, iy, ix]
            for f in range(3):
                assert np.abs(got[f] - ref[f]).max() < 1e-6 * np.abs(ref[f]).max(), (b, f)
        ctx.close()


def _gpu_analysis(torch, dev, cfg, ens32, cells, y, aidx, max_obs):
    from paper_1910_01031_amd import Context
    ctx = Context(cfg, max_obs=max_obs)
    st = torch.from_numpy(np.ascontiguousarray(ens32)).to(dev)
    stats = ctx.assimilate(st, cells, y, analysis_index=aidx)
    torch.cuda.synchronize()
    sc = ctx.particle_scalars()
    out = st.cpu().numpy().astype(np.float64)
    ctx.close()
    return out, stats, sc


def _check_scalars(stats, sc, info, n_psi):
    assert abs(stats["beta"] - info["beta"]) < 1e-9 * abs(info["beta"])
    assert abs(stats["cbar"] - info["cbar"]) < 1e-9 * abs(info["cbar"])
    assert np.abs(sc[:, 0] - info["c"]).max() < 1e-9 * np.abs(info["c"]).max()
    assert np.abs(sc[:, 1] - info["gamma"]).max() < 1e-7 * n_psi
    assert np.abs(sc[:, 2] - info["zeta"]).max() < 1e-7 * n_psi
    assert np.abs(sc[:, 3] - info["alpha"]).max() < 1e-7
    # equal weights on the GPU's own float64 scalars
    w = oiewpf.realized_weight(sc[:, 3], sc[:, 1], sc[:, 2], stats["beta"], sc[:, 0], n_psi)
    assert np.abs(w - stats["cbar"]).max() < 1e-9 * n_psi


def test_analysis_parity_tiny(torch_dev):
    torch, dev = torch_dev
    _say("analysis parity tiny (32x32, 10 particles, 4 moorings)")
    cfg = W.tiny()
    ens, truth = _ensemble_near(cfg, cfg.n_particles, 0.003)
    cells = np.array([[8, 8], [24, 8], [8, 24], [24, 24]], dtype=np.int32)
    noise = ophil.normals(8, cfg.seed, 0, ophil.TAG_OBS, 77, 0).reshape(4, 2)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, noise)
    got, stats, sc = _gpu_analysis(torch, dev, cfg, ens, cells, y, 5, 8)
    ref, info = oiewpf.analysis(ens.astype(np.float64), cells, y, cfg, 5)
    _check_scalars(stats, sc, info, cfg.n_psi)
    for f in range(3):
        err = np.abs(got[:, f] - ref[:, f]).max() / np.abs(ref[:, f]).max()
        _say(f"  field {f} rel err {err}")
        assert err < TOL


def test_repeated_cells_reuse_lists_bit_identical(torch_dev):
    """Analyses on one context whose cells repeat (the device lists are reused, only y is
    uploaded), change, return, and follow an observation synthesis that rewrites the device
    cells: each equals the same analysis on a fresh context, bit for bit."""
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    cfg = W.tiny()
    ens, truth = _ensemble_near(cfg, cfg.n_particles, 0.003)
    cells_a = np.array([[8, 8], [24, 8], [8, 24], [24, 24]], dtype=np.int32)
    cells_b = np.array([[3, 30], [17, 5], [29, 12]], dtype=np.int32)
    plan = [(cells_a, 1), (cells_a, 2), (cells_b, 3), (cells_a, 4), ("observe", 5), (cells_a, 6)]
    ctx = Context(cfg, max_obs=8)
    tr = torch.from_numpy(np.ascontiguousarray(W.as_f32(truth[None]))).to(dev)
    st = torch.from_numpy(np.ascontiguousarray(ens)).to(dev)
    for cells, aidx in plan:
        if isinstance(cells, str):
            _say("  observation synthesis on the same context (cells b)")
            ctx.observe_moorings(tr, cells_b, analysis_index=aidx)
            continue
        _say(f"  analysis {aidx}: {len(cells)} cells")
        noise = ophil.normals(2 * len(cells), cfg.seed, aidx, ophil.TAG_OBS, 77, 0).reshape(-1, 2)
        y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, noise)
        before = st.cpu().numpy()
        ctx.assimilate(st, cells, y, analysis_index=aidx)
        torch.cuda.synchronize()
        fresh, _, _ = _gpu_analysis(torch, dev, cfg, before, cells, y, aidx, 8)
        assert np.array_equal(st.cpu().numpy().astype(np.float64), fresh), aidx
    ctx.close()


def test_analysis_parity_overlapping_drifters(torch_dev):
    # drifters closer than the pull radius, two in the same cell, blocks overlapping
    torch, dev = torch_dev
    _say("analysis parity, overlapping observations (64x48)")
    cfg = W.Config(nx=64, ny=48, dx=1e4, dy=1e4, c_omega=4, n_particles=6, me_std=2e-3)
    ens, truth = _ensemble_near(cfg, 6, 0.003)
    cells = np.array([[10, 10], [12, 11], [12, 11], [40, 30], [63, 47], [0, 0]], dtype=np.int32)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, np.zeros((6, 2)))
    got, stats, sc = _gpu_analysis(torch, dev, cfg, ens, cells, y, 2, 8)
    ref, info = oiewpf.analysis(ens.astype(np.float64), cells, y, cfg, 2)
    _check_scalars(stats, sc, info, cfg.n_psi)
    for f in range(3):
        err = np.abs(got[:, f] - ref[:, f]).max() / np.abs(ref[:, f]).max()
        assert err < TOL, (f, err)


def test_analysis_parity_more_observations_than_lanes(torch_dev):
    # 83 moorings on 64x48: every strip of the update sees more observations than a wave
    # has lanes (the ones past 64 are read from the list), 5 particles (a partial group)
    torch, dev = torch_dev
    _say("analysis parity, 83 observations per strip (64x48)")
    cfg = W.Config(nx=64, ny=48, dx=1e4, dy=1e4, c_omega=4, n_particles=5, me_std=2e-3)
    ens, truth = _ensemble_near(cfg, 5, 0.003)
    rng = np.random.default_rng(83)
    flat = rng.choice(cfg.nx * cfg.ny, size=83, replace=False)
    cells = np.stack([flat % cfg.nx, flat // cfg.nx], axis=1).astype(np.int32)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, np.zeros((83, 2)))
    got, stats, sc = _gpu_analysis(torch, dev, cfg, ens, cells, y, 3, 96)
    ref, info = oiewpf.analysis(ens.astype(np.float64), cells, y, cfg, 3)
    _check_scalars(stats, sc, info, cfg.n_psi)
    for f in range(3):
        err = np.abs(got[:, f] - ref[:, f]).max() / np.abs(ref[:, f]).max()
        _say(f"  field {f} rel err {err}")
        assert err < TOL, (f, err)


def test_analysis_no_observations(torch_dev):
    torch, dev = torch_dev
    cfg = W.tiny().replace(n_particles=4)
    ens, _ = _ensemble_near(cfg, 4, 0.003)
    cells = np.zeros((0, 2), dtype=np.int32)
    y = np.zeros((0, 2))
    got, stats, sc = _gpu_analysis(torch, dev, cfg, ens, cells, y, 1, 4)
    ref, info = oiewpf.analysis(ens.astype(np.float64), cells, y, cfg, 1)
    assert stats["beta"] == info["beta"] == 1.0
    for f in range(3):
        err = np.abs(got[:, f] - ref[:, f]).max() / np.abs(ref[:, f]).max()
        assert err < TOL


def test_analysis_paper_scale_sampled(torch_dev):
    # 500x300, 100 particles, 225 buoys: all per-particle scalars, two sampled states
    torch, dev = torch_dev
    _say("analysis parity paper scale (sampled particles)")
    cfg = W.paper_scale()
    jet = W.jet_state(cfg)
    base = oens.init_member(cfg, jet, 0, 999)
    ens, truth = _ensemble_near(cfg, cfg.n_particles, 0.01, base_state=base)
    cells = W.buoy_cells(cfg.nx, cfg.ny, 15, 15)
    noise = ophil.normals(2 * len(cells), cfg.seed, 0, ophil.TAG_OBS, 77, 0).reshape(-1, 2)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, noise)
    got, stats, sc = _gpu_analysis(torch, dev, cfg, ens, cells, y, 0, 256)
    ref, info = oiewpf.analysis(ens.astype(np.float64), cells, y, cfg, 0, particles=[3, 77])
    _check_scalars(stats, sc, info, cfg.n_psi)
    for n, i in enumerate((3, 77)):
        for f in range(3):
            err = np.abs(got[i, f] - ref[n, f]).max() / np.abs(ref[n, f]).max()
            _say(f"  particle {i} field {f} rel err {err}")
            assert err < TOL


def test_beta_error_reported(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context, abi
    cfg = W.tiny().replace(n_particles=4)
    ens = W.as_f32(np.stack([oens.init_member(cfg, None, 0, i) for i in range(4)]))
    truth = oens.init_member(cfg.replace(ensemble_id=77), None, 0, 0)
    cells = np.array([[8, 8], [24, 8], [8, 24], [24, 24]], dtype=np.int32)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, np.zeros((4, 2)))
    ctx = Context(cfg, max_obs=8)
    st = torch.from_numpy(ens).to(dev)
    with pytest.raises(abi.IewpfError) as e:
        ctx.assimilate(st, cells, y, analysis_index=0)
    assert e.value.code == abi.IEWPF_E_BETA
    ctx.close()


def test_observe_moorings_parity(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    cfg = W.paper_scale(1).replace(ensemble_id=77)
    truth = W.as_f32(W.jet_state(cfg) + 0.1 * W.random_state(cfg, np.random.default_rng(2)))
    cells = W.buoy_cells(cfg.nx, cfg.ny, 15, 15)
    ctx = Context(cfg, max_obs=256)
    y = ctx.observe_moorings(torch.from_numpy(truth).to(dev), cells, analysis_index=9)
    noise = ophil.normals(2 * len(cells), cfg.seed, 9, ophil.TAG_OBS, 77, 0).reshape(-1, 2)
    ref = oobs.mooring_obs(truth.astype(np.float64), cells, cfg.H, cfg.obs_sigma, noise)
    assert np.abs(y - ref).max() < 1e-12 * np.abs(ref).max()
    ctx.close()


def test_drifter_advection_parity(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    cfg = W.tiny().replace(n_particles=3)
    rng = np.random.default_rng(5)
    a = W.as_f32(np.stack([W.random_state(cfg, rng) for _ in range(3)]))
    b = W.as_f32(np.stack([W.random_state(cfg, rng) for _ in range(3)]))
    pos = np.stack([W.drifter_lattice(cfg, 4, 4) + rng.normal(scale=3e3, size=(16, 2))
                    for _ in range(3)])
    pos[0, 0] = [-5.0, 319999.0]  # wraps
    ctx = Context(cfg, max_obs=16)
    p = torch.from_numpy(pos.copy()).to(dev)
    ctx.advect_drifters(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), p)
    got = p.cpu().numpy()
    for i in range(3):
        ref = odr.heun_step(pos[i], a[i].astype(np.float64), b[i].astype(np.float64), cfg, cfg.dt)
        assert np.abs(got[i] - ref).max() < 1e-9
    ctx.close()


def test_forecast_drifters_parity(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    cfg = W.tiny().replace(n_particles=2, me_std=0.01)
    rng = np.random.default_rng(6)
    ens = W.as_f32(np.stack([W.random_state(cfg, rng, q_amp=30.0) for _ in range(2)]))
    pos0 = np.stack([W.drifter_lattice(cfg, 3, 3) for _ in range(2)])
    ctx = Context(cfg, max_obs=9)
    st = torch.from_numpy(ens.copy()).to(dev)
    p = torch.from_numpy(pos0.copy()).to(dev)
    traj = torch.zeros((4, 2, 9, 2), dtype=torch.float64, device=dev)
    ctx.forecast_drifters(st, p, 3, first_step=20, traj=traj)
    got_traj = traj.cpu().numpy()
    for i in range(2):
        psi = ens[i].astype(np.float64)
        pp = pos0[i].copy()
        for s in range(3):
            nxt = oens.step_member(psi, cfg, i, 20 + s, 1, noise_on_last=True)
            pp = odr.heun_step(pp, psi, nxt, cfg, cfg.dt)
            psi = nxt
            assert np.abs(got_traj[s + 1, i] - pp).max() < 1e-3, (i, s)
    ctx.close()


def test_resampling_bit_exact(torch_dev):
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    cfg = W.tiny().replace(n_particles=37)
    rng = np.random.default_rng(8)
    ens = W.as_f32(rng.normal(size=(37, 3, 32, 32)))
    ctx = Context(cfg, max_obs=4)
    for rep in range(5):
        lw = rng.normal(scale=2.0, size=37)
        st = torch.from_numpy(ens.copy()).to(dev)
        par = torch.zeros(37, dtype=torch.int32, device=dev)
        ctx.resample(st, torch.from_numpy(lw).to(dev), analysis_index=rep, parents=par)
        got = par.cpu().numpy()
        u = ores.resample_uniforms(37, cfg.seed, rep, cfg.ensemble_id)
        ref, counts = ores.residual_resample(lw, u)
        assert np.array_equal(got, ref)
        assert np.array_equal(st.cpu().numpy(), ens[ref])
    ctx.close()
