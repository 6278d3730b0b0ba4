"""GPU parity of the full innovation covariance (S over all observations together instead of
the paper's independent 2x2 blocks) against the oracle's s_full and analysis(full_innovation)."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import iewpf as oiewpf
from oracle import model_error as ome
from oracle import observe as oobs
from test_gpu_analysis import TOL, _check_scalars, _ensemble_near

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


def _run(torch, dev, cfg, ens32, cells, y, aidx, max_obs, full=True):
    from paper_1910_01031_amd import Context
    ctx = Context(cfg, max_obs=max_obs)
    ctx.set_full_innovation(full)
    st = torch.from_numpy(np.ascontiguousarray(ens32)).to(dev)
    stats = ctx.assimilate(st, cells, y, analysis_index=aidx)
    torch.cuda.synchronize()
    sc = ctx.particle_scalars()
    n = 2 * len(cells)
    S = ctx.read_buffer(9, (n, n), np.float64) if full else None
    out = st.cpu().numpy().astype(np.float64)
    ctx.close()
    return out, stats, sc, S


def test_full_s_matches_oracle_and_analysis_parity(torch_dev):
    torch, dev = torch_dev
    _say("full innovation covariance: S and analysis vs oracle (64x48, 6 overlapping obs)")
    cfg = W.Config(nx=64, ny=48, dx=1e4, dy=1e4, c_omega=4, n_particles=6, me_std=2e-3)
    ens, truth = _ensemble_near(cfg, 6, 0.003)
    cells = np.array([[10, 10], [12, 11], [15, 13], [40, 30], [63, 47], [0, 0]], dtype=np.int32)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, np.zeros((6, 2)))
    got, stats, sc, S = _run(torch, dev, cfg, ens, cells, y, 2, 8)
    w = ome.model_error_stencil(cfg)
    Sref = oiewpf.s_full(cfg, w, cells)
    assert np.abs(S - Sref).max() < 1e-9 * np.abs(Sref).max()
    ref, info = oiewpf.analysis(ens.astype(np.float64), cells, y, cfg, 2, full_innovation=True)
    _check_scalars(stats, sc, info, cfg.n_psi)
    for f in range(3):
        err = np.abs(got[:, f] - ref[:, f]).max() / np.abs(ref[:, f]).max()
        _say(f"  field {f} rel err {err}")
        assert err < TOL, (f, err)
    # the paper's independent blocks give a different analysis for these observations
    blk, _, _, _ = _run(torch, dev, cfg, ens, cells, y, 2, 8, full=False)
    assert np.abs(blk - got).max() > 10 * TOL * np.abs(got).max()


def test_separated_observations_full_equals_blocks(torch_dev):
    torch, dev = torch_dev
    cfg = W.tiny().replace(c_omega=1, n_particles=4)
    ens, truth = _ensemble_near(cfg, 4, 0.003)
    cells = np.array([[2, 2], [18, 18]], dtype=np.int32)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, np.zeros((2, 2)))
    full, sf, _, _ = _run(torch, dev, cfg, ens, cells, y, 1, 4)
    blk, sb, _, _ = _run(torch, dev, cfg, ens, cells, y, 1, 4, full=False)
    assert abs(sf["cbar"] - sb["cbar"]) < 1e-9 * abs(sb["cbar"])
    assert np.abs(full - blk).max() < 1e-6 * np.abs(blk).max()


def test_full_covariance_follows_moving_observations(torch_dev):
    """Drifter-like use: the observed cells change between analyses, so the factor and S are
    rebuilt for the second one; that analysis matches the oracle on the state the first one
    left."""
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    _say("full covariance, observed cells moving between two analyses")
    cfg = W.Config(nx=64, ny=48, dx=1e4, dy=1e4, c_omega=4, n_particles=5, me_std=2e-3)
    ens, truth = _ensemble_near(cfg, 5, 0.003)
    cells_a = np.array([[10, 10], [13, 11], [40, 30], [50, 8]], dtype=np.int32)
    cells_b = np.array([[11, 10], [14, 12], [41, 31], [52, 9], [30, 40]], dtype=np.int32)
    ctx = Context(cfg, max_obs=8)
    ctx.set_full_innovation(True)
    st = torch.from_numpy(np.ascontiguousarray(ens)).to(dev)
    y_a = oobs.mooring_obs(truth, cells_a, cfg.H, cfg.obs_sigma, np.zeros((4, 2)))
    ctx.assimilate(st, cells_a, y_a, analysis_index=1)
    torch.cuda.synchronize()
    mid = st.cpu().numpy().astype(np.float64)
    y_b = oobs.mooring_obs(truth, cells_b, cfg.H, cfg.obs_sigma, np.zeros((5, 2)))
    stats = ctx.assimilate(st, cells_b, y_b, analysis_index=2)
    torch.cuda.synchronize()
    sc = ctx.particle_scalars()
    S = ctx.read_buffer(9, (10, 10), np.float64)
    got = st.cpu().numpy().astype(np.float64)
    ctx.close()
    w = ome.model_error_stencil(cfg)
    Sref = oiewpf.s_full(cfg, w, cells_b)
    assert np.abs(S - Sref).max() < 1e-9 * np.abs(Sref).max()
    ref, info = oiewpf.analysis(mid, cells_b, y_b, cfg, 2, full_innovation=True)
    _check_scalars(stats, sc, info, cfg.n_psi)
    for f in range(3):
        err = np.abs(got[:, f] - ref[:, f]).max() / np.abs(ref[:, f]).max()
        assert err < TOL, (f, err)


@pytest.mark.parametrize("bx,by", [(15, 15), (20, 15)])
def test_full_s_inverse_at_paper_scale(torch_dev, bx, by):
    """225 (300) buoys on 500x300 (neighbours 20 rows apart overlap): the device S (450x450;
    600x600 takes the 16-slot solve) times the matrix assembled independently from the
    oracle's translation-invariant pull response is the identity."""
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    _say(f"full S at paper scale ({bx * by} buoys)")
    cfg = W.paper_scale(2)
    cells = W.buoy_cells(cfg.nx, cfg.ny, bx, by)
    ctx = Context(cfg, max_obs=len(cells))
    ctx.set_full_innovation(True)
    st = torch.from_numpy(W.as_f32(np.stack([W.jet_state(cfg)] * 2))).to(dev)
    ctx.assimilate(st, cells, np.zeros((len(cells), 2)), analysis_index=0)
    torch.cuda.synchronize()
    n = 2 * len(cells)
    S = ctx.read_buffer(9, (n, n), np.float64)
    ctx.close()
    # M from the oracle chain: one pull per unit vector at an observed cell, read at offsets
    w = ome.model_error_stencil(cfg)
    j0, k0 = int(cells[0, 0]), int(cells[0, 1])
    resp = [oiewpf.pull_one(1.0, 0.0, j0, k0, cfg, w), oiewpf.pull_one(0.0, 1.0, j0, k0, cfg, w)]
    M = np.zeros((n, n))
    for o in range(len(cells)):
        dj = cells[:, 0] - cells[o, 0]
        dk = cells[:, 1] - cells[o, 1]
        jj = (j0 + dj) % cfg.nx
        kk = (k0 + dk) % cfg.ny
        for b in range(2):
            M[0::2, 2 * o + b] = resp[b][1, kk, jj]
            M[1::2, 2 * o + b] = resp[b][2, kk, jj]
    A = 0.5 * (M + M.T) + cfg.obs_sigma ** 2 * np.eye(n)
    assert np.abs(S @ A - np.eye(n)).max() < 1e-9
    assert np.abs(S - S.T).max() < 1e-12 * np.abs(S).max()


@pytest.mark.parametrize("full", [False, True])
def test_one_stage_scheme_parity(torch_dev, full):
    """The one-stage scheme (target weight max c, no nu term) against the oracle, with the
    paper's 2x2 blocks and with the full innovation covariance."""
    torch, dev = torch_dev
    from paper_1910_01031_amd import Context
    _say(f"one-stage scheme parity (full covariance {full})")
    cfg = W.Config(nx=64, ny=48, dx=1e4, dy=1e4, c_omega=4, n_particles=6, me_std=2e-3)
    ens, truth = _ensemble_near(cfg, 6, 0.003)
    cells = np.array([[10, 10], [12, 11], [40, 30], [63, 47]], dtype=np.int32)
    y = oobs.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, np.zeros((4, 2)))
    ctx = Context(cfg, max_obs=8)
    ctx.set_scheme(True)
    ctx.set_full_innovation(full)
    st = torch.from_numpy(np.ascontiguousarray(ens)).to(dev)
    stats = ctx.assimilate(st, cells, y, analysis_index=4)
    torch.cuda.synchronize()
    sc = ctx.particle_scalars()
    got = st.cpu().numpy().astype(np.float64)
    ctx.close()
    ref, info = oiewpf.analysis(ens.astype(np.float64), cells, y, cfg, 4, full_innovation=full,
                                one_stage=True)
    assert stats["beta"] == 0.0
    assert abs(stats["cbar"] - info["cbar"]) < 1e-9 * abs(info["cbar"])
    assert stats["argmin_beta"] == int(np.argmax(info["c"]))
    assert np.abs(sc[:, 0] - info["c"]).max() < 1e-9 * np.abs(info["c"]).max()
    assert np.abs(sc[:, 3] - info["alpha"]).max() < 1e-7
    # every particle reaches the target weight (one-stage form, no nu term)
    w = (sc[:, 3] - 1.0) * sc[:, 1] - cfg.n_psi * np.log(sc[:, 3]) + sc[:, 0]
    assert np.abs(w - stats["cbar"]).max() < 1e-9 * cfg.n_psi
    for f in range(3):
        err = np.abs(got[:, f] - ref[:, f]).max() / np.abs(ref[:, f]).max()
        assert err < TOL, (f, err)
