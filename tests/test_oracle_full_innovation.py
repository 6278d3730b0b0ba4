"""Pins of the full innovation covariance: S = (H Q H^T + R)^{-1} over all observations
together, which the paper approximates by independent 2x2 blocks (eq. S_extended and the
remark after it that observations are assumed far apart)."""
import numpy as np

import workloads as W
from oracle import iewpf, model_error as me
from oracle import observe as ob
from test_oracle_pull import _dense_qhalf, _h_matrix


def test_overlapping_observations_pull_equals_dense_kalman_gain():
    # c_Omega = 1: the chain is exactly Q H^T, so with the full S the summed pulls of three
    # observations two and three cells apart equal the dense Kalman gain K d
    cfg = W.Config(nx=16, ny=12, dx=1e4, dy=8e3, c_omega=1, me_std=0.02, obs_sigma=0.7)
    w = me.model_error_stencil(cfg)
    Qh = _dense_qhalf(cfg, w)
    Q = Qh @ Qh.T
    cells = np.array([[5, 7], [7, 7], [5, 4]], dtype=np.int32)
    Hm = _h_matrix(cfg, cells)
    HQH = Hm @ Q @ Hm.T
    assert np.abs(HQH[:2, 2:4]).max() > 1e-3 * np.abs(HQH).max()  # they do overlap
    Sd = np.linalg.inv(HQH + cfg.obs_sigma ** 2 * np.eye(6))
    Sf = iewpf.s_full(cfg, w, cells)
    assert np.abs(Sf - Sd).max() < 1e-11 * np.abs(Sd).max()
    d = np.array([0.8, -1.3, 0.4, 0.9, -0.6, 0.2])
    dense = (Q @ Hm.T @ Sd @ d).reshape(3, cfg.ny, cfg.nx)
    sd = (Sf @ d).reshape(3, 2)
    tot = sum(iewpf.pull_one(sd[o, 0], sd[o, 1], cells[o, 0], cells[o, 1], cfg, w)
              for o in range(3))
    assert np.abs(tot - dense).max() < 1e-10 * np.abs(dense).max()
    # the independent-block approximation differs here
    S2 = iewpf.s_matrix(cfg, w)
    assert np.abs(np.kron(np.eye(3), S2) - Sd).max() > 1e-3 * np.abs(Sd).max()


def test_separated_observations_reduce_to_blocks():
    cfg = W.tiny()
    w = me.model_error_stencil(cfg)
    # the chain reaches 7 c cells: 28 on the 32-cell torus at c = 4, so separate at c = 1
    cells = np.array([[2, 2], [18, 18]], dtype=np.int32)
    cfg = cfg.replace(c_omega=1)
    w = me.model_error_stencil(cfg)
    M = iewpf.hqht_full(cfg, w, cells)
    assert np.abs(M[:2, 2:]).max() == 0.0 and np.abs(M[2:, :2]).max() == 0.0
    Sf = iewpf.s_full(cfg, w, cells)
    S2 = iewpf.s_matrix(cfg, w)
    assert np.abs(Sf - np.kron(np.eye(2), S2)).max() < 1e-12 * np.abs(S2).max()


def test_full_operator_symmetry_and_definiteness():
    rng = np.random.default_rng(3)
    cells = np.stack([rng.integers(0, 32, 6), rng.integers(0, 32, 6)], axis=1).astype(np.int32)
    # c_Omega = 1: one coarse grid for all observations, M = H Q H^T exactly (symmetric)
    cfg1 = W.tiny().replace(c_omega=1)
    M1 = iewpf.hqht_full(cfg1, me.model_error_stencil(cfg1), cells)
    assert np.abs(M1 - M1.T).max() < 1e-12 * np.abs(M1).max()
    # c_Omega = 4: every observation's pull uses a coarse grid aligned on its own cell, so the
    # cross blocks of the chain are only nearly symmetric and their symmetric part need not be
    # semidefinite; s_full inverts the symmetric part plus R, which must be definite
    cfg = W.tiny()
    M = iewpf.hqht_full(cfg, me.model_error_stencil(cfg), cells)
    assert np.abs(M - M.T).max() < 0.1 * np.abs(M).max()
    for o in range(6):  # the diagonal blocks are the paper's 2x2 H Q H^T
        blk = M[2 * o:2 * o + 2, 2 * o:2 * o + 2]
        assert np.abs(blk - iewpf.hqht(cfg, me.model_error_stencil(cfg))).max() < 1e-12
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert ev.min() > -0.2 * ev.max()
    assert ev.min() + cfg.obs_sigma ** 2 > 0.5 * cfg.obs_sigma ** 2


def test_post_pull_innovation_is_r_s_d_for_overlapping_observations():
    # d' = d - H(sum of pulls) = (I - M S) d = R S d at every observed cell (c_Omega = 1,
    # where the chain's M is the symmetric H Q H^T that s_full inverts)
    cfg = W.tiny().replace(c_omega=1)
    w = me.model_error_stencil(cfg)
    cells = np.array([[7, 19], [9, 20], [12, 15]], dtype=np.int32)
    Sf = iewpf.s_full(cfg, w, cells)
    psi = W.random_state(cfg, np.random.default_rng(4))
    y = np.array([[30.0, -12.0], [10.0, 5.0], [-20.0, 8.0]])
    d = ob.innovations(psi, cells, y, cfg.H).reshape(-1)
    sd = (Sf @ d).reshape(3, 2)
    psi_a = psi.copy()
    for o in range(3):
        psi_a += iewpf.pull_one(sd[o, 0], sd[o, 1], cells[o, 0], cells[o, 1], cfg, w)
    eta0 = np.array([psi[0, k, j] for j, k in cells])
    d_after = (y * ((cfg.H + eta0) / cfg.H)[:, None] - ob.observe(psi_a, cells)).reshape(-1)
    assert np.abs(d_after - cfg.obs_sigma ** 2 * (Sf @ d)).max() < 1e-11 * np.abs(d).max()


def test_analysis_full_equals_blocks_for_separated_observations():
    cfg = W.tiny().replace(c_omega=1, n_particles=3)
    from oracle import ensemble as oens
    base = oens.init_member(cfg, None, 0, 999)
    small = cfg.replace(init_std=0.003)
    ens = np.stack([oens.init_member(small, base, 1, i) for i in range(3)])
    cells = np.array([[2, 2], [18, 18]], dtype=np.int32)
    y = np.array([[5.0, -3.0], [2.0, 4.0]])
    a, ia = iewpf.analysis(ens, cells, y, cfg, 3)
    b, ib = iewpf.analysis(ens, cells, y, cfg, 3, full_innovation=True)
    assert np.abs(ia["c"] - ib["c"]).max() < 1e-10 * np.abs(ia["c"]).max()
    assert np.abs(a - b).max() < 1e-10 * np.abs(a).max()
