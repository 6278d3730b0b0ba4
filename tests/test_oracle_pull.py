"""Pins of the oracle's optimal-proposal pull and S (Section "Optimal proposal particles")."""
import json
import os

import numpy as np

import workloads as W
from oracle import iewpf, model_error as me
from oracle import observe as ob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense_qhalf(cfg, w):
    nr = cfg.nrx * cfg.nry
    Qh = np.zeros((3 * cfg.nx * cfg.ny, nr))
    for col in range(nr):
        e = np.zeros((cfg.nry, cfg.nrx))
        e.flat[col] = 1.0
        Qh[:, col] = me.apply_qhalf(e, w, cfg).reshape(-1)
    return Qh


def _h_matrix(cfg, cells):
    n = cfg.nx * cfg.ny
    Hm = np.zeros((2 * len(cells), 3 * n))
    for o, (j, k) in enumerate(cells):
        Hm[2 * o, n + k * cfg.nx + j] = 1.0
        Hm[2 * o + 1, 2 * n + k * cfg.nx + j] = 1.0
    return Hm


def test_s_is_position_independent_and_diagonal():
    cfg = W.tiny()
    w = me.model_error_stencil(cfg)
    S0 = iewpf.s_matrix(cfg, w, 0, 0)
    for (j, k) in ((5, 9), (31, 31), (2, 17)):
        assert np.abs(iewpf.s_matrix(cfg, w, j, k) - S0).max() < 1e-14
    # reflection symmetry about the observed cell: no hu/hv coupling; dx = dy: equal terms
    M = iewpf.hqht(cfg, w)
    assert abs(M[0, 1]) < 1e-15 * M[0, 0] and abs(M[1, 0]) < 1e-15 * M[0, 0]
    assert abs(M[0, 0] - M[1, 1]) < 1e-13 * M[0, 0]
    assert M[0, 0] > 0


def test_pull_equals_dense_kalman_gain_at_unit_coarsening():
    # with c_Omega = 1 the approximate adjoint is the exact transpose, so the pull of one
    # observation is exactly Q H^T (H Q H^T + R)^{-1} d with Q = Q^{1/2} Q^{1/2,T}
    cfg = W.Config(nx=16, ny=12, dx=1e4, dy=8e3, c_omega=1, me_std=0.02, obs_sigma=0.7)
    w = me.model_error_stencil(cfg)
    Qh = _dense_qhalf(cfg, w)
    Q = Qh @ Qh.T
    cells = np.array([[5, 7]], dtype=np.int32)
    Hm = _h_matrix(cfg, cells)
    Sd = np.linalg.inv(Hm @ Q @ Hm.T + cfg.obs_sigma ** 2 * np.eye(2))
    S = iewpf.s_matrix(cfg, w, 5, 7)
    assert np.abs(S - Sd).max() < 1e-12 * np.abs(Sd).max()
    d = np.array([0.8, -1.3])
    dense = (Q @ Hm.T @ Sd @ d).reshape(3, cfg.ny, cfg.nx)
    sd = S @ d
    pull = iewpf.pull_one(sd[0], sd[1], 5, 7, cfg, w)
    assert np.abs(pull - dense).max() < 1e-11 * np.abs(dense).max()


def test_separated_observations_block_diagonal_gain():
    cfg = W.Config(nx=32, ny=24, dx=1e4, dy=1e4, c_omega=1, me_std=0.02)
    w = me.model_error_stencil(cfg)
    Qh = _dense_qhalf(cfg, w)
    Q = Qh @ Qh.T
    cells = np.array([[3, 3], [20, 15]], dtype=np.int32)
    Hm = _h_matrix(cfg, cells)
    HQH = Hm @ Q @ Hm.T
    assert np.abs(HQH[:2, 2:]).max() == 0.0
    d = np.array([0.5, -0.2, 1.1, 0.9])
    dense = (Q @ Hm.T @ np.linalg.inv(HQH + np.eye(4)) @ d).reshape(3, cfg.ny, cfg.nx)
    S = iewpf.s_matrix(cfg, w)
    tot = np.zeros_like(dense)
    for o in range(2):
        sd = S @ d[2 * o:2 * o + 2]
        tot += iewpf.pull_one(sd[0], sd[1], cells[o, 0], cells[o, 1], cfg, w)
    assert np.abs(tot - dense).max() < 1e-11 * np.abs(dense).max()


def test_post_pull_innovation_is_r_s_d():
    # for any c_Omega: d' = d - H(pull) = (I - M S) d = R S d at the observed cell
    cfg = W.tiny()
    w = me.model_error_stencil(cfg)
    S = iewpf.s_matrix(cfg, w)
    psi = W.random_state(cfg, np.random.default_rng(4))
    cells = np.array([[7, 19]], dtype=np.int32)
    y = np.array([[30.0, -12.0]])
    d = ob.innovations(psi, cells, y, cfg.H)[0]
    sd = S @ d
    psi_a = psi + iewpf.pull_one(sd[0], sd[1], 7, 19, cfg, w)
    eta0 = psi[0, 19, 7]
    d_after = y[0] * (cfg.H + eta0) / cfg.H - ob.observe(psi_a, cells)[0]
    assert np.abs(d_after - cfg.obs_sigma ** 2 * (S @ d)).max() < 1e-12 * np.abs(d).max()


def test_pull_window_radius():
    # dipole (+-1), two SOAR passes (+-4) and the bicubic taps reach 7 c - 1 fine cells in
    # eta; the geostrophic difference adds one more
    cfg = W.Config(nx=80, ny=72, dx=1e4, dy=1e4, c_omega=4)
    w = me.model_error_stencil(cfg)
    p = iewpf.pull_one(1.0, 0.7, 40, 36, cfg, w)
    nz = np.argwhere(np.abs(p).max(axis=0) > 0)
    r = 7 * cfg.c_omega
    assert nz[:, 0].min() >= 36 - r and nz[:, 0].max() <= 36 + r
    assert nz[:, 1].min() >= 40 - r and nz[:, 1].max() <= 40 + r
    nz_eta = np.argwhere(np.abs(p[0]) > 0)
    assert nz_eta[:, 1].max() == 40 + r - 1


def test_local_structure_counts_match_paper():
    g = json.load(open(os.path.join(GOLDEN, "localsvd_structure.json")))
    nx, ny = g["grid"]
    cfg = W.Config(nx=nx, ny=ny, dx=1e4, dy=1e4, c_omega=1)
    w = me.model_error_stencil(cfg)
    QS, G, Hm = iewpf.coarse_operator_matrices(cfg, w, n=nx)
    N = nx * ny
    PS = QS != 0
    PG = G != 0
    PGS = (PG.astype(int) @ PS.astype(int)) > 0
    assert set(PS.sum(axis=1)) == {g["soar_row_nnz"]}
    assert set(PGS[N:2 * N].sum(axis=1)) == {g["gb_soar_row_nnz_hu"]}
    assert set(PGS[2 * N:].sum(axis=1)) == {g["gb_soar_row_nnz_hv"]}
    # the hu rows span 7 cells in y and 5 in x; hv rows the transpose
    row = PGS[N + 5 * nx + 5].reshape(ny, nx)
    ys, xs = np.nonzero(row)
    assert (ys.max() - ys.min() + 1, xs.max() - xs.min() + 1) == tuple(g["gb_soar_hu_block"])
    PH = Hm != 0
    PK = (PH.astype(int) @ PGS.astype(int)) > 0
    assert set(PK.sum(axis=1)) == {g["obs_rows_nnz"]}
    PB = (PK.T.astype(int) @ np.ones((2, 2), int) @ PK.astype(int)) > 0
    rows = np.nonzero(PB.sum(axis=1))[0]
    assert len(rows) == g["final_nonidentity_rows"]
    assert set(PB[rows].sum(axis=1)) == {g["final_row_nnz"]}
    ys, xs = np.divmod(rows, nx)
    assert (ys.max() - ys.min() + 1, xs.max() - xs.min() + 1) == tuple(g["local_block"])
    assert 49 - len(rows) == g["local_block_missing_corners"]
