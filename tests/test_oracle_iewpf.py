"""Pins of the oracle's IEWPF stages 3-6 (Section "Sampling perpendicular random vectors",
"Target weight and beta", "Solving the implicit equation", "Posterior particle states",
Appendix A)."""
import math

import mpmath
import numpy as np
import pytest
import scipy.special

import workloads as W
from oracle import ensemble, iewpf, lambertw, model_error as me, observe as ob, philox


def test_perpendicular_vectors():
    xi = philox.normals(9375, 1, 0, philox.TAG_XI, 0, 0)
    nut = philox.normals(9375, 1, 0, philox.TAG_NU, 0, 0)
    nu, (xx, nn, nx_) = iewpf.perpendicular(xi, nut)
    assert abs(np.dot(nu, xi)) < 1e-12 * math.sqrt(xx * nn)
    assert abs(np.dot(nu, nu) - nn) < 1e-12 * nn


@pytest.mark.parametrize("x,cn", [(0.3, 0.0), (0.5, 0.2), (2.0, 0.0), (1.7, 0.05), (0.9, 1e-3),
                                  (4.0, 3.0), (0.05, 0.5)])
def test_w0_branch_form_matches_scipy(x, cn):
    z = -x * math.exp(-x - cn)
    ref = scipy.special.lambertw(z, 0).real
    got = lambertw.w0_branch_form(x, cn)
    assert abs(got - ref) < 1e-13 * abs(ref)
    assert abs(lambertw.lambert_w0(z) - ref) < 1e-13 * abs(ref)


@pytest.mark.parametrize("eps,cstar", [(0.002, 0.0), (-0.002, 0.0), (0.002, 450.0), (-0.002, 450.0),
                                       (1e-6, 3.0), (-3e-4, 1e4), (0.01, 1.0), (2e-9, 0.0)])
def test_alpha_solves_the_implicit_equation(eps, cstar):
    # reference: the root of (alpha-1) gamma - N log alpha = c* on alpha <= 1 in 50 digits
    N = 450000.0
    gamma = N * (1 + eps)
    a = lambertw.iewpf_alpha(gamma, cstar, N)
    mpmath.mp.dps = 50
    G, NN, C = mpmath.mpf(gamma), mpmath.mpf(N), mpmath.mpf(cstar)
    f = lambda al: (al - 1) * G - NN * mpmath.log(al) - C
    # f decreases on (0, N/gamma] from +inf to -N (x - 1 - ln x) - c* <= 0: bisection
    lo, hi = mpmath.mpf("1e-300"), NN / G
    if f(hi) == 0:
        lo = hi
    for _ in range(400):
        mid = (lo + hi) / 2
        if f(mid) > 0:
            lo = mid
        else:
            hi = mid
    ref = (lo + hi) / 2
    assert a <= 1.0
    assert abs(a - float(ref)) < 1e-12 * float(ref)


def test_alpha_is_one_on_the_target_when_gamma_small():
    assert lambertw.iewpf_alpha(449000.0, 0.0, 450000.0) == 1.0
    assert lambertw.iewpf_alpha(451000.0, 0.0, 450000.0) < 1.0


def test_beta_makes_every_cstar_nonnegative():
    rng = np.random.default_rng(5)
    c = 450 + 30 * rng.normal(size=100)
    zeta = 450000 + 950 * rng.normal(size=100)
    cbar, beta, cstar = iewpf.beta_and_cstar(c, zeta)
    assert np.all(cstar >= 0)
    i = int(np.argmin((cbar - c) / zeta + 1))
    assert cstar[i] <= 1e-10 * abs(cbar - c[i])
    assert beta < 1.0


def test_local_block_spectrum_and_root():
    cfg = W.tiny()
    w = me.model_error_stencil(cfg)
    A, Sc = iewpf.local_a_block(cfg, w)
    lam = np.sort(np.linalg.eigvalsh(A))
    Mc = np.linalg.inv(Sc) - cfg.obs_sigma ** 2 * np.eye(2)
    mu = np.sort(cfg.obs_sigma ** 2 / (np.linalg.eigvalsh(Mc) + cfg.obs_sigma ** 2))
    assert np.abs(lam[2:] - 1.0).max() < 1e-12
    assert np.abs(lam[:2] - mu).max() < 1e-12
    R = iewpf.sym_sqrt(A)
    assert np.abs(R @ R - A).max() < 1e-12
    assert np.abs(R - R.T).max() < 1e-14


def test_posterior_covariance_dense_at_unit_coarsening():
    # c_Omega = 1: Q^{1/2} A^{1/2} (Q^{1/2} A^{1/2})^T = Q - Q H^T S H Q (eq. PcovExpression)
    cfg = W.Config(nx=14, ny=12, dx=1e4, dy=1e4, c_omega=1, me_std=0.02, obs_sigma=0.5)
    w = me.model_error_stencil(cfg)
    A, Sc = iewpf.local_a_block(cfg, w)
    Ah = iewpf.sym_sqrt(A)
    cells = np.array([[5, 6]], dtype=np.int32)
    nr = cfg.nrx * cfg.nry
    L = np.zeros((3 * cfg.nx * cfg.ny, nr))
    Qh = np.zeros_like(L)
    for col in range(nr):
        e = np.zeros((cfg.nry, cfg.nrx))
        e.flat[col] = 1.0
        Qh[:, col] = me.apply_qhalf(e, w, cfg).reshape(-1)
        L[:, col] = me.apply_qhalf(iewpf.apply_local_blocks(e, Ah, cells, 1), w, cfg).reshape(-1)
    Q = Qh @ Qh.T
    n = cfg.nx * cfg.ny
    Hm = np.zeros((2, 3 * n))
    Hm[0, n + 6 * cfg.nx + 5] = 1
    Hm[1, 2 * n + 6 * cfg.nx + 5] = 1
    S = np.linalg.inv(Hm @ Q @ Hm.T + cfg.obs_sigma ** 2 * np.eye(2))
    assert np.abs(S - Sc).max() < 1e-12 * np.abs(S).max()
    P = Q - Q @ Hm.T @ S @ Hm @ Q
    assert np.abs(L @ L.T - P).max() < 1e-11 * np.abs(Q).max()


def _tiny_ensemble(cfg, ne, spread=0.003):
    """Particles and truth scattered around one random balanced state, as after a common
    spin-up, so that the ensemble is consistent with the observations."""
    base = ensemble.init_member(cfg, None, 0, 999)
    small = cfg.replace(init_std=spread)
    ens = np.stack([ensemble.init_member(small, base, 1, i) for i in range(ne)])
    truth = ensemble.init_member(small.replace(ensemble_id=77), base, 1, 0)
    return ens, truth


def test_equal_weights_after_analysis():
    cfg = W.tiny()
    ens, truth = _tiny_ensemble(cfg, cfg.n_particles)
    cells = np.array([[8, 8], [24, 8], [8, 24], [24, 24]], dtype=np.int32)
    noise = philox.normals(8, cfg.seed, 0, philox.TAG_OBS, 77, 0).reshape(4, 2)
    y = ob.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, noise)
    out, info = iewpf.analysis(ens, cells, y, cfg, analysis_index=3, particles=[0, 4])
    n_psi = cfg.n_psi
    wts = iewpf.realized_weight(info["alpha"], info["gamma"], info["zeta"], info["beta"],
                                info["c"], n_psi)
    assert 0 < info["beta"] <= 1.0
    assert np.abs(wts - info["cbar"]).max() < 1e-10 * n_psi
    assert np.all(info["alpha"] <= 1.0) and np.all(info["cstar"] >= 0)
    assert np.min(info["cstar"]) <= 1e-9
    assert out.shape == (2, 3, 32, 32) and np.isfinite(out).all()


def test_negative_beta_is_an_error():
    # beta is real only while N_psi >> N_y (eq. betaTwoStage); an ensemble far from the
    # observations on a small grid violates it and the analysis must refuse
    cfg = W.tiny()
    ens = np.stack([ensemble.init_member(cfg, None, 0, i) for i in range(4)])
    truth = ensemble.init_member(cfg.replace(ensemble_id=77), None, 0, 0)
    cells = np.array([[8, 8], [24, 8], [8, 24], [24, 24]], dtype=np.int32)
    y = ob.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, np.zeros((4, 2)))
    with pytest.raises(ValueError):
        iewpf.analysis(ens, cells, y, cfg, analysis_index=0, particles=[])


def test_pull_reduces_innovations():
    cfg = W.tiny().replace(me_std=0.05)
    ens, truth = _tiny_ensemble(cfg, 4)
    cells = np.array([[8, 8], [24, 24]], dtype=np.int32)
    y = ob.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, np.zeros((2, 2)))
    consts = iewpf.AnalysisConstants(cfg)
    d = ob.innovations(ens[0], cells, y, cfg.H)
    psi = ens[0].copy()
    for o in range(2):
        sd = consts.S @ d[o]
        psi += iewpf.pull_one(sd[0], sd[1], cells[o, 0], cells[o, 1], cfg, consts.w)
    d2 = y * ((cfg.H + ens[0][0, cells[:, 1], cells[:, 0]]) / cfg.H)[:, None] - ob.observe(psi, cells)
    assert np.abs(d2).sum() < np.abs(d).sum()
