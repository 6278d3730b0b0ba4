"""Pins of the oracle's drifter advection and residual resampling."""
import math

import numpy as np

import workloads as W
from oracle import drifters, philox, resample


def _flow_state(cfg, ufun, vfun):
    x = (np.arange(cfg.nx) + 0.5) * cfg.dx
    y = (np.arange(cfg.ny) + 0.5) * cfg.dy
    X, Y = np.meshgrid(x, y)
    psi = np.zeros((3, cfg.ny, cfg.nx))
    psi[0] = 0.3
    h = cfg.H + psi[0]
    psi[1] = h * ufun(X, Y)
    psi[2] = h * vfun(X, Y)
    return psi


def test_uniform_flow_moves_exactly():
    cfg = W.tiny()
    psi = _flow_state(cfg, lambda X, Y: 0.7 + 0 * X, lambda X, Y: -0.2 + 0 * X)
    pos = W.drifter_lattice(cfg, 2, 2) + np.array([[1234.5, -77.0]])
    p = pos.copy()
    for _ in range(50):
        p = drifters.heun_step(p, psi, psi, cfg, 30.0)
    assert np.abs(p - (pos + 50 * 30.0 * np.array([0.7, -0.2]))).max() < 1e-9


def test_solid_body_rotation_second_order():
    # linear velocity field => bilinear sampling exact away from the wrap; Heun's radius
    # drift over a fixed time must shrink ~4x when dt halves
    cfg = W.Config(nx=64, ny=64, dx=1e3, dy=1e3)
    om = 1e-4
    c0 = 32e3
    psi = _flow_state(cfg, lambda X, Y: -om * (Y - c0), lambda X, Y: om * (X - c0))
    errs = []
    for dt in (200.0, 100.0):
        p = np.array([[c0 + 8e3, c0]])
        for _ in range(int(round(2 * math.pi / om / 4 / dt))):
            p = drifters.heun_step(p, psi, psi, cfg, dt)
        errs.append(abs(math.hypot(p[0, 0] - c0, p[0, 1] - c0) - 8e3))
    assert errs[0] / errs[1] > 3.5
    # forward Euler is first order and drifts outward
    p = np.array([[c0 + 8e3, c0]])
    for _ in range(100):
        p = drifters.euler_step(p, psi, cfg, 100.0)
    assert math.hypot(p[0, 0] - c0, p[0, 1] - c0) > 8e3


def test_error_norm_definitions():
    lx = ly = 1e5
    ens = np.zeros((3, 2, 2))
    ens[:, :, 0] = [[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]]
    truth = np.zeros((2, 2))
    ref = math.sqrt(np.mean(ens[..., 0] ** 2))
    assert abs(drifters.forecast_error(ens, truth, lx, ly) - ref) < 1e-12
    # minimum image across the periodic boundary
    e2 = np.array([[[lx - 1.0, 0.0]]])
    assert abs(drifters.forecast_error(e2, np.array([[0.0, 0.0]]), lx, ly) - 1.0) < 1e-9


def test_residual_resampling_counts():
    rng = np.random.default_rng(0)
    for ne in (10, 100, 37):
        lw = rng.normal(scale=3.0, size=ne)
        u = philox.uniforms(ne, 5, 1, philox.TAG_RESAMPLE, 0, 0)
        parents, counts = resample.residual_resample(lw, u)
        w = np.exp(lw - lw.max())
        w /= w.sum()
        assert counts.sum() == ne and len(parents) == ne
        assert np.all(counts >= np.floor(ne * w) - 0)
        assert np.all(counts <= np.floor(ne * w) + ne)
        assert np.all(np.diff(parents) >= 0)


def test_exact_multiples_need_no_residual():
    lw = np.array([0.0, -np.inf, 0.0, -np.inf, 0.0, 0.0, -np.inf, -np.inf, 0.0, -np.inf])
    parents, counts = resample.residual_resample(lw, np.full(10, 0.999))
    assert list(counts) == [2, 0, 2, 0, 2, 2, 0, 0, 2, 0]
    parents, counts = resample.residual_resample(np.zeros(7), np.zeros(7))
    assert list(counts) == [1] * 7


def test_residual_draws_are_unbiased():
    # E[count_i] = N_e w_i: average over many independent uniform streams
    ne = 8
    lw = np.log(np.array([0.31, 0.05, 0.17, 0.02, 0.2, 0.11, 0.09, 0.05]))
    acc = np.zeros(ne)
    n_rep = 3000
    for rep in range(n_rep):
        u = philox.uniforms(ne, 11, rep, philox.TAG_RESAMPLE, 0, 0)
        acc += resample.residual_resample(lw, u)[1]
    w = np.exp(lw) / np.exp(lw).sum()
    assert np.abs(acc / n_rep - ne * w).max() < 0.05


def test_sir_log_weights():
    d = np.array([[[1.0, 2.0]], [[0.0, 0.0]]])
    lw = resample.sir_log_weights(d, 2.0)
    assert np.allclose(lw, [-0.5 * 5 / 4, 0.0])


def test_sir_weights_are_the_normalised_gaussian_likelihood():
    # eq. standardParticleFilterWeight: w_i proportional to p(y | psi_i), Gaussian with
    # R = sigma^2 I; held against scipy's normal density of every innovation component
    from scipy.stats import norm
    rng = np.random.default_rng(12)
    d = rng.normal(scale=1.3, size=(9, 6, 2))
    for sigma in (0.8, 1.0, 2.5):
        lw = resample.sir_log_weights(d, sigma)
        w = np.exp(lw - lw.max())
        w /= w.sum()
        lik = np.prod(norm.pdf(d, loc=0.0, scale=sigma), axis=(1, 2))
        assert np.abs(w - lik / lik.sum()).max() < 1e-13
