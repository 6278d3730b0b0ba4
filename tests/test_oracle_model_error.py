"""Pins of the oracle's model-error operator Q^{1/2} = Q_GB I_Omega Q_SOAR."""
import json
import math
import os

import numpy as np

import workloads as W
from oracle import model_error as me
from oracle import philox, swe

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_soar_dense_operator_is_autoconvolution():
    # Cov(z) = Q_S Q_S^T; its entries are the autoconvolution of the 5x5 stencil (the
    # SOAR stencil is the square root's kernel, not the covariance itself)
    n = 12
    w = me.soar_stencil(0.7, 3.0e4, 4e4, 3e4)
    Q = np.zeros((n * n, n * n))
    for col in range(n * n):
        e = np.zeros((n, n))
        e.flat[col] = 1.0
        Q[:, col] = me.soar_apply(e, w).reshape(-1)
    C = Q @ Q.T
    for (dq, dp) in ((0, 0), (0, 1), (1, 0), (1, 1), (2, -3), (4, 4), (0, 5)):
        ref = 0.0
        for q in range(-2, 3):
            for p in range(-2, 3):
                q2, p2 = q - dq, p - dp
                if abs(q2) <= 2 and abs(p2) <= 2:
                    ref += w[q + 2, p + 2] * w[q2 + 2, p2 + 2]
        a = 5 * n + 5
        b = ((5 + dq) % n) * n + (5 + dp) % n
        assert abs(C[a, b] - ref) < 1e-14 * abs(C[a, a])
    assert C[5 * n + 5, ((5 + 5) % n) * n + 5] == 0.0


def test_soar_sample_covariance():
    cfg = W.tiny()
    w = me.model_error_stencil(cfg)
    n_draw = 4000
    z = np.stack([me.soar_apply(philox.normals(64, 7, s, philox.TAG_MODEL_ERROR, 0, 0)
                                .reshape(8, 8), w) for s in range(n_draw)])
    var = z.var(axis=0).mean()
    # the coarse field's pointwise std is cfg.me_std by construction of q0
    assert abs(var - cfg.me_std ** 2) < 4 * cfg.me_std ** 2 * math.sqrt(2 / (n_draw * 64)) * 3
    cov1 = np.mean(z[:, 3, 3] * z[:, 3, 4])
    ref1 = sum(w[q + 2, p + 2] * w[q + 2, p + 1] for q in range(-2, 3) for p in range(-1, 3))
    assert abs(cov1 - ref1) < 4 * cfg.me_std ** 2 / math.sqrt(n_draw) * 1.5


def test_q0_from_std_norms():
    # ||k||_2 of the unit SOAR 5x5 stencil for L0 = 3/4 and 1 coarse spacing
    assert abs(1 / me.q0_from_std(1.0, 0.75, 1.0, 1.0) - 1.97843) < 1e-5
    assert abs(1 / me.q0_from_std(1.0, 1.0, 1.0, 1.0) - 2.52279) < 1e-5


def test_bicubic_reproduces_quadratics():
    c, nrx, nry = 4, 24, 20
    a = np.arange(nrx, dtype=float)
    b = np.arange(nry, dtype=float)
    for poly in (lambda s: 1.5 + 0 * s, lambda s: 0.3 * s - 2, lambda s: 0.05 * s * s - 0.4 * s + 1):
        z = poly(b)[:, None] * poly(a)[None, :]
        fine = me.bicubic(z, c, nrx * c, nry * c)
        j = np.arange(nrx * c)
        s = (2 * j + 1 - c) / (2.0 * c)
        k = np.arange(nry * c)
        t = (2 * k + 1 - c) / (2.0 * c)
        ref = poly(t)[:, None] * poly(s)[None, :]
        inner = np.ix_((t > 1.5) & (t < nry - 3), (s > 1.5) & (s < nrx - 3))
        assert np.abs(fine[inner] - ref[inner]).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_bicubic_colocated_for_odd_coarsening():
    c = 3
    z = np.random.default_rng(0).normal(size=(7, 9))
    fine = me.bicubic(z, c, 27, 21)
    assert np.abs(fine[1::3, 1::3] - z).max() < 1e-15


def test_bicubic_shifted_hits_the_observed_cell():
    c = 4
    z = np.random.default_rng(1).normal(size=(8, 10))
    fine = me.bicubic_shifted(z, c, 40, 32, j0=13, k0=6)
    for m in range(10):
        for n in range(8):
            assert abs(fine[(6 + n * c) % 32, (13 + m * c) % 40] - z[n, m]) < 1e-15


def test_geostrophic_balance_of_perturbation():
    cfg = W.tiny()
    xi = philox.normals(64, 3, 0, philox.TAG_MODEL_ERROR, 0, 0).reshape(8, 8)
    pert = me.apply_qhalf(xi, me.model_error_stencil(cfg), cfg)
    deta, dhu, dhv = pert
    Dx = lambda a: (np.roll(a, -1, 1) - np.roll(a, 1, 1)) / (2 * cfg.dx)
    Dy = lambda a: (np.roll(a, -1, 0) - np.roll(a, 1, 0)) / (2 * cfg.dy)
    scale = np.abs(dhu).max() / cfg.dx
    assert np.abs(Dx(dhu) + Dy(dhv)).max() < 1e-13 * scale      # non-divergent
    assert abs(dhu.sum()) < 1e-12 * np.abs(dhu).sum()
    assert abs(dhv.sum()) < 1e-12 * np.abs(dhv).sum()
    # f (dhv, -dhu) = g H grad(deta) in central differences
    a = cfg.g * cfg.H
    assert np.abs(cfg.f * dhv - a * Dx(deta)).max() < 1e-12 * np.abs(cfg.f * dhv).max()
    assert np.abs(-cfg.f * dhu - a * Dy(deta)).max() < 1e-12 * np.abs(cfg.f * dhu).max()


def test_geostrophic_direction_and_magnitude_on_smooth_bump():
    # a high-pressure bump with f > 0 gives clockwise flow: eastward (hu > 0) north of it;
    # central differences match the analytic gradient to O(dx^2)
    n, dx = 128, 2e3
    x = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(x, x)
    s = 2e4
    eta = 0.1 * np.exp(-((X - 128e3) ** 2 + (Y - 128e3) ** 2) / (2 * s * s))
    dhu, dhv = me.geostrophic(eta, 230.0, 9.81, 1.2e-4, dx, dx)
    a = 9.81 * 230.0 / 1.2e-4
    ex_hu = -a * eta * (-(Y - 128e3) / (s * s))
    ex_hv = a * eta * (-(X - 128e3) / (s * s))
    assert dhu[80, 64] > 0 and dhu[48, 64] < 0 and dhv[64, 80] < 0
    assert np.abs(dhu - ex_hu).max() < 5e-3 * np.abs(ex_hu).max()
    assert np.abs(dhv - ex_hv).max() < 5e-3 * np.abs(ex_hv).max()


def test_paper_constants_cfl_reading():
    # the double-jet case (dx = 2220 m, dt = 60 s, Courant 0.8) takes "typically eight"
    # scheme steps per model step; the CFL reading gives 7-8 for speeds up to ~3 m/s
    k = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    c = math.sqrt(k["g"] * k["H"])
    for umax in (0.5, 3.0):
        dt_cfl = k["courant"] * 0.25 * k["dx"] / (umax + c)
        n = math.ceil(k["dt_model"] / dt_cfl)
        assert 7 <= n <= 8
