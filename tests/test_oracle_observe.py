"""Pins of the oracle's observation operators (Section "Synthetic truth and observations").

Both observation types measure the depth-averaged current times the equilibrium depth,
u H: a mooring through (hu, hv) H / (H + eta) (eq. buoyObservation), a drifter through its
displacement over the observation interval times H (eq. drifterObservation).  The
eta-compensated innovation (eq. etaCompensatedInnovation) rescales y by (H + eta_i)/H, so a
particle whose current equals the observed one has zero innovation whatever its eta.  The
checks below build states from a prescribed current, so each formula is held against that
meaning on its own: a scale written upside down (H/(H + eta) in the innovation, (H + eta)/H
in the mooring formula) or a displacement not divided by the interval fails one of them."""
import numpy as np

import workloads as W
from oracle import drifters, observe


def _state_with_current(cfg, rng, u_of, v_of, eta_amp=0.8):
    """eta random (order 1 m, so H + eta differs from H by ~0.3 %), hu = (H + eta) u,
    hv = (H + eta) v for the prescribed current (u, v) at cell centres."""
    x = (np.arange(cfg.nx) + 0.5) * cfg.dx
    y = (np.arange(cfg.ny) + 0.5) * cfg.dy
    X, Y = np.meshgrid(x, y)
    psi = np.zeros((3, cfg.ny, cfg.nx))
    psi[0] = eta_amp * rng.uniform(-1.0, 1.0, size=(cfg.ny, cfg.nx))
    h = cfg.H + psi[0]
    psi[1] = h * u_of(X, Y)
    psi[2] = h * v_of(X, Y)
    return psi


def _current(X, Y):
    return 0.4 * np.sin(2e-5 * X) + 0.1, -0.3 * np.cos(3e-5 * Y)


def test_mooring_observes_current_times_depth():
    cfg = W.tiny()
    rng = np.random.default_rng(3)
    psi = _state_with_current(cfg, rng, lambda X, Y: _current(X, Y)[0],
                              lambda X, Y: _current(X, Y)[1])
    cells = np.array([[0, 0], [5, 17], [31, 31], [12, 3]], dtype=np.int32)
    y = observe.mooring_obs(psi, cells, cfg.H, cfg.obs_sigma, np.zeros((4, 2)))
    X = (cells[:, 0] + 0.5) * cfg.dx
    Y = (cells[:, 1] + 0.5) * cfg.dy
    u, v = _current(X, Y)
    ref = np.stack([u, v], axis=1) * cfg.H
    assert np.abs(y - ref).max() < 1e-13 * np.abs(ref).max()
    # the eta scale matters at this size: observing (hu, hv) itself misses by ~1e-3
    assert np.abs(observe.observe(psi, cells) - ref).max() > 1e-4 * np.abs(ref).max()


def test_innovation_vanishes_for_a_particle_with_the_observed_current():
    # y = u H from the truth's current (written out, not through mooring_obs); particles
    # with the same current but their own eta have d = 0, particles with another current
    # have d = (H + eta_i)(u_true - u_i)
    cfg = W.tiny()
    rng = np.random.default_rng(4)
    cells = np.array([[1, 2], [30, 9], [16, 16], [7, 28]], dtype=np.int32)
    X = (cells[:, 0] + 0.5) * cfg.dx
    Y = (cells[:, 1] + 0.5) * cfg.dy
    u, v = _current(X, Y)
    y = np.stack([u, v], axis=1) * cfg.H
    for _ in range(3):
        psi = _state_with_current(cfg, rng, lambda X, Y: _current(X, Y)[0],
                                  lambda X, Y: _current(X, Y)[1])
        d = observe.innovations(psi, cells, y, cfg.H)
        assert np.abs(d).max() < 1e-12 * np.abs(y).max()
    psi = _state_with_current(cfg, rng, lambda X, Y: _current(X, Y)[0] + 0.05,
                              lambda X, Y: _current(X, Y)[1] - 0.02)
    eta = psi[0, cells[:, 1], cells[:, 0]]
    d = observe.innovations(psi, cells, y, cfg.H)
    ref = np.stack([-0.05 * (cfg.H + eta), 0.02 * (cfg.H + eta)], axis=1)
    assert np.abs(d - ref).max() < 1e-11 * np.abs(ref).max()


def test_noise_free_mooring_of_a_state_has_zero_innovation_for_it():
    cfg = W.paper_scale(1)
    rng = np.random.default_rng(5)
    psi = W.random_state(cfg, rng, eta_amp=1.5, q_amp=80.0)
    cells = W.buoy_cells(cfg.nx, cfg.ny, 15, 15)
    y = observe.mooring_obs(psi, cells, cfg.H, cfg.obs_sigma, np.zeros((len(cells), 2)))
    d = observe.innovations(psi, cells, y, cfg.H)
    assert np.abs(d).max() < 1e-13 * np.abs(psi[1:]).max()


def test_mooring_noise_is_sigma_times_the_normals():
    cfg = W.tiny().replace(obs_sigma=2.5)
    rng = np.random.default_rng(6)
    psi = W.random_state(cfg, rng)
    cells = np.array([[3, 4], [20, 25]], dtype=np.int32)
    n = rng.standard_normal((2, 2))
    y0 = observe.mooring_obs(psi, cells, cfg.H, cfg.obs_sigma, np.zeros((2, 2)))
    y1 = observe.mooring_obs(psi, cells, cfg.H, cfg.obs_sigma, n)
    assert np.abs((y1 - y0) - 2.5 * n).max() < 1e-12


def _uniform_current_state(cfg, rng, U, V):
    return _state_with_current(cfg, rng, lambda X, Y: U + 0 * X, lambda X, Y: V + 0 * X)


def test_drifter_observation_in_a_uniform_current_is_current_times_depth():
    # a uniform current moves Heun drifters exactly, whatever eta is; over the observation
    # interval (10 model steps of 30 s) the observation is (U, V) H, equal to the noise-free
    # mooring observation at the drifter's cell; a drifter that crosses the periodic
    # boundary (unwrapped positions) observes the same value
    cfg = W.tiny()
    rng = np.random.default_rng(7)
    U, V = 0.61, -0.37
    psi = _uniform_current_state(cfg, rng, U, V)
    lx = cfg.nx * cfg.dx
    pos0 = np.concatenate([W.drifter_lattice(cfg, 2, 2),
                           np.array([[lx - 50.0, 3.3e4]])])  # crosses x = L within the interval
    p = pos0.copy()
    dt_obs = 10 * cfg.dt
    for _ in range(10):
        p = drifters.heun_step(p, psi, psi, cfg, cfg.dt)
    y = observe.drifter_obs(p, pos0, dt_obs, cfg.H, cfg.obs_sigma, np.zeros((5, 2)))
    ref = np.array([U, V]) * cfg.H
    assert np.abs(y - ref[None]).max() < 1e-9 * np.abs(ref).max()
    assert p[4, 0] > lx  # unwrapped: no jump by the domain length
    cells = observe.obs_cell(p, cfg.dx, cfg.dy, cfg.nx, cfg.ny)
    assert cells[4, 0] == 0
    ym = observe.mooring_obs(psi, cells, cfg.H, cfg.obs_sigma, np.zeros((5, 2)))
    assert np.abs(y - ym).max() < 1e-9 * np.abs(ref).max()
    # the eta-compensated innovation of the truth itself vanishes for drifter observations too
    d = observe.innovations(psi, cells, y, cfg.H)
    assert np.abs(d).max() < 1e-9 * np.abs(ref).max()


def test_drifter_observation_noise_and_interval():
    cfg = W.tiny().replace(obs_sigma=0.7)
    prev = np.array([[1.0e4, 2.0e4], [5.0, 3.1e5]])
    now = prev + np.array([[150.0, -60.0], [-90.0, 30.0]])
    n = np.array([[0.3, -1.2], [2.0, 0.1]])
    y = observe.drifter_obs(now, prev, 300.0, cfg.H, cfg.obs_sigma, n)
    ref = (now - prev) / 300.0 * cfg.H + 0.7 * n
    assert np.abs(y - ref).max() < 1e-12
    # half the interval for the same displacement: twice the current
    y2 = observe.drifter_obs(now, prev, 150.0, cfg.H, cfg.obs_sigma, np.zeros((2, 2)))
    assert np.abs(y2 - 2.0 * (ref - 0.7 * n)).max() < 1e-11


def test_observed_cell_is_floor_of_position_modulo_the_grid():
    cfg = W.tiny()
    lx, ly = cfg.nx * cfg.dx, cfg.ny * cfg.dy
    pos = np.array([[0.0, 0.0], [cfg.dx, 2 * cfg.dy - 1e-6], [-1.0, ly + 1.0],
                    [lx - 1e-3, -ly - 0.5 * cfg.dy], [3 * lx + 5.5 * cfg.dx, 7.25 * cfg.dy]])
    cells = observe.obs_cell(pos, cfg.dx, cfg.dy, cfg.nx, cfg.ny)
    assert cells.tolist() == [[0, 0], [1, 1], [31, 0], [31, 31], [5, 7]]
