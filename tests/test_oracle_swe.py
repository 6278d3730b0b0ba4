"""Pins of the oracle's shallow-water scheme (invariants, symmetries, closed forms, the
exact dam-break solution).

The paper cites its scheme without printing it, so these checks pin the properties any
correct well-balanced central-upwind SSP-RK2 scheme for eq. swe_full must have."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import swe


def _cfg(nx=40, ny=32, dx=1e4, **kw):
    return W.Config(nx=nx, ny=ny, dx=dx, dy=dx, **kw)


def test_mass_conserved_to_roundoff():
    cfg = _cfg()
    p = swe.SweParams.of(cfg)
    psi = W.random_state(cfg, np.random.default_rng(1))
    out = psi
    for _ in range(5):
        out = swe.model_step(out, p, 30.0, 2)
    assert abs(out[0].sum() - psi[0].sum()) < 1e-11 * np.abs(psi[0]).sum()
    assert np.abs(out - psi).max() > 1e-3  # the state does evolve


def test_lake_at_rest_exact():
    cfg = _cfg()
    p = swe.SweParams.of(cfg)
    z = np.zeros((3, cfg.ny, cfg.nx))
    assert np.array_equal(swe.model_step(z, p, 30.0, 1), z)


def test_zonal_jet_well_balanced():
    # eta and the normal momentum hv are steady to roundoff; only hu (tangential) diffuses
    cfg = W.paper_scale().replace(nx=24, ny=300)
    p = swe.SweParams.of(cfg)
    jet = W.jet_state(cfg)
    r = swe.rhs(jet, p)
    assert np.abs(r[0]).max() < 1e-15 * 1e3
    assert np.abs(r[2]).max() < 1e-12
    assert np.abs(r[1]).max() > 1e-6


def test_meridional_jet_well_balanced():
    cfg = W.paper_scale().replace(nx=24, ny=300)
    jet = W.jet_state(cfg)
    # transpose: v(x) = -u(y) keeps g eta_x = f v in the discrete sense
    tcfg = cfg.replace(nx=300, ny=24)
    jt = np.stack([jet[0].T, jet[2].T, -jet[1].T])
    r = swe.rhs(jt, swe.SweParams.of(tcfg))
    assert np.abs(r[0]).max() < 1e-12
    assert np.abs(r[1]).max() < 1e-12
    assert np.abs(r[2]).max() > 1e-6


def test_tangential_diffusion_second_order():
    # the jet's only motion is diffusion of the tangential momentum; for a smooth profile
    # it shrinks at second order in the mean (factor ~4 per refinement) and at first order
    # in the max norm, where the minmod limiter clips the slopes at the jet extrema
    l1, linf = [], []
    for ny in (100, 200, 400):
        cfg = W.paper_scale().replace(nx=8, ny=ny, dy=1.5e6 / ny, dx=1.5e6 / ny)
        jet = W.jet_state(cfg)
        r = swe.rhs(jet, swe.SweParams.of(cfg))
        l1.append(np.abs(r[1]).mean())
        linf.append(np.abs(r[1]).max())
    for a, b in zip(l1[:-1], l1[1:]):
        assert 3.6 < a / b < 4.4
    for a, b in zip(linf[:-1], linf[1:]):
        assert 1.8 < a / b < 2.2


def test_translation_commutes():
    cfg = _cfg()
    p = swe.SweParams.of(cfg)
    psi = W.random_state(cfg, np.random.default_rng(2))
    a = np.roll(swe.model_step(psi, p, 30.0, 2), (3, -5), axis=(1, 2))
    b = swe.model_step(np.roll(psi, (3, -5), axis=(1, 2)), p, 30.0, 2)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


def test_transpose_equals_reflected_rotation():
    # x<->y with hu<->hv is a reflection: equal to the step with f -> -f
    cfg = _cfg(nx=32, ny=32)
    p = swe.SweParams.of(cfg)
    pm = swe.SweParams(p.H, p.g, -p.f, p.dx, p.dy, p.theta)
    psi = W.random_state(cfg, np.random.default_rng(3))
    T = lambda s: np.stack([s[0].T, s[2].T, s[1].T])
    a = T(swe.model_step(psi, p, 30.0, 1))
    b = swe.model_step(T(psi), pm, 30.0, 1)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


def _inertia_gravity_error(n):
    # eigenmode eta = A cos kx, hu = A w/k cos kx, hv = A f/k sin kx of the linearised
    # equations, w^2 = f^2 + g H k^2; compare after one period
    L = 2.0e6
    cfg = W.Config(nx=n, ny=4, dx=L / n, dy=L / n)
    p = swe.SweParams.of(cfg)
    k = 2 * math.pi / L
    w = math.sqrt(cfg.f ** 2 + cfg.g * cfg.H * k * k)
    A = 1e-4
    x = (np.arange(n) + 0.5) * cfg.dx
    def mode(t):
        th = k * x - w * t
        return np.stack([np.tile(A * np.cos(th), (4, 1)), np.tile(A * w / k * np.cos(th), (4, 1)),
                         np.tile(A * cfg.f / k * np.sin(th), (4, 1))])
    T = 2 * math.pi / w
    dt = swe.cfl_dt(mode(0), p)
    nsteps = int(math.ceil(T / dt))
    psi = mode(0)
    for _ in range(nsteps):
        psi = swe.substep(psi, p, T / nsteps)
    return np.abs(psi[0] - mode(T)[0]).max() / A


def test_inertia_gravity_wave_dispersion():
    e1, e2 = _inertia_gravity_error(32), _inertia_gravity_error(64)
    assert e2 < 0.02
    assert e1 / e2 > 3.0


def test_cfl_substeps_for_workloads():
    for cfg, nsub in ((W.tiny(), 1), (W.paper_scale(), 2)):
        p = swe.SweParams.of(cfg)
        base = W.jet_state(cfg)
        assert swe.n_substeps(base, p, cfg.dt, cfg.courant) <= nsub == cfg.n_sub


def _dam_break_exact(xi, hL, hR, g):
    """Exact depth of the wet dam break (still water of depth hL left of the dam, hR < hL
    right of it) at x / t = xi: a rarefaction into hL, the middle state, a shock into hR
    (Stoker's solution).  The middle depth equates the rarefaction's velocity
    2 (sqrt(g hL) - sqrt(g hm)) and the shock's (hm - hR) sqrt(g/2 (1/hm + 1/hR))."""
    cL = math.sqrt(g * hL)

    def gap(hm):
        return 2.0 * (cL - math.sqrt(g * hm)) - (hm - hR) * math.sqrt(0.5 * g * (1 / hm + 1 / hR))

    lo, hi = hR, hL
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if gap(mid) > 0 else (lo, mid)
    hm = 0.5 * (lo + hi)
    cm = math.sqrt(g * hm)
    um = 2.0 * (cL - cm)
    s = hm * um / (hm - hR)  # shock speed from the mass jump
    h = np.where(xi < -cL, hL, 0.0)
    fan = (xi >= -cL) & (xi < um - cm)
    h = np.where(fan, (2.0 * cL - xi) ** 2 / (9.0 * g), h)
    h = np.where((xi >= um - cm) & (xi < s), hm, h)
    return np.where(xi >= s, hR, h)


def _dam_break_error(nx):
    """L1 error of the depth against the exact dam-break solution, without rotation: the
    flux, wave-speed bounds, limiter and time stepping all enter.  A periodic strip holds
    two dams (at L/2 and at 0); the comparison covers [L/4, 3L/4], which only the dam at
    L/2 reaches before the end time."""
    L, H, g = 2.0, 1.0, 9.81
    hL, hR = 2.0, 1.0
    dx = L / nx
    p = swe.SweParams(H=H, g=g, f=0.0, dx=dx, dy=dx)
    x = (np.arange(nx) + 0.5) * dx
    psi = np.zeros((3, 4, nx))
    psi[0] = np.where(x < L / 2, hL - H, hR - H)[None, :]
    t_end = 0.08  # the waves of the two dams meet after ~0.11
    n = int(math.ceil(t_end / swe.cfl_dt(psi, p)))
    for _ in range(n):
        psi = swe.substep(psi, p, t_end / n)
    assert np.abs(psi[:, 1:] - psi[:, :1]).max() < 1e-12  # stays uniform across the strip
    assert np.abs(psi[2]).max() < 1e-12
    win = (x >= L / 4) & (x < 3 * L / 4)
    exact = _dam_break_exact((x[win] - L / 2) / t_end, hL, hR, g)
    return np.abs(H + psi[0, 0, win] - exact).mean() / hR


def test_dam_break_converges_to_exact_riemann_solution():
    e1, e2 = _dam_break_error(200), _dam_break_error(400)
    assert e2 < 4e-3, (e1, e2)
    assert e1 / e2 > 1.5, (e1, e2)
