"""Model error beta = Q^{1/2} xi = Q_GB^{1/2} I_Omega Q_SOAR^{1/2} xi.

Paper: Section "Small scale model errors".
  * xi ~ N(0, I) on the coarse random grid Omega^R, cells c_Omega dx x c_Omega dy, values
    are point values at coarse-cell centres (fig. nestedGrids);
  * Q_SOAR^{1/2}: 5x5 (c_SOAR = 2) periodic stencil q0 (1 + d/L0) exp(-d/L0)
    (eq. soar_function, eq. local_soar_on_eta), d the distance between coarse points;
  * I_Omega: bicubic interpolation Omega^R -> Omega^M from the 4x4 surrounding coarse
    points (read as Catmull-Rom cubic convolution, evaluated at fine cell centres);
  * Q_GB^{1/2}: central-difference geostrophic balance on the fine grid
    (eq. geostrophic_balance_disc) with depth H.
The perturbation is added to the state after a model step (never stored).

Readings where the paper is silent or in conflict: even c_Omega is allowed (coarse points
then sit on fine-cell corners); q0 is set from the requested pointwise std of the coarse
SOAR field, q0 = std / ||k||_2 with k the unit-amplitude 5x5 SOAR stencil.
"""
from __future__ import annotations

import math

import numpy as np


def soar_stencil(q0: float, L0: float, dxc: float, dyc: float) -> np.ndarray:
    """5x5 SOAR weights, index [q+2, p+2] for coarse offset (p in x, q in y)."""
    p = np.arange(-2, 3, dtype=np.float64)
    d = np.sqrt((p[None, :] * dxc) ** 2 + (p[:, None] * dyc) ** 2)
    return q0 * (1.0 + d / L0) * np.exp(-d / L0)


def q0_from_std(std: float, L0: float, dxc: float, dyc: float) -> float:
    """Amplitude q0 giving the coarse SOAR field a pointwise standard deviation `std`."""
    k = soar_stencil(1.0, L0, dxc, dyc)
    return std / math.sqrt(float(np.sum(k * k)))


def soar_apply(xi: np.ndarray, w: np.ndarray) -> np.ndarray:
    """z[b, a] = sum_{|p|,|q|<=2} w[q+2, p+2] xi[b+q, a+p], periodic (eq. local_soar_on_eta)."""
    z = np.zeros_like(xi, dtype=np.float64)
    for q in range(-2, 3):
        for p in range(-2, 3):
            z += w[q + 2, p + 2] * np.roll(np.roll(xi, -q, axis=-2), -p, axis=-1)
    return z


def catmull_rom(t):
    """Cubic-convolution weights (Keys, a = -1/2) for taps at -1, 0, 1, 2 and phase t."""
    t = np.asarray(t, dtype=np.float64)
    t2, t3 = t * t, t * t * t
    return np.stack([0.5 * (-t3 + 2 * t2 - t),
                     0.5 * (3 * t3 - 5 * t2 + 2),
                     0.5 * (-3 * t3 + 4 * t2 + t),
                     0.5 * (t3 - t2)], axis=-1)


def _axis_taps(n_fine: int, c: int):
    """Base coarse index and phase of every fine cell on the unshifted coarse grid.

    Coarse point a sits at x = (a + 1/2) c dx; fine cell centre j at (j + 1/2) dx, so its
    coarse coordinate is s = (2 j + 1 - c) / (2 c); base = floor(s), phase t = s - base."""
    j = np.arange(n_fine)
    num = 2 * j + 1 - c
    base = np.floor_divide(num, 2 * c)
    t = (num - 2 * c * base) / (2.0 * c)
    return base, t


def _axis_taps_shifted(n_fine: int, c: int, j0: int):
    """Same for a coarse grid shifted so that coarse point 0 sits on fine cell j0."""
    rel = np.mod(np.arange(n_fine) - j0, n_fine)
    base = rel // c
    t = (rel % c) / float(c)
    return base, t


def _interp(z: np.ndarray, bx, tx, by, ty) -> np.ndarray:
    nry, nrx = z.shape
    wx = catmull_rom(tx)  # [nx, 4]
    wy = catmull_rom(ty)  # [ny, 4]
    ny, nx = len(by), len(bx)
    out = np.zeros((ny, nx))
    for m in range(4):
        ix = np.mod(bx + m - 1, nrx)
        for n in range(4):
            iy = np.mod(by + n - 1, nry)
            out += wy[:, n][:, None] * wx[:, m][None, :] * z[np.ix_(iy, ix)]
    return out


def bicubic(z: np.ndarray, c: int, nx: int, ny: int) -> np.ndarray:
    """I_Omega: coarse field [nry, nrx] -> fine [ny, nx] (unshifted coarse grid)."""
    bx, tx = _axis_taps(nx, c)
    by, ty = _axis_taps(ny, c)
    return _interp(z, bx, tx, by, ty)


def bicubic_shifted(z: np.ndarray, c: int, nx: int, ny: int, j0: int, k0: int) -> np.ndarray:
    """I_Omega from a coarse grid offset so that its point (0, 0) is co-located with the
    centre of fine cell (j0, k0) (fig. nestedGrids caption)."""
    bx, tx = _axis_taps_shifted(nx, c, j0)
    by, ty = _axis_taps_shifted(ny, c, k0)
    return _interp(z, bx, tx, by, ty)


def geostrophic(deta: np.ndarray, H: float, g: float, f: float, dx: float, dy: float):
    """Q_GB^{1/2}: (dhu, dhv) from deta by central differences (eq. geostrophic_balance_disc)."""
    a = g * H / f
    dhu = -a * (np.roll(deta, -1, axis=-2) - np.roll(deta, 1, axis=-2)) / (2.0 * dy)
    dhv = a * (np.roll(deta, -1, axis=-1) - np.roll(deta, 1, axis=-1)) / (2.0 * dx)
    return dhu, dhv


def apply_qhalf(coarse: np.ndarray, w: np.ndarray, cfg) -> np.ndarray:
    """Q^{1/2} applied to a coarse field: SOAR, bicubic, geostrophic balance -> [3, ny, nx]."""
    z = soar_apply(coarse, w)
    deta = bicubic(z, cfg.c_omega, cfg.nx, cfg.ny)
    dhu, dhv = geostrophic(deta, cfg.H, cfg.g, cfg.f, cfg.dx, cfg.dy)
    return np.stack([deta, dhu, dhv])


def model_error_stencil(cfg) -> np.ndarray:
    """SOAR stencil of the model-error covariance for a configuration."""
    dxc, dyc = cfg.c_omega * cfg.dx, cfg.c_omega * cfg.dy
    q0 = q0_from_std(cfg.me_std, cfg.L0, dxc, dyc)
    return soar_stencil(q0, cfg.L0, dxc, dyc)


def init_stencil(cfg) -> np.ndarray:
    """SOAR stencil of the initial-state perturbation (std cfg.init_std, length cfg.init_L)."""
    dxc, dyc = cfg.c_omega * cfg.dx, cfg.c_omega * cfg.dy
    q0 = q0_from_std(cfg.init_std, cfg.init_L, dxc, dyc)
    return soar_stencil(q0, cfg.init_L, dxc, dyc)
