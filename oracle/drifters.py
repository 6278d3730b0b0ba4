"""Passive drifters advected by the model currents.

Paper: Section "Synthetic truth and observations" (drifters follow the current; the
paper's truth uses forward Euler) and the drift-forecast experiments.  One integrator is
used for truth and forecasts (reading): Heun / RK2 over one model step,
    k1 = u(p; psi^n),  p* = p + dt k1,  k2 = u(p*; psi^{n+1}),  p' = p + dt (k1 + k2)/2,
with u = (hu, hv)/(H + eta) at cell centres interpolated bilinearly (periodic).
Positions are unwrapped metres; sampling wraps them into the domain.
Forecast errors: eq. errorPerEnsembleDrifter and eq. errorNorm.
"""
from __future__ import annotations

import numpy as np


def velocity(psi: np.ndarray, pos: np.ndarray, cfg) -> np.ndarray:
    """Bilinear (u, v) at positions [n, 2] from cell-centre velocities of psi [3, ny, nx]."""
    h = cfg.H + psi[0]
    uc = psi[1] / h
    vc = psi[2] / h
    fx = pos[:, 0] / cfg.dx - 0.5
    fy = pos[:, 1] / cfg.dy - 0.5
    j0 = np.floor(fx).astype(np.int64)
    k0 = np.floor(fy).astype(np.int64)
    tx = fx - j0
    ty = fy - k0
    j0m, j1m = np.mod(j0, cfg.nx), np.mod(j0 + 1, cfg.nx)
    k0m, k1m = np.mod(k0, cfg.ny), np.mod(k0 + 1, cfg.ny)
    out = np.zeros_like(pos, dtype=np.float64)
    for comp, fld in enumerate((uc, vc)):
        out[:, comp] = ((1 - tx) * (1 - ty) * fld[k0m, j0m] + tx * (1 - ty) * fld[k0m, j1m]
                        + (1 - tx) * ty * fld[k1m, j0m] + tx * ty * fld[k1m, j1m])
    return out


def heun_step(pos: np.ndarray, psi_n: np.ndarray, psi_np1: np.ndarray, cfg, dt: float) -> np.ndarray:
    k1 = velocity(psi_n, pos, cfg)
    pstar = pos + dt * k1
    k2 = velocity(psi_np1, pstar, cfg)
    return pos + 0.5 * dt * (k1 + k2)


def euler_step(pos: np.ndarray, psi_n: np.ndarray, cfg, dt: float) -> np.ndarray:
    return pos + dt * velocity(psi_n, pos, cfg)


def _min_image(d: np.ndarray, length: float) -> np.ndarray:
    return d - length * np.round(d / length)


def forecast_error(pos_ens: np.ndarray, pos_true: np.ndarray, lx: float, ly: float) -> float:
    """E(t): sqrt(mean_d mean_i |x_id - x_true,d|^2) with minimum-image distances."""
    dx = _min_image(pos_ens[..., 0] - pos_true[None, :, 0], lx)
    dy = _min_image(pos_ens[..., 1] - pos_true[None, :, 1], ly)
    return float(np.sqrt(np.mean(dx * dx + dy * dy)))


def forecast_rmse(pos_ens: np.ndarray, lx: float, ly: float) -> float:
    """RMSE(t): as forecast_error but about the ensemble mean (spread)."""
    mean = pos_ens.mean(axis=0)
    return forecast_error(pos_ens, mean, lx, ly)
