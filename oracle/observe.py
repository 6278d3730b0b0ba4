"""Observations, observation operator and innovations.

Paper: Section "Synthetic truth and observations".
  * H picks (hu, hv) of the cell containing the observation (eq. stateObservation);
  * drifter observation: displacement over the observation interval times H, plus noise
    (eq. drifterObservation);
  * mooring observation: true (hu, hv) scaled by H/(H + eta_true), plus noise
    (eq. buoyObservation);
  * eta-compensated innovation d = y (H + eta_i)/H - H(psi_i) (eq. etaCompensatedInnovation).
R = obs_sigma^2 I.  The observed cell of a position (x, y) is (floor(x/dx) mod n_x,
floor(y/dy) mod n_y).
"""
from __future__ import annotations

import numpy as np


def obs_cell(pos: np.ndarray, dx: float, dy: float, nx: int, ny: int) -> np.ndarray:
    """Cell (j, k) containing each position [n, 2] (periodic)."""
    j = np.mod(np.floor(pos[:, 0] / dx).astype(np.int64), nx)
    k = np.mod(np.floor(pos[:, 1] / dy).astype(np.int64), ny)
    return np.stack([j, k], axis=1).astype(np.int32)


def observe(psi: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """H(psi): (hu, hv) at each observed cell, [n_obs, 2]."""
    j, k = cells[:, 0], cells[:, 1]
    return np.stack([psi[1, k, j], psi[2, k, j]], axis=1).astype(np.float64)


def innovations(psi: np.ndarray, cells: np.ndarray, y: np.ndarray, H: float) -> np.ndarray:
    """d_o = y_o (H + eta[k_o, j_o]) / H - (hu, hv)[k_o, j_o], [n_obs, 2]."""
    j, k = cells[:, 0], cells[:, 1]
    eta = np.asarray(psi[0, k, j], dtype=np.float64)
    scale = (H + eta) / H
    return y * scale[:, None] - observe(psi, cells)


def mooring_obs(truth: np.ndarray, cells: np.ndarray, H: float, sigma: float,
                noise: np.ndarray) -> np.ndarray:
    """y_o = (hu, hv)_true H / (H + eta_true) + sigma * noise_o; noise [n_obs, 2] N(0,1)."""
    j, k = cells[:, 0], cells[:, 1]
    eta = np.asarray(truth[0, k, j], dtype=np.float64)
    return observe(truth, cells) * (H / (H + eta))[:, None] + sigma * noise


def drifter_obs(pos_now: np.ndarray, pos_prev: np.ndarray, dt_obs: float, H: float,
                sigma: float, noise: np.ndarray) -> np.ndarray:
    """y_d = (pos_now - pos_prev) / dt_obs * H + sigma * noise_d (unwrapped positions)."""
    return (pos_now - pos_prev) / dt_obs * H + sigma * noise
