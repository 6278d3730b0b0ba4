"""Ensemble-level drivers: initial ensemble, stochastic model steps, perturbation.

Paper: eq. model_equation -- psi_i^n = M(psi_i^{n-1}) + beta_i^{n-1}, particles
independent; the model error is added after each model step except the step that ends
at an observation time (Section "Observations and innovations": the forecast to the
observation time is taken without the stochastic term).

Random streams (see philox): model error of particle i after model step n uses
(step = n, tag = MODEL_ERROR); the initial perturbation uses (step = stream index,
tag = INIT).
"""
from __future__ import annotations

import numpy as np

from . import model_error as me
from . import philox
from .swe import SweParams, model_step


def coarse_normals(cfg, step: int, tag: int, particle: int, ensemble_id=None) -> np.ndarray:
    ens = cfg.ensemble_id if ensemble_id is None else ensemble_id
    n = cfg.nrx * cfg.nry
    return philox.normals(n, cfg.seed, step, tag, ens, particle).reshape(cfg.nry, cfg.nrx)


def perturbation(cfg, step: int, particle: int, w=None) -> np.ndarray:
    """beta = Q^{1/2} xi for one particle after model step `step` -> [3, ny, nx]."""
    if w is None:
        w = me.model_error_stencil(cfg)
    xi = coarse_normals(cfg, step, philox.TAG_MODEL_ERROR, particle)
    return me.apply_qhalf(xi, w, cfg)


def init_member(cfg, base: np.ndarray | None, stream: int, particle: int) -> np.ndarray:
    """base + Q_init^{1/2} xi (SOAR eta perturbation in geostrophic balance)."""
    w = me.init_stencil(cfg)
    xi = coarse_normals(cfg, stream, philox.TAG_INIT, particle)
    pert = me.apply_qhalf(xi, w, cfg)
    if base is None:
        return pert
    return np.asarray(base, dtype=np.float64) + pert


def step_member(psi: np.ndarray, cfg, particle: int, first_step: int, n_steps: int,
                noise_on_last: bool = True) -> np.ndarray:
    """n_steps model steps of one particle; model error after each step (step index
    first_step + s), skipped after the last one when noise_on_last is False."""
    p = SweParams.of(cfg)
    w = me.model_error_stencil(cfg)
    out = np.asarray(psi, dtype=np.float64)
    for s in range(n_steps):
        out = model_step(out, p, cfg.dt, cfg.n_sub)
        if s < n_steps - 1 or noise_on_last:
            out = out + perturbation(cfg, first_step + s, particle, w)
    return out
