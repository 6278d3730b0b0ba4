"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the benchmark.

This module holds configuration constants and input recipes only (grid sizes, physics
constants, observation placement, base states, random test states).  It contains none of
the filter's arithmetic: no scheme, no covariance operator, no analysis step.

The paper's experiments are identical-twin runs on a 500x300 periodic grid with moored
buoys and drifters (Section "Experimental results"); its truth/observation files are not
available, so every input here is synthetic, seeded and shaped like those workloads.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# Philox key base for the workloads below: key = SEED_BASE + workload index.
SEED_BASE = 0x191001031


@dataclasses.dataclass
class Config:
    """One ensemble's grid, physics, model-error and filter constants.

    Symbols follow the paper: grid n_x x n_y of dx x dy cells (eq. cell_center), depth H,
    gravity g, Coriolis f (eq. swe_full), model time step dt split into n_sub scheme steps
    (eq. swecfl), coarse random grid with coarsening c_omega (Section "Small scale model
    errors"), observation error std obs_sigma (R = obs_sigma^2 I).
    """

    nx: int
    ny: int
    dx: float
    dy: float
    H: float = 230.0
    g: float = 9.81
    f: float = 1.2e-4
    dt: float = 30.0
    n_sub: int = 1
    c_omega: int = 4
    me_std: float = 1e-3          # model-error pointwise std of the coarse SOAR field [m]
    me_L0: Optional[float] = None  # SOAR length scale; None -> 0.75 * coarse spacing
    obs_sigma: float = 1.0
    n_particles: int = 10
    seed: int = SEED_BASE
    ensemble_id: int = 0
    theta: float = 1.3            # generalized-minmod parameter
    courant: float = 0.8
    init_std: float = 0.5         # initial-state SOAR eta std [m]
    init_L0: Optional[float] = None
    obs_every: int = 10           # model steps per observation interval (5 min at dt=30 s)

    @property
    def L0(self) -> float:
        return self.me_L0 if self.me_L0 is not None else 0.75 * self.c_omega * self.dx

    @property
    def init_L(self) -> float:
        return self.init_L0 if self.init_L0 is not None else 0.75 * self.c_omega * self.dx

    @property
    def nrx(self) -> int:
        return self.nx // self.c_omega

    @property
    def nry(self) -> int:
        return self.ny // self.c_omega

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny

    @property
    def n_psi(self) -> int:
        return 3 * self.nx * self.ny

    @property
    def n_r(self) -> int:
        return self.nrx * self.nry

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


def tiny() -> Config:
    """32x32 periodic, dx=10 km, 10 particles, 4 drifters, 1 h window (12 analyses)."""
    return Config(nx=32, ny=32, dx=1e4, dy=1e4, n_sub=1, c_omega=4, me_std=1e-3,
                  n_particles=10, seed=SEED_BASE + 0, init_std=0.5, init_L0=4e4)


def paper_scale(n_particles: int = 100) -> Config:
    """500x300 periodic, dx=5 km, 100 particles, 225 moored buoys, model error on a
    1/4-resolution coarse grid; jet + SOAR eta perturbation initial states."""
    return Config(nx=500, ny=300, dx=5e3, dy=5e3, n_sub=2, c_omega=4, me_std=1e-3,
                  n_particles=n_particles, seed=SEED_BASE + 1, init_std=0.05, init_L0=None)


def large_ensemble() -> Config:
    """500x300, 1000 particles (the large drift-forecast ensemble)."""
    return paper_scale(1000).replace(seed=SEED_BASE + 4)


def batched() -> List[Tuple[Config, Tuple[int, int]]]:
    """Eight independent ensembles of uneven size, each with its own buoy lattice."""
    spec = [((200, 120), 4, 50, (6, 5)), ((256, 256), 4, 75, (8, 8)),
            ((300, 200), 4, 100, (12, 8)), ((500, 300), 4, 200, (15, 15)),
            ((500, 300), 4, 150, (15, 10)), ((400, 400), 4, 125, (14, 14)),
            ((128, 512), 4, 60, (4, 16)), ((350, 250), 5, 90, (12, 10))]
    out = []
    for e, ((nx, ny), c, ne, lat) in enumerate(spec):
        cfg = Config(nx=nx, ny=ny, dx=5e3, dy=5e3, n_sub=2, c_omega=c, n_particles=ne,
                     seed=SEED_BASE + 2, ensemble_id=e, init_std=0.05)
        out.append((cfg, lat))
    return out


# --------------------------------------------------------------------------------------
# Observation placement
# --------------------------------------------------------------------------------------

def buoy_cells(nx: int, ny: int, nbx: int, nby: int) -> np.ndarray:
    """Equidistant moored buoys: buoy (m, l) sits in cell (floor((m+1/2) nx/nbx),
    floor((l+1/2) ny/nby)).  Returns int32 [nbx*nby, 2] of (j, k), l-major."""
    cells = []
    for l in range(nby):
        for m in range(nbx):
            cells.append((((2 * m + 1) * nx) // (2 * nbx), ((2 * l + 1) * ny) // (2 * nby)))
    return np.asarray(cells, dtype=np.int32)


def drifter_lattice(cfg: Config, nbx: int, nby: int) -> np.ndarray:
    """Drifters released on an nbx x nby lattice at ((m+1/2) L_x/nbx, (l+1/2) L_y/nby) in
    metres.  Returns float64 [nbx*nby, 2]."""
    lx, ly = cfg.nx * cfg.dx, cfg.ny * cfg.dy
    pos = [((m + 0.5) * lx / nbx, (l + 0.5) * ly / nby) for l in range(nby) for m in range(nbx)]
    return np.asarray(pos, dtype=np.float64)


# --------------------------------------------------------------------------------------
# Base states and random test states (float64 arrays [3, ny, nx] = eta, hu, hv)
# --------------------------------------------------------------------------------------

def jet_state(cfg: Config, u0: float = 1.0, wavenumber: int = 1) -> np.ndarray:
    """Zonal double jet u_k = u0 sin(2 pi m (k+1/2)/n_y) with eta from the discrete
    balance g (eta_{k+1} - eta_k) = -f dy (u_k + u_{k+1}) / 2, re-centred to zero mean;
    hu = (H + eta) u, hv = 0.  Stands in for the paper's Galewsky-like double jet, whose
    profile is only given as a figure."""
    k = np.arange(cfg.ny)
    u = u0 * np.sin(2.0 * math.pi * wavenumber * (k + 0.5) / cfg.ny)
    eta = np.zeros(cfg.ny)
    for kk in range(cfg.ny - 1):
        eta[kk + 1] = eta[kk] - cfg.f * cfg.dy * (u[kk] + u[kk + 1]) / (2.0 * cfg.g)
    eta -= eta.mean()
    psi = np.zeros((3, cfg.ny, cfg.nx))
    psi[0] = eta[:, None]
    psi[1] = ((cfg.H + eta) * u)[:, None]
    return psi


def random_state(cfg: Config, rng: np.random.Generator, eta_amp: float = 0.5,
                 q_amp: float = 60.0, n_modes: int = 6) -> np.ndarray:
    """Smooth random state: a few random periodic Fourier modes per field.  Not balanced;
    used for per-step scheme tests."""
    ny, nx = cfg.ny, cfg.nx
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    out = np.zeros((3, ny, nx))
    for fld, amp in enumerate((eta_amp, q_amp, q_amp)):
        acc = np.zeros((ny, nx))
        for _ in range(n_modes):
            kx = rng.integers(0, 4)
            ky = rng.integers(0, 4)
            ph = rng.uniform(0, 2 * math.pi)
            a = rng.normal()
            acc += a * np.cos(2 * math.pi * (kx * x[None, :] + ky * y[:, None]) + ph)
        acc += 0.05 * rng.normal(size=(ny, nx))  # small-scale roughness exercises the limiter
        out[fld] = amp * acc / max(1e-12, np.abs(acc).max())
    return out


def as_f32(a: np.ndarray) -> np.ndarray:
    """Round to the FP32 grid (both paths then consume identical values)."""
    return np.asarray(a, dtype=np.float32)
