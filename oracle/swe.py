"""Rotating shallow-water model M: well-balanced central-upwind finite volumes + SSP-RK2.

Paper: Section "The simplified ocean model" -- conservation law eq. swe_full for
psi = [eta, hu, hv] with h = H + eta and Coriolis source (0, f hv, -f hu); cell (j, k)
centred at ((j+1/2) dx, (k+1/2) dy) (eq. cell_center); second-order strong-stability-
preserving Runge-Kutta in time; step restricted by eq. swecfl with Courant number 0.8.
The paper cites, but does not print, the central-upwind scheme of Chertock et al. with a
local reformulation of the Coriolis potential.  This module fixes one exact definition of
such a scheme (documented reading; both the oracle and the HIP path follow it):

  * velocities u = hu/h, v = hv/h at cell centres;
  * x-reconstruction at cell j uses the Coriolis potential local to cell j:
      K_j = g eta_j,  K_{j+-1} = g eta_{j+-1} -+ (f dx / 2)(v_j + v_{j+-1}),
    generalized-minmod slopes (parameter theta) of K, u, v, and face values
      eta^{E,W} = eta_j +- (sigma_K + f dx v_j) / (2 g),  u^{E,W} = u_j +- sigma_u/2, ...
  * y-reconstruction symmetrically with L_{k+-1} = g eta_{k+-1} +- (f dy/2)(u_k + u_{k+-1})
    and eta^{N,S} = eta_k +- (sigma_L - f dy u_k) / (2 g);
  * Kurganov-Petrova central-upwind flux at each face between the reconstructed states,
    with the momentum flux written as q u + g eta (H + eta/2) (the constant g H^2/2 part of
    g h^2/2 cancels in every flux difference);
  * SSP-RK2: psi* = psi + dt L(psi);  psi^{n+1} = psi/2 + (psi* + dt L(psi*))/2.

The scheme is exactly steady for lake at rest and for axis-aligned jets in the discrete
balance g (eta_{k+1} - eta_k) = -f dy (u_k + u_{k+1})/2 (well-balanced w.r.t. eq.
geostrophic_balance_cont).  The paper prints no scheme, so this definition is the
reference; its pins (tests/test_oracle_swe.py) are mass conservation, the two steady
states, second-order convergence, translation and reflection symmetry, the inertia-
gravity dispersion relation, and, without rotation, convergence to the exact dam-break
(Riemann) solution.  The rotating reconstruction itself (the local Coriolis potential)
is pinned only through the steady jets and the dispersion relation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class SweParams:
    H: float
    g: float
    f: float
    dx: float
    dy: float
    theta: float = 1.3

    @staticmethod
    def of(cfg) -> "SweParams":
        return SweParams(cfg.H, cfg.g, cfg.f, cfg.dx, cfg.dy, cfg.theta)


def _east(a):   # value of cell j+1 at cell j
    return np.roll(a, -1, axis=-1)


def _west(a):   # value of cell j-1
    return np.roll(a, 1, axis=-1)


def _north(a):  # value of cell k+1
    return np.roll(a, -1, axis=-2)


def _south(a):  # value of cell k-1
    return np.roll(a, 1, axis=-2)


def minmod3(a, b, c):
    """Generalized minmod: min if all positive, max if all negative, else 0."""
    pos = (a > 0) & (b > 0) & (c > 0)
    neg = (a < 0) & (b < 0) & (c < 0)
    return np.where(pos, np.minimum(a, np.minimum(b, c)),
                    np.where(neg, np.maximum(a, np.maximum(b, c)), 0.0))


def limited_slope(qm, q0, qp, theta):
    return minmod3(theta * (q0 - qm), 0.5 * (qp - qm), theta * (qp - q0))


def central_upwind_flux(eL, unL, utL, eR, unR, utR, H, g):
    """Kurganov-Petrova flux between left (-) and right (+) face states given as
    (eta, normal velocity, tangential velocity).  Returns (mass, normal momentum,
    tangential momentum) fluxes."""
    hL = H + eL
    hR = H + eR
    qL, qR = hL * unL, hR * unR          # normal momentum
    tL, tR = hL * utL, hR * utR          # tangential momentum
    cL, cR = np.sqrt(g * hL), np.sqrt(g * hR)
    ap = np.maximum(np.maximum(unL + cL, unR + cR), 0.0)
    am = np.minimum(np.minimum(unL - cL, unR - cR), 0.0)
    FL = (qL, qL * unL + g * eL * (H + 0.5 * eL), qL * utL)
    FR = (qR, qR * unR + g * eR * (H + 0.5 * eR), qR * utR)
    UL = (eL, qL, tL)
    UR = (eR, qR, tR)
    den = ap - am
    out = []
    for k in range(3):
        out.append((ap * FL[k] - am * FR[k]) / den + ap * am / den * (UR[k] - UL[k]))
    return out


def rhs(psi: np.ndarray, p: SweParams) -> np.ndarray:
    """Semi-discrete operator L(psi) for one state [3, ny, nx] (or [..., 3, ny, nx])."""
    eta, hu, hv = psi[..., 0, :, :], psi[..., 1, :, :], psi[..., 2, :, :]
    H, g, f, dx, dy, th = p.H, p.g, p.f, p.dx, p.dy, p.theta
    h = H + eta
    u = hu / h
    v = hv / h

    # ---- x direction: faces j+1/2 between cell j (east face) and cell j+1 (west face)
    Kc = g * eta
    Kp = g * _east(eta) - 0.5 * f * dx * (v + _east(v))
    Km = g * _west(eta) + 0.5 * f * dx * (v + _west(v))
    sK = limited_slope(Km, Kc, Kp, th)
    su = limited_slope(_west(u), u, _east(u), th)
    sv = limited_slope(_west(v), v, _east(v), th)
    off = (sK + f * dx * v) / (2.0 * g)
    eE, eW = eta + off, eta - off
    uE, uW = u + 0.5 * su, u - 0.5 * su
    vE, vW = v + 0.5 * sv, v - 0.5 * sv
    Fm, Fu, Fv = central_upwind_flux(eE, uE, vE, _east(eW), _east(uW), _east(vW), H, g)

    # ---- y direction: faces k+1/2 between cell k (north face) and cell k+1 (south face)
    Lc = g * eta
    Lp = g * _north(eta) + 0.5 * f * dy * (u + _north(u))
    Lm = g * _south(eta) - 0.5 * f * dy * (u + _south(u))
    sL = limited_slope(Lm, Lc, Lp, th)
    su_y = limited_slope(_south(u), u, _north(u), th)
    sv_y = limited_slope(_south(v), v, _north(v), th)
    offy = (sL - f * dy * u) / (2.0 * g)
    eN, eS = eta + offy, eta - offy
    uN, uS = u + 0.5 * su_y, u - 0.5 * su_y
    vN, vS = v + 0.5 * sv_y, v - 0.5 * sv_y
    Gm, Gv, Gu = central_upwind_flux(eN, vN, uN, _north(eS), _north(vS), _north(uS), H, g)

    out = np.empty_like(psi)
    out[..., 0, :, :] = -(Fm - _west(Fm)) / dx - (Gm - _south(Gm)) / dy
    out[..., 1, :, :] = -(Fu - _west(Fu)) / dx - (Gu - _south(Gu)) / dy + f * hv
    out[..., 2, :, :] = -(Fv - _west(Fv)) / dx - (Gv - _south(Gv)) / dy - f * hu
    return out


def substep(psi: np.ndarray, p: SweParams, dt: float) -> np.ndarray:
    """One SSP-RK2 scheme step of size dt."""
    s1 = psi + dt * rhs(psi, p)
    return 0.5 * psi + 0.5 * (s1 + dt * rhs(s1, p))


def model_step(psi: np.ndarray, p: SweParams, dt: float, n_sub: int) -> np.ndarray:
    """Deterministic model operator M over one model step dt = n_sub equal scheme steps
    (the model step is decoupled from the scheme step, Section "The simplified ocean
    model")."""
    out = np.asarray(psi, dtype=np.float64)
    for _ in range(n_sub):
        out = substep(out, p, dt / n_sub)
    return out


def cfl_dt(psi: np.ndarray, p: SweParams, courant: float = 0.8) -> float:
    """Largest admissible scheme step, eq. swecfl with the Courant number applied:
    courant * 1/4 * min(dx / max(|u| + c), dy / max(|v| + c)), c = sqrt(g (H + eta))."""
    eta, hu, hv = psi[..., 0, :, :], psi[..., 1, :, :], psi[..., 2, :, :]
    h = p.H + eta
    c = np.sqrt(p.g * h)
    sx = np.max(np.abs(hu / h) + c)
    sy = np.max(np.abs(hv / h) + c)
    return courant * 0.25 * min(p.dx / sx, p.dy / sy)


def n_substeps(psi: np.ndarray, p: SweParams, dt: float, courant: float = 0.8) -> int:
    return int(math.ceil(dt / cfl_dt(psi, p, courant) - 1e-12))
