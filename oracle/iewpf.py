"""Two-stage implicit equal-weights particle filter analysis (float64).

Paper: Section "Efficient implementation of the IEWPF scheme" (six stages) and Appendix A.

Stage 1  innovations d_i (eq. etaCompensatedInnovation);
Stage 2  pull psi^a = psi^f + Q H^T S d with the per-observation chain of eq.
         detailedOPDUpdate: S d -> H^T -> coarse grid shifted onto the observed cell ->
         Q_GB^{1/2,T} (eq. adjointGeoBalance) -> Q_SOAR -> Q_SOAR -> I_Omega -> Q_GB;
         observations are treated independently with 2x2 blocks S, pulls summed (or,
         optionally, S is the inverse of the full H Q H^T + R over all observations);
         c_i = sum_o d^T S d (eq. ciMultiDrifter; the previous weights are equal after an
         IEWPF step, so their constant term is dropped).  All weights are in -2 log w units.
Stage 3  xi, nu~ ~ N(0, I) on Omega^R, nu = nu~ made perpendicular to xi with preserved
         length (eq. nuPerpendicular), gamma = xi^T xi N_psi/N_R, zeta = nu^T nu N_psi/N_R
         (eq. scalingGammaZeta);
Stage 4  w_target = mean c, beta = min_i ((cbar - c_i)/zeta_i + 1) (eq. betaTwoStage);
Stage 5  c*_i = cbar - c_i - (beta - 1) zeta_i (eq. cistarTwoStage), alpha_i by Lambert W
         (eq. iewpfAlphaSol);
Stage 6  psi = psi^a + Q^{1/2} A^{1/2} (beta^{1/2} nu + alpha^{1/2} xi)
         (eq. optUpdateEquationTwoStage), with the local 49x49 block of
         A = I - Q_SOAR Q_GB^T H^T S H Q_GB Q_SOAR computed on the coarse grid as model grid
         (fig. localsvd and the text around it).

Readings: the adjoint geostrophic coefficient is g H/f (the transpose of eq.
geostrophic_balance_disc; the printed g/(H f) is dimensionally inconsistent); A uses the
coarse-grid S_c = (H Q_c H^T + R)^{-1} so that its spectrum lies in (0, 1]; the square root
of A is the symmetric root V diag(sqrt(lambda)) V^T (equal in distribution to U Sigma^{1/2}
xi); overlapping 7x7 blocks are applied additively to the unmodified field; c*_i is
clamped at 0.
"""
from __future__ import annotations

import math

import numpy as np

from . import model_error as me
from . import observe as ob
from . import philox
from .lambertw import iewpf_alpha

BLOCK_R = 3          # 7x7 coarse block half width
BLOCK_N = 7 * 7


# --------------------------------------------------------------------------------------
# Stage 2: the pull and S
# --------------------------------------------------------------------------------------

def adjoint_gb_dipole(su: float, sv: float, cfg, nry: int, nrx: int) -> np.ndarray:
    """Q_GB^{1/2,T} C H^T (su, sv) on a coarse grid whose point (0,0) is the observed cell
    (eq. adjointGeoBalance, coefficient g H / f, coarse spacing c dx)."""
    a = cfg.g * cfg.H / cfg.f
    dxc, dyc = cfg.c_omega * cfg.dx, cfg.c_omega * cfg.dy
    D = np.zeros((nry, nrx))
    D[1 % nry, 0] += -a * su / (2.0 * dyc)
    D[(-1) % nry, 0] += a * su / (2.0 * dyc)
    D[0, 1 % nrx] += a * sv / (2.0 * dxc)
    D[0, (-1) % nrx] += -a * sv / (2.0 * dxc)
    return D


def pull_one(su: float, sv: float, jo: int, ko: int, cfg, w: np.ndarray) -> np.ndarray:
    """Q^{1/2} Q^{1/2,T} H^T (su, sv) for one observation in cell (jo, ko) -> [3, ny, nx]
    (eq. detailedOPDUpdate read right to left)."""
    nrx, nry = cfg.nx // cfg.c_omega, cfg.ny // cfg.c_omega
    D = adjoint_gb_dipole(su, sv, cfg, nry, nrx)
    Z = me.soar_apply(me.soar_apply(D, w), w)
    deta = me.bicubic_shifted(Z, cfg.c_omega, cfg.nx, cfg.ny, jo, ko)
    dhu, dhv = me.geostrophic(deta, cfg.H, cfg.g, cfg.f, cfg.dx, cfg.dy)
    return np.stack([deta, dhu, dhv])


def hqht(cfg, w: np.ndarray, jo: int = 0, ko: int = 0) -> np.ndarray:
    """2x2 H Q~ H^T obtained by pushing the unit vectors through the pull chain and reading
    (hu, hv) at the observed cell (eq. S_extended and the text after it)."""
    M = np.zeros((2, 2))
    for b, (su, sv) in enumerate(((1.0, 0.0), (0.0, 1.0))):
        p = pull_one(su, sv, jo, ko, cfg, w)
        M[0, b] = p[1, ko, jo]
        M[1, b] = p[2, ko, jo]
    return M


def inverse_via_cholesky(A: np.ndarray) -> np.ndarray:
    """Inverse of a symmetric positive definite matrix through its Cholesky factor."""
    L = np.linalg.cholesky(0.5 * (A + A.T))
    Li = np.linalg.inv(L)
    return Li.T @ Li


def s_matrix(cfg, w: np.ndarray, jo: int = 0, ko: int = 0) -> np.ndarray:
    """S = (H Q~ H^T + R)^{-1}, R = sigma^2 I (eq. S_extended)."""
    M = hqht(cfg, w, jo, ko)
    return inverse_via_cholesky(M + cfg.obs_sigma ** 2 * np.eye(2))


def hqht_full(cfg, w: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """H Q~ H^T over all observations together, [2 n_obs, 2 n_obs] with rows/columns ordered
    (observation, component): column (o, b) pushes the unit vector e_b at observation o
    through the pull chain and reads (hu, hv) at every observed cell.  Blocks between
    observations further apart than the chain's reach are exactly zero; the 2x2 diagonal
    blocks equal hqht().  (The paper treats observations independently, i.e. keeps only the
    diagonal blocks; this is the exact operator it approximates.)"""
    n = len(cells)
    M = np.zeros((2 * n, 2 * n))
    for o in range(n):
        jo, ko = int(cells[o, 0]), int(cells[o, 1])
        for b, (su, sv) in enumerate(((1.0, 0.0), (0.0, 1.0))):
            p = pull_one(su, sv, jo, ko, cfg, w)
            for o2 in range(n):
                j2, k2 = int(cells[o2, 0]), int(cells[o2, 1])
                M[2 * o2, 2 * o + b] = p[1, k2, j2]
                M[2 * o2 + 1, 2 * o + b] = p[2, k2, j2]
    return M


def s_full(cfg, w: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """S = (H Q~ H^T + R)^{-1} over all observations (eq. S_extended without the
    independence assumption), through a Cholesky factorisation of the symmetric part.  With
    c_Omega = 1 the chain's matrix is symmetric (it is H Q H^T); with c_Omega > 1 each
    observation's pull uses a coarse grid aligned on its own cell, so the cross blocks are
    only nearly symmetric and their symmetric part is used."""
    M = hqht_full(cfg, w, cells)
    return inverse_via_cholesky(M + cfg.obs_sigma ** 2 * np.eye(M.shape[0]))


# --------------------------------------------------------------------------------------
# Stage 6 operator: the local block of A = I - Q^{1/2,T} H^T S H Q^{1/2} on the coarse grid
# --------------------------------------------------------------------------------------

def coarse_operator_matrices(cfg, w: np.ndarray, n: int = 16):
    """Dense matrices of the coarse grid used as model grid (interpolation and coarsening
    are the identity): Q_S [N, N], G = Q_GB^{1/2} [3N, N] with spacing c dx, and H [2, 3N]
    observing the point (n//2, n//2).  Grid n x n, periodic, n >= 8 so no stencil wraps."""
    N = n * n
    dxc, dyc = cfg.c_omega * cfg.dx, cfg.c_omega * cfg.dy
    QS = np.zeros((N, N))
    for col in range(N):
        e = np.zeros((n, n))
        e.flat[col] = 1.0
        QS[:, col] = me.soar_apply(e, w).reshape(-1)
    G = np.zeros((3 * N, N))
    for col in range(N):
        e = np.zeros((n, n))
        e.flat[col] = 1.0
        dhu, dhv = me.geostrophic(e, cfg.H, cfg.g, cfg.f, dxc, dyc)
        G[:N, col] = e.reshape(-1)
        G[N:2 * N, col] = dhu.reshape(-1)
        G[2 * N:, col] = dhv.reshape(-1)
    c0 = (n // 2) * n + n // 2
    Hm = np.zeros((2, 3 * N))
    Hm[0, N + c0] = 1.0
    Hm[1, 2 * N + c0] = 1.0
    return QS, G, Hm


def local_a_block(cfg, w: np.ndarray, n: int = 16):
    """Returns (A_blk [49, 49], S_c [2, 2]).  A_blk is the 7x7-block restriction of
    I - Q_S G^T H^T S_c H G Q_S around the observed coarse point, block index
    (dk + 3) * 7 + (dj + 3) for coarse offsets dj (x) and dk (y) in [-3, 3]."""
    QS, G, Hm = coarse_operator_matrices(cfg, w, n)
    K = Hm @ G @ QS                              # 2 x N
    Mc = K @ K.T
    Sc = inverse_via_cholesky(Mc + cfg.obs_sigma ** 2 * np.eye(2))
    B = K.T @ Sc @ K
    ctr = n // 2
    idx = [(ctr + dk) * n + (ctr + dj) for dk in range(-BLOCK_R, BLOCK_R + 1)
           for dj in range(-BLOCK_R, BLOCK_R + 1)]
    A = np.eye(BLOCK_N) - B[np.ix_(idx, idx)]
    return A, Sc


def sym_sqrt(A: np.ndarray) -> np.ndarray:
    """Symmetric square root V diag(sqrt(max(lambda, 0))) V^T."""
    lam, V = np.linalg.eigh(0.5 * (A + A.T))
    return (V * np.sqrt(np.maximum(lam, 0.0))) @ V.T


def apply_local_blocks(r: np.ndarray, Ahalf: np.ndarray, cells: np.ndarray, c: int) -> np.ndarray:
    """r' = r + sum_o (A^{1/2} - I) r restricted to the 7x7 block around the coarse point
    (floor(j_o/c), floor(k_o/c)) of each observation; every block reads the unmodified r."""
    nry, nrx = r.shape
    out = r.copy()
    D = Ahalf - np.eye(BLOCK_N)
    for j, k in cells:
        a, b = int(j) // c, int(k) // c
        iy = [(b + dk) % nry for dk in range(-BLOCK_R, BLOCK_R + 1)]
        ix = [(a + dj) % nrx for dj in range(-BLOCK_R, BLOCK_R + 1)]
        blk = r[np.ix_(iy, ix)].reshape(-1)
        out[np.ix_(iy, ix)] += (D @ blk).reshape(7, 7)
    return out


# --------------------------------------------------------------------------------------
# Stages 3-5
# --------------------------------------------------------------------------------------

def perpendicular(xi: np.ndarray, nut: np.ndarray):
    """nu = sqrt(nu~.nu~ / (nu~.nu~ - a nu~.xi)) (nu~ - a xi), a = nu~.xi / xi.xi
    (eq. nuPerpendicular).  Returns (nu, (xi.xi, nu~.nu~, nu~.xi))."""
    xx = float(np.dot(xi.ravel(), xi.ravel()))
    nn = float(np.dot(nut.ravel(), nut.ravel()))
    nx_ = float(np.dot(nut.ravel(), xi.ravel()))
    a = nx_ / xx
    scale = math.sqrt(nn / (nn - a * nx_))
    return scale * (nut - a * xi), (xx, nn, nx_)


def beta_and_cstar(c: np.ndarray, zeta: np.ndarray):
    """cbar = mean c;  beta = min_i ((cbar - c_i)/zeta_i + 1);  c*_i = max(0, cbar - c_i -
    (beta - 1) zeta_i)  (eq. betaTwoStage, eq. cistarTwoStage)."""
    cbar = float(np.mean(c))
    beta = float(np.min((cbar - c) / zeta + 1.0))
    cstar = np.maximum(0.0, cbar - c - (beta - 1.0) * zeta)
    return cbar, beta, cstar


# --------------------------------------------------------------------------------------
# Whole analysis
# --------------------------------------------------------------------------------------

class AnalysisConstants:
    """Everything the analysis precomputes once per configuration."""

    def __init__(self, cfg):
        self.w = me.model_error_stencil(cfg)
        self.S = s_matrix(cfg, self.w)
        A, Sc = local_a_block(cfg, self.w)
        self.A = A
        self.Sc = Sc
        self.Ahalf = sym_sqrt(A)


def analysis(ens_f: np.ndarray, cells: np.ndarray, y: np.ndarray, cfg, analysis_index: int,
             consts: AnalysisConstants | None = None, particles=None,
             full_innovation: bool = False, one_stage: bool = False):
    """Two-stage IEWPF analysis of a forecast ensemble [Ne, 3, ny, nx] (float64 result).

    `particles` optionally restricts stage 6 (the state update) to a subset of particle
    indices; stages 1-5 always use the whole ensemble (stage 4 couples all particles).
    `full_innovation` replaces the paper's independent 2x2 blocks of S by the inverse of the
    full H Q H^T + R over all observations (s_full) in the pull and in c_i; stage 6 keeps
    the paper's local blocks.  Returns (ens_out, info) where ens_out holds only the updated
    particles in `particles` order.

    `one_stage` runs the original one-stage IEWPF instead (Appendix A, eq.
    iewpfUpdateAgain): no nu term (beta = 0), target weight w_target = max_i c_i (eq.
    iewpf_targetWeight), c*_i = w_target - c_i (eq. iewpfCStar), alpha_i by the Lambert W
    limit of eq. numericalEqForAlpha; info["cbar"] then holds w_target."""
    if consts is None:
        consts = AnalysisConstants(cfg)
    ne = ens_f.shape[0]
    n_r = cfg.nrx * cfg.nry
    n_psi = 3 * cfg.nx * cfg.ny
    S = consts.S

    # Stage 1 + part of 2: innovations and c_i
    d_all = np.stack([ob.innovations(ens_f[i], cells, y, cfg.H) for i in range(ne)])
    if full_innovation and len(cells):
        Sf = s_full(cfg, consts.w, cells)
        sd_all = (d_all.reshape(ne, -1) @ Sf.T).reshape(d_all.shape)
    else:
        sd_all = d_all @ S.T                                # S d_o per observation
    c = np.einsum("iok,iok->i", d_all, sd_all)

    # Stage 3
    xis, nus, dots = [], [], []
    for i in range(ne):
        xi = philox.normals(n_r, cfg.seed, analysis_index, philox.TAG_XI, cfg.ensemble_id, i)
        nut = philox.normals(n_r, cfg.seed, analysis_index, philox.TAG_NU, cfg.ensemble_id, i)
        xi = xi.reshape(cfg.nry, cfg.nrx)
        nut = nut.reshape(cfg.nry, cfg.nrx)
        nu, d3 = perpendicular(xi, nut)
        xis.append(xi)
        nus.append(nu)
        dots.append(d3)
    dots = np.asarray(dots)
    gamma = dots[:, 0] * n_psi / n_r
    zeta = dots[:, 1] * n_psi / n_r

    # Stage 4-5
    if one_stage:
        cbar = float(np.max(c)) if ne else 0.0       # w_target
        beta = 0.0
        cstar = np.maximum(0.0, cbar - c)
    else:
        cbar, beta, cstar = beta_and_cstar(c, zeta)
        if not beta > 0.0:
            raise ValueError(f"beta = {beta} <= 0: the ensemble violates N_psi >> N_y")
    alpha = np.array([iewpf_alpha(gamma[i], cstar[i], n_psi) for i in range(ne)])

    # Stage 6
    if particles is None:
        particles = list(range(ne))
    out = []
    for i in particles:
        psi = np.asarray(ens_f[i], dtype=np.float64).copy()
        for o in range(len(cells)):
            psi += pull_one(sd_all[i, o, 0], sd_all[i, o, 1], int(cells[o, 0]), int(cells[o, 1]),
                            cfg, consts.w)
        r = math.sqrt(beta) * nus[i] + math.sqrt(alpha[i]) * xis[i]
        r2 = apply_local_blocks(r, consts.Ahalf, cells, cfg.c_omega)
        psi += me.apply_qhalf(r2, consts.w, cfg)
        out.append(psi)
    info = dict(c=c, gamma=gamma, zeta=zeta, dots=dots, cbar=cbar, beta=beta, cstar=cstar,
                alpha=alpha, d=d_all, sd=sd_all)
    return np.stack(out) if out else np.zeros((0,) + ens_f.shape[1:]), info


def realized_weight(alpha, gamma, zeta, beta, c, n_psi):
    """-2 log w_i realised by the update: (alpha-1) gamma + (beta-1) zeta - N log alpha + c_i
    (large-N form of eq. unfinishedImplicitEquationTwoStage with nu perpendicular to xi)."""
    return (alpha - 1.0) * gamma + (beta - 1.0) * zeta - n_psi * np.log(alpha) + c
