"""Pins of the one-stage IEWPF (Appendix A: eq. iewpfUpdateAgain, iewpf_targetWeight,
iewpfCStar) and of the exact alpha equation with incomplete gamma functions (eq.
numericalEqForAlpha) against high-precision arithmetic and its Lambert W limit (eq.
iewpfAlphaSol)."""
import math

import mpmath
import numpy as np
import pytest

import workloads as W
from oracle import ensemble as oens
from oracle import iewpf
from oracle.lambertw import iewpf_alpha, iewpf_alpha_incomplete_gamma


def _alpha_mp(gamma, cstar, n):
    """Root alpha in (0, 1] of P(n/2, alpha gamma/2) = exp(-c*/2) P(n/2, gamma/2) by
    bisection in 50-digit arithmetic."""
    mpmath.mp.dps = 50
    s, x = mpmath.mpf(n) / 2, mpmath.mpf(gamma) / 2
    rhs = mpmath.exp(-mpmath.mpf(cstar) / 2) * mpmath.gammainc(s, 0, x, regularized=True)
    lo, hi = mpmath.mpf(0), mpmath.mpf(1)
    for _ in range(200):
        mid = (lo + hi) / 2
        if mpmath.gammainc(s, 0, mid * x, regularized=True) < rhs:
            lo = mid
        else:
            hi = mid
    return float((lo + hi) / 2)


@pytest.mark.parametrize("n,gamma,cstar", [(10, 9.0, 1.5), (10, 14.0, 0.2), (40, 35.0, 4.0),
                                           (40, 52.0, 0.01), (400, 420.0, 30.0)])
def test_incomplete_gamma_alpha_matches_high_precision(n, gamma, cstar):
    a = iewpf_alpha_incomplete_gamma(gamma, cstar, n)
    ref = _alpha_mp(gamma, cstar, n)
    assert 0.0 < a < 1.0
    assert abs(a - ref) < 1e-11 * ref


def test_incomplete_gamma_alpha_converges_to_lambert_w():
    # gamma and c* at the same number of standard deviations as N grows: the exact root
    # approaches the large-N Lambert W solution (observed: the difference falls about 4x
    # per decade of N)
    diffs = []
    for n in (100, 1000, 10000, 100000, 1000000):
        gamma = n + 0.7 * math.sqrt(2.0 * n)
        cstar = 0.5 * math.sqrt(n)
        diffs.append(abs(iewpf_alpha_incomplete_gamma(gamma, cstar, n) - iewpf_alpha(gamma, cstar, n)))
    assert all(d2 < 0.4 * d1 for d1, d2 in zip(diffs, diffs[1:])), diffs
    assert diffs[-1] < 1e-3


def test_one_stage_analysis_reaches_the_target_weight():
    cfg = W.tiny().replace(n_particles=6)
    base = oens.init_member(cfg, None, 0, 999)
    small = cfg.replace(init_std=0.003)
    ens = np.stack([oens.init_member(small, base, 1, i) for i in range(6)])
    truth = oens.init_member(small.replace(ensemble_id=77), base, 1, 0)
    cells = np.array([[8, 8], [24, 8], [8, 24], [24, 24]], dtype=np.int32)
    from oracle import observe as ob
    y = ob.mooring_obs(truth, cells, cfg.H, cfg.obs_sigma, np.zeros((4, 2)))
    out, info = iewpf.analysis(ens, cells, y, cfg, 3, one_stage=True)
    c, g, a = info["c"], info["gamma"], info["alpha"]
    assert info["beta"] == 0.0 and info["cbar"] == c.max()
    assert np.all(info["cstar"] >= 0.0) and info["cstar"][np.argmax(c)] == 0.0
    w = (a - 1.0) * g - cfg.n_psi * np.log(a) + c      # -2 log w realised, no nu term
    assert np.abs(w - c.max()).max() < 1e-9 * cfg.n_psi
    # the two-stage target is the mean instead, and it moves particles less
    out2, info2 = iewpf.analysis(ens, cells, y, cfg, 3)
    assert info2["cbar"] < info["cbar"]
