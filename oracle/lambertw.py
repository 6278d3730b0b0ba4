"""Principal-branch Lambert W for the IEWPF alpha equation (float64).

Paper: Appendix A, eq. iewpfAlphaSol -- alpha_i = -(N/gamma_i) W_0(z_i) with
z_i = -(gamma_i/N) exp(-gamma_i/N) exp(-c*_i/N), only the principal branch (alpha < 1)
accepted.  N = N_psi (the appendix's N_x is read as N_psi).

Writing x = gamma/N and y = -W_0(z) in (0, 1], the definition W e^W = z is equivalent to
    y - ln y = x - ln x + c*/N,                                         (*)
and alpha = y / x.  Near the branch point z = -1/e (x close to 1, c* small, the usual
regime since gamma ~ N +- sqrt(2N)) z itself is poorly conditioned in float64, so W_0 is
evaluated from (*) with y = 1 - delta:  -delta - ln(1 - delta) = rho,
rho = (x - 1 - ln x) + c*/N >= 0, solved by Newton from the right (the left side is convex
and increasing in delta on [0, 1), so the iteration decreases monotonically to the root).
"""
from __future__ import annotations

import math


def _x_minus_1_minus_log_x(eps: float) -> float:
    """(x - 1) - ln x for x = 1 + eps, without cancellation for small eps."""
    if abs(eps) < 1e-2:
        s = 0.0
        term = eps * eps
        for k in range(2, 24):
            s += term / k if k % 2 == 0 else -term / k
            term *= eps
        return s
    return eps - math.log1p(eps)


def w0_branch_form(x: float, cn: float) -> float:
    """W_0(-x exp(-x - cn)) for x > 0, cn >= 0 (argument in [-1/e, 0))."""
    rho = _x_minus_1_minus_log_x(x - 1.0) + cn
    if rho <= 0.0:
        return -1.0
    if rho < 0.5:
        # y = 1 - delta close to 1: solve -delta - ln(1 - delta) = rho by Newton from the
        # right, starting at sqrt(2 rho) >= delta (the left side is >= delta^2/2)
        d = math.sqrt(2.0 * rho)
        for _ in range(100):
            step = (-d - math.log1p(-d) - rho) * (1.0 - d) / d
            if step <= 0.0:
                break
            d -= step
            if step <= 1e-17 * d:
                break
        return -(1.0 - d)
    # y far from 1: solve y - ln y = 1 + rho by Newton from the left, starting at
    # exp(-(1 + rho)) <= y (y = exp(y - R) > exp(-R)); h(y) = y - ln y - R is convex and
    # decreasing on (0, 1), so the iterates increase monotonically to the root
    big_r = 1.0 + rho
    y = math.exp(-big_r)
    for _ in range(200):
        step = (y - math.log(y) - big_r) / (1.0 / y - 1.0)
        if step <= 0.0:
            break
        y += step
        if step <= 1e-17 * y:
            break
    return -y


def lambert_w0(z: float) -> float:
    """W_0(z) for real z >= -1/e, by Halley iteration on w e^w = z (used to cross-check the
    branch form away from the branch point)."""
    if z == 0.0:
        return 0.0
    if z < -1.0 / math.e:
        raise ValueError("z below the branch point")
    if z < -0.3:
        p = math.sqrt(max(0.0, 2.0 * (math.e * z + 1.0)))
        w = -1.0 + p - p * p / 3.0 + 11.0 / 72.0 * p ** 3
    elif z < 3.0:
        w = math.log1p(z)
    else:
        lz = math.log(z)
        w = lz - math.log(lz)
    for _ in range(100):
        ew = math.exp(w)
        fw = w * ew - z
        denom = ew * (w + 1.0) - (w + 2.0) * fw / (2.0 * w + 2.0) if w != -1.0 else 0.0
        if denom == 0.0:
            break
        dw = fw / denom
        w -= dw
        if abs(dw) <= 1e-16 * (1.0 + abs(w)):
            break
    return w


def iewpf_alpha(gamma: float, cstar: float, n_psi: float) -> float:
    """alpha = -(N/gamma) W_0(-(gamma/N) e^{-gamma/N} e^{-c*/N}) (eq. iewpfAlphaSol).

    With c* = 0 and gamma <= N the principal branch returns exactly alpha = 1."""
    x = gamma / n_psi
    cn = max(cstar, 0.0) / n_psi
    if cn == 0.0 and x <= 1.0:
        return 1.0
    w = w0_branch_form(x, cn)
    return -w / x


def iewpf_alpha_incomplete_gamma(gamma: float, cstar: float, n: float) -> float:
    """alpha from the exact equation of the one-stage scheme (eq. numericalEqForAlpha):
        P(N/2, alpha gamma/2) = exp(-c*/2) P(N/2, gamma/2),
    P the regularised lower incomplete gamma function, solved for alpha < 1 by Newton in
    u = ln alpha on F(u) = ln P(s, x e^u) - ln P(s, x) + c*/2 (s = N/2, x = gamma/2).
    F is increasing in u with F(0) = c*/2 >= 0, so the root is at u <= 0.  Feasible while
    ln P(s, x) stays representable, i.e. for small N (for large N the Lambert W limit
    iewpf_alpha applies, which this converges to as N grows)."""
    from scipy.special import gammainc, gammaln
    s, x = 0.5 * n, 0.5 * gamma
    cs = max(cstar, 0.0)
    if cs == 0.0:
        return 1.0
    lp_x = math.log(gammainc(s, x))

    def F(u):  # -inf where P underflows (far left of the root)
        p = gammainc(s, x * math.exp(u))
        return math.log(p) - lp_x + 0.5 * cs if p > 0.0 else -math.inf

    def dF(u):  # d/du ln P(s, x e^u) = (x e^u)^s e^{-x e^u} / (Gamma(s) P(s, x e^u))
        xu = x * math.exp(u)
        return math.exp(s * math.log(xu) - xu - gammaln(s) - math.log(gammainc(s, xu)))

    # bracket F(lo) <= 0 <= F(0), starting from twice the large-N (Lambert W) estimate
    lo = 2.0 * math.log(iewpf_alpha(gamma, cs, n)) - 1e-3
    while F(lo) > 0.0:
        lo *= 2.0
    hi, u = 0.0, 0.5 * lo
    for _ in range(200):
        f = F(u)
        if f > 0.0:
            hi = u
        else:
            lo = u
        un = u - f / dF(u) if math.isfinite(f) else 0.5 * (lo + hi)
        if not (lo < un < hi):  # keep Newton inside the bracket, else bisect
            un = 0.5 * (lo + hi)
        if abs(un - u) <= 1e-15 * max(1.0, abs(u)):
            u = un
            break
        u = un
    return math.exp(u)
