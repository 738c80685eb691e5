"""Bulk thermodynamics for setting up runs (coexisting densities, couplings).

For psi = exp(-1/n) the measure of the coexistence rule, eq. (SCMaxwell), is
dn psi'/psi = d(-1/n), so with s = 1/n and the bulk pressure
P(n) = n c^2 + (G c^2 e2 / 2) psi^2 = c^2 / s + (G c^2 e2 / 2) exp(-2 s) the equal-area
integral has the closed form
    int_{s_l}^{s_g} (p0 - P) ds = p0 (s_g - s_l) - c^2 [ln s - (G e2 / 4) exp(-2 s)]_{s_l}^{s_g} = 0,
and coexistence is the pair of outer roots of P(n) = p0 for which that integral vanishes
(bisection on p0 between the spinodal pressures). The critical point of psi = exp(-1/n) is
n_c = 1, G_c = -e^2 / e2.
"""
from __future__ import annotations

import math

import numpy as np

CS2 = 1.0 / 3.0


def critical_coupling_exp(e2: float = 1.0) -> float:
    return -math.e ** 2 / e2


def coupling_for_reduced_temperature(dT: float, e2: float = 1.0) -> float:
    """G with G / G_c - 1 = dT for psi = exp(-1/n)."""
    return (1.0 + dT) * critical_coupling_exp(e2)


def _pressure(n, G, e2):
    return n * CS2 + 0.5 * G * CS2 * e2 * np.exp(-2.0 / n)


def epsilon(e4: float, e2: float = 1.0) -> float:
    """eq. (eps_moments): eps = (6 e4 - 2 e2) / (6 e4 + e2)."""
    return (6.0 * e4 - 2.0 * e2) / (6.0 * e4 + e2)


def coexistence_exp(G: float, e2: float = 1.0, eps: float = 0.0):
    """(n_gas, n_liquid, p0) for psi = exp(-1/n) at coupling G < G_c.

    eps is the exponent of the measure psi' / psi^(1 + eps) of eq. (SCMaxwell) (eps(e4) of the
    stencil, eq. (eps_moments)); with s = 1/n it is exp(eps s) ds. For eps = 0 the equal-area
    integral has the closed form above; otherwise it is integrated numerically (composite
    Simpson rule on s, whose integrand is smooth between the two bulk roots).

    For a trial p0 between the spinodal pressures the two outer roots of P(n) = p0 are found by
    bisection on the monotone gas and liquid branches; the equal-area residual
    E(p0) = p0 (s_g - s_l) - c^2 [ln s - (a/2) exp(-2 s)]_{s_l}^{s_g}, a = G e2 / 2, s = 1/n,
    is then driven to zero by bisection on p0.
    """
    if not G < critical_coupling_exp(e2):
        raise ValueError("G must be below the critical coupling")
    a = 0.5 * G * e2

    def P(n):
        return CS2 * (n + a * math.exp(-2.0 / n))

    def slope(n):
        return 1.0 + a * 2.0 / (n * n) * math.exp(-2.0 / n)

    def bisect(f, lo, hi, it=200):
        flo = f(lo)
        for _ in range(it):
            mid = 0.5 * (lo + hi)
            fm = f(mid)
            if (fm > 0) == (flo > 0):
                lo, flo = mid, fm
            else:
                hi = mid
            if hi - lo <= 1e-16 * max(1.0, abs(hi)):
                break
        return 0.5 * (lo + hi)

    # spinodals (slope = 0) around the critical density n = 1
    n_lo = bisect(slope, 1e-3, 1.0)
    n_hi = bisect(slope, 1.0, 100.0)
    p_max, p_min = P(n_lo), P(n_hi)

    def branches(p0):
        ng = bisect(lambda n: P(n) - p0, 1e-6, n_lo)
        nl = bisect(lambda n: P(n) - p0, n_hi, 1e3)
        return ng, nl

    def F(s):
        return CS2 * (math.log(s) - 0.5 * a * math.exp(-2.0 * s))

    def area(p0):
        ng, nl = branches(p0)
        sg, sl = 1.0 / ng, 1.0 / nl
        if eps == 0.0:
            return p0 * (sg - sl) - (F(sg) - F(sl))
        s_ = np.linspace(sl, sg, 4001)
        f = (p0 - CS2 / s_ - CS2 * a * np.exp(-2.0 * s_)) * np.exp(eps * s_)
        h = (sg - sl) / 4000
        return h / 3.0 * (f[0] + f[-1] + 4.0 * f[1:-1:2].sum() + 2.0 * f[2:-1:2].sum())

    p0 = bisect(area, max(p_min, 1e-300) * (1 + 1e-12), p_max * (1 - 1e-12))
    ng, nl = branches(p0)
    return ng, nl, p0
