"""Bulk thermodynamics of the Shan-Chen fluid (oracle side).

TEST INFRASTRUCTURE ONLY. Follows Sec. "Bulk Physics" and Sec. "Interface Physics":

* bulk pressure P_b(n) = n c_s^2 + (G c_s^2 e_2 / 2) psi(n)^2;
* critical coupling G_c where dP_b/dn = d^2P_b/dn^2 = 0, reduced temperature
  Delta T = G / G_c - 1 (Laplace-law paragraph of the sigma_1 tuning section);
* liquid/gas coexistence from eq. (SCMaxwell): p0 = P_b(n_g) = P_b(n_l) and
  int_{n_g}^{n_l} dn psi'/psi^(eps+1) (p0 - P_b) = 0, with eps from eq. (eps_moments);
* spinodal densities where dP_b/dn = 0.

Plain numerics (scipy quadrature and bracketing root finders) in FP64.
"""
from __future__ import annotations

import math

from scipy import integrate, optimize

CS2 = 1.0 / 3.0


def psi_funcs(kind: int, eps: float = 0.0):
    """(psi, dpsi/dn) for kind 0 = exp(-1/n), 1 = (n/(eps+n))^(1/eps), 2 = 1 - exp(-n)."""
    if kind == 0:
        return (lambda n: math.exp(-1.0 / n)), (lambda n: math.exp(-1.0 / n) / (n * n))
    if kind == 1:
        ps = lambda n: (n / (eps + n)) ** (1.0 / eps)
        return ps, (lambda n: ps(n) / (n * (eps + n)))
    return (lambda n: 1.0 - math.exp(-n)), (lambda n: math.exp(-n))


def bulk_pressure(n, G, kind=0, eps=0.0, e2=1.0):
    ps, _ = psi_funcs(kind, eps)
    return n * CS2 + 0.5 * G * CS2 * e2 * ps(n) ** 2


def critical(kind=0, eps=0.0, e2=1.0):
    """(n_c, G_c): psi psi' is maximal at n_c and G_c = -1 / (e2 psi psi'(n_c))."""
    ps, dps = psi_funcs(kind, eps)
    res = optimize.minimize_scalar(lambda n: -ps(n) * dps(n), bounds=(1e-3, 50.0), method="bounded",
                                   options={"xatol": 1e-13})
    nc = res.x
    return nc, -1.0 / (e2 * ps(nc) * dps(nc))


def spinodal(G, kind=0, eps=0.0, e2=1.0):
    """Densities bounding the mechanically unstable region (dP_b/dn < 0)."""
    ps, dps = psi_funcs(kind, eps)
    nc, Gc = critical(kind, eps, e2)
    slope = lambda n: 1.0 + G * e2 * ps(n) * dps(n)
    if G >= Gc:
        raise ValueError("G is not below the critical coupling")
    lo = optimize.brentq(slope, 1e-3, nc, xtol=1e-15)
    hi = optimize.brentq(slope, nc, 100.0, xtol=1e-15)
    return lo, hi


def coexistence(G, kind=0, eps=None, e2=1.0, e4=None):
    """(n_g, n_l, p0) from the equal-area rule of eq. (SCMaxwell).

    ``eps`` (the measure exponent) defaults to eq. (eps_moments) evaluated at ``e4``; for
    kind 1 the pseudopotential parameter is the same eps (thermodynamic consistency).
    """
    if eps is None:
        eps = 0.0 if e4 is None else (6 * e4 - 2 * e2) / (6 * e4 + e2)
    ps, dps = psi_funcs(kind, eps)
    P = lambda n: bulk_pressure(n, G, kind, eps, e2)
    lo, hi = spinodal(G, kind, eps, e2)
    Pmax, Pmin = P(lo), P(hi)   # local max on the gas side, local min on the liquid side
    measure = lambda n: dps(n) / ps(n) ** (eps + 1.0)

    def branches(p0):
        ng = optimize.brentq(lambda n: P(n) - p0, 1e-6, lo, xtol=1e-15)
        nl = optimize.brentq(lambda n: P(n) - p0, hi, 200.0, xtol=1e-15)
        return ng, nl

    def area(p0):
        ng, nl = branches(p0)
        val, _ = integrate.quad(lambda n: measure(n) * (p0 - P(n)), ng, nl, epsabs=1e-15, epsrel=1e-13,
                                limit=200)
        return val

    a = max(Pmin, 1e-12) + 1e-12 * abs(Pmax)
    b = Pmax - 1e-12 * abs(Pmax)
    p0 = optimize.brentq(area, a, b, xtol=1e-15, rtol=1e-15)
    ng, nl = branches(p0)
    return ng, nl, p0


def G_for_reduced_temperature(dT, kind=0, eps=0.0, e2=1.0):
    """G such that Delta T = G / G_c - 1."""
    return (1.0 + dT) * critical(kind, eps, e2)[1]
