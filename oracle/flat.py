"""Flat-interface observables of the oracle (test infrastructure only).

A flat slab varies along x only; with periodic boundaries it has two interfaces, one in each
half of the domain. These routines take the oracle's density field and lattice pressure
tensor of such a slab and return, per interface:

* sigma_0, eq. (sigma0pnpt): the site sum of P_N - P_T over the half domain;
* z_s, eq. (ZSDef): the first moment of P_N - P_T over the same sites, divided by sigma_0;
* z_e: the position of a sharp step between the two bulk densities holding the same mass as
  the half domain (vanishing adsorbance, Sec. Tolman Length);
* delta = z_e - z_s, eq. (zemzs), and delta_ads = Gamma(z_s) / (n_l - n_g), eq. (deltaads);
* the analytic estimates eq. (SCTolmanFlat) for delta and eq. (HOSigmaInt) for sigma_0, with
  the profile derivatives of eqs. (PSIProfile) and (d2psi).

Discrete reading: site x stands for the unit cell [x - 1/2, x + 1/2), so a half domain of
sites lo .. hi-1 spans [lo - 1/2, hi - 1/2) and positions are site coordinates.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

CS2 = 1.0 / 3.0


def halves(nx: int):
    """Site ranges [lo, hi) of the two half domains of a slab centred at nx/2."""
    return [(0, nx // 2), (nx // 2, nx)]


def sigma0(PN, PT, lo, hi):
    """eq. (sigma0pnpt) on the sites lo .. hi-1."""
    return float(np.sum(PN[lo:hi] - PT[lo:hi]))


def z_s(PN, PT, lo, hi):
    """eq. (ZSDef): first moment of P_N - P_T over the sites lo .. hi-1."""
    x = np.arange(lo, hi, dtype=np.float64)
    d = PN[lo:hi] - PT[lo:hi]
    return float(np.sum(x * d) / np.sum(d))


def _sides(n, lo, hi, n_l, n_g):
    """(density on the low side, density on the high side) of the interface in [lo, hi)."""
    return (n_l, n_g) if n[lo] > n[hi - 1] else (n_g, n_l)


def adsorbance(n, lo, hi, n_l, n_g, z):
    """Gamma(z): mass of the half domain minus that of a sharp step at z between the bulks."""
    a, b = lo - 0.5, hi - 0.5
    n_lo, n_hi = _sides(n, lo, hi, n_l, n_g)
    return float(np.sum(n[lo:hi]) - (n_lo * (z - a) + n_hi * (b - z)))


def z_e(n, lo, hi, n_l, n_g):
    """Equimolar position: Gamma(z_e) = 0 (Gamma is linear in z)."""
    a, b = lo - 0.5, hi - 0.5
    n_lo, n_hi = _sides(n, lo, hi, n_l, n_g)
    return float((np.sum(n[lo:hi]) + n_lo * a - n_hi * b) / (n_lo - n_hi))


def orientation(n, lo, hi):
    """+1 if the liquid lies on the low-x side of the interface in [lo, hi) (x then runs from
    liquid to vapour, like the radius of a droplet), else -1."""
    return 1.0 if n[lo] > n[hi - 1] else -1.0


def delta_zemzs(n, PN, PT, lo, hi, n_l, n_g):
    """eq. (zemzs): delta = z_e - z_s along the liquid-to-vapour direction."""
    return orientation(n, lo, hi) * (z_e(n, lo, hi, n_l, n_g) - z_s(PN, PT, lo, hi))


def delta_ads(n, PN, PT, lo, hi, n_l, n_g):
    """eq. (deltaads): Gamma(z_s) / (n_l - n_g)."""
    return adsorbance(n, lo, hi, n_l, n_g, z_s(PN, PT, lo, hi)) / (n_l - n_g)


def delta_sc(G, sig0, dhat0, psi_l, psi_g):
    """eq. (SCTolmanFlat): -(G c_s^2 / (2 sigma_0)) dhat_0 [psi^2(n_l) - psi^2(n_g)]."""
    return -(G * CS2 / (2.0 * sig0)) * dhat0 * (psi_l ** 2 - psi_g ** 2)


def sigma0_estimate(G, shat0, shat1, n_g, n_l, p0, psi, dpsi, eps=0.0, e2=1.0):
    """eq. (HOSigmaInt): G c_s^2 (shat_0 Sigma_11 + shat_1 Sigma_22), with (dpsi/dx)^2 from
    eq. (PSIProfile) and d2psi/dx2 from eq. (d2psi), integrated over the density across the
    interface (dx = dpsi / |dpsi/dx|)."""
    pref = 8.0 * (1.0 - eps) / (G * CS2 * e2)

    def inner(nb):
        return dpsi(nb) / psi(nb) ** (eps + 1.0) * (p0 - nb * CS2 - 0.5 * G * CS2 * e2 * psi(nb) ** 2)

    def psix2(n):
        val, _ = integrate.quad(inner, n_g, n, epsabs=1e-14, epsrel=1e-12, limit=200)
        return max(pref * psi(n) ** eps * val, 0.0)

    def psixx(n, px2):
        return (eps * px2 + (pref * (p0 - n * CS2 - 0.5 * G * CS2 * e2 * psi(n) ** 2))) / (2.0 * psi(n))

    def s11(n):  # (psi_x)^2 dx = |psi_x| dpsi
        return math.sqrt(psix2(n)) * dpsi(n)

    def s22(n):  # (psi_xx)^2 dx = (psi_xx)^2 / |psi_x| dpsi
        px2 = psix2(n)
        if px2 <= 0.0:
            return 0.0
        return psixx(n, px2) ** 2 / math.sqrt(px2) * dpsi(n)

    S11, _ = integrate.quad(s11, n_g, n_l, epsabs=1e-13, epsrel=1e-10, limit=200)
    S22, _ = integrate.quad(s22, n_g, n_l, epsabs=1e-13, epsrel=1e-10, limit=200)
    return G * CS2 * (shat0 * S11 + shat1 * S22), S11, S22
