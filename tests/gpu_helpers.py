"""Shared helpers of the GPU tests: oracle runs and comparisons in matching layouts."""
from __future__ import annotations

import sys
from fractions import Fraction as Fr

import numpy as np

import oracle
from oracle import stencil_algebra as sa
from oracle import thermo

E4_2D = ([1, 2], [1 / 3, 1 / 12])
E8_2D = ([1, 2, 4, 5, 8], [4 / 21, 4 / 45, 1 / 60, 2 / 315, 1 / 5040])


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def family2d_weights(e4, e8):
    return [float(v) for v in sa.family2d(Fr(e4).limit_denominator(10 ** 12), Fr(e8).limit_denominator(10 ** 12)).values()]


def family3d_weights(e4, e8, w6):
    W = sa.family3d(Fr(e4).limit_denominator(10 ** 12), Fr(e8).limit_denominator(10 ** 12),
                    Fr(w6).limit_denominator(10 ** 12))
    return [float(W[c]) for c in (1, 2, 3, 4, 5, 6, 8)]


def coupling(dT=0.2):
    return thermo.G_for_reduced_temperature(dT)


def perm_to_oracle(lat_xi, d):
    """Index map: oracle population k  <-  library population perm[k]."""
    oxi, _ = oracle.velset(d)
    perm = []
    for v in oxi:
        hits = [i for i, u in enumerate(lat_xi) if tuple(u) == tuple(v)]
        assert len(hits) == 1
        perm.append(hits[0])
    return np.array(perm)


def rel_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def oracle_run(dims, tau, G, codes, W, n0, steps, psi_kind=0, psi_param=0.0):
    s = oracle.Sim(dims, tau, G, codes, W, psi_kind, psi_param).init_density(n0)
    rc = s.run(steps)
    return s, rc


def patch_oracle(n0_full, dims, center, half, tau, G, codes, W, steps, psi_kind=0, psi_param=0.0):
    """Oracle value of the populations at one site after ``steps`` steps, computed on a
    periodic patch of half-width ``half`` around it. Exact when half >= steps * (reach + 1):
    information travels at most reach + 1 sites per step (pull of the neighbours' psi at
    distance reach, one more site for the streaming)."""
    d = len(dims)
    n0 = n0_full.reshape(tuple(reversed(dims)))
    idx = [np.arange(c - half, c + half + 1) % L for c, L in zip(center, dims)]
    if d == 2:
        patch = n0[np.ix_(idx[1], idx[0])]
    else:
        patch = n0[np.ix_(idx[2], idx[1], idx[0])]
    P = 2 * half + 1
    s = oracle.Sim((P,) * d, tau, G, codes, W, psi_kind, psi_param).init_density(patch.reshape(-1))
    s.run(steps)
    cidx = half + P * half + (P * P * half if d == 3 else 0)
    return s.f[:, cidx].copy()
