"""Forcing-stencil weight design (Sec. "Computing the Weights").

The weights W(|e|^2) are the method's tunable degrees of freedom. Fixing the second moment
e_2 = 1 and the isotropy conditions leaves free moments; the closed forms below give the
weights of the nearest shells as functions of those moments:

* 2D, shells {1,2,4,5,8}: e_2 = 1, I_4,0 = I_6,0 = 0, free (e_4, e_8). The sixth moment is
  then fixed, e_6 = e_4 - 4/15.
* 3D, shells {1,2,3,4,5,6,8}: e_2 = 1, I_4,0 = I_6,0 = I_6,1 = 0, free (e_4, e_8) and W(6).

At e_4 = 4/7, e_8 = 16/105 (and W(6) = 1/630 in 3D) they reduce to the maximally isotropic
E(8) stencils. Knobs of the paper: sigma_0 = -e_4/2 (eq. hatsigma01eI) and the flat-profile
exponent eps(e_4) = (6 e_4 - 2)/(6 e_4 + 1) (eq. eps_moments).
"""
from __future__ import annotations

import numpy as np

SHELLS_2D = (1, 2, 4, 5, 8)
SHELLS_3D = (1, 2, 3, 4, 5, 6, 8)
E4_2D = ((1, 2), (1 / 3, 1 / 12))
E4_3D = ((1, 2), (1 / 6, 1 / 12))


def family2d(e4: float, e8: float) -> np.ndarray:
    """W(1), W(2), W(4), W(5), W(8) of the 2D family."""
    return np.array([(44 - 25 * e4 - 45 * e8) / 120,
                     (32 - 40 * e4 + 45 * e8) / 180,
                     (4 - 5 * e4 + 45 * e8) / 480,
                     (11 * e4 - 9 * e8 - 4) / 144,
                     (8 - 25 * e4 + 45 * e8) / 2880])


def family3d(e4: float, e8: float, w6: float) -> np.ndarray:
    """W(1), W(2), W(3), W(4), W(5), W(6), W(8) of the 3D family."""
    t = w6
    return np.array([(35 * e4 - 45 * e8 - 2400 * t - 4) / 60,
                     (-85 * e4 + 45 * e8 + 3960 * t + 44) / 180,
                     (15 * e4 - 1440 * t - 4) / 120,
                     (-35 * e4 + 45 * e8 + 960 * t + 14) / 240,
                     (11 * e4 - 9 * e8 - 288 * t - 4) / 144,
                     t,
                     (8 - 25 * e4 + 45 * e8) / 2880])


def epsilon(e4: float, e2: float = 1.0) -> float:
    return (6 * e4 - 2 * e2) / (6 * e4 + e2)


def seeded_family2d(u_e4: float, u_e8: float):
    """Weights from two uniform draws: e4 = 0.45 + 0.25 u, e8 = e4^2 (16/105)/(4/7)^2 (0.8 + 0.4 u')
    (the E(8) ratio e8/e4^2, perturbed by +-20%)."""
    e4 = 0.45 + 0.25 * u_e4
    e8 = e4 ** 2 * (16 / 105) / (4 / 7) ** 2 * (0.8 + 0.4 * u_e8)
    return e4, e8, family2d(e4, e8)


def seeded_family3d(u_e4: float, u_e8: float, u_w6: float):
    """3D weights near E(8): e4 = 4/7 (1 + 0.1 (2u - 1)), e8 scaled likewise, W(6) = 1/630 (0.8 + 0.4 u'')."""
    e4 = 4 / 7 * (1 + 0.1 * (2 * u_e4 - 1))
    e8 = 16 / 105 * (1 + 0.1 * (2 * u_e8 - 1))
    w6 = 1 / 630 * (0.8 + 0.4 * u_w6)
    return e4, e8, w6, family3d(e4, e8, w6)


# ---------------------------------------------------------------------- knob -> weight solver
# The moments of a weighted stencil are linear in the weights, so fixing as many of them as
# there are shells gives the weights by one linear solve (Sec. "Computing the Weights"). The
# 2D moment names follow the definitions of the isotropy and anisotropy coefficients:
#   e2 = <x^2>, e4 = <x^2 y^2>, e6 = <x^4 y^2>/3, e8 = <x^4 y^4>/9,
#   I40 = <x^4> - 3 <x^2 y^2>, I60 = <x^6> - 15 e6, I80 = <x^6 y^2> - 15 e8,
#   I81 = <x^8> - 7 <x^6 y^2>,
# where <x^a y^b> = sum over stencil vectors of W(|e|^2) e_x^a e_y^b.

TOLMAN_SHELLS_2D = (1, 2, 4, 5, 8, 9, 18)


def shell_vectors_2d(code: int):
    """All integer (x, y) with x^2 + y^2 = code."""
    r = int(np.ceil(np.sqrt(code)))
    return [(x, y) for x in range(-r, r + 1) for y in range(-r, r + 1) if x * x + y * y == code]


def _moment_rows_2d(codes):
    def m(a, b):
        return np.array([sum(float(x) ** a * float(y) ** b for x, y in shell_vectors_2d(c)) for c in codes])

    e6 = m(4, 2) / 3
    e8 = m(4, 4) / 9
    return {"e2": m(2, 0), "e4": m(2, 2), "e6": e6, "e8": e8,
            "I40": m(4, 0) - 3 * m(2, 2), "I60": m(6, 0) - 15 * e6,
            "I80": m(6, 2) - 15 * e8, "I81": m(8, 0) - 7 * m(6, 2)}


def moments2d(codes, W):
    """Named moments of a 2D stencil with weights W (one per shell code)."""
    rows = _moment_rows_2d(codes)
    return {k: float(v @ np.asarray(W, dtype=np.float64)) for k, v in rows.items()}


def solve_weights_2d(codes, targets: dict) -> np.ndarray:
    """Weights of the shells ``codes`` whose named moments take the values ``targets``
    (exactly as many targets as shells)."""
    if len(targets) != len(codes):
        raise ValueError("need one target per shell")
    rows = _moment_rows_2d(codes)
    A = np.array([rows[k] for k in targets])
    b = np.array([float(v) for v in targets.values()])
    return np.linalg.solve(A, b)


def moments_for_knobs(sigma0: float, sigma1: float, delta0: float):
    """(e4, e6, e8) from the interface knobs: sigma_0 = -e4/2, sigma_1 = e6/4
    (eq. hatsigma01eI) and delta_0 = 1/12 + 95 e4/432 + 7 e6/72 - 5 e8/144 (eq. hatdelta0eI)."""
    e4 = -2.0 * sigma0
    e6 = 4.0 * sigma1
    e8 = (1.0 / 12 + 95.0 * e4 / 432 + 7.0 * e6 / 72 - delta0) * 144.0 / 5.0
    return e4, e6, e8


def tolman_stencil_2d(sigma0: float, sigma1: float, delta0: float) -> np.ndarray:
    """Weights on the shells {1,2,4,5,8,9,18} with e2 = 1, sixth-order isotropy (I40 = I60 = 0),
    I80 = 0 and the three knobs (sigma_0, sigma_1, delta_0): the stencil of the paper's
    Tolman-length tuning (Sec. "Higher-order Tolman length tuning")."""
    e4, e6, e8 = moments_for_knobs(sigma0, sigma1, delta0)
    return solve_weights_2d(TOLMAN_SHELLS_2D, {"e2": 1.0, "e4": e4, "e6": e6, "e8": e8,
                                               "I40": 0.0, "I60": 0.0, "I80": 0.0})


def surface_tension_stencil_2d(sigma0: float, sigma1: float) -> np.ndarray:
    """Weights on the shells {1,2,4,5,8,9,18} with e2 = 1, e4 = -2 sigma_0, e6 = 4 sigma_1 and
    eighth-order isotropy (I40 = I60 = I80 = I81 = 0): the stencil of the paper's higher-order
    surface-tension tuning (Sec. "Higher-order surface tension tuning")."""
    return solve_weights_2d(TOLMAN_SHELLS_2D, {"e2": 1.0, "e4": -2.0 * sigma0, "e6": 4.0 * sigma1,
                                               "I40": 0.0, "I60": 0.0, "I80": 0.0, "I81": 0.0})


# ---------------------------------------------------------------------- 3D tuning stencil
# In 3D the squared length 9 holds two symmetry groups; the shell code 9 names the (2,2,1)
# group and 1009 the (3,0,0) group, 18 is the (3,3,0) group. Moments <x^a y^b z^c> of the
# isotropic tensors give e_2 = <x^2>, e_4 = <x^2 y^2>, e_6 = <x^2 y^2 z^2>, e_8 = <x^4 y^2 z^2>/3
# and the isotropy conditions (each zero on an isotropic stencil)
#   order 4:  <x^4> - 3 e_4
#   order 6:  <x^6> - 15 e_6,  <x^4 y^2> - 3 e_6
#   order 8:  <x^8> - 105 e_8, <x^6 y^2> - 15 e_8, <x^4 y^4> - 9 e_8
#   order 10 (one of them): 9 <x^6 y^2 z^2> - 15 <x^4 y^4 z^2>.
# With all conditions of orders 4 to 8 zero they span the same space as the paper's I_4,0 ...
# I_8,2 (Appendix "Defining the stencil"). The 3D table of the Tolman-length tuning
# (tab. e4e6e8_tuning_6_3d, 11 shells) satisfies the conditions of orders 4 to 8 and, as one
# more equation fixing its last degree of freedom, the order-10 condition above.

TOLMAN_SHELLS_3D = (1, 2, 3, 4, 5, 6, 8, 9, 1009, 16, 18)
_GEN3 = {1: (0, 0, 1), 2: (0, 1, 1), 3: (1, 1, 1), 4: (0, 0, 2), 5: (0, 1, 2), 6: (1, 1, 2), 8: (0, 2, 2),
         9: (1, 2, 2), 1009: (0, 0, 3), 16: (0, 0, 4), 18: (0, 3, 3)}


def shell_vectors_3d(code: int):
    """All integer (x, y, z) of the 3D symmetry group named by ``code``."""
    g = _GEN3[code]
    r = g[2]
    return [(x, y, z) for x in range(-r, r + 1) for y in range(-r, r + 1) for z in range(-r, r + 1)
            if sorted((abs(x), abs(y), abs(z))) == list(g)]


def _moment_rows_3d(codes):
    def m(a, b, c):
        return np.array([sum(float(x) ** a * float(y) ** b * float(z) ** c for x, y, z in shell_vectors_3d(k))
                         for k in codes])

    e6 = m(2, 2, 2)
    e8 = m(4, 2, 2) / 3
    return {"e2": m(2, 0, 0), "e4": m(2, 2, 0), "e6": e6, "e8": e8,
            "C40": m(4, 0, 0) - 3 * m(2, 2, 0),
            "C60": m(6, 0, 0) - 15 * e6, "C61": m(4, 2, 0) - 3 * e6,
            "C80": m(8, 0, 0) - 105 * e8, "C81": m(6, 2, 0) - 15 * e8, "C82": m(4, 4, 0) - 9 * e8,
            "C10": 9 * m(6, 2, 2) - 15 * m(4, 4, 2)}


def moments3d(codes, W):
    """Named moments and isotropy conditions of a 3D stencil with weights W (one per shell)."""
    rows = _moment_rows_3d(codes)
    return {k: float(v @ np.asarray(W, dtype=np.float64)) for k, v in rows.items()}


def solve_weights_3d(codes, targets: dict) -> np.ndarray:
    """Weights of the 3D shells ``codes`` whose named moments take the values ``targets``
    (exactly as many targets as shells)."""
    if len(targets) != len(codes):
        raise ValueError("need one target per shell")
    rows = _moment_rows_3d(codes)
    A = np.array([rows[k] for k in targets])
    b = np.array([float(v) for v in targets.values()])
    return np.linalg.solve(A, b)


def tolman_stencil_3d(sigma0: float, sigma1: float, delta0: float) -> np.ndarray:
    """Weights on the 3D shells of TOLMAN_SHELLS_3D with e_2 = 1, the three knobs through
    (e_4, e_6, e_8) as in 2D (eqs. hatsigma01eI, hatdelta0eI) and the isotropy conditions of
    orders 4, 6, 8 and the one of order 10 listed above: the 3D stencil of the paper's
    Tolman-length tuning."""
    e4, e6, e8 = moments_for_knobs(sigma0, sigma1, delta0)
    return solve_weights_3d(TOLMAN_SHELLS_3D, {"e2": 1.0, "e4": e4, "e6": e6, "e8": e8, "C40": 0.0,
                                               "C60": 0.0, "C61": 0.0, "C80": 0.0, "C81": 0.0, "C82": 0.0,
                                               "C10": 0.0})
