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
