"""The product's weight design: closed-form families against the oracle's exact linear solve,
and the knob -> weight solver against the tuning tables printed in the paper."""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import stencil_algebra as sa
from paper_2505_23647_amd import stencil

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.mark.parametrize("e4,e8", [(Fr(4, 7), Fr(16, 105)), (Fr(1, 2), Fr(1, 10)), (Fr(3, 5), Fr(1, 7))])
def test_family2d_closed_form(e4, e8):
    ref = sa.family2d(e4, e8)
    got = stencil.family2d(float(e4), float(e8))
    assert np.allclose(got, [float(ref[c]) for c in stencil.SHELLS_2D], rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("e4,e8,w6", [(Fr(4, 7), Fr(16, 105), Fr(1, 630)), (Fr(3, 5), Fr(1, 6), Fr(1, 500))])
def test_family3d_closed_form(e4, e8, w6):
    ref = sa.family3d(e4, e8, w6)
    got = stencil.family3d(float(e4), float(e8), float(w6))
    assert np.allclose(got, [float(ref[c]) for c in stencil.SHELLS_3D], rtol=1e-13, atol=1e-16)


def test_seeded_families_are_isotropic():
    rng = np.random.default_rng(2)
    for _ in range(3):
        e4, e8, W = stencil.seeded_family2d(*rng.uniform(size=2))
        c = sa.coefficients(2, {k: Fr(float(w)) for k, w in zip(stencil.SHELLS_2D, W)})
        assert abs(float(c["e2"]) - 1) < 1e-14 and abs(float(c["I40"])) < 1e-13 and abs(float(c["I60"])) < 1e-12
        assert abs(float(c["e4"]) - e4) < 1e-14 and abs(float(c["e8"]) - e8) < 1e-14


def _table(tab, **kn):
    """Weights of a printed tuning table (exact rationals) at the given knobs."""
    from fractions import Fraction as Fr
    W = {}
    for code, e in tab.items():
        v = Fr(e.get("1", "0"))
        for k in ("s0", "s1", "d0"):
            if k in e:
                v += Fr(e[k]) * Fr(kn[k]).limit_denominator(10 ** 9)
        W[int(code)] = float(v)
    return W


KNOBS = [(-1 / 6, 1 / 30, 1 / 5), (-0.4, 0.17888543819998318, 0.30660373), (-0.25, 0.05, 0.3)]


@pytest.mark.parametrize("s0,s1,d0", KNOBS)
def test_tolman_stencil_matches_paper_table(s0, s1, d0):
    """The product's solver reproduces Table tab:e4e6e8_tuning_6_2d (sigma_0, sigma_1, delta_0
    tuning on {1,2,4,5,8,9,18}) from the knob relations eqs. (hatsigma01eI), (hatdelta0eI)."""
    tab = _table(GOLD["tab_e4e6e8_tuning_6_2d"]["d2"], s0=s0, s1=s1, d0=d0)
    W = stencil.tolman_stencil_2d(s0, s1, d0)
    for c, w in zip(stencil.TOLMAN_SHELLS_2D, W):
        assert abs(w - tab.get(c, 0.0)) < 1e-12 * max(1.0, abs(tab.get(c, 0.0))), c


@pytest.mark.parametrize("s0,s1,d0", KNOBS)
def test_surface_tension_stencil_matches_paper_table(s0, s1, d0):
    """Table tab:e4e6_tuning_8 (sigma_0, sigma_1 tuning, eighth-order isotropy)."""
    tab = _table(GOLD["tab_e4e6_tuning_8"]["d2"], s0=s0, s1=s1)
    W = stencil.surface_tension_stencil_2d(s0, s1)
    for c, w in zip(stencil.TOLMAN_SHELLS_2D, W):
        assert abs(w - tab.get(c, 0.0)) < 1e-12 * max(1.0, abs(tab.get(c, 0.0))), c


def test_moments_of_maximally_isotropic_e8():
    """E(8) on {1,2,4,5,8} (weights printed in Sec. "Leading order surface tension tuning"):
    e2 = 1, e4 = 4/7, e8 = 16/105 and vanishing I40, I60, I80, I81."""
    m = stencil.moments2d(stencil.SHELLS_2D, [4 / 21, 4 / 45, 1 / 60, 2 / 315, 1 / 5040])
    assert abs(m["e2"] - 1) < 1e-15 and abs(m["e4"] - 4 / 7) < 1e-15 and abs(m["e8"] - 16 / 105) < 1e-15
    for k in ("I40", "I60", "I80", "I81"):
        assert abs(m[k]) < 1e-14, k
