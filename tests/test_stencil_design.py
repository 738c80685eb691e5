"""The product's closed-form weight families against the oracle's exact linear solve."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import stencil_algebra as sa
from paper_2505_23647_amd import stencil


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
