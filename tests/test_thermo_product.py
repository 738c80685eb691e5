"""The product's closed-form coexistence against the oracle's quadrature construction."""
import math

import pytest

from oracle import thermo as othermo
from paper_2505_23647_amd import thermo


@pytest.mark.parametrize("dT", [0.05, 0.1, 0.2, 0.4])
def test_coexistence_matches_oracle(dT):
    G = thermo.coupling_for_reduced_temperature(dT)
    assert abs(G - othermo.G_for_reduced_temperature(dT)) < 1e-12
    ng, nl, p0 = thermo.coexistence_exp(G)
    og, ol, op = othermo.coexistence(G)
    assert abs(ng - og) < 1e-9 and abs(nl - ol) < 1e-9 and abs(p0 - op) < 1e-11


def test_critical_coupling():
    assert thermo.critical_coupling_exp() == -math.e ** 2


@pytest.mark.parametrize("e4", [4 / 7, 0.5, 0.65])
def test_coexistence_with_stencil_measure_matches_oracle(e4):
    """eq. (SCMaxwell) with the measure psi'/psi^(1+eps), eps = eps(e4) of eq. (eps_moments)."""
    G = thermo.coupling_for_reduced_temperature(0.2)
    ng, nl, p0 = thermo.coexistence_exp(G, eps=thermo.epsilon(e4))
    og, ol, op = othermo.coexistence(G, e4=e4)
    assert abs(ng - og) < 1e-9 and abs(nl - ol) < 1e-9 and abs(p0 - op) < 1e-11
