"""D3Q19 interface readouts on the GPU: the 3D lattice pressure tensor (App. on the lattice
pressure tensor, d = 3) and 3D droplet observables against the oracle's readout of the same
populations, and the 3D Laplace law, Delta P R_e = 2 sigma_0, with sigma_0 from a converged 3D
flat slab (eq. sigma0pnpt)."""
import numpy as np
import pytest

import oracle
from oracle import flat, thermo
from paper_2505_23647_amd import SCL_FP32_SHIFTED, SCL_FP64, Lattice, stencil, synth
from tests.gpu_helpers import perm_to_oracle, rel_err, say

pytestmark = pytest.mark.gpu

SH3 = [1, 2, 3, 4, 5, 6, 8]
W3 = list(stencil.family3d(4 / 7, 16 / 105, 1 / 630))


def test_pressure_tensor_3d_matches_oracle():
    say("case: 3D pressure tensor vs oracle, 20x18x16 fp64")
    G = thermo.G_for_reduced_temperature(0.2)
    dims = (20, 18, 16)
    n0 = synth.uniform(dims, 0.8, 1.2, seed=41)
    lat = Lattice([dims], SCL_FP64).set_physics(1.0, G).set_stencil(SH3, W3).init_density(n0)
    lat.step(15)
    P = lat.pressure_tensor()
    s = oracle.Sim(dims, 1.0, G, SH3, W3)
    s.f = np.ascontiguousarray(lat.domain_populations(0)[perm_to_oracle(lat.xi, 3)])
    ref = s.pressure_tensor_general()
    e = rel_err(P, ref)
    say(f"  rel err {e:.2e}")
    assert e < 1e-13


def _sigma0_flat3d(G):
    ng, nl, _ = thermo.coexistence(G, e4=4 / 7)
    nx = 48
    s = oracle.Sim((nx, 4, 4), 1.0, G, SH3, W3).init_density(np.tile(synth.slab(nx, nl, ng, 12.0), 16))
    assert s.run(20000) == 0
    P = s.pressure_tensor_general().reshape(6, 4, 4, nx).mean(axis=(1, 2))
    lo, hi = flat.halves(nx)[0]
    return flat.sigma0(P[0], P[1], lo, hi), ng, nl


def test_droplet_observables_3d_and_laplace():
    G = thermo.G_for_reduced_temperature(0.2)
    sigma0, ng, nl = _sigma0_flat3d(G)
    say(f"case: 3D droplets, sigma_0 (flat, 3D) = {sigma0:.6f}")
    sides, radii = [40, 48, 56], [9.0, 11.0, 13.0]
    dims = [(L, L, L) for L in sides]
    n0 = np.concatenate([synth.droplet(d, R, nl, ng, noise=1e-3, seed=60 + k) for k, (d, R) in enumerate(zip(dims, radii))])
    centers = np.array([(L // 2,) * 3 for L in sides])
    # FP64 readout parity on an early state
    lat = Lattice(dims, SCL_FP64).set_physics(1.0, G).set_stencil(SH3, W3).init_density(n0)
    lat.step(200)
    obs = lat.droplet_observables(centers)
    perm = perm_to_oracle(lat.xi, 3)
    for k in (0, 2):
        s = oracle.Sim(dims[k], 1.0, G, SH3, W3)
        s.f = np.ascontiguousarray(lat.domain_populations(k)[perm])
        ref = s.droplet_observables3d(centers[k])
        assert np.array_equal(np.isnan(obs[k]), np.isnan(ref))
        ok = ~np.isnan(ref)
        rel = np.abs(obs[k][ok] - ref[ok]) / np.abs(ref[ok])
        say(f"  domain {k}: readout vs oracle max rel diff {rel.max():.2e}")
        assert rel.max() < 1e-10
    lat.close()
    # Laplace law after relaxation (FP32 shifted storage)
    lat = Lattice(dims, SCL_FP32_SHIFTED).set_physics(1.0, G).set_stencil(SH3, W3).init_density(n0)
    lat.set_graph_steps(50)
    lat.step(6000)
    obs = lat.droplet_observables(centers)
    for k, R in enumerate(radii):
        lap = obs[k, 0] * obs[k, 4] / (2.0 * sigma0)
        say(f"  R0={R}: dP={obs[k, 0]:.4e} R_e={obs[k, 4]:.3f} R_s={obs[k, 2]:.3f} sigma_s={obs[k, 3]:.5f} "
            f"dP R_e / (2 sigma_0) = {lap:.4f}")
        assert abs(lap - 1.0) < 0.15
