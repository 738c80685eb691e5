"""The paper's tuning stencils on the GPU: shells {1,2,4,5,8,9,18} (reach 4 sites) with weights
from the knob solver, and the flat-interface observables read out by the library.

* FP64 parity with the oracle on a ragged droplet domain and on a slab (populations within
  1e-12), FP32-shifted against FP64.
* The library's flat-interface readout (sigma_0, z_s, z_e, delta, delta_ads) against the
  oracle's flat-interface module on the same populations.
* The flat Tolman-length tuning of Sec. "Higher-order Tolman length tuning": with
  psi = (n/(eps+n))^(1/eps), eps = 14/29, e4 = 4/5, e6 = e4^(3/2), e8 = e4^2 as reference and
  delta_0 = delta_0,ref (1 + Delta_delta), converged slabs keep their bulk densities (to
  machine precision, as the paper reports), delta changes linearly with Delta_delta and
  sigma_0 only at the 1e-3 level; eq. (zemzs) and eq. (deltaads) agree.
"""
import numpy as np
import pytest

import oracle
from oracle import flat, thermo
from paper_2505_23647_amd import SCL_FP32_SHIFTED, SCL_FP64, Lattice, stencil, synth
from tests.gpu_helpers import perm_to_oracle, rel_err, say

pytestmark = pytest.mark.gpu

SH = list(stencil.TOLMAN_SHELLS_2D)
EPS = 14 / 29
E4 = 0.8
KNOB_REF = (-E4 / 2, E4 ** 1.5 / 4, 1 / 12 + 95 * E4 / 432 + 7 * E4 ** 1.5 / 72 - 5 * E4 ** 2 / 144)


def _weights(ddelta=0.0):
    s0, s1, d0 = KNOB_REF
    return stencil.tolman_stencil_2d(s0, s1, d0 * (1.0 + ddelta))


def _physics(dT):
    G = thermo.G_for_reduced_temperature(dT, kind=1, eps=EPS)
    ng, nl, _ = thermo.coexistence(G, kind=1, eps=EPS)
    return G, ng, nl


def _lattice(dims, prec, G, W, n0, tiling=None):
    lat = Lattice(dims, prec).set_physics(1.0, G, 1, EPS).set_stencil(SH, W)
    if tiling:
        lat.set_tiling(*tiling)
    return lat.init_density(n0)


def _oracle(dims, G, W, n0, steps):
    s = oracle.Sim(dims, 1.0, G, SH, W, oracle.PSI_EPS, EPS).init_density(n0)
    assert s.run(steps) == 0
    return s


@pytest.mark.parametrize("tiling", [(256, 0), (128, 9)])
def test_reach4_droplet_fp64_parity(tiling):
    say(f"case: reach-4 tuning stencil droplet 300x70 fp64, tiling {tiling}")
    G, ng, nl = _physics(0.1)
    W = _weights(0.2)
    dims = (300, 70)
    n0 = synth.droplet(dims, 22.0, nl, ng, noise=1e-3, seed=5)
    lat = _lattice([dims], SCL_FP64, G, W, n0, tiling)
    lat.step(300)
    ora = _oracle(dims, G, W, n0, 300)
    perm = perm_to_oracle(lat.xi, 2)
    e = rel_err(lat.domain_populations(0)[perm], ora.f)
    say(f"  populations rel err {e:.2e}")
    assert e <= 1e-12
    l32 = _lattice([dims], SCL_FP32_SHIFTED, G, W, n0, tiling)
    l32.step(300)
    e32 = rel_err(l32.density(), lat.density())
    say(f"  fp32 shifted vs fp64 density rel err {e32:.2e}")
    assert e32 < 1e-4


def test_flat_observables_match_oracle_readout():
    say("case: flat readout vs oracle, reach-4 stencil slab 128x2")
    G, ng, nl = _physics(0.1)
    W = _weights(0.0)
    dims = (128, 2)
    n0 = synth.slab(128, nl, ng, 32.0, ny=2)
    lat = _lattice([dims], SCL_FP64, G, W, n0)
    lat.step(3000)
    ora = _oracle(dims, G, W, n0, 3000)
    perm = perm_to_oracle(lat.xi, 2)
    assert rel_err(lat.domain_populations(0)[perm], ora.f) <= 1e-12
    got = lat.flat_observables([[nl, ng]])[0]
    # the oracle's readout of the GPU populations, row-mean profiles as in the library
    s = oracle.Sim(dims, 1.0, G, SH, W, oracle.PSI_EPS, EPS)
    s.f = np.ascontiguousarray(lat.domain_populations(0)[perm])
    n = s.fields()["n"].reshape(2, 128).mean(axis=0)
    P = s.pressure_tensor().reshape(3, 2, 128).mean(axis=1)
    for h, (lo, hi) in enumerate(flat.halves(128)):
        ref = [flat.sigma0(P[0], P[1], lo, hi), flat.z_s(P[0], P[1], lo, hi), flat.z_e(n, lo, hi, nl, ng),
               flat.delta_zemzs(n, P[0], P[1], lo, hi, nl, ng), flat.delta_ads(n, P[0], P[1], lo, hi, nl, ng)]
        say(f"  interface {h}: gpu {np.array2string(got[h], precision=6)} oracle {np.array2string(np.array(ref), precision=6)}")
        np.testing.assert_allclose(got[h], ref, rtol=1e-9, atol=1e-12)


def test_flat_tolman_length_tuning():
    say("case: flat Tolman tuning, Delta_delta in (-0.2, 0, 0.2), 128x1 slabs, 60000 steps")
    G, ng, nl = _physics(0.1)
    nx = 128
    n0 = synth.slab(nx, nl, ng, 32.0)
    res = {}
    for dd in (-0.2, 0.0, 0.2):
        lat = _lattice([(nx, 1)], SCL_FP64, G, _weights(dd), n0)
        lat.set_graph_steps(100)
        lat.step(60000)
        n = lat.density()
        P = lat.pressure_tensor()
        spread = (P[0].max() - P[0].min()) / abs(P[0].mean())
        obs = lat.flat_observables()[0]
        res[dd] = (n.max(), n.min(), obs, spread)
        say(f"  Delta_delta={dd:+.1f}: n_l={n.max():.12f} n_g={n.min():.12f} P_N spread {spread:.1e} "
            f"sigma_0={obs[0, 0]:.6f} delta={obs[0, 3]:.5f} delta_ads={obs[0, 4]:.5f}")
        lat.close()
    for dd, (nlx, ngx, obs, spread) in res.items():
        assert spread < 1e-9
        # the two Tolman definitions agree (per interface), the interfaces mirror each other
        assert np.allclose(obs[:, 3], obs[:, 4], rtol=1e-9)
        assert abs(obs[0, 3] - obs[1, 3]) < 1e-5 * abs(obs[0, 3])
        # bulk densities untouched by the Tolman knob
        assert abs(nlx - res[0.0][0]) < 1e-12 * nlx and abs(ngx - res[0.0][1]) < 1e-12 * ngx
    d = {dd: res[dd][2][0, 3] for dd in res}
    sig = {dd: res[dd][2][0, 0] for dd in res}
    slope = (d[0.2] - d[-0.2]) / (0.4 * d[0.0])
    say(f"  delta: {d[-0.2]:.5f} {d[0.0]:.5f} {d[0.2]:.5f}; d delta / (delta d Delta_delta) = {slope:.4f}")
    # linear in the knob, with the relative slope near the tuning target 1 (a constant offset of
    # the measured delta from eq. (SCTolmanFlat), as the paper notes, tilts it), and the surface
    # tension changed at the 1e-3 level
    assert abs((d[0.2] - d[0.0]) / (d[0.0] - d[-0.2]) - 1.0) < 0.01
    assert 0.9 < slope < 1.3
    assert max(abs(sig[dd] / sig[0.0] - 1.0) for dd in (-0.2, 0.2)) < 1e-2


def test_closed_interface_tolman_tuning_2d():
    """Sec. "Higher-order Tolman length tuning", closed interfaces in d = 2: droplets and bubbles
    of 16 radii (12..96, side 4R + 32) with the reach-4 tuning stencil at Delta_delta in
    (-0.2, 0, 0.2), 40000 steps in one batched launch each (FP32 shifted storage, graphs). The
    fit of dP R_s / sigma_0 against the signed curvature (-1)^b / R_s gives the surface tension
    (intercept) and -delta (slope). Asserted: the Laplace law holds at a fixed slope for every
    Delta_delta and the surface tension moves by under 3%, as the paper reports. The fitted
    delta (5.1, 5.8, 4.9 on MI355X) is not resolved well enough at these radii and this
    relaxation time to show the knob's +-20%; only its range is checked (the flat interface
    resolves the knob: test_flat_tolman_length_tuning)."""
    from oracle import flat as oflat
    from paper_2505_23647_amd import SCL_FP32_SHIFTED
    say("case: closed-interface Tolman tuning, 2D, 32 domains x 3 knob values, 40000 steps")
    G, ng, nl = _physics(0.1)
    # sigma_0 of the flat interface at the reference knobs (FP64 slab)
    lat = _lattice([(128, 1)], SCL_FP64, G, _weights(0.0), synth.slab(128, nl, ng, 32.0))
    lat.set_graph_steps(100)
    lat.step(60000)
    sigma0 = lat.flat_observables()[0][0, 0]
    lat.close()
    radii = np.exp(np.linspace(np.log(12.0), np.log(96.0), 16))
    dims, n0, centers, bubble = [], [], [], []
    for k, R in enumerate(radii):
        L = int(round(4 * R + 32))
        for b in (0, 1):
            n_in, n_out = (ng, nl) if b else (nl, ng)
            dims.append((L, L))
            n0.append(synth.droplet((L, L), R, n_in, n_out, noise=1e-3, seed=300 + 2 * k + b))
            centers.append((L // 2, L // 2))
            bubble.append(b)
    n0 = np.concatenate(n0)
    centers, bubble = np.array(centers), np.array(bubble, dtype=np.int8)
    sgn = np.where(bubble == 1, -1.0, 1.0)
    fits = {}
    for dd in (-0.2, 0.0, 0.2):
        lat = _lattice(dims, SCL_FP32_SHIFTED, G, _weights(dd), n0)
        lat.set_graph_steps(100)
        lat.step(40000)
        obs = lat.droplet_observables(centers, bubble)
        lat.close()
        dP, Rs, Re = obs[:, 0], obs[:, 2], obs[:, 4]
        ok = np.isfinite(Rs) & (np.repeat(radii, 2) >= 16)
        slope, icpt = np.polyfit(sgn[ok] / Rs[ok], dP[ok] * Rs[ok] / sigma0, 1)
        lap = dP[ok] * Re[ok] / sigma0
        fits[dd] = (icpt, -slope)
        say(f"  Delta_delta={dd:+.1f}: {ok.sum()} domains, intercept {icpt:.4f}, delta {-slope:.3f}, "
            f"dP R_e / sigma_0 in {lap.min():.3f}..{lap.max():.3f}")
        assert ok.sum() >= 20
        assert np.all(np.abs(lap - 1.0) < 0.15)
    d = {k: v[1] for k, v in fits.items()}
    say(f"  sigma_0 (flat) {sigma0:.6f}; delta ratios {d[-0.2] / d[0.0]:.3f}, {d[0.2] / d[0.0]:.3f}")
    for dd in (-0.2, 0.2):
        assert abs(fits[dd][0] / fits[0.0][0] - 1.0) < 0.03
    assert all(2.0 < v < 10.0 for v in d.values())
