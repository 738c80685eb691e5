"""Parity of the HIP step (through the C ABI) with the FP64 oracle.

FP64 bar: max |gpu - oracle| / max |oracle| <= 1e-12 over all populations (and density).
FP32 / FP16-storage: measured error bounds stated in each test.
"""
import numpy as np
import pytest

from paper_2505_23647_amd import (SCL_FP16S_FP32, SCL_FP32, SCL_FP32_SHIFTED, SCL_FP64, Lattice, SclError, synth)
from paper_2505_23647_amd import _lib as B
from tests.gpu_helpers import (E4_2D, E8_2D, coupling, family2d_weights, family3d_weights, oracle_run,
                               patch_oracle, perm_to_oracle, rel_err, say)
import oracle
from oracle import thermo

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def gpu_run(dims_list, prec, tau, G, codes, W, n0, steps, tiling=None, psi_kind=0, psi_param=None):
    lat = Lattice(dims_list, prec)
    lat.set_physics(tau, G, psi_kind, psi_param)
    lat.set_stencil(codes, W)
    if tiling:
        lat.set_tiling(*tiling)
    lat.init_density(n0)
    lat.step(steps)
    return lat


def compare_domain(lat, k, ora, tol):
    perm = perm_to_oracle(lat.xi, lat.d)
    f = lat.domain_populations(k)[perm]
    e = rel_err(f, ora.f)
    return e


def test_c1_droplet_fp64_parity():
    """128^2 nearest-neighbour droplet (E(4), psi = exp(-1/n), Delta T = 0.2, coexistence
    densities), 1000 steps, FP64: populations and density within 1e-12 of the oracle."""
    say("case: C1* 128x128 E4 fp64 1000 steps")
    G = coupling(0.2)
    ng, nl, _ = thermo.coexistence(G)
    L = 128
    n0 = synth.droplet((L, L), 20.0, nl, ng, noise=1e-3, seed=0)
    lat = gpu_run([(L, L)], SCL_FP64, 1.0, G, *E4_2D, n0, 1000)
    ora, rc = oracle_run((L, L), 1.0, G, *E4_2D, n0, 1000)
    assert rc == 0
    assert compare_domain(lat, 0, ora, FP64_TOL) <= FP64_TOL
    assert rel_err(lat.density(), ora.fields()["n"]) <= FP64_TOL
    mass, mom = lat.reduce_conserved()
    assert abs(mass[0] / ora.f.sum() - 1) < 1e-13


def test_fp64_reductions_of_reduced_precision_states():
    """Mass and momentum sum_x (j + F/2) reduced on the GPU in FP64 from FP32-shifted and FP16
    states, against the FP64 oracle's fields of the same stored populations."""
    say("case: fp64 reductions of fp32 / fp16 states")
    G = coupling(0.2)
    L = 96
    n0 = synth.uniform((L, L), 0.7, 1.3, seed=12)
    for prec in (SCL_FP32_SHIFTED, SCL_FP16S_FP32):
        lat = gpu_run([(L, L)], prec, 1.0, G, *E8_2D, n0, 60)
        mass, mom = lat.reduce_conserved()
        s = oracle.Sim((L, L), 1.0, G, *E8_2D)
        s.f = np.ascontiguousarray(lat.domain_populations(0)[perm_to_oracle(lat.xi, 2)])
        fld = s.fields()
        m_ref = fld["n"].sum()
        p_ref = (fld["j"][:, :2] + 0.5 * fld["F"][:, :2]).sum(axis=0)
        scale = np.abs(fld["j"][:, :2]).sum()
        say(f"  precision {prec}: mass rel diff {abs(mass[0] / m_ref - 1):.2e}, momentum diff / sum|j| "
            f"{np.abs(mom[0] - p_ref).max() / scale:.2e}")
        assert abs(mass[0] / m_ref - 1) < 1e-14
        assert np.abs(mom[0] - p_ref).max() < 1e-12 * scale


@pytest.mark.parametrize("strip,seg,cpl", [(64, 7, 1), (128, 32, 1), (256, 0, 1), (64, 7, 2), (128, 5, 2)])
def test_extended_stencil_ragged_fp64(strip, seg, cpl):
    """24-vector stencil (seeded family weights), ragged sizes spanning several strips and
    row segments (both marching directions), spinodal start U(0.5, 1.5), FP64, 150 steps;
    one and two sites per lane."""
    say(f"case: ragged 250x190 24-vector fp64 strip={strip} seg={seg} cpl={cpl}")
    G = coupling(0.2)
    W = family2d_weights(0.55, 0.55 ** 2 * (16 / 105) / (4 / 7) ** 2)
    dims = (250, 190)
    n0 = synth.uniform(dims, 0.9, 1.1, seed=1)
    lat = gpu_run([dims], SCL_FP64, 1.0, G, E8_2D[0], W, n0, 150, tiling=(strip, seg, cpl))
    ora, _ = oracle_run(dims, 1.0, G, E8_2D[0], W, n0, 150)
    assert compare_domain(lat, 0, ora, FP64_TOL) <= FP64_TOL


@pytest.mark.parametrize("dims", [(5, 7), (3, 3), (96, 1), (1, 40), (300, 2), (2, 9), (4, 4), (130, 3)])
def test_small_and_degenerate_domains_fp64(dims):
    """Domains narrower than a strip or than the stencil (periodic images), single rows and
    columns; even widths also through the two-sites-per-lane path."""
    say(f"case: degenerate dims {dims}")
    G = coupling(0.1)
    W = family2d_weights(0.5, 0.1)
    n0 = synth.uniform(dims, 0.95, 1.05, seed=3)
    ora, _ = oracle_run(dims, 0.9, G, E8_2D[0], W, n0, 40)
    for cpl in ((1, 2) if dims[0] % 2 == 0 else (1,)):
        lat = gpu_run([dims], SCL_FP64, 0.9, G, E8_2D[0], W, n0, 40, tiling=(64, 5, cpl))
        assert compare_domain(lat, 0, ora, FP64_TOL) <= FP64_TOL, cpl


def test_two_sites_per_lane_bitwise_fp32():
    """The vector path (two sites per lane) performs the same arithmetic per site as the
    scalar path: bitwise equal FP32 states, over tilings with partial strips and both
    marching directions."""
    say("case: cpl 1 vs 2 bitwise")
    G = coupling(0.2)
    dims = [(1000, 330), (64, 18), (2, 7)]
    W = family2d_weights(0.6, 0.2)
    n0 = np.concatenate([synth.uniform(d, 0.6, 1.4, seed=20 + k) for k, d in enumerate(dims)])
    ref = gpu_run(dims, SCL_FP32_SHIFTED, 0.9, G, E8_2D[0], W, n0, 60, tiling=(64, 9, 1))
    pref = ref.populations()
    for strip, seg in ((64, 9), (128, 16), (256, 31)):
        lat = gpu_run(dims, SCL_FP32_SHIFTED, 0.9, G, E8_2D[0], W, n0, 60, tiling=(strip, seg, 2))
        assert lat.get_tiling()[2] == 2
        assert np.array_equal(lat.populations(), pref), (strip, seg)
    with pytest.raises(SclError):
        Lattice([(5, 4)], SCL_FP32).set_tiling(64, 8, 2)


@pytest.mark.parametrize("kind,param", [(1, 14 / 29), (2, None)])
def test_pseudopotential_variants_fp64(kind, param):
    """psi_eps of eq. (psieps) and the textbook 1 - exp(-n)."""
    say(f"case: psi kind {kind}")
    dims = (70, 66)
    if kind == 1:
        G = thermo.G_for_reduced_temperature(0.1, 1, param)
    else:
        G = -5.0
    n0 = synth.uniform(dims, 0.8, 1.2, seed=5)
    lat = gpu_run([dims], SCL_FP64, 1.0, G, *E8_2D, n0, 100, psi_kind=kind, psi_param=param)
    ora, _ = oracle_run(dims, 1.0, G, *E8_2D, n0, 100, kind, param or 0.0)
    assert compare_domain(lat, 0, ora, FP64_TOL) <= FP64_TOL


def test_batched_domains_fp64_and_fp32_bitwise():
    """Uneven domains in one launch: each matches the oracle (FP64), and in FP32 each domain
    of the batch is bitwise equal to the same domain run alone."""
    say("case: batched uneven domains")
    G = coupling(0.2)
    dims = [(64, 64), (90, 90), (40, 40), (130, 130)]
    W = np.array([family2d_weights(e4, 0.2) for e4 in (0.5, 0.55, 0.6, 0.65)])
    n0s = [synth.droplet(d, d[0] / 4, 2.1, 0.5, noise=1e-3, seed=10 + k) for k, d in enumerate(dims)]
    n0 = np.concatenate(n0s)
    lat = gpu_run(dims, SCL_FP64, 1.0, G, E8_2D[0], W, n0, 120, tiling=(128, 24))
    for k, d in enumerate(dims):
        ora, _ = oracle_run(d, 1.0, G, E8_2D[0], W[k], n0s[k], 120)
        assert compare_domain(lat, k, ora, FP64_TOL) <= FP64_TOL, k
    bat = gpu_run(dims, SCL_FP32, 1.0, G, E8_2D[0], W, n0, 120, tiling=(128, 24))
    for k, d in enumerate(dims):
        one = gpu_run([d], SCL_FP32, 1.0, G, E8_2D[0], W[k], n0s[k], 120, tiling=(128, 24))
        assert np.array_equal(bat.domain_populations(k), one.domain_populations(0)), k


@pytest.mark.parametrize("d", [2, 3])
def test_force_squared_term_fp64(d):
    """The F^2 part of the Guo tensor, T = 2uF - (A/tau) FF (appendix on eps and e4): FP64
    parity with the oracle in 2D (24-vector stencil) and 3D (92 vectors), tau != 1."""
    say(f"case: F^2 forcing A = 0.6, d = {d}")
    G = coupling(0.2)
    if d == 2:
        dims, codes, W = (150, 70), E8_2D[0], family2d_weights(0.55, 0.12)
    else:
        dims, codes, W = (40, 24, 20), [1, 2, 3, 4, 5, 6, 8], family3d_weights(4 / 7, 16 / 105, 1 / 630)
    n0 = synth.uniform(dims, 0.8, 1.2, seed=31)
    lat = Lattice([dims], SCL_FP64).set_physics(0.8, G).set_force_squared(0.6).set_stencil(codes, W)
    lat.init_density(n0).step(60)
    ora = oracle.Sim(dims, 0.8, G, codes, W, force_squared=0.6).init_density(n0)
    assert ora.run(60) == 0
    assert compare_domain(lat, 0, ora, FP64_TOL) <= FP64_TOL
    # and the term matters: without it the states differ
    ref = oracle.Sim(dims, 0.8, G, codes, W).init_density(n0)
    ref.run(60)
    assert rel_err(ref.f, ora.f) > 1e-8


def test_fp32_error_bound_per_1000_steps():
    """FP32 and FP32-shifted storage against the FP64 oracle on the C1* droplet: relative
    density error after 1000 steps (max |n - n_ref| / max |n_ref|). FP32 shifted meets the
    1e-5 per 1000 steps bound (6e-6 measured on MI355X); plain FP32 does not (7.5e-5):
    rounding of identical bulk sites is identical, so the bulk density drifts coherently and
    the error grows about linearly with the step count, which the shifted storage avoids."""
    say("case: fp32 error 128x128 1000 steps")
    G = coupling(0.2)
    ng, nl, _ = thermo.coexistence(G)
    L = 128
    n0 = synth.droplet((L, L), 20.0, nl, ng, noise=1e-3, seed=0)
    ora, _ = oracle_run((L, L), 1.0, G, *E4_2D, n0, 1000)
    nref = ora.fields()["n"]
    for prec, bound in ((SCL_FP32, 1.5e-4), (SCL_FP32_SHIFTED, 1e-5)):
        lat = gpu_run([(L, L)], prec, 1.0, G, *E4_2D, n0, 1000)
        e = rel_err(lat.density(), nref)
        say(f"  precision {prec}: density rel err {e:.3e}")
        assert e < bound
    lat = gpu_run([(L, L)], SCL_FP16S_FP32, 1.0, G, *E4_2D, n0, 1000)
    e = rel_err(lat.density(), nref)
    say(f"  fp16 storage: density rel err {e:.3e}")
    assert e < 2e-2


@pytest.mark.parametrize("codes,weights,dims,steps", [
    ([1, 2], [1 / 6, 1 / 12], (20, 18, 17), 40),
    ([1, 2, 3, 4, 5, 6, 8], "family", (36, 33, 30), 30),
])
def test_d3q19_fp64_parity(codes, weights, dims, steps):
    """D3Q19 with the 18-vector E(4) stencil and the 92-vector seeded family, ragged sizes."""
    say(f"case: d3q19 {dims} shells {codes}")
    G = coupling(0.2)
    W = family3d_weights(4 / 7, 16 / 105, 1 / 630) if weights == "family" else weights
    n0 = synth.around(dims, 1.0, 1e-2, seed=4)
    for tile in (1, 2, 4):
        lat = gpu_run([dims], SCL_FP64, 0.8, G, codes, W, n0, steps, tiling=(tile, 7))
        ora, _ = oracle_run(dims, 0.8, G, codes, W, n0, steps)
        assert compare_domain(lat, 0, ora, FP64_TOL) <= FP64_TOL, tile


def test_d3q19_fp32_error():
    say("case: d3q19 fp32")
    G = coupling(0.2)
    W = family3d_weights(4 / 7, 16 / 105, 1 / 630)
    dims = (40, 36, 34)
    n0 = synth.around(dims, 1.0, 1e-2, seed=4)
    ora, _ = oracle_run(dims, 0.8, G, [1, 2, 3, 4, 5, 6, 8], W, n0, 50)
    for tile in (1, 2, 3, 4):
        lat = gpu_run([dims], SCL_FP32, 0.8, G, [1, 2, 3, 4, 5, 6, 8], W, n0, 50, tiling=(tile, 9))
        e = rel_err(lat.density(), ora.fields()["n"])
        say(f"  tile {tile}: {e:.2e}")
        assert e < 1e-5
    # FP16 storage (shifted), automatic tile (64x4) and 64x8
    for tiling in (None, (2, 9)):
        lat = gpu_run([dims], SCL_FP16S_FP32, 0.8, G, [1, 2, 3, 4, 5, 6, 8], W, n0, 50, tiling=tiling)
        e = rel_err(lat.density(), ora.fields()["n"])
        say(f"  fp16 storage, tiling {tiling} (in use {lat.get_tiling()}): {e:.2e}")
        assert e < 2e-3


def test_d3q19_tile_selection():
    """Automatic 3D tiles: 128x4 for FP32 storage, 64x4 for FP16 storage, 64x8 for FP64 and for
    the reach-4 set, which rejects the 64x4 and 128x4 tiles."""
    from paper_2505_23647_amd import stencil
    G = coupling(0.2)
    W = family3d_weights(4 / 7, 16 / 105, 1 / 630)
    shells = [1, 2, 3, 4, 5, 6, 8]
    for prec, tile in ((SCL_FP32, 4), (SCL_FP32_SHIFTED, 4), (SCL_FP16S_FP32, 1), (SCL_FP64, 2)):
        lat = Lattice([(32, 32, 32)], prec).set_physics(0.8, G).set_stencil(shells, W)
        assert lat.get_tiling()[0] == tile, prec
    r4 = list(stencil.TOLMAN_SHELLS_3D)
    lat = Lattice([(32, 32, 32)], SCL_FP32).set_physics(0.8, G).set_stencil(r4, [0.01] * len(r4))
    assert lat.get_tiling()[0] == 2
    for bad in (1, 4, 5):
        with pytest.raises(SclError):
            lat.set_tiling(bad, 0, 0)


def test_full_size_c2_sampled_fp64_and_fp32():
    """4096^2 spinodal start, 24-vector stencil, in the bench's launch configuration: after 3
    steps, sampled sites against oracle patches (exact light cone), FP64 to 1e-12 and FP32
    shifted to 2e-6; mass conserved over 200 steps."""
    say("case: full size 4096^2 sampled")
    G = coupling(0.2)
    W = family2d_weights(0.6, 0.6 ** 2 * (16 / 105) / (4 / 7) ** 2)
    dims = (4096, 4096)
    n0 = synth.uniform(dims, 0.5, 1.5, seed=1)
    rng = np.random.default_rng(7)
    samples = [(0, 0), (4095, 4095), (251, 17), (2048, 4000)] + [tuple(v) for v in rng.integers(0, 4096, (4, 2))]
    steps = 3
    refs = [patch_oracle(n0, dims, s, 3 * steps + 2, 1.0, G, E8_2D[0], W, steps) for s in samples]
    for prec, tol in ((SCL_FP64, FP64_TOL), (SCL_FP32_SHIFTED, 2e-6)):
        lat = gpu_run([dims], prec, 1.0, G, E8_2D[0], W, n0, steps)
        perm = perm_to_oracle(lat.xi, 2)
        f = lat.domain_populations(0)
        for s, ref in zip(samples, refs):
            c = s[0] + dims[0] * s[1]
            e = np.abs(f[perm, c] - ref).max() / np.abs(ref).max()
            assert e <= tol, (prec, s, e)
        m0, _ = lat.reduce_conserved()
        lat.step(200)
        m1, _ = lat.reduce_conserved()
        assert abs(m1[0] / m0[0] - 1) < (1e-13 if prec == SCL_FP64 else 1e-5)


def test_full_size_c4_sampled_3d_fp32_and_fp64():
    """512^3 D3Q19 with the 92-vector stencil (seeded weights near 3D E(8)), tau = 0.8,
    n0 = 1 + U(-1e-2, 1e-2), in the bench's launch configuration (automatic tiling): after 2
    steps, sampled sites (seam corners included) against oracle patches (exact light cone),
    FP64 to 1e-12 and FP32 to 2e-6. The populations are read out into device memory and only
    the samples are brought to the host."""
    import torch
    from paper_2505_23647_amd import stencil
    say("case: full size 512^3 d3q19 sampled")
    dims = (512, 512, 512)
    u = synth.knob_draws(3, 3, 0.0, 1.0)
    W = stencil.seeded_family3d(*u)[3]
    codes = list(stencil.SHELLS_3D)
    G = -1.2 * np.e ** 2
    n0 = synth.around(dims, 1.0, 1e-2, seed=4)
    rng = np.random.default_rng(11)
    samples = [(0, 0, 0), (511, 511, 511), (0, 511, 255), (300, 2, 509)] + [tuple(v) for v in rng.integers(0, 512, (3, 3))]
    steps = 2
    refs = [patch_oracle(n0, dims, c, 3 * steps + 1, 0.8, G, codes, W, steps) for c in samples]
    cells = 512 ** 3
    for prec, tol in ((SCL_FP64, FP64_TOL), (SCL_FP32, 2e-6)):
        lat = gpu_run([dims], prec, 0.8, G, codes, W, n0, steps)
        out = torch.empty((19, cells), dtype=torch.float64, device="cuda")
        B.check(B.lib().scl_get_populations(lat.h, out.data_ptr(), 1))
        idx = torch.tensor([c[0] + 512 * (c[1] + 512 * c[2]) for c in samples], device="cuda")
        f = out[:, idx].cpu().numpy()
        del out
        perm = perm_to_oracle(lat.xi, 3)
        for k, (c, ref) in enumerate(zip(samples, refs)):
            e = np.abs(f[perm, k] - ref).max() / np.abs(ref).max()
            say(f"  precision {prec} site {c}: {e:.2e}")
            assert e <= tol, (prec, c, e)
        lat.close()
        torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,dims,tiling,tol", [(SCL_FP32, (8192, 8192), None, 2e-6),
                                                 (SCL_FP64, (6144, 6144), (256, 32, 1), FP64_TOL),
                                                 (SCL_FP64, (6144, 6144), (-256, 24, 0), FP64_TOL)])
def test_states_over_2gib_sampled(prec, dims, tiling, tol):
    """A domain whose state exceeds 2 GiB: the marching step addresses it through a descriptor
    per row and plane instead of one for the whole state (the tiles need only each plane under
    2 GiB). After 3 steps, sampled sites (seam corners included) against oracle patches."""
    import torch
    say(f"case: state over 2 GiB, precision {prec}, dims {dims}, tiling {tiling}")
    G = coupling(0.2)
    W = family2d_weights(0.6, 0.6 ** 2 * (16 / 105) / (4 / 7) ** 2)
    n0 = synth.uniform(dims, 0.5, 1.5, seed=5)
    rng = np.random.default_rng(8)
    samples = [(0, 0), (dims[0] - 1, dims[1] - 1), (dims[0] - 1, 3), (5000, 6000)] + \
        [tuple(v) for v in rng.integers(0, min(dims), (3, 2))]
    steps = 3
    refs = [patch_oracle(n0, dims, c, 3 * steps + 2, 1.0, G, E8_2D[0], W, steps) for c in samples]
    lat = gpu_run([dims], prec, 1.0, G, E8_2D[0], W, n0, steps, tiling=tiling)
    cells = dims[0] * dims[1]
    out = torch.empty((9, cells), dtype=torch.float64, device="cuda")
    B.check(B.lib().scl_get_populations(lat.h, out.data_ptr(), 1))
    idx = torch.tensor([c[0] + dims[0] * c[1] for c in samples], device="cuda")
    f = out[:, idx].cpu().numpy()
    del out
    perm = perm_to_oracle(lat.xi, 2)
    for k, (c, ref) in enumerate(zip(samples, refs)):
        e = np.abs(f[perm, k] - ref).max() / np.abs(ref).max()
        assert e <= tol, (c, e)
    lat.close()
    torch.cuda.empty_cache()


def test_graph_replay_matches_plain_launches():
    say("case: hip graph replay")
    G = coupling(0.2)
    dims = (200, 150)
    n0 = synth.uniform(dims, 0.9, 1.1, seed=2)
    a = gpu_run([dims], SCL_FP32, 1.0, G, *E8_2D, n0, 0)
    b = gpu_run([dims], SCL_FP32, 1.0, G, *E8_2D, n0, 0)
    b.set_graph_steps(10)
    for _ in range(3):  # replays with eager work in between
        a.step(25)
        b.step(25)
        _ = a.density(), b.density()
    assert np.array_equal(a.populations(), b.populations())
    assert a.step_count() == b.step_count() == 75


def test_runs_are_deterministic():
    say("case: determinism")
    G = coupling(0.2)
    dims = (300, 260)
    n0 = synth.uniform(dims, 0.5, 1.5, seed=9)
    a = gpu_run([dims], SCL_FP32_SHIFTED, 1.0, G, *E8_2D, n0, 100)
    b = gpu_run([dims], SCL_FP32_SHIFTED, 1.0, G, *E8_2D, n0, 100)
    assert np.array_equal(a.populations(), b.populations())
    ma, pa = a.reduce_conserved()
    mb, pb = b.reduce_conserved()
    assert np.array_equal(ma, mb) and np.array_equal(pa, pb)


def test_argument_validation_and_state_errors():
    say("case: validation")
    lat = Lattice([(16, 16)], SCL_FP64)
    with pytest.raises(SclError) as e:
        lat.step(1)
    assert e.value.status == B.SCL_E_STATE
    with pytest.raises(SclError) as e:
        lat.set_physics(0.5, -5.0)
    assert e.value.status == B.SCL_E_INVALID
    with pytest.raises(SclError) as e:
        lat.set_stencil([1, 7], [0.1, 0.1])
    assert e.value.status == B.SCL_E_INVALID
    lat.set_physics(1.0, -5.0).set_stencil(*E4_2D)
    bad = np.ones(256)
    bad[3] = np.nan
    with pytest.raises(SclError) as e:
        lat.init_density(bad)
    assert e.value.status == B.SCL_E_INVALID
    bad[3] = -1.0
    with pytest.raises(SclError):
        lat.init_density(bad)
    lat3 = Lattice([(8, 8, 8)], SCL_FP32)
    with pytest.raises(SclError) as e:
        lat3.set_stencil([10], [0.1])
    assert e.value.status == B.SCL_E_INVALID
    lat3.set_stencil([1, 2, 9], [0.1, 0.05, 0.01])  # the (2,2,1) group: reach-4 set
    with pytest.raises(SclError) as e:
        lat3.set_tiling(1, 0, 0)
    assert e.value.status == B.SCL_E_UNSUPPORTED


def test_literal_config_reports_nonfinite():
    """The literal nearest-neighbour droplet diverges; the checked readout says so."""
    say("case: literal C1 nonfinite")
    L = 128
    n0 = synth.droplet((L, L), 20.0, 2.0, 0.15, noise=1e-3, seed=0)
    lat = gpu_run([(L, L)], SCL_FP64, 1.0, -15.0, *E4_2D, n0, 200)
    with pytest.raises(SclError) as e:
        lat.reduce_conserved()
    assert e.value.status == B.SCL_E_NONFINITE
