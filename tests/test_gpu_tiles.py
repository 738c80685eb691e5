"""One-shot tiles of the 2D step (a workgroup per 64 x seg tile, no march) through the C ABI.

* FP64 against the oracle (populations within 1e-12) on ragged domains whose sizes leave
  partial tiles in x and y, for every tile shape, and on domains smaller than a tile or than
  the stencil's reach (periodic images inside one tile's rim).
* Bitwise equality with the marching strips in every storage precision and for the three
  compiled shell sets (reach 1, 2 and 4), batched uneven domains included: both kernels
  perform the same arithmetic per site in the same order.
* HIP-graph replays with tiles, the automatic choice for FP64, argument validation, and the
  adjoint (whose recording pass marches) on a lattice that steps through tiles.
"""
import numpy as np
import pytest

from paper_2505_23647_amd import (SCL_FP16S_FP32, SCL_FP32, SCL_FP32_SHIFTED, SCL_FP64, Lattice, SclError,
                                  stencil, synth)
from tests.gpu_helpers import E4_2D, E8_2D, coupling, family2d_weights, oracle_run, perm_to_oracle, rel_err, say

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
TILES = [(-256, 8, 1), (-256, 16, 1), (-256, 24, 1), (-256, 32, 1), (-512, 16, 1), (-512, 24, 1), (-512, 32, 1),
         (-256, 8, 2), (-256, 16, 2), (-512, 16, 2), (-512, 32, 2)]
REACH4 = list(stencil.TOLMAN_SHELLS_2D)


def _lat(dims, prec, G, codes, W, n0, tiling, tau=1.0):
    lat = Lattice(dims, prec).set_physics(tau, G).set_stencil(codes, W)
    if tiling:
        lat.set_tiling(*tiling)
    return lat.init_density(n0)


@pytest.mark.parametrize("strip,seg,width", TILES)
def test_tiles_ragged_fp64_vs_oracle(strip, seg, width):
    """250 x 190 (3 full tiles + 58 columns; rows not a multiple of any tile height), 24-vector
    stencil, spinodal start, 150 steps."""
    say(f"case: tiles {strip}x{seg} width {64 * width} ragged 250x190 fp64")
    G = coupling(0.2)
    W = family2d_weights(0.55, 0.55 ** 2 * (16 / 105) / (4 / 7) ** 2)
    dims = (250, 190)
    n0 = synth.uniform(dims, 0.9, 1.1, seed=1)
    lat = _lat([dims], SCL_FP64, G, E8_2D[0], W, n0, (strip, seg, width))
    assert tuple(lat.get_tiling()) == (strip, seg, width)
    lat.step(150)
    ora, _ = oracle_run(dims, 1.0, G, E8_2D[0], W, n0, 150)
    e = rel_err(lat.domain_populations(0)[perm_to_oracle(lat.xi, 2)], ora.f)
    say(f"  rel err {e:.2e}")
    assert e <= FP64_TOL


@pytest.mark.parametrize("dims", [(5, 7), (3, 3), (96, 1), (1, 40), (300, 2), (2, 9), (4, 4), (130, 3), (64, 16), (65, 17)])
def test_tiles_small_and_degenerate_fp64(dims):
    """Domains narrower or lower than one tile or than the stencil (the rim wraps onto the
    tile itself), single rows and columns, exact and one-past tile sizes."""
    say(f"case: tiles degenerate dims {dims}")
    G = coupling(0.1)
    W = family2d_weights(0.5, 0.1)
    n0 = synth.uniform(dims, 0.95, 1.05, seed=3)
    ora, _ = oracle_run(dims, 0.9, G, E8_2D[0], W, n0, 40)
    for tiling in ((-256, 8, 0), (-512, 16, 0), (-256, 8, 2)):
        lat = _lat([dims], SCL_FP64, G, E8_2D[0], W, n0, tiling, tau=0.9)
        lat.step(40)
        e = rel_err(lat.domain_populations(0)[perm_to_oracle(lat.xi, 2)], ora.f)
        assert e <= FP64_TOL, (tiling, e)


@pytest.mark.parametrize("prec", [SCL_FP64, SCL_FP32, SCL_FP32_SHIFTED, SCL_FP16S_FP32])
@pytest.mark.parametrize("shells", ["E4", "E8", "reach4"])
def test_tiles_bitwise_equal_marching(prec, shells):
    """Tiles and marching strips give bitwise equal states after 40 steps on three uneven
    domains in one launch."""
    say(f"case: tiles vs march bitwise prec={prec} shells={shells}")
    G = coupling(0.2)
    if shells == "E4":
        codes, W = E4_2D
    elif shells == "E8":
        codes, W = E8_2D[0], family2d_weights(0.6, 0.2)
    else:
        codes = REACH4
        W = stencil.tolman_stencil_2d(-0.4, 0.8 ** 1.5 / 4, 1 / 12 + 95 * 0.8 / 432 + 7 * 0.8 ** 1.5 / 72 - 5 * 0.64 / 144)
    dims = [(200, 77), (64, 64), (130, 33), (9, 5)]
    n0 = np.concatenate([synth.uniform(d, 0.9, 1.1, seed=10 + k) for k, d in enumerate(dims)])
    ref = _lat(dims, prec, G, codes, W, n0, (128, 9, 1))
    ref.step(40)
    pref = ref.populations()
    assert np.all(np.isfinite(pref))
    for strip, seg, width in ((-256, 8, 1), (-256, 24, 1), (-512, 32, 1), (-256, 8, 2), (-256, 16, 2), (-512, 24, 2)):
        lat = _lat(dims, prec, G, codes, W, n0, (strip, seg, width))
        lat.step(40)
        assert np.array_equal(lat.populations(), pref), (strip, seg, width)


def test_tiles_graph_replay():
    """HIP-graph replays of tile steps, with eager readouts between replays, equal plain
    launches of the marching strips."""
    say("case: tiles under hip graphs")
    G = coupling(0.2)
    dims = (200, 150)
    n0 = synth.uniform(dims, 0.9, 1.1, seed=2)
    a = _lat([dims], SCL_FP32, G, *E8_2D, n0, (256, 32, 1))
    b = _lat([dims], SCL_FP32, G, *E8_2D, n0, (-256, 16, 0))
    b.set_graph_steps(10)
    for _ in range(3):
        a.step(25)
        b.step(25)
        _ = a.density(), b.density()
    assert np.array_equal(a.populations(), b.populations())


def test_tiles_selection_and_validation():
    """FP64 lattices with the reach-1 and reach-2 sets step through 256-lane 128 x 8 tiles unless
    a tiling is requested, narrow batched domains through 512-lane 64 x 16 tiles and FP16
    lattices through 256-lane 128 x 16 tiles; FP32 lattices march; bad tile shapes are
    rejected."""
    say("case: tile selection and validation")
    G = coupling(0.2)
    lat = Lattice([(128, 96)], SCL_FP64).set_physics(1.0, G).set_stencil(*E8_2D)
    assert tuple(lat.get_tiling()) == (-256, 8, 2)
    lat.set_tiling(128, 0, 0)
    assert lat.get_tiling()[0] == 128
    lat.set_tiling(-512, 24, 0)
    assert tuple(lat.get_tiling()) == (-512, 24, 1)
    l4 = Lattice([(128, 96)], SCL_FP64).set_physics(1.0, G).set_stencil(REACH4, [0.1] * len(REACH4))
    assert l4.get_tiling()[0] > 0
    l32 = Lattice([(128, 96)], SCL_FP32_SHIFTED).set_physics(1.0, G).set_stencil(*E8_2D)
    assert l32.get_tiling()[0] > 0
    l16 = Lattice([(512, 512)], SCL_FP16S_FP32).set_physics(1.0, G).set_stencil(*E8_2D)
    assert tuple(l16.get_tiling()) == (-256, 16, 2)
    # narrow batched domains: 256-lane strips would leave 48% of their lanes idle
    narrow = Lattice([(64, 64), (100, 100), (544, 544)], SCL_FP32_SHIFTED).set_physics(1.0, G).set_stencil(*E8_2D)
    assert tuple(narrow.get_tiling()) == (-512, 16, 1)
    wide = Lattice([(256, 256)] * 4, SCL_FP32_SHIFTED).set_physics(1.0, G).set_stencil(*E8_2D)
    assert wide.get_tiling()[0] == 256
    for bad in ((-128, 16, 0), (-256, 12, 0), (-512, 8, 0), (-64, 0, 0), (-256, 16, 3)):
        with pytest.raises(SclError):
            lat.set_tiling(*bad)
    with pytest.raises(SclError):
        Lattice([(16, 16, 16)], SCL_FP64).set_tiling(-256, 16, 0)


def test_adjoint_on_a_tiled_lattice():
    """The adjoint's recording pass marches while the lattice steps through tiles; the
    gradients equal those of a lattice that marches throughout."""
    say("case: adjoint with tiles")
    G = coupling(0.2)
    dims = (96, 80)
    n0 = synth.droplet(dims, 18.0, 1.9, 0.5, noise=1e-3, seed=4)
    grads = []
    for tiling in ((-256, 16, 0), (128, 16, 1)):
        lat = _lat([dims], SCL_FP64, G, *E8_2D, n0, tiling)
        lat.checkpointed_forward(60, 7)
        gW, gG = lat.adjoint(seed_n=np.linspace(0.5, 1.5, dims[0] * dims[1]))
        assert lat.get_tiling()[0] == tiling[0]
        grads.append((gW, gG))
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])
