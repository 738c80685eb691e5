"""Device memory from a caller's allocator (scl_set_allocator), here torch's caching allocator.

Lattices created after the hook is installed take every device buffer, and the temporaries of
their calls, from it and return all of it by scl_destroy; their results are bitwise those of
lattices on hipMalloc, through steps, readouts (pressure tensor in 2D and 3D, droplet
observables) and the adjoint. A lattice keeps the source it was created with.
"""
import numpy as np
import pytest
import torch

from paper_2505_23647_amd import SCL_FP32_SHIFTED, SCL_FP64, Lattice, SclError, set_allocator, synth
from paper_2505_23647_amd import _lib as B
from tests.gpu_helpers import E8_2D, coupling, family3d_weights, say

pytestmark = pytest.mark.gpu


class Counting:
    def __init__(self):
        self.live, self.nalloc, self.nfree, self.peak = {}, 0, 0, 0

    def alloc(self, n, stream):
        p = torch.cuda.caching_allocator_alloc(n, stream=stream)
        self.live[p] = n
        self.nalloc += 1
        self.peak = max(self.peak, sum(self.live.values()))
        return p

    def free(self, p, stream):
        assert p in self.live, "freed a pointer the hook did not hand out"
        torch.cuda.caching_allocator_delete(p)
        del self.live[p]
        self.nfree += 1


def _run(dims, prec, codes, W, n0, tau=1.0):
    lat = Lattice(dims, prec).set_physics(tau, coupling(0.2)).set_stencil(codes, W).init_density(n0)
    lat.step(30)
    out = {"pops": lat.populations(), "P": lat.pressure_tensor()}
    if len(dims[0]) == 2:
        out["obs"] = lat.droplet_observables([(d[0] // 2, d[1] // 2) for d in dims])
        lat.checkpointed_forward(20, 6)
        out["grad"] = lat.adjoint(seed_n=np.linspace(0.5, 1.5, lat.cells))
    return lat, out


def test_allocator_hook_serves_all_device_memory():
    torch.cuda.init()
    say("case: allocator hook (torch caching allocator)")
    dims2 = [(96, 96), (64, 64)]
    n2 = np.concatenate([synth.droplet(d, 14.0, 1.9, 0.5, noise=1e-3, seed=3 + k) for k, d in enumerate(dims2)])
    dims3 = [(24, 20, 18)]
    n3 = synth.around(dims3[0], 1.0, 1e-2, seed=4)
    W3 = family3d_weights(4 / 7, 16 / 105, 1 / 630)
    cases = [(dims2, SCL_FP64, E8_2D[0], E8_2D[1], n2, 1.0), (dims2, SCL_FP32_SHIFTED, E8_2D[0], E8_2D[1], n2, 1.0),
             (dims3, SCL_FP64, [1, 2, 3, 4, 5, 6, 8], W3, n3, 0.8)]
    for dims, prec, codes, W, n0, tau in cases:
        ref_lat, ref = _run(dims, prec, codes, W, n0, tau)
        ref_lat.close()
        hook = Counting()
        set_allocator(hook.alloc, hook.free)
        try:
            lat = Lattice(dims, prec)
        finally:
            set_allocator()  # the lattice keeps the hook it was created with
        lat.close()
        assert hook.nalloc >= 2 and not hook.live
        hook = Counting()
        set_allocator(hook.alloc, hook.free)
        try:
            lat, got = _run(dims, prec, codes, W, n0, tau)
        finally:
            set_allocator()
        say(f"  dims {dims} precision {prec}: {hook.nalloc} allocations, peak {hook.peak / 2**20:.1f} MiB")
        state = lat.Q * lat.cells * (8 if prec == SCL_FP64 else 4)
        assert hook.nalloc > 2 and hook.peak >= 2 * state
        for k in ref:
            a, b = ref[k], got[k]
            # (observables of a droplet 30 steps from its start may be NaN: C_d < 0 at this age)
            if isinstance(a, tuple):
                assert all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b)), k
            else:
                assert np.array_equal(a, b, equal_nan=True), k
        lat.close()
        assert not hook.live and hook.nfree == hook.nalloc


def test_allocator_failure_is_reported():
    """An allocator that cannot allocate makes scl_create fail with SCL_E_NOMEM."""
    set_allocator(lambda n, stream: 0, lambda p, stream: None)
    try:
        with pytest.raises(SclError) as e:
            Lattice([(32, 32)], SCL_FP64)
        assert e.value.status == B.SCL_E_NOMEM
    finally:
        set_allocator()
    Lattice([(32, 32)], SCL_FP64).close()
