"""Python face of libscl: a handle class whose methods map one-to-one onto the C ABI.

Host arrays are numpy; device arrays may be passed as torch tensors on the GPU (their
data pointer is handed to the library with is_device_ptr = 1). Nothing here computes.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as B
from ._lib import check, lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _is_torch_cuda(a):
    return hasattr(a, "is_cuda") and a.is_cuda


_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
# Every callback pair ever installed stays referenced: lattices created with it free through
# it until they are destroyed, even after another source has been installed.
_installed_hooks = []


def set_allocator(alloc=None, free=None):
    """Device-memory source of the lattices created afterwards (scl_set_allocator).

    alloc(nbytes, stream) -> device pointer as an int (0 if it cannot allocate);
    free(ptr, stream). stream is the lattice's hipStream_t as an int (0: the null stream).
    Both None restores hipMalloc / hipFree.
    """
    if alloc is None and free is None:
        check(lib().scl_set_allocator(None, None, None))
        return
    if alloc is None or free is None:
        raise ValueError("give both functions, or neither")
    a = _ALLOC_T(lambda n, ctx, stream: alloc(int(n), stream or 0) or None)
    f = _FREE_T(lambda p, ctx, stream: free(int(p), stream or 0))
    _installed_hooks.append((a, f))
    check(lib().scl_set_allocator(ctypes.cast(a, ctypes.c_void_p), ctypes.cast(f, ctypes.c_void_p), None))


def use_torch_allocator():
    """Lattices created afterwards take their device memory from torch's caching allocator."""
    import torch

    set_allocator(lambda n, stream: torch.cuda.caching_allocator_alloc(n, stream=stream),
                  lambda p, stream: torch.cuda.caching_allocator_delete(p))


def velocity_set(vs: int):
    xi = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    q = lib().scl_velocity_set(vs, _dptr(xi), _dptr(w))
    if q < 0:
        raise ValueError("unknown velocity set")
    return xi[:q].copy(), w[:q].copy()


class Lattice:
    """A batch of independent periodic domains (one or more) on the GPU.

    dims: list of (nx, ny) or (nx, ny, nz); D2Q9 for 2D, D3Q19 for 3D.
    stream: a hipStream_t handle as int (e.g. torch.cuda.current_stream().cuda_stream) or None.
    """

    def __init__(self, dims, precision=B.SCL_FP64, stream=None):
        dims = [tuple(int(v) for v in d) for d in dims]
        self.d = len(dims[0])
        if any(len(d) != self.d for d in dims):
            raise ValueError("all domains must have the same dimension")
        self.vs = B.SCL_D2Q9 if self.d == 2 else B.SCL_D3Q19
        self.precision = precision
        self.dims = [d if self.d == 3 else d + (1,) for d in dims]
        self.ndom = len(dims)
        self.cells_per_dom = [int(np.prod(d)) for d in self.dims]
        self.cells = sum(self.cells_per_dom)
        self.offsets = np.concatenate([[0], np.cumsum(self.cells_per_dom)[:-1]]).astype(np.int64)
        arr = np.ascontiguousarray(np.array(self.dims, dtype=np.int32).reshape(-1))
        h = ctypes.c_void_p()
        check(lib().scl_create(self.vs, precision, self.ndom, _dptr(arr), ctypes.c_void_p(stream or 0),
                               ctypes.byref(h)))
        self.h = h
        self.xi, self.w = velocity_set(self.vs)
        self.Q = len(self.w)

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "h", None):
            lib().scl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ setup
    def set_physics(self, tau, G, psi_kind=B.SCL_PSI_EXP, psi_param=None):
        tau = np.ascontiguousarray(np.broadcast_to(np.asarray(tau, dtype=np.float64), (self.ndom,)))
        G = np.ascontiguousarray(np.broadcast_to(np.asarray(G, dtype=np.float64), (self.ndom,)))
        pp = None
        if psi_param is not None:
            pp = np.ascontiguousarray(np.broadcast_to(np.asarray(psi_param, dtype=np.float64), (self.ndom,)))
        check(lib().scl_set_physics(self.h, _dptr(tau), _dptr(G), psi_kind, _dptr(pp) if pp is not None else None))
        return self

    def set_force_squared(self, A):
        """A per domain (scalar broadcast) of T = 2uF - (A/tau) FF in the Guo term (default 0)."""
        A = np.ascontiguousarray(np.broadcast_to(np.asarray(A, dtype=np.float64), (self.ndom,)))
        check(lib().scl_set_force_squared(self.h, _dptr(A)))
        return self

    def set_stencil(self, codes, W):
        codes = np.ascontiguousarray(codes, dtype=np.int32)
        W = np.asarray(W, dtype=np.float64)
        if W.ndim == 1:
            W = np.tile(W, (self.ndom, 1))
        W = np.ascontiguousarray(W)
        check(lib().scl_set_stencil(self.h, len(codes), _dptr(codes), _dptr(W)))
        self._nshells = len(codes)
        return self

    def init_density(self, n0):
        if _is_torch_cuda(n0):
            check(lib().scl_init_density(self.h, ctypes.c_void_p(n0.data_ptr()), 1))
        else:
            n0 = np.ascontiguousarray(np.asarray(n0, dtype=np.float64).reshape(-1))
            if n0.size != self.cells:
                raise ValueError("n0 has the wrong size")
            check(lib().scl_init_density(self.h, _dptr(n0), 0))
        return self

    # ------------------------------------------------------------------ stepping
    def step(self, nsteps=1):
        check(lib().scl_step(self.h, int(nsteps)))
        return self

    def step_timed(self, nsteps):
        ms = ctypes.c_double()
        check(lib().scl_step_timed(self.h, int(nsteps), ctypes.byref(ms)))
        return ms.value

    def step_count(self):
        v = ctypes.c_int64()
        check(lib().scl_get_step_count(self.h, ctypes.byref(v)))
        return v.value

    def set_tiling(self, strip=0, seg=0, cpl=0):
        check(lib().scl_set_tiling(self.h, int(strip), int(seg), int(cpl)))
        return self

    def get_tiling(self):
        """(strip, seg, sites per lane)."""
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().scl_get_tiling(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def tune(self, cache_path=None):
        check(lib().scl_tune(self.h, cache_path.encode() if cache_path else None))
        return self.get_tiling()

    def set_graph_steps(self, k):
        check(lib().scl_set_graph_steps(self.h, int(k)))
        return self

    # ------------------------------------------------------------------ readouts
    def _get(self, fn, count):
        out = np.empty(count)
        check(fn(self.h, _dptr(out), 0))
        return out

    def density(self):
        return self._get(lib().scl_get_density, self.cells)

    def velocity(self):
        return self._get(lib().scl_get_velocity, self.d * self.cells).reshape(self.d, self.cells)

    def force(self):
        return self._get(lib().scl_get_force, self.d * self.cells).reshape(self.d, self.cells)

    def populations(self):
        """Populations f_i(x, t) as doubles, domain by domain [Q][cells_of_domain] blocks."""
        return self._get(lib().scl_get_populations, self.Q * self.cells)

    def domain_populations(self, k):
        p = self.populations()
        o, c = int(self.offsets[k]) * self.Q, self.cells_per_dom[k]
        return p[o:o + self.Q * c].reshape(self.Q, c)

    def set_populations(self, f):
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
        check(lib().scl_set_populations(self.h, _dptr(f), 0))
        return self

    def pressure_tensor(self):
        """2D: [3, cells] (xx, yy, xy); 3D: [6, cells] (xx, yy, zz, xy, xz, yz)."""
        nc = 3 if self.d == 2 else 6
        return self._get(lib().scl_get_pressure_tensor, nc * self.cells).reshape(nc, self.cells)

    def reduce_conserved(self):
        mass = np.empty(self.ndom)
        mom = np.empty((self.ndom, self.d))
        check(lib().scl_reduce_conserved(self.h, _dptr(mass), _dptr(mom)))
        return mass, mom

    def droplet_observables(self, centers, is_bubble=None):
        c = np.ascontiguousarray(np.asarray(centers, dtype=np.int32).reshape(self.ndom, self.d))
        b = None
        if is_bubble is not None:
            b = np.ascontiguousarray(np.asarray(is_bubble, dtype=np.int8).reshape(self.ndom))
        out = np.empty((self.ndom, 6))
        check(lib().scl_droplet_observables(self.h, _dptr(c), _dptr(b) if b is not None else None, _dptr(out)))
        return out

    def flat_observables(self, bulk=None):
        """[ndom, 2, 5]: (sigma_0, z_s, z_e, delta, delta_ads) of the lower and upper interface
        of a slab varying along x; bulk: [ndom, 2] (n_l, n_g) or None."""
        b = None
        if bulk is not None:
            b = np.ascontiguousarray(np.asarray(bulk, dtype=np.float64).reshape(self.ndom, 2))
        out = np.empty((self.ndom, 2, 5))
        check(lib().scl_flat_observables(self.h, _dptr(b) if b is not None else None, _dptr(out)))
        return out

    # ------------------------------------------------------------------ adjoint
    def checkpointed_forward(self, nsteps, every):
        check(lib().scl_checkpointed_forward(self.h, int(nsteps), int(every)))
        return self

    def adjoint(self, seed_n=None, seed_f=None):
        """Gradients (dL/dW [ndom, nshells], dL/dG [ndom]) through the last checkpointed forward.

        seed_n / seed_f: dL/dn(x) (cells) and dL/df (populations) at the final time, as torch
        tensors on the GPU or numpy arrays (copied to the GPU).
        """
        import torch

        def dev(a):
            if a is None:
                return None
            if _is_torch_cuda(a):
                return a.to(torch.float64).contiguous()
            return torch.as_tensor(np.asarray(a, dtype=np.float64)).cuda().contiguous()

        sn, sf = dev(seed_n), dev(seed_f)
        nsh = self._nshells
        gW = np.zeros((self.ndom, nsh))
        gG = np.zeros(self.ndom)
        check(lib().scl_adjoint(self.h, ctypes.c_void_p(sn.data_ptr()) if sn is not None else None,
                                ctypes.c_void_p(sf.data_ptr()) if sf is not None else None, _dptr(gW), _dptr(gG)))
        return gW, gG

    def adjoint_populations(self):
        return self._get(lib().scl_get_adjoint_populations, self.Q * self.cells)

    def droplet_observables_vjp(self, centers, g_obs, is_bubble=None):
        """(seed_n [cells] host array, direct dL/dW [ndom, nshells], direct dL/dG [ndom])."""
        c = np.ascontiguousarray(np.asarray(centers, dtype=np.int32).reshape(self.ndom, 2))
        b = None
        if is_bubble is not None:
            b = np.ascontiguousarray(np.asarray(is_bubble, dtype=np.int8).reshape(self.ndom))
        g = np.ascontiguousarray(np.asarray(g_obs, dtype=np.float64).reshape(self.ndom, 6))
        seed = np.zeros(self.cells)
        gW = np.zeros((self.ndom, self._nshells))
        gG = np.zeros(self.ndom)
        check(lib().scl_droplet_observables_vjp(self.h, _dptr(c), _dptr(b) if b is not None else None, _dptr(g),
                                                _dptr(seed), 0, _dptr(gW), _dptr(gG)))
        return seed, gW, gG
