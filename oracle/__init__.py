"""Oracle for the Shan-Chen extended-stencil lattice Boltzmann step (arXiv 2505.23647).

TEST INFRASTRUCTURE ONLY: a plain, slow FP64 CPU reference. Only the tests, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product library never does, and
the two share no code. See ``sc_oracle.cpp`` for the equations each routine follows.

Sub-modules:
  * ``stencil_algebra`` - exact-rational forcing-stencil algebra (moments, isotropy and
    anisotropy coefficients, projected pressure-tensor coefficients, knobs).
  * ``thermo`` - bulk thermodynamics of the Shan-Chen fluid (critical coupling, coexistence).
  * ``flat`` - flat-interface observables (sigma_0, z_s, z_e, Tolman length, analytic estimates).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

PSI_EXP, PSI_EPS, PSI_CLASSIC = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the C++ oracle with g++ (plain FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", _SRC, "-o", _LIB_PATH + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def velset(d: int):
    """Return (xi [Q,3] int, w [Q] float) of D2Q9 (d=2) or D3Q19 (d=3)."""
    xi = np.zeros((27, 3), dtype=np.int32)
    w = np.zeros(27)
    q = lib().orc_velset(d, _ip(xi), _dp(w))
    return xi[:q].copy(), w[:q].copy()


def stencil(d: int, codes):
    """Forcing vectors of the given shell codes: (e [N,3] int, shell_index [N] int)."""
    codes = np.ascontiguousarray(codes, dtype=np.int32)
    cap = 1024
    e = np.zeros((cap, 3), dtype=np.int32)
    sh = np.zeros(cap, dtype=np.int32)
    m = lib().orc_stencil(d, len(codes), _ip(codes), cap, _ip(e), _ip(sh))
    if m < 0:
        raise ValueError(f"unknown shell code in {codes.tolist()} for d={d}")
    return e[:m].copy(), sh[:m].copy()


class Sim:
    """A single periodic domain advanced by the oracle.

    ``dims`` is (nx, ny) or (nx, ny, nz); arrays are indexed [z][y][x] with x fastest.
    Populations are stored as ``f[Q, N]`` in the order given by :func:`velset`.
    """

    def __init__(self, dims, tau, G, codes, W, psi_kind=PSI_EXP, psi_param=0.0, force_squared=0.0):
        dims = tuple(int(v) for v in dims)
        self.d = len(dims)
        self.nx, self.ny = dims[0], dims[1]
        self.nz = dims[2] if self.d == 3 else 1
        self.N = self.nx * self.ny * self.nz
        self.tau, self.G = float(tau), float(G)
        self.codes = np.ascontiguousarray(codes, dtype=np.int32)
        self.W = np.ascontiguousarray(W, dtype=np.float64)
        self.kind, self.p = int(psi_kind), float(psi_param)
        self.aF = float(force_squared)  # A of T = 2uF - (A/tau) FF (0: the paper's Guo forcing)
        self.xi, self.w = velset(self.d)
        self.Q = len(self.w)
        self.f = np.zeros((self.Q, self.N))

    def init_density(self, n0):
        n0 = np.ascontiguousarray(np.asarray(n0, dtype=np.float64).reshape(-1))
        assert n0.size == self.N
        lib().orc_init(self.d, self.nx, self.ny, self.nz, _dp(n0), _dp(self.f))
        return self

    def run(self, nsteps: int) -> int:
        """Advance ``nsteps``; returns 0, or 5 if the mass became non-finite."""
        L = lib()
        L.orc_run.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double] * 3 + [ctypes.c_int, ctypes.c_double,
                              ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long]
        self.f = np.ascontiguousarray(self.f)
        return L.orc_run(self.d, self.nx, self.ny, self.nz, self.tau, self.aF, self.G, self.kind, self.p,
                         len(self.codes), self.codes.ctypes.data, self.W.ctypes.data, self.f.ctypes.data,
                         int(nsteps))

    def fields(self):
        """Return dict of n [N], j [N,3], psi [N], F [N,3], u [N,3] for the current state."""
        L = lib()
        L.orc_fields.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_int] + [ctypes.c_void_p] * 8
        n = np.zeros(self.N); psi = np.zeros(self.N)
        j = np.zeros((self.N, 3)); F = np.zeros((self.N, 3)); u = np.zeros((self.N, 3))
        rc = L.orc_fields(self.d, self.nx, self.ny, self.nz, self.G, self.kind, self.p, len(self.codes),
                          self.codes.ctypes.data, self.W.ctypes.data, self.f.ctypes.data, n.ctypes.data,
                          j.ctypes.data, psi.ctypes.data, F.ctypes.data, u.ctypes.data)
        assert rc == 0
        return {"n": n, "j": j, "psi": psi, "F": F, "u": u}

    def pressure_tensor(self):
        """Lattice pressure tensor (d=2): array [3, N] of (Pxx, Pyy, Pxy)."""
        assert self.d == 2
        L = lib()
        L.orc_ptensor2d.argtypes = [ctypes.c_int] * 2 + [ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int] + [ctypes.c_void_p] * 4
        out = np.zeros((3, self.N))
        rc = L.orc_ptensor2d(self.nx, self.ny, self.G, self.kind, self.p, len(self.codes),
                             self.codes.ctypes.data, self.W.ctypes.data, self.f.ctypes.data, out.ctypes.data)
        assert rc == 0
        return out

    def pressure_tensor_general(self):
        """Lattice pressure tensor by the link-sharing rule, d = 2 or 3: [6, N] planes
        (xx, yy, zz, xy, xz, yz)."""
        L = lib()
        L.orc_ptensor.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int] + [ctypes.c_void_p] * 4
        out = np.zeros((6, self.N))
        rc = L.orc_ptensor(self.d, self.nx, self.ny, self.nz, self.G, self.kind, self.p, len(self.codes),
                           self.codes.ctypes.data, self.W.ctypes.data, self.f.ctypes.data, out.ctypes.data)
        assert rc == 0
        return out

    def droplet_observables3d(self, center, bubble=False):
        """(dP, C_d, R_s, sigma_s, R_e, delta) of the current state (d=3, cubic domain)."""
        L = lib()
        L.orc_droplet_obs3d.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int] + [ctypes.c_void_p] * 3 + [ctypes.c_int] * 4 + [ctypes.c_void_p]
        out = np.zeros(6)
        assert self.d == 3 and self.nx == self.ny == self.nz
        rc = L.orc_droplet_obs3d(self.nx, self.G, self.kind, self.p, len(self.codes), self.codes.ctypes.data,
                                 self.W.ctypes.data, self.f.ctypes.data, int(center[0]), int(center[1]),
                                 int(center[2]), int(bool(bubble)), out.ctypes.data)
        assert rc == 0
        return out

    def droplet_observables(self, center, bubble=False):
        """(dP, C_d, R_s, sigma_s, R_e, R_e - R_s) of the current state (d=2, square domain)."""
        L = lib()
        L.orc_droplet_obs2d.argtypes = [ctypes.c_int] * 2 + [ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int] + [ctypes.c_void_p] * 3 + [ctypes.c_int] * 3 + [ctypes.c_void_p]
        out = np.zeros(6)
        rc = L.orc_droplet_obs2d(self.nx, self.ny, self.G, self.kind, self.p, len(self.codes),
                                 self.codes.ctypes.data, self.W.ctypes.data, self.f.ctypes.data,
                                 int(center[0]), int(center[1]), int(bool(bubble)), out.ctypes.data)
        assert rc == 0
        return out


def droplet_tangent_linear(dims, tau, G, codes, W, n0, nsteps, center, bubble=False,
                           psi_kind=PSI_EXP, psi_param=0.0, force_squared=0.0):
    """Forward-mode (dual-number) run of the plain step loop from f = w n0.

    Returns (obs[6], jac[6, nshells+1]) where jac holds d obs / d (W_0..W_{k-1}, G).
    """
    nx, ny = int(dims[0]), int(dims[1])
    codes = np.ascontiguousarray(codes, dtype=np.int32)
    W = np.ascontiguousarray(W, dtype=np.float64)
    n0 = np.ascontiguousarray(np.asarray(n0, dtype=np.float64).reshape(-1))
    L = lib()
    L.orc_droplet_tl2d.argtypes = [ctypes.c_int] * 2 + [ctypes.c_double] * 3 + [ctypes.c_int, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p]
    obs = np.zeros(6)
    jac = np.zeros((6, len(codes) + 1))
    rc = L.orc_droplet_tl2d(nx, ny, float(tau), float(force_squared), float(G), int(psi_kind), float(psi_param), len(codes),
                            codes.ctypes.data, W.ctypes.data, n0.ctypes.data, int(nsteps), int(center[0]),
                            int(center[1]), int(bool(bubble)), obs.ctypes.data, jac.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle tangent-linear run failed ({rc})")
    return obs, jac


def num_threads() -> int:
    """Threads used by the oracle's OpenMP loops."""
    return int(lib().orc_num_threads())
