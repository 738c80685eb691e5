"""Differentiable droplet observables: torch.autograd.Function over the library's adjoint.

forward(W, G): runs the checkpointed forward on the GPU and returns the droplet observables
(dP, C_d, R_s, sigma_s, R_e, delta) of every domain. backward: the observables' vector-
Jacobian product (explicit dependence on W and G plus dL/dn of the final state), then the
adjoint through the time loop. All the arithmetic runs in libscl; this file only marshals.
"""
from __future__ import annotations

import numpy as np
import torch

from .lattice import Lattice


class DropletProblem:
    """A batch of droplet (or bubble) domains run for a fixed number of steps.

    dims: list of square (L, L); n0: concatenated initial densities; centers: (ndom, 2);
    codes: shell codes; tau: per-domain relaxation times; psi_kind / psi_param as in scl.h;
    force_squared: A of the F^2 part of the Guo tensor (per domain or scalar, default 0).
    equilibrate: if > 0, the first load() relaxes n0 for that many steps with the parameters
    it is given, and that state becomes the fixed initial state of every later run, so the
    differentiated window starts from a droplet at mechanical equilibrium.
    """

    def __init__(self, dims, n0, centers, codes, tau, nsteps, every, precision, is_bubble=None,
                 psi_kind=0, psi_param=None, stream=None, equilibrate=0, force_squared=0.0):
        self.lat = Lattice(dims, precision, stream=stream)
        self.n0 = np.ascontiguousarray(n0, dtype=np.float64)
        self.centers = np.asarray(centers, dtype=np.int32)
        self.codes = list(codes)
        self.tau = np.broadcast_to(np.asarray(tau, dtype=np.float64), (self.lat.ndom,)).copy()
        self.nsteps, self.every = int(nsteps), int(every)
        self.is_bubble = is_bubble
        self.psi_kind, self.psi_param = psi_kind, psi_param
        self.equilibrate = int(equilibrate)
        self.force_squared = force_squared
        self.f0 = None

    def load(self, W, G):
        """Set the parameters and the initial state of the differentiated window."""
        lat = self.lat
        lat.set_physics(self.tau, G, self.psi_kind, self.psi_param)
        lat.set_force_squared(self.force_squared)
        lat.set_stencil(self.codes, W)
        lat.init_density(self.n0)
        if self.equilibrate > 0:
            if self.f0 is None:
                lat.step(self.equilibrate)
                self.f0 = lat.populations()
            lat.set_populations(self.f0)

    def forward(self):
        """Checkpointed forward of the window, then the observables of its final state."""
        self.lat.checkpointed_forward(self.nsteps, self.every)
        return self.lat.droplet_observables(self.centers, self.is_bubble)

    def run(self, W, G):
        self.load(W, G)
        return self.forward()

    def vjp(self, g_obs):
        seed, gW_direct, gG_direct = self.lat.droplet_observables_vjp(self.centers, g_obs, self.is_bubble)
        gW, gG = self.lat.adjoint(seed_n=seed)
        return gW + gW_direct, gG + gG_direct


class DropletObservables(torch.autograd.Function):
    """obs = DropletObservables.apply(W, G, problem); W: (ndom, nshells), G: (ndom,) float64."""

    @staticmethod
    def forward(ctx, W, G, problem):
        ctx.problem = problem
        obs = problem.run(W.detach().cpu().numpy(), G.detach().cpu().numpy())
        return torch.as_tensor(obs, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g_obs):
        gW, gG = ctx.problem.vjp(g_obs.detach().cpu().numpy())
        return torch.as_tensor(gW, dtype=torch.float64), torch.as_tensor(gG, dtype=torch.float64), None
