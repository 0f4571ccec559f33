"""Gradient of the final transfer fidelity with respect to the guide profile.

The quantity is the final population of the target guide (Morgan et al.,
arXiv:1309.2451, Sec. V and Fig. 6: fidelity of the transfer into the right
guide).  The two moving guides follow x_g(z) = sum_m c_gm B_m(z) with M
clamped cubic B-splines over the z box; the middle guide is fixed.

Forward: real-time steps with checkpoints every `every` steps
(ssf_step_ckpt), then F = P3 of the last state.  Backward: for each segment
from the last to the first, the states are recomputed from the checkpoint
(ssf_step_seq, bitwise identical to the forward run) and the adjoint walks
the segment backwards (ssf_adjoint_segment), accumulating dF/dx_g(z) on the
device; ssf_profile_grad applies the B-spline chain rule.  Everything runs
in libssf; this module only allocates buffers and sequences the calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Solver, bspline_basis, bspline_eval


class FidelityProblem:
    """Holds the solver, the fixed initial state and the buffers of one
    gradient computation.

    solver   Solver with the grid (and storage type) to use
    psi0     initial state (torch tensor on the solver's device), held fixed
    v0, sigma  depths and widths of the three guides
    x_mid    (Nz,) centre of the fixed middle guide
    M        B-spline functions per moving guide; zrange = (a, b)
    moving   indices of the guides whose centres are parameterised
    """

    def __init__(self, solver: Solver, psi0, v0, sigma, x_mid, M, zrange, x_lo, x_hi, dt, nsteps, every,
                 moving=(0, 2)):
        torch = solver.torch
        self.s = solver
        self.torch = torch
        self.psi0 = psi0
        self.v0 = np.asarray(v0, dtype=np.float64)
        self.sigma = np.asarray(sigma, dtype=np.float64)
        self.x_mid = np.asarray(x_mid, dtype=np.float64)
        self.M = int(M)
        self.moving = tuple(moving)
        self.dt = float(dt)
        self.nsteps = int(nsteps)
        self.every = int(every)
        z = solver.lo[2] + np.arange(solver.n[2]) * (solver.hi[2] - solver.lo[2]) / solver.n[2]
        self.z = z
        self.zrange = (float(zrange[0]), float(zrange[1]))
        self.B = bspline_basis(self.M, zrange[0], zrange[1], z)               # (Nz, M), host
        self.B_dev = torch.from_numpy(self.B).to(solver.device).contiguous()
        solver.set_partition(x_lo, x_hi)
        self.nseg = -(-self.nsteps // self.every)
        self.ckpt = solver.empty(self.nseg)
        self.seq = solver.empty(self.every + 1)
        self.psi = solver.empty()
        self.lam = solver.empty()
        self.G = torch.zeros(3 * solver.n[2], dtype=torch.float64, device=solver.device)
        self.grad3 = torch.zeros(3 * self.M, dtype=torch.float64, device=solver.device)

    def profile(self, coeffs):
        """(3, Nz) guide centres for coefficients of shape (len(moving), M)."""
        c = np.asarray(coeffs, dtype=np.float64).reshape(len(self.moving), self.M)
        prof = bspline_eval(self.M, self.zrange[0], self.zrange[1], c, self.z)   # the library's map
        xc = np.zeros((3, self.s.n[2]))
        xc[1] = self.x_mid
        for k, g in enumerate(self.moving):
            xc[g] = prof[k]
        return xc

    def forward(self, coeffs) -> float:
        self.s.set_guides(self.v0, self.sigma, self.profile(coeffs))
        self.psi.copy_(self.psi0)
        self.s.step_ckpt(self.psi, self.nsteps, self.dt, self.every, self.ckpt)
        return float(self.s.observables(self.psi)["pop"][2])

    def backward(self):
        """dF/dc, shape (len(moving), M), after forward() with the same coefficients."""
        s = self.s
        s.adjoint_init(self.psi, self.lam)
        self.G.zero_()
        for k in reversed(range(self.nseg)):
            steps = min(self.every, self.nsteps - k * self.every)
            s.step_seq(self.ckpt[k], steps, self.dt, self.seq)
            s.adjoint_segment(self.lam, self.seq, steps, self.dt, self.G)
        s.profile_grad(self.G, self.B_dev, 3, self.grad3)
        g = self.grad3.view(3, self.M)
        return g[list(self.moving)].clone()

    def dF_dxc(self):
        """dF/dx_g(z) of the last backward(), shape (3, Nz)."""
        return self.G.view(3, self.s.n[2]).clone()


class FidelityFn(torch.autograd.Function):
    """F = FidelityFn.apply(coeffs, problem): final target-guide population;
    F.backward() gives coeffs.grad through the adjoint split-step."""

    @staticmethod
    def forward(ctx, coeffs, problem):
        ctx.problem = problem
        ctx.shape = coeffs.shape
        F = problem.forward(coeffs.detach().cpu().numpy())
        return torch.tensor(F, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gF):
        g = ctx.problem.backward().to(gF.device).reshape(ctx.shape)
        return gF * g, None
