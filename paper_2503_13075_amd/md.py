"""Constrained leapfrog around the device solve (the Verlet scheme of the
main text's section on constrained dynamics, Eqs. (nonlinear:1a)-(1c)):

    v_{k+1/2} = v_{k-1/2} + h M^-1 f_k,   r_u = r_k + h v_{k+1/2}
    r_{k+1}   = r_u - M^-1 G(r_k)^T lambda  with g(r_{k+1}) = 0   (the solve)
    v_{k+1/2} = (r_{k+1} - r_k) / h

Every step runs in the library's kernels (kick/drift, solve, finish); this
module only holds the device buffers and the order of the calls.  Forces are
the caller's (a device tensor, or a callable returning one).  The solve of a
step may start from lambda = 0, from each constraint's decoupled solution, or
from the previous step's multipliers (which change little from one step to
the next; the first step then starts from 0).
"""
from __future__ import annotations

import numpy as np

from . import _lib as L
from .synth import System, soa


class ConstrainedLeapfrog:
    def __init__(self, sysm: System, v0: np.ndarray, h: float, tol: float = 1e-12, precision: int = L.PREC_FP64,
                 variant: int = L.VARIANT_NEWTON, device: str = "cuda", plan: L.Plan = None, warm: str = "zero"):
        import torch
        self.torch = torch
        self.sysm = sysm
        self.h = float(h)
        self.tol = float(tol)
        self.precision = precision
        self.variant = variant
        if warm not in ("zero", "decoupled", "previous"):
            raise ValueError("warm must be 'zero', 'decoupled' or 'previous'")
        self.warm = warm
        self.steps = 0
        self.plan = plan or L.Plan(sysm.n_atoms, sysm.pairs, sysm.d)
        dev = device
        self.r = torch.from_numpy(soa(sysm.r)).to(dev)
        self.v = torch.from_numpy(soa(np.asarray(v0, dtype=np.float64))).to(dev)
        self.mass = torch.from_numpy(np.ascontiguousarray(sysm.mass, dtype=np.float64)).to(dev)
        self.r_u = torch.empty_like(self.r)
        self.r_new = torch.empty_like(self.r)
        nm = max(1, self.plan.n_molecules)
        self.lam = torch.zeros(max(1, sysm.n_constraints), dtype=torch.float64, device=dev)[:sysm.n_constraints]
        self.iters = torch.zeros(nm, dtype=torch.int32, device=dev)
        self.status = torch.zeros(nm, dtype=torch.int32, device=dev)
        self.worst = torch.zeros(nm, dtype=torch.int32, device=dev)

    def step(self, f, stream=None):
        """One step with forces f (device tensor [3, n_atoms]); the status of
        every solve is folded into ``worst`` (elementwise maximum)."""
        torch = self.torch
        L.md_kick_drift(self.r, self.v, f, self.mass, self.h, self.r_u, stream)
        warm = {"zero": L.WARM_ZERO, "decoupled": L.WARM_DECOUPLED,
                "previous": L.WARM_CALLER if self.steps > 0 else L.WARM_ZERO}[self.warm]
        self.plan.solve(self.r, self.r_u, self.mass, self.tol, self.r_new, self.lam, self.iters, self.status,
                        precision=self.precision, variant=self.variant, warm_start=warm, stream=stream)
        self.steps += 1
        L.md_finish(self.r, self.r_new, self.h, self.v, stream)
        torch.maximum(self.worst, self.status, out=self.worst)

    def state(self):
        """Host copies (AoS) of positions and half-step velocities."""
        return self.r.cpu().numpy().T.copy(), self.v.cpu().numpy().T.copy()

    def tangent_velocities(self, stream=None):
        """The current half-step velocities projected onto the tangent space of
        the constraints at the current positions (RATTLE's velocity
        constraint, ilves_project_velocities); returns the device tensor
        [3, n_atoms] and the per-molecule status."""
        torch = self.torch
        if not hasattr(self, "v_tan"):
            self.v_tan = torch.empty_like(self.v)
            self.mu = torch.zeros_like(self.lam)
            self.p_iters = torch.zeros_like(self.iters)
            self.p_status = torch.zeros_like(self.status)
        self.plan.project_velocities(self.r, self.v, self.mass, 1e-12, self.v_tan, self.mu, self.p_iters,
                                     self.p_status, precision=self.precision, stream=stream)
        return self.v_tan, self.p_status


def pendulum(length: float = 1.0, mass: float = 1.0, pivot_mass: float = 1e20, v0: float = 1.0):
    """The simple pendulum of the supplement's table: bob of mass 1 at the
    origin hanging from a pivot at (0, length), initial velocity (v0, 0).
    The pivot is an atom of huge mass that receives no force, so it stays
    put.  Returns (System, v0 [2, 3], force [2, 3] for gravity g)."""
    r = np.array([[0.0, length, 0.0], [0.0, 0.0, 0.0]])
    sm = System(pairs=np.array([[0, 1]], np.int32), d=np.array([length]), mass=np.array([pivot_mass, mass]),
                r=r, kind=np.zeros(1, np.int8), elem=["X", "X"])
    v = np.array([[0.0, 0.0, 0.0], [v0, 0.0, 0.0]])
    return sm, v


def gravity(sysm: System, g: float, fixed=()) -> np.ndarray:
    """Force -m g y^ on every atom except the fixed ones (AoS [n, 3])."""
    f = np.zeros((sysm.n_atoms, 3))
    f[:, 1] = -sysm.mass * g
    for i in fixed:
        f[i] = 0.0
    return f
