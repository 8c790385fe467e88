"""Device-side helpers around a Plan: uploads a system's inputs into HBM as
torch tensors (torch provides memory and streams only) and runs solves."""
from __future__ import annotations

import numpy as np

from . import _lib as L
from .synth import soa


class DeviceSystem:
    """Inputs and outputs of one system resident on the current GPU."""

    def __init__(self, sysm, device="cuda"):
        import torch
        self.torch = torch
        self.n_atoms = sysm.n_atoms
        self.n_constraints = sysm.n_constraints
        self.r = torch.from_numpy(soa(sysm.r)).to(device)
        self.mass = torch.from_numpy(np.ascontiguousarray(sysm.mass, dtype=np.float64)).to(device)
        self.r_out = torch.empty_like(self.r)
        self.lam = torch.zeros(max(1, sysm.n_constraints), dtype=torch.float64, device=device)[:sysm.n_constraints]
        self.device = device

    def alloc_status(self, n_molecules):
        torch = self.torch
        self.iters = torch.zeros(max(1, n_molecules), dtype=torch.int32, device=self.device)
        self.status = torch.zeros(max(1, n_molecules), dtype=torch.int32, device=self.device)
        return self

    def upload_ru(self, r_u_aos):
        return self.torch.from_numpy(soa(r_u_aos)).to(self.device)


def solve_once(sysm, r_u, tol=1e-12, precision=L.PREC_FP64, variant=L.VARIANT_NEWTON, max_iter=0,
               lam0=None, plan=None, warm=None, **plan_kw):
    """Plans (unless given), uploads, solves once, and returns host arrays."""
    import torch
    own = plan is None
    if own:
        plan = L.Plan(sysm.n_atoms, sysm.pairs, sysm.d, **plan_kw)
    ds = DeviceSystem(sysm).alloc_status(plan.n_molecules)
    ru = ds.upload_ru(r_u)
    warm = L.WARM_ZERO if warm is None else warm
    if lam0 is not None:
        ds.lam.copy_(torch.from_numpy(np.asarray(lam0, dtype=np.float64)))
        warm = L.WARM_CALLER
    plan.solve(ds.r, ru, ds.mass, tol, ds.r_out, ds.lam, ds.iters, ds.status, precision=precision,
               variant=variant, warm_start=warm, max_iter=max_iter)
    torch.cuda.synchronize()
    out = {"r_out": ds.r_out.cpu().numpy().T.copy(), "lam": ds.lam.cpu().numpy().copy(),
           "iters": ds.iters[:plan.n_molecules].cpu().numpy().copy(),
           "status": ds.status[:plan.n_molecules].cpu().numpy().copy(), "plan": plan}
    return out
