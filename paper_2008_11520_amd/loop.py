"""The closed DNN-MG time loop (Algorithm 2) on one flow.

Per time step n:
  coarse:    the coarse Newton solve for (v_n, p_n) on level L with the
             right-hand side b_L of the previous step (coarse.CoarseNS);
  fine:      the fine step on level L+K (prolongation, defect, GRU + MLP
             correction, right-hand side of the corrected velocity, its
             restriction), whose b_L is the next coarse right-hand side.
The first coarse solve takes the coarse right-hand side of v_0,
(1/dt) M_L v_0 - (1 - theta) T_L(v_0) (no fine step before it).
Dirichlet values at step n are the flow's boundary values at t_n.

The fine step is an object with step(v, p) -> b_L (coarse (N, 2) arrays,
FP64); GpuFineStep drives the library.  The coarse solve runs on the host
and is timed apart from the fine step.
"""
from __future__ import annotations

import time

import numpy as np

from .coarse import CoarseNS


class GpuFineStep:
    """dnnmg_step + dnnmg_restrict_rhs on the device: the coarse fields go
    to the device as FP32, b_L comes back as FP64."""

    def __init__(self, flow, K, H, Hm, weights, nu, precision="fp32", theta=1.0):
        import torch
        from . import DNNMG_F_CRANK_NICOLSON, DnnMG, make_config
        if theta not in (1.0, 0.5):
            raise ValueError("theta must be 1 (implicit Euler) or 1/2 (Crank-Nicolson)")
        flags = DNNMG_F_CRANK_NICOLSON if theta == 0.5 else 0
        self.g = DnnMG(make_config(flow.nx, flow.ny, K, H, Hm, flow.dt, nu, precision, flow.dirichlet, flags),
                       flow.cxy, weights)
        nc = (flow.nx + 1) * (flow.ny + 1)
        self.v = torch.empty(2 * nc, dtype=torch.float32, device="cuda")
        self.p = torch.empty(nc, dtype=torch.float32, device="cuda")
        self.b = torch.empty(2 * nc, dtype=torch.float64, device="cuda")
        self.seconds = 0.0

    def step(self, v, p):
        import torch
        t0 = time.perf_counter()
        self.v.copy_(torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32).reshape(-1)))
        self.p.copy_(torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32).reshape(-1)))
        self.g.step(self.v, self.p)
        self.g.restrict_rhs(self.b)
        out = self.b.cpu().numpy().reshape(-1, 2)
        self.seconds += time.perf_counter() - t0
        return out

    def close(self):
        self.g.close()


def boundary_values(flow, n):
    """The flow's coarse velocity at t_n (its Dirichlet values on the
    Dirichlet sides)."""
    v, _ = flow.fields(n)
    return v.astype(np.float64)


def run(flow, nu, steps, fine=None, coarse=None, theta=1.0):
    """Run `steps` DNN-MG time steps of `flow` (a synth.Flow) with the time
    scheme's weight theta (1 implicit Euler, 1/2 Crank-Nicolson; the fine
    step must use the same).  fine=None runs the coarse solver alone (b the
    coarse right-hand side of v_{n-1}: plain coarse multigrid in the paper's
    comparison).  Returns the coarse velocities and pressures per step, the
    Newton step counts and the coarse-solve time."""
    ns = coarse if coarse is not None else CoarseNS(flow.cxy, flow.dt, nu, flow.dirichlet, theta=theta)
    v = boundary_values(flow, 0)
    p = np.zeros(ns.N)
    b = ns.rhs_of(v)
    vs, ps, newton = [], [], []
    t_coarse = 0.0
    for n in range(1, steps + 1):
        t0 = time.perf_counter()
        v, p, it = ns.solve(b, boundary_values(flow, n), v, p)
        t_coarse += time.perf_counter() - t0
        vs.append(v.copy())
        ps.append(p.copy())
        newton.append(it)
        # the fine step's coarse inputs are FP32 (the library's boundary)
        vf, pf = v.astype(np.float32), p.astype(np.float32)
        b = fine.step(vf, pf) if fine is not None else ns.rhs_of(v)
    return dict(v=np.array(vs), p=np.array(ps), newton=newton, coarse_s=t_coarse)
