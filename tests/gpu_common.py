"""Shared helpers of the GPU parity tests: seeded flows, the GPU runner and
the oracle runner on identical FP32 inputs, and error metrics."""
import numpy as np

import oracle
from paper_2008_11520_amd import synth


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_max(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m = np.abs(b).max()
    return float(np.abs(a - b).max() / (m if m > 0 else 1.0))


# FP32 unit roundoff
EPS32 = 2.0 ** -24
# fine elements per side of a defect / rhs tile (tile-edge nodes are where
# neighbouring tiles' halos and staged edge nodes meet)
TILE_FINE = 32


def node_errors(got, ref, nx, ny, K, dirichlet, name="Dbar"):
    """Element-wise errors of a fine nodal field (Fn x 2): relative L2, max
    abs error over max |oracle| for all nodes, for the nodes on defect/rhs
    tile edges (fine index a multiple of 32), and the count of Dirichlet
    nodes where the GPU value is not exactly zero."""
    n = 1 << K
    NX, NY = nx * n, ny * n
    g = np.asarray(got, np.float64).reshape(NY + 1, NX + 1, 2)
    r = np.asarray(ref, np.float64).reshape(NY + 1, NX + 1, 2)
    mask = oracle.dirichlet_mask(nx, ny, K, dirichlet).reshape(NY + 1, NX + 1)
    edge = (np.arange(NX + 1)[None, :] % TILE_FINE == 0) | (np.arange(NY + 1)[:, None] % TILE_FINE == 0)
    m = np.abs(r).max()
    m = m if m > 0 else 1.0
    err = np.abs(g - r).max(axis=2)
    sel = edge & ~mask
    return {name: rel_l2(g, r), name + "_max": float(err.max() / m),
            name + "_edge_max": float(err[sel].max() / m) if sel.any() else 0.0,
            name + "_dirichlet_nonzero": int(np.count_nonzero(g[mask]))}


def step_errors(got, ref, h_ref, nx, ny, K, dirichlet):
    """Errors of one step's outputs: D-bar (element-wise, see node_errors),
    the per-patch outputs and the state (relative L2 and max-relative), and
    b_L (relative L2 and max-relative)."""
    e = node_errors(got["Dbar"], ref["Dbar"], nx, ny, K, dirichlet)
    for k, r in (("dpatch", ref.get("dpatch")), ("h", h_ref), ("bL", ref["bL"])):
        if r is None:
            continue
        e[k] = rel_l2(got[k], r)
        e[k + "_max"] = rel_max(got[k], r)
    return e


def merge_worst(worst, errs):
    for k, v in errs.items():
        worst[k] = max(worst.get(k, 0), v)
    return worst


def assert_step_errors(worst, tol, bl_tol):
    """The bound applies to relative L2 and to max-relative alike; D-bar is
    exactly zero at Dirichlet nodes."""
    assert worst["Dbar_dirichlet_nonzero"] == 0, worst
    for k in ("Dbar", "Dbar_max", "Dbar_edge_max", "dpatch", "dpatch_max", "h", "h_max"):
        if k in worst:
            assert worst[k] < tol, (k, worst)
    assert worst["bL"] < bl_tol and worst["bL_max"] < bl_tol, worst


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def make_gpu_flow(flow, K, H, Hm, nu, weights, precision="fp32", share=None, flags=None):
    """A GPU flow; by default it keeps its per-patch outputs (DNNMG_F_PATCH_OUTPUTS),
    so that the tests can compare them."""
    import paper_2008_11520_amd as pam
    if flags is None:
        flags = pam.DNNMG_F_PATCH_OUTPUTS
    cfg = pam.make_config(flow.nx, flow.ny, K, H, Hm, flow.dt, nu, precision, flow.dirichlet, flags)
    return pam.DnnMG(cfg, flow.cxy, None if share is not None else weights, share=share)


def make_oracle_flow(flow, K, H, Hm, nu, weights, theta=1.0):
    return oracle.OracleFlow(flow.nx, flow.ny, K, H, Hm, flow.dt, nu, flow.dirichlet,
                             flow.cxy, weights.astype(np.float64), theta=theta)


class GpuRunner:
    """Steps a GPU flow and reads back the correction, rhs and state."""

    def __init__(self, g):
        import torch
        self.g = g
        s = g.s
        self.dbar = torch.empty(2 * s["Fn"], dtype=torch.float32, device="cuda")
        self.bL = torch.empty(2 * s["Nc"], dtype=torch.float64, device="cuda")
        self.h = torch.empty(s["P"] * g.cfg.H, dtype=torch.float32, device="cuda")
        self.dp = torch.empty(s["P"] * s["nout"], dtype=torch.float32, device="cuda")

    def step(self, v, p):
        import torch
        import paper_2008_11520_amd as pam
        vd, pd = to_dev(v.reshape(-1)), to_dev(p.reshape(-1))
        self.g.step(vd, pd, self.dbar)
        self.g.restrict_rhs(self.bL)
        self.g.get_state(self.h, None)
        try:
            self.g.patch_output(self.dp)
            kept = True
        except pam.DnnmgError as e:
            # a one-launch step without DNNMG_F_PATCH_OUTPUTS keeps none
            assert e.code == pam.DNNMG_ESTATE, e
            kept = False
        torch.cuda.synchronize()
        s = self.g.s
        out = dict(Dbar=self.dbar.cpu().numpy().reshape(s["Fn"], 2).copy(),
                   bL=self.bL.cpu().numpy().reshape(s["Nc"], 2).copy(),
                   h=self.h.cpu().numpy().reshape(s["P"], -1).copy())
        if kept:
            out["dpatch"] = self.dp.cpu().numpy().reshape(s["P"], s["nout"]).copy()
        return out


def window(flow, i0, i1, j0, j1):
    """Sub-flow on coarse elements [i0,i1) x [j0,j1) of `flow` (for sampled
    comparisons at full size); Dirichlet flags only where the window touches
    the domain's own boundary."""
    g = flow.cxy
    sub = synth.Flow(i1 - i0, j1 - j0, g[j0:j1 + 1, i0:i1 + 1].copy(), 0, flow.dt, flow.fourier,
                     flow.inflow_max)
    d = 0
    if i0 == 0: d |= flow.dirichlet & synth.DIR_XMIN
    if i1 == flow.nx: d |= flow.dirichlet & synth.DIR_XMAX
    if j0 == 0: d |= flow.dirichlet & synth.DIR_YMIN
    if j1 == flow.ny: d |= flow.dirichlet & synth.DIR_YMAX
    sub.dirichlet = d
    return sub


def window_fields(flow, step, i0, i1, j0, j1):
    v, p = flow.fields(step)
    v = v.reshape(flow.ny + 1, flow.nx + 1, 2)[j0:j1 + 1, i0:i1 + 1].reshape(-1, 2)
    p = p.reshape(flow.ny + 1, flow.nx + 1)[j0:j1 + 1, i0:i1 + 1].reshape(-1)
    return np.ascontiguousarray(v), np.ascontiguousarray(p)


class OracleFineStep:
    """The oracle's fine step as the fine step of the closed DNN-MG loop
    (paper_2008_11520_amd.loop.run): coarse v, p in, b_L out (FP64)."""

    def __init__(self, flow, K, H, Hm, weights, nu, fp8=False, theta=1.0):
        self.o = oracle.OracleFlow(flow.nx, flow.ny, K, H, Hm, flow.dt, nu, flow.dirichlet, flow.cxy,
                                   np.asarray(weights, dtype=np.float64), fp8=fp8, theta=theta)

    def step(self, v, p):
        return self.o.step(np.asarray(v, np.float64), np.asarray(p, np.float64), want=("bL",))["bL"]
