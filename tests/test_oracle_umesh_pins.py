"""Pins of the oracle's unstructured-mesh step (explicit connectivity,
isoparametric refinement of curved edges) against the structured oracle
(itself pinned), the mesh's topology and closed forms.

* A structured mesh handed over as an unstructured one -- elements in
  shuffled order, nodes renumbered, each element's corners cyclically
  rotated -- gives the same prolongation, defect, mass products and restricted
  right-hand side at the same fine points; without the rotation (the patch's
  local node order is then the structured one) the whole step, network
  included, is the same.
* Counts: Fn = Nc + E (n - 1) + P (n - 1)^2 with E from Euler's formula.
* Curved edges: their fine nodes lie on the circle; the fine mesh's area
  (the mass matrix's total) converges to the exact area at second order.
* The affine exact Navier-Stokes solution has zero defect at every interior
  fine node of the (straight) O-grid mesh with its five-element vertices.
* Duplicate averaging divides by the number of patches that hold a node.
"""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from paper_2008_11520_amd import synth


def _match(a, b, tol=1e-12):
    """Index into b of every point of a (same point set)."""
    d, idx = cKDTree(b).query(a)
    assert d.max() <= tol, d.max()
    assert len(set(idx.tolist())) == len(idx)
    return idx


def _structured(nx=6, ny=4, seed=7):
    flow = synth.channel_flow(nx, ny, 3, 0.005, perturb_seed=seed)
    return flow


@pytest.mark.parametrize("K", [1, 2, 3])
def test_counts_follow_euler(K):
    n = 1 << K
    for mesh, holes in ((synth.structured_as_umesh(synth.rect_mesh(5, 3), 15)[0], 0),
                        (synth.cylinder_channel_umesh(4), 1)):
        f = oracle.UFine(mesh, K)
        assert f.E == f.nc + f.ne - 1 + holes
        assert f.Fn == f.nc + f.E * (n - 1) + f.ne * (n - 1) ** 2
        # every fine node is used, each patch's nodes are distinct
        assert np.array_equal(np.unique(f.pmap), np.arange(f.Fn))
        assert all(len(set(r.tolist())) == f.nf for r in f.pmap)


@pytest.mark.parametrize("K", [1, 2])
def test_structured_mesh_as_unstructured_operators(K):
    flow = _structured()
    nx, ny = flow.nx, flow.ny
    cxy = flow.cxy.reshape(-1, 2)
    mesh, order, rot, perm = synth.structured_as_umesh(flow.cxy, flow.dirichlet, order_seed=1, rotate_seed=2,
                                                       renumber_seed=3)
    f = oracle.UFine(mesh, K)
    sfxy = oracle.fine_coords(nx, ny, K, cxy)
    m = _match(sfxy, f.fxy)                      # structured fine node -> unstructured index
    v, p = flow.fields(2)
    vu, pu = np.empty_like(v, dtype=np.float64), np.empty_like(p, dtype=np.float64)
    vu[perm], pu[perm] = v, p
    pv = oracle.prolong(nx, ny, K, v.astype(np.float64))
    pvu = f.prolong(vu)
    assert np.abs(pvu[m] - pv).max() <= 1e-14 * np.abs(pv).max()
    pp = oracle.prolong(nx, ny, K, p.astype(np.float64))
    rng = np.random.default_rng(4)
    up = rng.standard_normal(pv.shape)
    upu = np.empty_like(up)
    upu[m] = up
    D = oracle.defect(nx, ny, K, cxy, pv, pp, up, flow.dt, 1e-3, flow.dirichlet)
    ppu = np.empty_like(pp)
    ppu[m] = pp
    pvu2 = np.empty_like(pv)
    pvu2[m] = pv
    Du = f.defect(pvu2, ppu, upu, flow.dt, 1e-3)
    assert np.array_equal(f.mask[m], oracle.dirichlet_mask(nx, ny, K, flow.dirichlet))
    assert np.abs(Du[m] - D).max() <= 1e-12 * np.abs(D).max()
    Mu = f.mass_apply(upu)
    Ms = oracle.mass_apply(nx, ny, K, cxy, up)
    assert np.abs(Mu[m] - Ms).max() <= 1e-13 * np.abs(Ms).max()
    dbar = 0.2 * rng.standard_normal(pv.shape)
    dbu = np.empty_like(dbar)
    dbu[m] = dbar
    b = oracle.rhs_restrict(nx, ny, K, cxy, v.astype(np.float64), dbar, flow.dt)
    bu = f.rhs_restrict(vu, dbu, flow.dt)
    assert np.abs(bu[perm] - b).max() <= 1e-12 * np.abs(b).max()
    # R = P^T: <R x, y> = <x, P y>
    x, y = rng.standard_normal((f.Fn, 2)), rng.standard_normal((f.nc, 2))
    assert abs(np.sum(f.restrict(x) * y) - np.sum(x * f.prolong(y))) <= 1e-12 * np.abs(x).sum()


@pytest.mark.parametrize("K,Hm", [(1, 0), (2, 16)])
def test_structured_mesh_as_unstructured_full_step(K, Hm):
    flow = _structured()
    nx, ny = flow.nx, flow.ny
    H = 16
    w = synth.xavier_weights(K, H, Hm, 9).astype(np.float64)
    mesh, order, rot, perm = synth.structured_as_umesh(flow.cxy, flow.dirichlet, order_seed=5, renumber_seed=6)
    ou = oracle.OracleUFlow(mesh, K, H, Hm, flow.dt, 1e-3, w)
    os_ = oracle.OracleFlow(nx, ny, K, H, Hm, flow.dt, 1e-3, flow.dirichlet, flow.cxy, w)
    m = _match(oracle.fine_coords(nx, ny, K, flow.cxy.reshape(-1, 2)), ou.f.fxy)
    for n in range(3):
        v, p = flow.fields(n)
        vu, pu = np.empty_like(v), np.empty_like(p)
        vu[perm], pu[perm] = v, p
        rs = os_.step(v, p, want=("Dbar", "bL", "dpatch"))
        ru = ou.step(vu, pu, want=("Dbar", "bL", "dpatch"))
        assert np.abs(ru["Dbar"][m] - rs["Dbar"]).max() <= 1e-11 * max(np.abs(rs["Dbar"]).max(), 1e-300)
        assert np.abs(ru["bL"][perm] - rs["bL"]).max() <= 1e-11 * np.abs(rs["bL"]).max()
        assert np.abs(ru["dpatch"][order] - rs["dpatch"]).max() <= 1e-11 * np.abs(rs["dpatch"]).max()
        assert np.abs(ou.h[order] - os_.h).max() <= 1e-11


@pytest.mark.parametrize("K", [1, 2, 3])
def test_curved_edges_put_fine_nodes_on_the_circle(K):
    mesh = synth.cylinder_channel_umesh(4)
    f = oracle.UFine(mesh, K)
    cx, cy, r = mesh.circles[0]
    n = 1 << K
    on = set()
    for e, el in enumerate(mesh.elems):
        ends = [(el[0], el[1]), (el[1], el[2]), (el[3], el[2]), (el[0], el[3])]
        for k, (a, b) in enumerate(ends):
            if any({a, b} == {c[0], c[1]} for c in mesh.curved):
                for t in range(n + 1):
                    aa = t if k in (0, 2) else (n if k == 1 else 0)
                    bb = t if k in (1, 3) else (n if k == 2 else 0)
                    on.add(int(f.pmap[e, bb * (n + 1) + aa]))
    on = np.array(sorted(on))
    assert on.size == len(mesh.curved) * n
    d = np.hypot(f.fxy[on, 0] - cx, f.fxy[on, 1] - cy)
    assert np.abs(d - r).max() <= 1e-15
    assert f.mask[on].all()


def test_curved_mesh_area_converges_at_second_order():
    mesh = synth.cylinder_channel_umesh(4)
    exact = synth.CHANNEL_LX * synth.CHANNEL_LY - math.pi * mesh.circles[0][2] ** 2
    errs = []
    for K in (1, 2, 3):
        f = oracle.UFine(mesh, K)
        area = f.mass_apply(np.ones((f.Fn, 2)))[:, 0].sum()
        errs.append(area - exact)
    # the polygon through points on the circle lies inside the disc: too large
    assert all(e > 0 for e in errs)
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0
    f = oracle.UFine(mesh, 2)
    assert np.abs(f.prolong(np.ones(f.nc)) - 1.0).max() <= 1e-15


@pytest.mark.parametrize("K", [1, 2])
def test_affine_solution_has_zero_interior_defect_on_the_ogrid(K):
    mesh = synth.cylinder_channel_umesh(4)
    mesh.curved = np.zeros((0, 3), dtype=np.int32)      # straight ring edges: the affine space is exact
    f = oracle.UFine(mesh, K)
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    al, be, de = 0.3, 0.7, -0.2
    v = np.stack([al + be * (x + y), de - be * (x + y)], axis=1)
    p = -be * (al + de) * (x - y)
    pv, pp = f.prolong(v), f.prolong(p)
    D = f.defect(pv, pp, pv, 0.01, 1e-3)
    # interior fine nodes: not on an edge that only one element holds
    n = 1 << K
    cnt = {}
    for el in mesh.elems:
        for a, b in ((el[0], el[1]), (el[1], el[2]), (el[3], el[2]), (el[0], el[3])):
            key = (min(a, b), max(a, b))
            cnt[key] = cnt.get(key, 0) + 1
    bnd = np.zeros(f.Fn, dtype=bool)
    for e, el in enumerate(mesh.elems):
        for k, (a, b) in enumerate(((el[0], el[1]), (el[1], el[2]), (el[3], el[2]), (el[0], el[3]))):
            if cnt[(min(a, b), max(a, b))] == 1:
                for t in range(n + 1):
                    aa = t if k in (0, 2) else (n if k == 1 else 0)
                    bb = t if k in (1, 3) else (n if k == 2 else 0)
                    bnd[f.pmap[e, bb * (n + 1) + aa]] = True
    # scale: the convection and the pressure terms alone (they cancel)
    scale = np.abs(f.defect(pv, 0 * pp, pv, 0.01, 0.0)).max() + np.abs(f.defect(0 * pv, pp, 0 * pv, 0.01, 0.0)).max()
    assert np.abs(D[~bnd]).max() <= 1e-12 * scale
    assert np.all(D[f.mask] == 0.0)


def test_averaging_counts_patches_at_irregular_vertices():
    mesh = synth.cylinder_channel_umesh(4)
    f = oracle.UFine(mesh, 1)
    dp = np.repeat(np.arange(f.ne, dtype=np.float64)[:, None], 2 * f.nf, axis=1)
    Db = f.average(dp)
    occ = {}
    for e in range(f.ne):
        for l in range(f.nf):
            occ.setdefault(int(f.pmap[e, l]), []).append(e)
    val5 = 0
    for node, es in occ.items():
        want = 0.0 if f.mask[node] else float(np.mean(es))
        assert abs(Db[node, 0] - want) <= 1e-12 * max(1.0, want)
        val5 += len(es) == 5
    assert val5 == 4


@pytest.mark.parametrize("K", [1, 2, 3])
def test_transfinite_refinement_reproduces_the_polar_map(K):
    """One ring of elements between two circles, both curved: the transfinite
    map of each element (two arcs, two radial segments) is the polar map, so
    fine node (a, b) sits at radius r0 + (a/n)(r1 - r0) and angle
    theta_i + (b/n) dtheta exactly."""
    m, r0, r1, cx, cy = 12, 0.5, 1.25, 0.3, -0.2
    th = [2 * math.pi * i / m for i in range(m)]
    xy = np.array([(cx + r * math.cos(t), cy + r * math.sin(t)) for r in (r0, r1) for t in th])
    elems, curved = [], []
    for i in range(m):
        j = (i + 1) % m
        elems.append((i, m + i, m + j, j))        # radial outward, then counter-clockwise
        curved += [(i, j, 0), (m + i, m + j, 1)]
    mesh = synth.UMesh(xy, np.array(elems, dtype=np.int32), np.zeros((0, 2), dtype=np.int32),
                       np.array([[cx, cy, r0], [cx, cy, r1]]), np.array(curved, dtype=np.int32))
    f = oracle.UFine(mesh, K)
    n = 1 << K
    for e in range(m):
        for b in range(n + 1):
            for a in range(n + 1):
                r = r0 + a / n * (r1 - r0)
                t = th[e] + b / n * (2 * math.pi / m)
                x = f.fxy[f.pmap[e, b * (n + 1) + a]]
                assert abs(x[0] - cx - r * math.cos(t)) <= 1e-14 and abs(x[1] - cy - r * math.sin(t)) <= 1e-14
