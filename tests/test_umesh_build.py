"""The library's unstructured-mesh construction (csrc/umesh_build.h, host C++)
against the FP64 reference implementation (oracle/dnnmg_oracle.c): the same
canonical fine numbering, patch maps, Dirichlet mask and fine coordinates
(to 1e-15 of the domain), valid gather lists, the same patch features (as
FP32), and rejection of invalid meshes with a reason.  CPU only."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2008_11520_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def ub(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("ub") / "libub.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-I",
                           os.path.join(ROOT, "paper_2008_11520_amd", "csrc"),
                           os.path.join(HERE, "umesh_build_check.cpp"), "-o", so])
    L = ctypes.CDLL(so)
    L.ub_error.restype = ctypes.c_char_p
    return L


def _args(mesh):
    xy = np.ascontiguousarray(mesh.xy, np.float64)
    el = np.ascontiguousarray(mesh.elems, np.int32)
    dr = np.ascontiguousarray(mesh.dirichlet_edges, np.int32).reshape(-1, 2)
    ci = np.ascontiguousarray(mesh.circles, np.float64).reshape(-1, 3)
    cu = np.ascontiguousarray(mesh.curved, np.int32).reshape(-1, 3)
    keep = (xy, el, dr, ci, cu)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    return keep, [xy.shape[0], el.shape[0], vp(xy), vp(el), dr.shape[0], vp(dr), ci.shape[0], vp(ci),
                  cu.shape[0], vp(cu)]


def _build(L, mesh, K):
    keep, a = _args(mesh)
    E, Fn = ctypes.c_int(), ctypes.c_int()
    if L.ub_counts(*a, K, ctypes.byref(E), ctypes.byref(Fn)) != 0:
        return L.ub_error().decode()
    ne, n = mesh.elems.shape[0], 1 << K
    nf, nc = (n + 1) ** 2, mesh.xy.shape[0]
    out = dict(pmap=np.empty((ne, nf), np.int32), fxy=np.empty((Fn.value, 2)), rel=np.empty((ne, nf, 2)),
               mask=np.empty(Fn.value, np.uint8), node_ptr=np.empty(Fn.value + 1, np.int32),
               node_occ=np.empty(ne * nf, np.int32), cnode_ptr=np.empty(nc + 1, np.int32),
               cnode_occ=np.empty(4 * ne, np.int32), feat=np.empty((ne, 4), np.float32))
    vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    assert L.ub_build(*a, K, *[vp(out[k]) for k in ("pmap", "fxy", "rel", "mask", "node_ptr", "node_occ",
                                                     "cnode_ptr", "cnode_occ", "feat")]) == 0
    out["E"], out["Fn"] = E.value, Fn.value
    return out


MESHES = {
    "cylinder_channel": lambda: synth.cylinder_channel_umesh(6),
    "structured_shuffled_rotated": lambda: synth.structured_as_umesh(
        synth.perturb_interior(synth.rect_mesh(7, 5, 2.2, 0.41), 0.1, 3), synth.DIR_CHANNEL,
        order_seed=1, rotate_seed=2, renumber_seed=3)[0],
}


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("K", [1, 2, 3])
def test_construction_matches_the_reference(ub, name, K):
    mesh = MESHES[name]()
    got = _build(ub, mesh, K)
    ref = oracle.UFine(mesh, K)
    assert got["E"] == ref.E and got["Fn"] == ref.Fn
    assert np.array_equal(got["pmap"], ref.pmap)
    assert np.abs(got["fxy"] - ref.fxy).max() <= 1e-15 * np.abs(ref.fxy).max()
    assert np.array_equal(got["mask"].astype(bool), ref.mask)
    corner0 = mesh.xy[mesh.elems[:, 0]]
    assert np.abs(got["rel"] - (ref.fxy[ref.pmap] - corner0[:, None, :])).max() <= 1e-15
    # gather lists: every (patch, local node) once, in patch order per node
    ptr, occ = got["node_ptr"], got["node_occ"]
    for f in range(0, ref.Fn, max(1, ref.Fn // 500)):
        lst = occ[ptr[f]:ptr[f + 1]]
        assert np.all(np.diff(lst) > 0)
        assert np.all(ref.pmap.reshape(-1)[lst] == f)
    assert np.array_equal(np.sort(occ), np.arange(ref.ne * ref.nf))
    cptr, cocc = got["cnode_ptr"], got["cnode_occ"]
    for c in range(ref.nc):
        lst = cocc[cptr[c]:cptr[c + 1]]
        assert np.all(mesh.elems.reshape(-1)[lst] == c) and np.all(np.diff(lst) > 0)
    assert np.array_equal(got["feat"], ref.features().astype(np.float32))


def test_invalid_meshes_are_rejected_with_a_reason(ub):
    good = synth.cylinder_channel_umesh(4)

    def variant(**kw):
        d = dict(xy=good.xy.copy(), elems=good.elems.copy(), dirichlet_edges=good.dirichlet_edges.copy(),
                 circles=good.circles.copy(), curved=good.curved.copy())
        d.update(kw)
        return synth.UMesh(**d)

    flipped = good.elems.copy()
    flipped[0] = flipped[0][::-1]
    bad_node = good.elems.copy()
    bad_node[3, 2] = good.xy.shape[0]
    off_circle = good.xy.copy()
    off_circle[good.curved[0, 0]] += 1e-3
    cases = {"oriented alike": variant(elems=flipped),
             "out of range": variant(elems=bad_node),
             "not on its circle": variant(xy=off_circle),
             "Dirichlet edge": variant(dirichlet_edges=np.array([[0, good.xy.shape[0] - 1]], np.int32)),
             "repeats a node": variant(elems=np.where(np.arange(4) == 1, good.elems[:, :1], good.elems))}
    for why, mesh in cases.items():
        msg = _build(ub, mesh, 2)
        assert isinstance(msg, str) and why in msg, (why, msg)
