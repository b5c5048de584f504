"""FP64 CPU oracle of the fine-level DNN-MG step -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never calls it.  numpy wrappers over the plain C implementation in
dnnmg_oracle.c; every array is float64 and C-contiguous.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_U8 = ctypes.POINTER(ctypes.c_uint8)


def lib():
    global _lib
    if _lib is None:
        # DNNMG_ORACLE_LIB lets the mutation test load a deliberately broken
        # build of this same source, to show that the pins catch it.
        path = os.environ.get("DNNMG_ORACLE_LIB") or _build.build(force=False)
        L = ctypes.CDLL(path)
        i, d, u = ctypes.c_int, ctypes.c_double, ctypes.c_uint
        L.orc_fine_coords.argtypes = [i, i, i, _D, _D]
        L.orc_prolong.argtypes = [i, i, i, i, _D, _D]
        L.orc_restrict.argtypes = [i, i, i, i, _D, _D]
        L.orc_dirichlet_mask.argtypes = [i, i, i, u, _U8]
        L.orc_defect.argtypes = [i, i, i, _D, _D, _D, _D, d, d, u, _D]
        L.orc_defect_abs.argtypes = [i, i, i, _D, _D, _D, _D, d, d, _D]
        L.orc_set_threads.argtypes = [i]
        L.orc_get_threads.restype = i
        L.orc_mass_apply.argtypes = [i, i, i, _D, _D, _D]
        L.orc_features.argtypes = [i, i, _D, _D]
        L.orc_gather_input.argtypes = [i, i, i, _D, _D, _D, _D]
        L.orc_gru.argtypes = [i, i, i, _D, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_mlp.argtypes = [i, i, i, i, _D, _D, _D, _D]
        L.orc_average.argtypes = [i, i, i, _D, u, _D]
        L.orc_rhs_restrict.argtypes = [i, i, i, _D, _D, _D, d, _D]
        L.orc_step.argtypes = [i, i, i, i, i, d, d, u, _D, _D, _D, _D, _D, _D, i,
                               _D, _D, _D, _D, _D, _D]
        L.orc_step.restype = i
        L.orc_step_prec.argtypes = [i, i, i, i, i, d, d, u, _D, _D, _D, _D, _D, _D, i, i,
                                    _D, _D, _D, _D, _D, _D]
        L.orc_step_prec.restype = i
        L.orc_step_theta.argtypes = [i, i, i, i, i, d, d, d, u, _D, _D, _D, _D, _D, _D, i, i,
                                     _D, _D, _D, _D, _D, _D]
        L.orc_step_theta.restype = i
        L.orc_transport_apply.argtypes = [i, i, i, _D, _D, d, _D]
        L.orc_defect_theta.argtypes = [i, i, i, _D, _D, _D, _D, d, d, d, u, _D]
        L.orc_rhs_restrict_theta.argtypes = [i, i, i, _D, _D, _D, d, d, d, _D]
        L.orc_step_form.argtypes = [i, i, i, i, i, d, d, d, u, i, i, _D, _D, _D, _D, _D, _D, i, i,
                                    _D, _D, _D, _D, _D, _D]
        L.orc_step_form.restype = i
        L.orc_continuity_rows.argtypes = [i, i, i, _D, _D, _D]
        L.orc_paper_geometry.argtypes = [i, i, _D, _D]
        L.orc_peclet.argtypes = [i, i, _D, _D, d, _D]
        L.orc_gather_input_paper.argtypes = [i, i, i, _D, _D, _D, _D, _D, _D]
        L.orc_gru_form.argtypes = [i, i, i, _D, _D, _D, _D, _D, _D, _D, _D, i, _D]
        L.orc_conv_head.argtypes = [i, i, i, _D, _D, _D, _D, _D, _D]
        L.orc_paper_weight_count.argtypes = [i, i]
        L.orc_paper_weight_count.restype = ctypes.c_long
        _I = ctypes.POINTER(ctypes.c_int)
        L.orc_umesh_count.argtypes = [i, i, _I, i, _I, _I]
        L.orc_umesh_refine.argtypes = [i, i, _D, _I, i, i, _I, _D, _D, _I]
        L.orc_u_prolong.argtypes = [i, i, _I, _I, i, i, _D, _D]
        L.orc_u_restrict.argtypes = [i, i, i, _I, _I, i, i, _D, _D]
        L.orc_u_mask.argtypes = [i, i, _I, _I, i, i, _I, _U8]
        L.orc_u_defect.argtypes = [i, i, _I, _D, i, _D, _D, _D, d, d, _U8, _D]
        L.orc_u_mass_apply.argtypes = [i, i, _I, _D, i, _D, _D]
        L.orc_u_features.argtypes = [i, _D, _I, _D]
        L.orc_u_average.argtypes = [i, i, _I, i, _D, _U8, _D]
        L.orc_u_rhs_restrict.argtypes = [i, i, i, _I, _I, _D, i, _D, _D, d, _D]
        L.orc_u_step.argtypes = [i, i, _D, _I, i, i, i, d, d, _I, _D, i, _U8, _D, _D, _D, _D, _D, i,
                                 _D, _D, _D, _D, _D, _D]
        L.orc_u_step.restype = i
        L.orc_e4m3_decode.argtypes = [u]
        L.orc_e4m3_decode.restype = d
        L.orc_e4m3_encode.argtypes = [ctypes.c_float]
        L.orc_e4m3_encode.restype = u
        L.orc_quantize_rows.argtypes = [i, i, ctypes.POINTER(ctypes.c_float), _U8, ctypes.POINTER(ctypes.c_float)]
        L.orc_qgemm.argtypes = [i, i, i, _D, _D, _D]
        L.orc_gru_fp8.argtypes = [i, i, i, _D, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_mlp_fp8.argtypes = [i, i, i, i, _D, _D, _D, _D]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def sizes(nx, ny, K):
    n = 1 << K
    return dict(n=n, nf=(n + 1) ** 2, Fn=(nx * n + 1) * (ny * n + 1),
                Nc=(nx + 1) * (ny + 1), P=nx * ny, nin=4 * (n + 1) ** 2 + 4,
                nout=2 * (n + 1) ** 2)


def fine_coords(nx, ny, K, cxy):
    s = sizes(nx, ny, K)
    out = np.empty((s["Fn"], 2))
    lib().orc_fine_coords(nx, ny, K, _p(_f64(cxy)), _p(out))
    return out


def prolong(nx, ny, K, coarse):
    c = _f64(coarse)
    ncomp = 1 if c.ndim == 1 else c.shape[-1]
    s = sizes(nx, ny, K)
    out = np.empty((s["Fn"], ncomp) if ncomp > 1 else (s["Fn"],))
    lib().orc_prolong(nx, ny, K, ncomp, _p(c), _p(out))
    return out


def restrict(nx, ny, K, fine):
    f = _f64(fine)
    ncomp = 1 if f.ndim == 1 else f.shape[-1]
    s = sizes(nx, ny, K)
    out = np.empty((s["Nc"], ncomp) if ncomp > 1 else (s["Nc"],))
    lib().orc_restrict(nx, ny, K, ncomp, _p(f), _p(out))
    return out


def dirichlet_mask(nx, ny, K, dirichlet):
    s = sizes(nx, ny, K)
    m = np.empty(s["Fn"], dtype=np.uint8)
    lib().orc_dirichlet_mask(nx, ny, K, dirichlet, m.ctypes.data_as(_U8))
    return m.astype(bool)


def defect(nx, ny, K, cxy, pv, pp, uprev, dt, nu, dirichlet):
    s = sizes(nx, ny, K)
    D = np.empty((s["Fn"], 2))
    lib().orc_defect(nx, ny, K, _p(_f64(cxy)), _p(_f64(pv)), _p(_f64(pp)), _p(_f64(uprev)),
                     dt, nu, dirichlet, _p(D))
    return D


def defect_abs(nx, ny, K, cxy, pv, pp, uprev, inv_dt, nu):
    """Error scale of the defect (orc_defect_abs): the element terms and the
    sums inside them in absolute value, assembled, unmasked.  inv_dt is the
    1/dt of the evaluation being judged (0 if it leaves the mass term out)."""
    s = sizes(nx, ny, K)
    S = np.empty((s["Fn"], 2))
    lib().orc_defect_abs(nx, ny, K, _p(_f64(cxy)), _p(_f64(pv)), _p(_f64(pp)), _p(_f64(uprev)),
                         inv_dt, nu, _p(S))
    return S


def transport_apply(nx, ny, K, cxy, w, nu):
    """T(w) = C(w) w + nu K w at the fine nodes (unmasked)."""
    s = sizes(nx, ny, K)
    out = np.empty((s["Fn"], 2))
    lib().orc_transport_apply(nx, ny, K, _p(_f64(cxy)), _p(_f64(w)), nu, _p(out))
    return out


def defect_theta(nx, ny, K, cxy, pv, pp, uprev, dt, nu, theta, dirichlet):
    s = sizes(nx, ny, K)
    D = np.empty((s["Fn"], 2))
    lib().orc_defect_theta(nx, ny, K, _p(_f64(cxy)), _p(_f64(pv)), _p(_f64(pp)), _p(_f64(uprev)),
                           dt, nu, theta, dirichlet, _p(D))
    return D


def rhs_restrict_theta(nx, ny, K, cxy, v, Dbar, dt, nu, theta):
    s = sizes(nx, ny, K)
    out = np.empty((s["Nc"], 2))
    lib().orc_rhs_restrict_theta(nx, ny, K, _p(_f64(cxy)), _p(_f64(v)), _p(_f64(Dbar)), dt, nu, theta, _p(out))
    return out


def set_threads(n):
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())


def mass_apply(nx, ny, K, cxy, u):
    s = sizes(nx, ny, K)
    out = np.empty((s["Fn"], 2))
    lib().orc_mass_apply(nx, ny, K, _p(_f64(cxy)), _p(_f64(u)), _p(out))
    return out


def features(nx, ny, cxy):
    out = np.empty((nx * ny, 4))
    lib().orc_features(nx, ny, _p(_f64(cxy)), _p(out))
    return out


def gather_input(nx, ny, K, pv, D, feat):
    s = sizes(nx, ny, K)
    X = np.empty((s["P"], s["nin"]))
    lib().orc_gather_input(nx, ny, K, _p(_f64(pv)), _p(_f64(D)), _p(_f64(feat)), _p(X))
    return X


def gru(X, h, Wz, Wr, Wh, Uz, Ur, Uh):
    X, h = _f64(X), _f64(h)
    P, nin = X.shape
    H = h.shape[1]
    out = np.empty((P, H))
    lib().orc_gru(P, nin, H, *[_p(_f64(w)) for w in (Wz, Wr, Wh, Uz, Ur, Uh)],
                  _p(X), _p(h), _p(out))
    return out


def mlp(h, M1, M2=None):
    h = _f64(h)
    P, H = h.shape
    if M2 is None:
        Hm, nout = 0, M1.shape[0]
        m2 = None
    else:
        Hm, nout = M1.shape[0], M2.shape[0]
        m2 = _f64(M2)
    out = np.empty((P, nout))
    lib().orc_mlp(P, H, Hm, nout, _p(_f64(M1)), _p(m2), _p(h), _p(out))
    return out


# ---- FP8 E4M3 operand form
def e4m3_decode(code):
    return lib().orc_e4m3_decode(int(code))


def e4m3_encode(x):
    return lib().orc_e4m3_encode(float(x))


def quantize_rows(a):
    """Per-row E4M3 quantisation of an FP32 matrix: (codes uint8, scales float32)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    rows, cols = a.shape
    q = np.empty((rows, cols), dtype=np.uint8)
    sc = np.empty(rows, dtype=np.float32)
    F = ctypes.POINTER(ctypes.c_float)
    lib().orc_quantize_rows(rows, cols, a.ctypes.data_as(F), q.ctypes.data_as(_U8), sc.ctypes.data_as(F))
    return q, sc


def qgemm(A, B):
    """A (M x K) times B (N x K)^T with per-row FP8 operands, exact accumulation."""
    A, B = _f64(A), _f64(B)
    out = np.empty((A.shape[0], B.shape[0]))
    lib().orc_qgemm(A.shape[0], B.shape[0], A.shape[1], _p(A), _p(B), _p(out))
    return out


def gru_fp8(X, h, Wz, Wr, Wh, Uz, Ur, Uh):
    X, h = _f64(X), _f64(h)
    P, nin = X.shape
    H = h.shape[1]
    out = np.empty((P, H))
    lib().orc_gru_fp8(P, nin, H, *[_p(_f64(w)) for w in (Wz, Wr, Wh, Uz, Ur, Uh)],
                      _p(X), _p(h), _p(out))
    return out


def mlp_fp8(h, M1, M2=None):
    h = _f64(h)
    P, H = h.shape
    if M2 is None:
        Hm, nout, m2 = 0, M1.shape[0], None
    else:
        Hm, nout, m2 = M1.shape[0], M2.shape[0], _f64(M2)
    out = np.empty((P, nout))
    lib().orc_mlp_fp8(P, H, Hm, nout, _p(_f64(M1)), _p(m2), _p(h), _p(out))
    return out


def average(nx, ny, K, dpatch, dirichlet):
    s = sizes(nx, ny, K)
    out = np.empty((s["Fn"], 2))
    lib().orc_average(nx, ny, K, _p(_f64(dpatch)), dirichlet, _p(out))
    return out


def rhs_restrict(nx, ny, K, cxy, v, Dbar, dt):
    s = sizes(nx, ny, K)
    out = np.empty((s["Nc"], 2))
    lib().orc_rhs_restrict(nx, ny, K, _p(_f64(cxy)), _p(_f64(v)), _p(_f64(Dbar)), dt, _p(out))
    return out


def continuity_rows(nx, ny, K, cxy, pv):
    """-(div Pv, xi_a) at the fine nodes (unmasked)."""
    s = sizes(nx, ny, K)
    out = np.empty(s["Fn"])
    lib().orc_continuity_rows(nx, ny, K, _p(_f64(cxy)), _p(_f64(pv)), _p(out))
    return out


def paper_geometry(nx, ny, cxy):
    out = np.empty((nx * ny, 12))
    lib().orc_paper_geometry(nx, ny, _p(_f64(cxy)), _p(out))
    return out


def peclet(nx, ny, cxy, v, nu):
    out = np.empty((nx * ny, 4))
    lib().orc_peclet(nx, ny, _p(_f64(cxy)), _p(_f64(v)), nu, _p(out))
    return out


def gather_input_paper(nx, ny, K, D, Rp, v, Pe, G):
    s = sizes(nx, ny, K)
    out = np.empty((s["P"], 3 * s["nf"] + 24))
    lib().orc_gather_input_paper(nx, ny, K, _p(_f64(D)), _p(_f64(Rp)), _p(_f64(v)), _p(_f64(Pe)), _p(_f64(G)),
                                 _p(out))
    return out


def gru_form(X, h, Wz, Wr, Wh, Uz, Ur, Uh, reset_after):
    X, h = _f64(X), _f64(h)
    P, nin = X.shape
    H = h.shape[1]
    out = np.empty((P, H))
    lib().orc_gru_form(P, nin, H, *[_p(_f64(w)) for w in (Wz, Wr, Wh, Uz, Ur, Uh)], _p(X), _p(h),
                       int(reset_after), _p(out))
    return out


def conv_head(K, h, M, WV, WS, wf):
    h = _f64(h)
    P, H = h.shape
    out = np.empty((P, 2 * (2 ** K + 1) ** 2))
    lib().orc_conv_head(P, K, H, _p(_f64(M)), _p(_f64(WV)), _p(_f64(WS)), _p(_f64(wf)), _p(h), _p(out))
    return out


def paper_weight_count(K, H):
    return int(lib().orc_paper_weight_count(K, H))


class OracleFlow:
    """Stateful wrapper: h (P x H) and u_prev (Fn x 2) in float64.
    form 0: the workloads' network; 1: the paper's (orc_step_form)."""

    def __init__(self, nx, ny, K, H, Hm, dt, nu, dirichlet, cxy, weights, fp8=False, theta=1.0, form=0,
                 reset_after=False):
        self.nx, self.ny, self.K, self.H, self.Hm = nx, ny, K, H, Hm
        self.fp8 = bool(fp8)
        self.theta = float(theta)
        self.form, self.reset_after = int(form), int(bool(reset_after))
        self.dt, self.nu, self.dirichlet = dt, nu, dirichlet
        self.cxy = _f64(cxy).reshape(-1, 2)
        self.w = _f64(weights).reshape(-1)
        s = sizes(nx, ny, K)
        if self.form:
            s["nin"] = 3 * s["nf"] + 24
        self.s = s
        self.h = np.zeros((s["P"], H))
        self.uprev = np.zeros((s["Fn"], 2))
        self.nsteps = 0

    def step(self, v, p, want=("Dbar", "bL")):
        s = self.s
        outs = {k: None for k in ("Pv", "D", "X", "dpatch", "Dbar", "bL")}
        shapes = dict(Pv=(s["Fn"], 2), D=(s["Fn"], 2), X=(s["P"], s["nin"]),
                      dpatch=(s["P"], s["nout"]), Dbar=(s["Fn"], 2), bL=(s["Nc"], 2))
        for k in want:
            outs[k] = np.empty(shapes[k])
        rc = lib().orc_step_form(self.nx, self.ny, self.K, self.H, self.Hm, self.dt, self.nu, self.theta,
                                 self.dirichlet, self.form, self.reset_after, _p(self.cxy), _p(self.w),
                                 _p(_f64(v).reshape(-1, 2)), _p(_f64(p).reshape(-1)),
                                 _p(self.h), _p(self.uprev), 1 if self.nsteps == 0 else 0, int(self.fp8),
                                 *[_p(outs[k]) for k in ("Pv", "D", "X", "dpatch", "Dbar", "bL")])
        if rc != 0:
            raise MemoryError("oracle step failed: %d" % rc)
        self.nsteps += 1
        return {k: outs[k] for k in want}


# ----------------------------------------------------- unstructured meshes
def _pi(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _i32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a.reshape(shape) if shape is not None else a


class UFine:
    """The refined fine mesh of an unstructured coarse mesh (orc_umesh_refine):
    fine node coordinates fxy (Fn x 2), patch maps pmap (ne x nf), the
    Dirichlet mask, and the wrappers of the mesh's operators."""

    def __init__(self, mesh, K):
        self.mesh, self.K = mesh, K
        self.xy = _f64(mesh.xy).reshape(-1, 2)
        self.elems = _i32(mesh.elems, (-1, 4))
        self.nc, self.ne = self.xy.shape[0], self.elems.shape[0]
        n = 1 << K
        self.nf = (n + 1) ** 2
        E, Fn = ctypes.c_int(), ctypes.c_int()
        lib().orc_umesh_count(self.nc, self.ne, _pi(self.elems), K, ctypes.byref(E), ctypes.byref(Fn))
        self.E, self.Fn = E.value, Fn.value
        self.curved = _i32(mesh.curved, (-1, 3)) if len(mesh.curved) else np.zeros((0, 3), np.int32)
        self.circles = _f64(mesh.circles).reshape(-1, 3) if len(mesh.circles) else np.zeros((0, 3))
        self.fxy = np.empty((self.Fn, 2))
        self.pmap = np.empty((self.ne, self.nf), dtype=np.int32)
        lib().orc_umesh_refine(self.nc, self.ne, _p(self.xy), _pi(self.elems), K, self.curved.shape[0],
                               _pi(self.curved), _p(self.circles) if self.circles.size else None,
                               _p(self.fxy), _pi(self.pmap))
        dirs = _i32(mesh.dirichlet_edges, (-1, 2)) if len(mesh.dirichlet_edges) else np.zeros((0, 2), np.int32)
        m = np.empty(self.Fn, dtype=np.uint8)
        lib().orc_u_mask(self.ne, K, _pi(self.elems), _pi(self.pmap), self.Fn, dirs.shape[0], _pi(dirs),
                         m.ctypes.data_as(_U8))
        self.mask_u8 = m
        self.mask = m.astype(bool)

    def prolong(self, coarse):
        c = _f64(coarse)
        ncomp = 1 if c.ndim == 1 else c.shape[-1]
        out = np.empty((self.Fn, ncomp) if ncomp > 1 else (self.Fn,))
        lib().orc_u_prolong(self.ne, self.K, _pi(self.elems), _pi(self.pmap), self.Fn, ncomp, _p(c), _p(out))
        return out

    def restrict(self, fine):
        f = _f64(fine)
        ncomp = 1 if f.ndim == 1 else f.shape[-1]
        out = np.empty((self.nc, ncomp) if ncomp > 1 else (self.nc,))
        lib().orc_u_restrict(self.nc, self.ne, self.K, _pi(self.elems), _pi(self.pmap), self.Fn, ncomp, _p(f),
                             _p(out))
        return out

    def defect(self, pv, pp, uprev, dt, nu):
        D = np.empty((self.Fn, 2))
        lib().orc_u_defect(self.ne, self.K, _pi(self.pmap), _p(self.fxy), self.Fn, _p(_f64(pv)), _p(_f64(pp)),
                           _p(_f64(uprev)), dt, nu, self.mask_u8.ctypes.data_as(_U8), _p(D))
        return D

    def mass_apply(self, u):
        out = np.empty((self.Fn, 2))
        lib().orc_u_mass_apply(self.ne, self.K, _pi(self.pmap), _p(self.fxy), self.Fn, _p(_f64(u)), _p(out))
        return out

    def features(self):
        out = np.empty((self.ne, 4))
        lib().orc_u_features(self.ne, _p(self.xy), _pi(self.elems), _p(out))
        return out

    def average(self, dpatch):
        out = np.empty((self.Fn, 2))
        lib().orc_u_average(self.ne, self.K, _pi(self.pmap), self.Fn, _p(_f64(dpatch)),
                            self.mask_u8.ctypes.data_as(_U8), _p(out))
        return out

    def rhs_restrict(self, v, Dbar, dt):
        out = np.empty((self.nc, 2))
        lib().orc_u_rhs_restrict(self.nc, self.ne, self.K, _pi(self.elems), _pi(self.pmap), _p(self.fxy), self.Fn,
                                 _p(_f64(v)), _p(_f64(Dbar)), dt, _p(out))
        return out


class OracleUFlow:
    """Stateful fine step on an unstructured mesh (orc_u_step): h (ne x H) and
    u_prev (Fn x 2) in float64."""

    def __init__(self, mesh, K, H, Hm, dt, nu, weights):
        self.f = UFine(mesh, K)
        self.K, self.H, self.Hm, self.dt, self.nu = K, H, Hm, dt, nu
        self.w = _f64(weights).reshape(-1)
        self.h = np.zeros((self.f.ne, H))
        self.uprev = np.zeros((self.f.Fn, 2))
        self.nsteps = 0

    def step(self, v, p, want=("Dbar", "bL")):
        f = self.f
        nf = f.nf
        shapes = dict(Pv=(f.Fn, 2), D=(f.Fn, 2), X=(f.ne, 4 * nf + 4), dpatch=(f.ne, 2 * nf), Dbar=(f.Fn, 2),
                      bL=(f.nc, 2))
        outs = {k: (np.empty(shapes[k]) if k in want else None) for k in shapes}
        rc = lib().orc_u_step(f.nc, f.ne, _p(f.xy), _pi(f.elems), self.K, self.H, self.Hm, self.dt, self.nu,
                              _pi(f.pmap), _p(f.fxy), f.Fn, f.mask_u8.ctypes.data_as(_U8), _p(self.w),
                              _p(_f64(v).reshape(-1, 2)), _p(_f64(p).reshape(-1)), _p(self.h), _p(self.uprev),
                              1 if self.nsteps == 0 else 0,
                              *[_p(outs[k]) for k in ("Pv", "D", "X", "dpatch", "Dbar", "bL")])
        if rc != 0:
            raise MemoryError("oracle step failed: %d" % rc)
        self.nsteps += 1
        return {k: outs[k] for k in want}
