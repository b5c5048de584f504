"""Fine-level DNN-MG step on AMD MI355X: Python binding of libdnnmg.so.

Argument marshalling only: every stage of the step runs in the library's HIP
kernels.  Device buffers are torch tensors on a HIP device; the stream is
torch's current stream unless one is passed.  There is no CPU fallback: if the
library is not built, or no GPU is present, calls raise.

The C ABI is declared in include/dnnmg.h; names here follow it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdnnmg.so")

DNNMG_OK, DNNMG_EINVAL, DNNMG_ENOMEM, DNNMG_EDEVICE, DNNMG_ESTATE, DNNMG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FP32, BF16, FP8_E4M3 = 0, 1, 2
DNNMG_F_UNFUSED = 1
DNNMG_F_NANCHECK = 2
DNNMG_F_CRANK_NICOLSON = 4
DNNMG_F_PAPER_NET = 8
DNNMG_F_GRU_RESET_AFTER = 16
DNNMG_F_PATCH_OUTPUTS = 32
DNNMG_NONFINITE_CORRECTION, DNNMG_NONFINITE_RHS = 1, 2
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8_E4M3}

SYMBOLS = [
    "dnnmg_weight_count", "dnnmg_workspace_bytes", "dnnmg_create", "dnnmg_create_shared",
    "dnnmg_step", "dnnmg_restrict_rhs", "dnnmg_batch_create", "dnnmg_batch_destroy",
    "dnnmg_batch_prepare", "dnnmg_batch_launch", "dnnmg_batch_captures", "dnnmg_step_batch", "dnnmg_destroy", "dnnmg_last_error", "dnnmg_prolong", "dnnmg_defect",
    "dnnmg_rhs_restrict", "dnnmg_get_state", "dnnmg_set_state", "dnnmg_patch_output",
    "dnnmg_step_count", "dnnmg_profile_enable", "dnnmg_profile_read", "dnnmg_quantize_e4m3",
    "dnnmg_noalloc_scratch_bytes", "dnnmg_rhs_restrict_noalloc", "dnnmg_nonfinite",
    "dnnmg_arena_create", "dnnmg_arena_destroy", "dnnmg_arena_block_bytes", "dnnmg_arena_usage",
    "dnnmg_create_in_arena", "dnnmg_arena_upload", "dnnmg_umesh_counts", "dnnmg_create_umesh",
]
DNNMG_NOALLOC_MAX_PATCHES = 1 << 18


class DnnmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("dnnmg error %d: %s" % (code, msg))
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("K", ctypes.c_int),
                ("H", ctypes.c_int), ("Hm", ctypes.c_int), ("dt", ctypes.c_double),
                ("nu", ctypes.c_double), ("precision", ctypes.c_int),
                ("dirichlet", ctypes.c_uint), ("flags", ctypes.c_uint)]


_lib = None


def lib():
    """Load libdnnmg.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- loads the HIP runtime the library links against
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdnnmg.so is not built; run `python -m paper_2008_11520_amd.build_lib`")
    L = ctypes.CDLL(LIB_PATH)
    vp, cp, i, sz = ctypes.c_void_p, ctypes.POINTER(Config), ctypes.c_int, ctypes.c_size_t
    L.dnnmg_weight_count.argtypes = [cp]; L.dnnmg_weight_count.restype = sz
    L.dnnmg_workspace_bytes.argtypes = [cp]; L.dnnmg_workspace_bytes.restype = sz
    L.dnnmg_create.argtypes = [cp, vp, vp, sz, vp, ctypes.POINTER(vp)]
    L.dnnmg_create_shared.argtypes = [cp, vp, vp, vp, ctypes.POINTER(vp)]
    L.dnnmg_step.argtypes = [vp, vp, vp, vp, vp]
    L.dnnmg_restrict_rhs.argtypes = [vp, vp, vp]
    L.dnnmg_batch_create.argtypes = [i, ctypes.POINTER(vp)]
    L.dnnmg_batch_destroy.argtypes = [vp]
    L.dnnmg_step_batch.argtypes = [vp, vp, i, vp, vp, vp, vp]
    L.dnnmg_batch_prepare.argtypes = [vp, vp, i, vp, vp, vp, vp, vp]
    L.dnnmg_batch_launch.argtypes = [vp, i, vp]
    L.dnnmg_batch_captures.argtypes = [vp]
    L.dnnmg_destroy.argtypes = [vp]
    L.dnnmg_last_error.restype = ctypes.c_char_p
    L.dnnmg_prolong.argtypes = [vp, vp, vp, vp, vp, vp]
    L.dnnmg_defect.argtypes = [vp, vp, vp, vp, vp]
    L.dnnmg_rhs_restrict.argtypes = [vp, vp, vp, vp, vp]
    L.dnnmg_get_state.argtypes = [vp, vp, vp, vp]
    L.dnnmg_set_state.argtypes = [vp, vp, vp, ctypes.c_longlong, vp]
    L.dnnmg_umesh_counts.argtypes = [ctypes.POINTER(UMeshC), i, ctypes.POINTER(i), ctypes.POINTER(i)]
    L.dnnmg_create_umesh.argtypes = [cp, ctypes.POINTER(UMeshC), vp, sz, vp, ctypes.POINTER(vp)]
    L.dnnmg_patch_output.argtypes = [vp, vp, vp]
    L.dnnmg_step_count.argtypes = [vp]; L.dnnmg_step_count.restype = ctypes.c_longlong
    L.dnnmg_profile_enable.argtypes = [vp, i]
    L.dnnmg_quantize_e4m3.argtypes = [vp, i, i, vp, vp, vp]
    L.dnnmg_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    L.dnnmg_noalloc_scratch_bytes.argtypes = []; L.dnnmg_noalloc_scratch_bytes.restype = sz
    L.dnnmg_nonfinite.argtypes = [vp, i, ctypes.POINTER(ctypes.c_int), vp]
    L.dnnmg_arena_create.argtypes = [sz, sz, ctypes.POINTER(vp)]
    L.dnnmg_arena_destroy.argtypes = [vp]
    L.dnnmg_arena_block_bytes.argtypes = [cp]; L.dnnmg_arena_block_bytes.restype = sz
    L.dnnmg_arena_usage.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.dnnmg_create_in_arena.argtypes = [vp, cp, vp, vp, vp, ctypes.POINTER(vp)]
    L.dnnmg_arena_upload.argtypes = [vp, vp, vp, sz, vp]
    L.dnnmg_rhs_restrict_noalloc.argtypes = [i, i, i, ctypes.c_double, vp, vp, vp, vp, vp]
    for name in SYMBOLS:
        getattr(L, name).restype = getattr(L, name).restype or ctypes.c_int
    L.dnnmg_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != DNNMG_OK:
        raise DnnmgError(rc, lib().dnnmg_last_error().decode())


def sizes(nx, ny, K):
    n = 1 << K
    nf = (n + 1) ** 2
    return dict(n=n, nf=nf, nin=4 * nf + 4, nout=2 * nf, P=nx * ny,
                Fn=(nx * n + 1) * (ny * n + 1), Nc=(nx + 1) * (ny + 1))


def make_config(nx, ny, K, H, Hm, dt, nu, precision=FP32, dirichlet=15, flags=0):
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    return Config(nx, ny, K, H, Hm, dt, nu, precision, dirichlet, flags)


def weight_count(cfg: Config) -> int:
    return int(lib().dnnmg_weight_count(ctypes.byref(cfg)))


def workspace_bytes(cfg: Config) -> int:
    return int(lib().dnnmg_workspace_bytes(ctypes.byref(cfg)))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype, numel, name):
    """Device pointer of a contiguous torch tensor of the given dtype and size."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError("%s must be contiguous %s with %d elements (got %s, %s, %d)"
                         % (name, dtype, numel, t.dtype, t.is_contiguous(), t.numel()))
    return ctypes.c_void_p(t.data_ptr())


class DnnMG:
    """One flow of the fine-level DNN-MG step (see include/dnnmg.h)."""

    def __init__(self, cfg: Config, coarse_xy: np.ndarray, weights: np.ndarray | None = None,
                 share: "DnnMG | None" = None, stream=None, arena: "Arena | None" = None):
        import torch
        self.cfg = cfg
        self.s = sizes(cfg.nx, cfg.ny, cfg.K)
        if cfg.flags & DNNMG_F_PAPER_NET:
            self.s["nin"] = (3 * self.s["nf"] + 24 + 7) // 8 * 8     # rows padded to 8 values
        self._cxy = np.ascontiguousarray(coarse_xy, dtype=np.float64).reshape(-1)
        if self._cxy.size != 2 * self.s["Nc"]:
            raise ValueError("coarse_xy must hold %d values" % (2 * self.s["Nc"]))
        h = ctypes.c_void_p()
        if arena is not None:
            if share is None:
                raise ValueError("a context in an arena shares a model's weights (share=...)")
            _check(lib().dnnmg_create_in_arena(arena.handle, ctypes.byref(cfg),
                                               self._cxy.ctypes.data_as(ctypes.c_void_p), share.handle,
                                               _stream(stream), ctypes.byref(h)))
        elif share is None:
            w = np.ascontiguousarray(weights, dtype=np.float32).reshape(-1)
            _check(lib().dnnmg_create(ctypes.byref(cfg), self._cxy.ctypes.data_as(ctypes.c_void_p),
                                      w.ctypes.data_as(ctypes.c_void_p), w.size, _stream(stream),
                                      ctypes.byref(h)))
        else:
            _check(lib().dnnmg_create_shared(ctypes.byref(cfg), self._cxy.ctypes.data_as(ctypes.c_void_p),
                                             share.handle, _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.device = torch.cuda.current_device()

    # -- the step
    def step(self, v, p=None, d_out=None, stream=None):
        import torch
        s = self.s
        _check(lib().dnnmg_step(self.handle, _ptr(v, torch.float32, 2 * s["Nc"], "v"),
                                _ptr(p, torch.float32, s["Nc"], "p"),
                                _ptr(d_out, torch.float32, 2 * s["Fn"], "d_out"), _stream(stream)))

    def restrict_rhs(self, b_out, stream=None):
        import torch
        _check(lib().dnnmg_restrict_rhs(self.handle, _ptr(b_out, torch.float64, 2 * self.s["Nc"], "b_out"),
                                        _stream(stream)))

    # -- stages
    def prolong(self, v, p=None, pv_out=None, pp_out=None, stream=None):
        import torch
        s = self.s
        _check(lib().dnnmg_prolong(self.handle, _ptr(v, torch.float32, 2 * s["Nc"], "v"),
                                   _ptr(p, torch.float32, s["Nc"], "p"),
                                   _ptr(pv_out, torch.float32, 2 * s["Fn"], "pv_out"),
                                   _ptr(pp_out, torch.float32, s["Fn"], "pp_out"), _stream(stream)))

    def defect(self, v, p, D_out, stream=None):
        import torch
        s = self.s
        _check(lib().dnnmg_defect(self.handle, _ptr(v, torch.float32, 2 * s["Nc"], "v"),
                                  _ptr(p, torch.float32, s["Nc"], "p"),
                                  _ptr(D_out, torch.float32, 2 * s["Fn"], "D_out"), _stream(stream)))

    def rhs_restrict(self, v, dbar, b_out, stream=None):
        import torch
        s = self.s
        _check(lib().dnnmg_rhs_restrict(self.handle, _ptr(v, torch.float32, 2 * s["Nc"], "v"),
                                        _ptr(dbar, torch.float32, 2 * s["Fn"], "dbar"),
                                        _ptr(b_out, torch.float64, 2 * s["Nc"], "b_out"), _stream(stream)))

    def get_state(self, h_out=None, u_out=None, stream=None):
        import torch
        s = self.s
        _check(lib().dnnmg_get_state(self.handle, _ptr(h_out, torch.float32, s["P"] * self.cfg.H, "h_out"),
                                     _ptr(u_out, torch.float32, 2 * s["Fn"], "u_out"), _stream(stream)))

    def set_state(self, h_in=None, u_in=None, steps=0, stream=None):
        import torch
        s = self.s
        _check(lib().dnnmg_set_state(self.handle, _ptr(h_in, torch.float32, s["P"] * self.cfg.H, "h_in"),
                                     _ptr(u_in, torch.float32, 2 * s["Fn"], "u_in"), steps, _stream(stream)))

    def patch_output(self, d_out, stream=None):
        import torch
        _check(lib().dnnmg_patch_output(self.handle, _ptr(d_out, torch.float32, self.s["P"] * self.s["nout"],
                                                          "d_out"), _stream(stream)))

    def nonfinite(self, clear=True, stream=None) -> int:
        """dnnmg_nonfinite: DNNMG_NONFINITE_* bits recorded since the last clear
        (waits for the stream's work)."""
        out = ctypes.c_int(0)
        _check(lib().dnnmg_nonfinite(self.handle, 1 if clear else 0, ctypes.byref(out), _stream(stream)))
        return int(out.value)

    def profile_enable(self, max_steps: int):
        _check(lib().dnnmg_profile_enable(self.handle, max_steps))

    def profile_read(self):
        """Per stage (defect, network, rhs, gather): (total ms, launches)."""
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int * 4)()
        _check(lib().dnnmg_profile_read(self.handle, ms, cnt))
        return list(ms), list(cnt)

    @property
    def steps(self) -> int:
        return int(lib().dnnmg_step_count(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().dnnmg_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def quantize_e4m3(a, q_out, scale_out, stream=None):
    """dnnmg_quantize_e4m3 on device tensors: a (rows, cols) float32 ->
    q_out (rows, cols) uint8 codes, scale_out (rows,) float32."""
    import torch
    rows, cols = a.shape
    _check(lib().dnnmg_quantize_e4m3(_ptr(a, torch.float32, rows * cols, "a"), rows, cols,
                                     _ptr(q_out, torch.uint8, rows * cols, "q_out"),
                                     _ptr(scale_out, torch.float32, rows, "scale_out"), _stream(stream)))


class Arena:
    """Device arena for serving (dnnmg_arena_*): contexts made with
    DnnMG(..., share=model, arena=arena) take their workspace from it."""

    def __init__(self, nbytes: int, staging_bytes: int = 8 << 20):
        h = ctypes.c_void_p()
        _check(lib().dnnmg_arena_create(int(nbytes), int(staging_bytes), ctypes.byref(h)))
        self.handle = h
        self.nbytes = int(nbytes)

    @staticmethod
    def block_bytes(cfg: Config) -> int:
        return int(lib().dnnmg_arena_block_bytes(ctypes.byref(cfg)))

    def upload(self, dst, src: np.ndarray, stream=None):
        """dnnmg_arena_upload: host array src into the device tensor dst (same
        number of bytes), asynchronously on the stream."""
        src = np.ascontiguousarray(src)
        if not dst.is_cuda or not dst.is_contiguous() or dst.numel() * dst.element_size() != src.nbytes:
            raise ValueError("dst must be a contiguous device tensor of %d bytes" % src.nbytes)
        _check(lib().dnnmg_arena_upload(self.handle, ctypes.c_void_p(dst.data_ptr()),
                                        src.ctypes.data_as(ctypes.c_void_p), src.nbytes, _stream(stream)))

    def usage(self):
        """(bytes in use, largest free block)."""
        used, largest = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().dnnmg_arena_usage(self.handle, ctypes.byref(used), ctypes.byref(largest)))
        return int(used.value), int(largest.value)

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().dnnmg_arena_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def noalloc_scratch_bytes() -> int:
    return int(lib().dnnmg_noalloc_scratch_bytes())


def rhs_restrict_noalloc(nx, ny, K, dt, coarse_xy, v, dbar, b_out, stream=None):
    """dnnmg_rhs_restrict_noalloc: b_out = P^T (1/dt) M_f (P v + dbar) with no
    context and no device allocation.  coarse_xy: device float64
    ((ny+1)(nx+1) x 2), v: float32 coarse velocity, dbar: float32 fine
    correction, b_out: float64 coarse output."""
    import torch
    s = sizes(nx, ny, K)
    _check(lib().dnnmg_rhs_restrict_noalloc(nx, ny, K, dt, _ptr(coarse_xy, torch.float64, 2 * s["Nc"], "coarse_xy"),
                                            _ptr(v, torch.float32, 2 * s["Nc"], "v"),
                                            _ptr(dbar, torch.float32, 2 * s["Fn"], "dbar"),
                                            _ptr(b_out, torch.float64, 2 * s["Nc"], "b_out"), _stream(stream)))


class UMeshC(ctypes.Structure):
    """dnnmg_umesh (include/dnnmg.h)."""
    _fields_ = [("n_nodes", ctypes.c_int), ("n_elems", ctypes.c_int), ("xy", ctypes.c_void_p),
                ("elems", ctypes.c_void_p), ("n_dirichlet", ctypes.c_int), ("dirichlet_edges", ctypes.c_void_p),
                ("n_circles", ctypes.c_int), ("circles", ctypes.c_void_p), ("n_curved", ctypes.c_int),
                ("curved_edges", ctypes.c_void_p)]


def _umesh_c(mesh):
    """(UMeshC, the arrays it points into) for a mesh with fields xy, elems,
    dirichlet_edges, circles, curved (numpy-like)."""
    keep = dict(xy=np.ascontiguousarray(mesh.xy, dtype=np.float64).reshape(-1, 2),
                elems=np.ascontiguousarray(mesh.elems, dtype=np.int32).reshape(-1, 4),
                dirs=np.ascontiguousarray(mesh.dirichlet_edges, dtype=np.int32).reshape(-1, 2),
                circ=np.ascontiguousarray(mesh.circles, dtype=np.float64).reshape(-1, 3),
                curved=np.ascontiguousarray(mesh.curved, dtype=np.int32).reshape(-1, 3))
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else None
    c = UMeshC(keep["xy"].shape[0], keep["elems"].shape[0], ptr(keep["xy"]), ptr(keep["elems"]),
               keep["dirs"].shape[0], ptr(keep["dirs"]), keep["circ"].shape[0], ptr(keep["circ"]),
               keep["curved"].shape[0], ptr(keep["curved"]))
    return c, keep


def umesh_counts(mesh, K):
    """dnnmg_umesh_counts: (edges, fine nodes) of the mesh refined K times."""
    c, _keep = _umesh_c(mesh)
    E, Fn = ctypes.c_int(), ctypes.c_int()
    _check(lib().dnnmg_umesh_counts(ctypes.byref(c), K, ctypes.byref(E), ctypes.byref(Fn)))
    return E.value, Fn.value


class UDnnMG(DnnMG):
    """One flow on an unstructured mesh (dnnmg_create_umesh): the same calls
    as DnnMG with fine arrays in the mesh's fine numbering."""

    def __init__(self, K, H, Hm, dt, nu, mesh, weights, precision=FP32, flags=0, stream=None):
        import torch
        c, keep = _umesh_c(mesh)
        ne, nc = keep["elems"].shape[0], keep["xy"].shape[0]
        self.cfg = make_config(ne, 1, K, H, Hm, dt, nu, precision, 0, flags)
        E, Fn = umesh_counts(mesh, K)
        n = 1 << K
        nf = (n + 1) ** 2
        self.s = dict(n=n, nf=nf, nin=4 * nf + 4, nout=2 * nf, P=ne, Fn=Fn, Nc=nc, E=E)
        w = np.ascontiguousarray(weights, dtype=np.float32).reshape(-1)
        h = ctypes.c_void_p()
        _check(lib().dnnmg_create_umesh(ctypes.byref(self.cfg), ctypes.byref(c), w.ctypes.data_as(ctypes.c_void_p),
                                        w.size, _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.device = torch.cuda.current_device()


class Batch:
    """Descriptor table for stepping many flows (sharing one weight set) together."""

    def __init__(self, max_flows: int):
        h = ctypes.c_void_p()
        _check(lib().dnnmg_batch_create(max_flows, ctypes.byref(h)))
        self.handle = h
        self.max_flows = max_flows

    @staticmethod
    def _arrays(flows, vs, ps, d_outs, b_outs):
        import torch
        nf = len(flows)
        arr = (ctypes.c_void_p * nf)(*[f.handle.value for f in flows])
        va = (ctypes.c_void_p * nf)(*[_ptr(v, torch.float32, 2 * f.s["Nc"], "v").value for f, v in zip(flows, vs)])
        pa = da = ba = None
        if ps is not None:
            pa = (ctypes.c_void_p * nf)(*[(_ptr(p, torch.float32, f.s["Nc"], "p").value if p is not None else None)
                                          for f, p in zip(flows, ps)])
        if d_outs is not None:
            da = (ctypes.c_void_p * nf)(*[(_ptr(d, torch.float32, 2 * f.s["Fn"], "d").value if d is not None else None)
                                          for f, d in zip(flows, d_outs)])
        if b_outs is not None:
            ba = (ctypes.c_void_p * nf)(*[_ptr(b, torch.float64, 2 * f.s["Nc"], "b").value
                                          for f, b in zip(flows, b_outs)])
        return nf, arr, va, pa, da, ba

    def step(self, flows, vs, ps=None, d_outs=None, stream=None):
        """dnnmg_step_batch: prepare + eager launch."""
        nf, arr, va, pa, da, _ = self._arrays(flows, vs, ps, d_outs, None)
        _check(lib().dnnmg_step_batch(self.handle, arr, nf, va, pa, da, _stream(stream)))

    def prepare(self, flows, vs, ps=None, d_outs=None, b_outs=None, stream=None):
        nf, arr, va, pa, da, ba = self._arrays(flows, vs, ps, d_outs, b_outs)
        _check(lib().dnnmg_batch_prepare(self.handle, arr, nf, va, pa, da, ba, _stream(stream)))

    def prepare_raw(self, n, handles, v_ptrs, p_ptrs=None, b_ptrs=None, stream=None):
        """dnnmg_batch_prepare from arrays of n context handles and device
        pointers (contiguous numpy uintp arrays, as the serving loop keeps
        them; p_ptrs and b_ptrs may be None).  No per-flow checks here beyond
        the library's own."""
        def arr(a):
            if a is None:
                return None
            if a.dtype != np.uintp or not a.flags.c_contiguous or a.size < n:
                raise ValueError("pointer arrays must be contiguous uintp with >= n entries")
            return ctypes.c_void_p(a.ctypes.data)
        _check(lib().dnnmg_batch_prepare(self.handle, arr(handles), int(n), arr(v_ptrs), arr(p_ptrs), None,
                                         arr(b_ptrs), _stream(stream)))

    def launch(self, graph=False, stream=None):
        _check(lib().dnnmg_batch_launch(self.handle, 1 if graph else 0, _stream(stream)))

    @property
    def captures(self) -> int:
        return int(lib().dnnmg_batch_captures(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().dnnmg_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
