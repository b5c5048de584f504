"""The C ABI library: it loads, exports every symbol include/dnnmg.h declares,
and rejects bad arguments on the host before touching the device.  No compute
call is made here (this suite runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dnnmg.h")

pam = pytest.importorskip("paper_2008_11520_amd")
if not os.path.exists(pam.LIB_PATH):
    pytest.skip("libdnnmg.so not built", allow_module_level=True)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dnnmg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = pam.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert sorted(pam.SYMBOLS) == names


def cfg(**kw):
    base = dict(nx=4, ny=3, K=2, H=64, Hm=64, dt=0.005, nu=1e-3, precision=0, dirichlet=13)
    base.update(kw)
    return pam.make_config(**base)


def test_weight_count_formula():
    c = cfg()
    s = pam.sizes(4, 3, 2)
    assert pam.weight_count(c) == 3 * 64 * s["nin"] + 3 * 64 * 64 + 64 * 64 + s["nout"] * 64
    c = cfg(K=1, H=32, Hm=0)
    assert pam.weight_count(c) == 3 * 32 * 40 + 3 * 32 * 32 + 18 * 32
    from paper_2008_11520_amd import synth
    for K, H, Hm in ((1, 32, 0), (2, 64, 64), (3, 128, 128)):
        assert synth.xavier_weights(K, H, Hm, 1).size == pam.weight_count(cfg(K=K, H=H, Hm=Hm))


def test_workspace_bytes():
    assert pam.workspace_bytes(cfg()) > 0
    big = pam.workspace_bytes(cfg(nx=1024, ny=256))
    # state alone: h (P x H f32) and the corrected velocity (Fn x 2 f32)
    assert big > 262144 * 64 * 4 + 4097 * 1025 * 8
    assert pam.workspace_bytes(cfg(K=4)) == 0
    assert pam.workspace_bytes(cfg(nx=0)) == 0


@pytest.mark.parametrize("bad,code", [
    (dict(nx=0), pam.DNNMG_EINVAL), (dict(ny=-1), pam.DNNMG_EINVAL), (dict(K=0), pam.DNNMG_EINVAL),
    (dict(K=4), pam.DNNMG_EINVAL), (dict(dt=0.0), pam.DNNMG_EINVAL), (dict(nu=-1.0), pam.DNNMG_EINVAL),
    (dict(precision=7), pam.DNNMG_EINVAL), (dict(dirichlet=16), pam.DNNMG_EINVAL),
    (dict(H=48), pam.DNNMG_EUNSUPPORTED), (dict(Hm=40), pam.DNNMG_EUNSUPPORTED),
])
def test_create_rejects_bad_config_on_host(bad, code):
    L = pam.lib()
    c = cfg(**bad)
    cxy = np.zeros(2 * (max(c.nx, 1) + 1) * (max(c.ny, 1) + 1))
    w = np.zeros(100000, dtype=np.float32)
    out = ctypes.c_void_p(1)
    rc = L.dnnmg_create(ctypes.byref(c), cxy.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p),
                        w.size, None, ctypes.byref(out))
    assert rc == code
    assert out.value is None
    assert len(L.dnnmg_last_error()) > 0


def test_create_rejects_null_and_size_mismatch():
    L = pam.lib()
    c = cfg()
    s = pam.sizes(4, 3, 2)
    cxy = np.zeros(2 * s["Nc"])
    w = np.zeros(pam.weight_count(c), dtype=np.float32)
    out = ctypes.c_void_p()
    vp = ctypes.c_void_p
    assert L.dnnmg_create(ctypes.byref(c), None, w.ctypes.data_as(vp), w.size, None, ctypes.byref(out)) == pam.DNNMG_EINVAL
    assert L.dnnmg_create(ctypes.byref(c), cxy.ctypes.data_as(vp), None, w.size, None, ctypes.byref(out)) == pam.DNNMG_EINVAL
    assert L.dnnmg_create(ctypes.byref(c), cxy.ctypes.data_as(vp), w.ctypes.data_as(vp), w.size - 1, None,
                          ctypes.byref(out)) == pam.DNNMG_EINVAL
    assert b"n_weights" in L.dnnmg_last_error()
    cxy[3] = np.nan
    assert L.dnnmg_create(ctypes.byref(c), cxy.ctypes.data_as(vp), w.ctypes.data_as(vp), w.size, None,
                          ctypes.byref(out)) == pam.DNNMG_EINVAL
    assert L.dnnmg_create(None, cxy.ctypes.data_as(vp), w.ctypes.data_as(vp), w.size, None,
                          ctypes.byref(out)) == pam.DNNMG_EINVAL
    assert L.dnnmg_create(ctypes.byref(c), cxy.ctypes.data_as(vp), w.ctypes.data_as(vp), w.size, None,
                          None) == pam.DNNMG_EINVAL


def test_calls_on_null_context_fail_cleanly():
    L = pam.lib()
    assert L.dnnmg_step(None, None, None, None, None) == pam.DNNMG_EINVAL
    assert L.dnnmg_restrict_rhs(None, None, None) == pam.DNNMG_EINVAL
    assert L.dnnmg_defect(None, None, None, None, None) == pam.DNNMG_EINVAL
    assert L.dnnmg_rhs_restrict(None, None, None, None, None) == pam.DNNMG_EINVAL
    assert L.dnnmg_get_state(None, None, None, None) == pam.DNNMG_EINVAL
    assert L.dnnmg_set_state(None, None, None, 0, None) == pam.DNNMG_EINVAL
    assert L.dnnmg_patch_output(None, None, None) == pam.DNNMG_EINVAL
    assert L.dnnmg_destroy(None) == pam.DNNMG_EINVAL
    assert L.dnnmg_step_count(None) == -1
    out = ctypes.c_void_p()
    assert L.dnnmg_batch_create(0, ctypes.byref(out)) == pam.DNNMG_EINVAL
    assert L.dnnmg_batch_create(100000, ctypes.byref(out)) == pam.DNNMG_EINVAL
    assert L.dnnmg_step_batch(None, None, 1, None, None, None, None) == pam.DNNMG_EINVAL


def test_fp8_config_sizes_and_quantiser_validation():
    c8, c16 = cfg(nx=64, ny=32, precision=2), cfg(nx=64, ny=32, precision=1)
    assert pam.workspace_bytes(c8) > 0
    # FP8 network input: 128 bytes + a 4-byte scale per patch instead of 208 BF16 bytes
    assert pam.workspace_bytes(c8) < pam.workspace_bytes(c16)
    L = pam.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.dnnmg_quantize_e4m3(None, 1, 1, fake, fake, None) == pam.DNNMG_EINVAL
    assert L.dnnmg_quantize_e4m3(fake, 0, 4, fake, fake, None) == pam.DNNMG_EINVAL
    assert L.dnnmg_quantize_e4m3(fake, 4, 0, fake, fake, None) == pam.DNNMG_EINVAL


def test_unknown_flags_rejected_on_host():
    L = pam.lib()
    c = cfg(flags=64)
    s = pam.sizes(4, 3, 2)
    cxy = np.zeros(2 * s["Nc"])
    w = np.zeros(pam.weight_count(c), dtype=np.float32)
    out = ctypes.c_void_p()
    rc = L.dnnmg_create(ctypes.byref(c), cxy.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p),
                        w.size, None, ctypes.byref(out))
    assert rc == pam.DNNMG_EINVAL and b"flags" in L.dnnmg_last_error()


def test_noalloc_entry_point_rejects_on_the_host():
    """dnnmg_rhs_restrict_noalloc validates before touching the device: NULL
    pointers, K, dt, and meshes beyond the static scratch's patch limit."""
    L = pam.lib()
    p = ctypes.c_void_p(256)    # never dereferenced: every case fails validation first
    assert pam.noalloc_scratch_bytes() >= 64 * pam.DNNMG_NOALLOC_MAX_PATCHES
    cases = [((4, 3, 2, 0.01, None, p, p, p), "NULL"),
             ((4, 3, 4, 0.01, p, p, p, p), "K must be"),
             ((4, 3, 2, 0.0, p, p, p, p), "dt"),
             ((0, 3, 2, 0.01, p, p, p, p), "nx, ny"),
             ((1024, 257, 2, 0.01, p, p, p, p), "allocation-free limit")]
    for args, msg in cases:
        rc = L.dnnmg_rhs_restrict_noalloc(*args, None)
        assert rc == pam.DNNMG_EINVAL, args
        assert msg in L.dnnmg_last_error().decode(), (args, L.dnnmg_last_error())


def test_crank_nicolson_flag_is_known_and_holds_fp64_maps():
    """DNNMG_F_CRANK_NICOLSON is a valid flag; its workspace adds the FP64
    map vectors (64 bytes per patch, 256-byte aligned)."""
    base = pam.workspace_bytes(cfg())
    cn = pam.workspace_bytes(cfg(flags=pam.DNNMG_F_CRANK_NICOLSON))
    P = 4 * 3
    assert cn - base == (64 * P + 255) // 256 * 256
    assert pam.workspace_bytes(cfg(flags=pam.DNNMG_F_CRANK_NICOLSON | pam.DNNMG_F_NANCHECK)) == cn


def test_paper_net_weight_counts_and_validation():
    """DNNMG_F_PAPER_NET: the weight vector of the paper's form (8634 values
    at K = 1, H = 32: Sec. 5.2); Hm must be 0, nu > 0, FP32/BF16 only; H = 96
    (the paper's K = 2 network) runs FP32 and BF16; the GRU flag is known."""
    P = pam.DNNMG_F_PAPER_NET
    assert pam.weight_count(cfg(K=1, H=32, Hm=0, flags=P)) == 8634
    assert pam.weight_count(cfg(K=2, H=96, Hm=0, flags=P)) == 60960 + 36 + 36 + 50
    assert pam.workspace_bytes(cfg(K=1, H=32, Hm=0, flags=P)) > 0
    assert pam.workspace_bytes(cfg(K=2, H=96, Hm=0, flags=P, precision=1)) > 0
    assert pam.workspace_bytes(cfg(K=2, H=64, Hm=64, flags=P)) == 0
    assert pam.workspace_bytes(cfg(K=2, H=64, Hm=0, flags=P, precision=2)) == 0
    assert pam.workspace_bytes(cfg(K=2, H=64, Hm=0, flags=P, nu=0.0)) == 0
    assert pam.workspace_bytes(cfg(H=96, Hm=0)) > 0
    assert pam.workspace_bytes(cfg(H=96, Hm=0, precision=2)) == 0
    assert pam.workspace_bytes(cfg(flags=pam.DNNMG_F_GRU_RESET_AFTER)) > 0
    assert pam.workspace_bytes(cfg(flags=pam.DNNMG_F_GRU_RESET_AFTER, precision=2)) == 0


def test_nancheck_flag_validation():
    """DNNMG_F_NANCHECK is a known flag (the configuration is valid); unknown
    flag bits are not; dnnmg_nonfinite rejects NULL arguments on the host."""
    assert pam.workspace_bytes(cfg(flags=pam.DNNMG_F_NANCHECK)) > pam.workspace_bytes(cfg()) - 1
    assert pam.workspace_bytes(cfg(flags=pam.DNNMG_F_NANCHECK | pam.DNNMG_F_UNFUSED)) > 0
    assert pam.workspace_bytes(cfg(flags=64)) == 0
    L = pam.lib()
    out = ctypes.c_int(7)
    assert L.dnnmg_nonfinite(None, 1, ctypes.byref(out), None) == pam.DNNMG_EINVAL
    assert out.value == 7


def test_patch_outputs_flag_and_tile_frame_workspace():
    """DNNMG_F_PATCH_OUTPUTS is a known flag that changes no buffer; the
    one-launch form (K=2, H=64, BF16) holds a tile frame of 280 (x, y) pairs
    per 8 x 8-patch tile (ragged tiles counted whole), the other forms none."""
    one = cfg(nx=20, ny=19, precision=1)
    assert pam.workspace_bytes(cfg(nx=20, ny=19, precision=1, flags=pam.DNNMG_F_PATCH_OUTPUTS)) == \
        pam.workspace_bytes(one)
    frame = 3 * 3 * 280 * 8
    unfused = pam.workspace_bytes(cfg(nx=20, ny=19, precision=1, flags=pam.DNNMG_F_UNFUSED))
    assert pam.workspace_bytes(one) - unfused >= frame
    assert pam.workspace_bytes(one) - unfused < frame + 512
