"""GPU path (through the C ABI) against the FP64 oracle on the same seeded inputs.

Tolerances (relative L2 over the whole output, and max |error| over
max |oracle|, unless stated):
  P v                  1e-6 max-rel: FP32 bilinear interpolation of FP32 values
  D (defect)           derived per test: FP32 assembly; see test docstrings
  d (correction), per-patch output, state
                       1e-5 FP32 operands, 2e-2 BF16 operands, on both norms;
                       tile-edge nodes reported separately; exactly 0 at
                       Dirichlet nodes
  b_L stage            1e-10 (FP64 right-hand side and restriction of given inputs)
  b_L end to end       1e-5 FP32 (bounded by the correction's error)
  zero weights         d == 0 bitwise; b_L per coarse node within the FP32
                       rounding of the stored state u = P v, carried through
                       the FP64 weights (zero_weight_bl_bound)
"""
import numpy as np
import pytest

import oracle
from paper_2008_11520_amd import synth

from gpu_common import (EPS32, GpuRunner, assert_step_errors, make_gpu_flow, make_oracle_flow, merge_worst,
                        node_errors, rel_l2, rel_max, step_errors, to_dev, window, window_fields)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2008_11520_amd as pam
    pam.lib()


def _flows():
    return {
        "unit16_k1": (synth.unit_square_flow(16, 16, 1, 0.01), 1, 32, 0),
        "ragged13x7_k2_perturbed": (synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5), 2, 64, 64),
        "stretched5x3_k3": (synth.stretched_flow(5, 3, 3.7, 4, 0.01), 3, 128, 128),
        "single1x1_k2": (synth.unit_square_flow(1, 1, 2, 0.01), 2, 32, 32),
        "strip9x1_k1": (synth.channel_flow(9, 1, 6, 0.005), 1, 64, 0),
    }


FLOWS = _flows()


@pytest.mark.parametrize("name", sorted(FLOWS))
def test_prolongation(name):
    import torch
    flow, K, H, Hm = FLOWS[name]
    w = synth.xavier_weights(K, H, Hm, 1234)
    g = make_gpu_flow(flow, K, H, Hm, 1e-3, w)
    v, p = flow.fields(3)
    s = g.s
    pv = torch.empty(2 * s["Fn"], dtype=torch.float32, device="cuda")
    pp = torch.empty(s["Fn"], dtype=torch.float32, device="cuda")
    g.prolong(to_dev(v.reshape(-1)), to_dev(p), pv, pp)
    torch.cuda.synchronize()
    ref_v = oracle.prolong(flow.nx, flow.ny, K, v.astype(np.float64))
    ref_p = oracle.prolong(flow.nx, flow.ny, K, p.astype(np.float64))
    assert rel_max(pv.cpu().numpy().reshape(-1, 2), ref_v) < 1e-6
    assert rel_max(pp.cpu().numpy(), ref_p) < 1e-6


@pytest.mark.parametrize("name", sorted(FLOWS))
def test_defect_with_given_previous_velocity(name):
    """Defect against a seeded previous corrected velocity (mass term active
    and dominant).  FP32 evaluation: each element term carries a few ulp of
    its own size, so 1e-5 relative L2 is ~100x the FP32 unit roundoff."""
    import torch
    flow, K, H, Hm = FLOWS[name]
    w = synth.xavier_weights(K, H, Hm, 1234)
    g = make_gpu_flow(flow, K, H, Hm, 1e-3, w)
    s = g.s
    rng = synth.SplitMix64(77)
    u_prev = rng.uniform(2 * s["Fn"], -1.0, 1.0).astype(np.float32)
    g.set_state(None, to_dev(u_prev), steps=1)
    v, p = flow.fields(2)
    D = torch.empty(2 * s["Fn"], dtype=torch.float32, device="cuda")
    g.defect(to_dev(v.reshape(-1)), to_dev(p), D)
    torch.cuda.synchronize()
    pv = oracle.prolong(flow.nx, flow.ny, K, v.astype(np.float64))
    pp = oracle.prolong(flow.nx, flow.ny, K, p.astype(np.float64))
    ref = oracle.defect(flow.nx, flow.ny, K, flow.cxy.reshape(-1, 2), pv, pp,
                        u_prev.astype(np.float64).reshape(-1, 2), flow.dt, 1e-3, flow.dirichlet)
    got = D.cpu().numpy().reshape(-1, 2)
    err = rel_l2(got, ref)
    S = oracle.defect_abs(flow.nx, flow.ny, K, flow.cxy.reshape(-1, 2), pv, pp,
                          u_prev.astype(np.float64).reshape(-1, 2), 1.0 / flow.dt, 1e-3)
    ratio = np.abs(got - ref) / (EPS32 * S + 1e-300)
    print("defect rel-L2 error", name, err, "max error / (eps32 * scale) %.2f" % ratio.max())
    assert err < 1e-5
    assert ratio.max() <= 64.0


@pytest.mark.parametrize("name", sorted(FLOWS))
def test_defect_first_step_without_mass_term(name):
    """Before the first step the previous velocity is P v itself, and the
    kernel leaves the mass term out, so only convection, diffusion and
    pressure remain.  Their element terms cancel in the node sums (a smooth
    field's residual is O(h^2) of its element terms), so the error is judged
    node by node against the running-error scale of those terms: the oracle's
    defect_abs with the mass term off (every term, and every sum inside one,
    in absolute value).  An FP32 evaluation of a few tens of operations per
    term stays within 64 eps32 of that scale."""
    import torch
    flow, K, H, Hm = FLOWS[name]
    w = synth.xavier_weights(K, H, Hm, 1234)
    g = make_gpu_flow(flow, K, H, Hm, 1e-3, w)
    s = g.s
    v, p = flow.fields(4)
    D = torch.empty(2 * s["Fn"], dtype=torch.float32, device="cuda")
    g.defect(to_dev(v.reshape(-1)), to_dev(p), D)
    torch.cuda.synchronize()
    pv = oracle.prolong(flow.nx, flow.ny, K, v.astype(np.float64))
    pp = oracle.prolong(flow.nx, flow.ny, K, p.astype(np.float64))
    ref = oracle.defect(flow.nx, flow.ny, K, flow.cxy.reshape(-1, 2), pv, pp, pv, flow.dt, 1e-3, flow.dirichlet)
    S = oracle.defect_abs(flow.nx, flow.ny, K, flow.cxy.reshape(-1, 2), pv, pp, pv, 0.0, 1e-3)
    mask = oracle.dirichlet_mask(flow.nx, flow.ny, K, flow.dirichlet)
    got = D.cpu().numpy().reshape(-1, 2)
    err = np.abs(got - ref)
    ratio = err / (EPS32 * S + 1e-300)
    print("defect (no mass term)", name, "max error / (eps32 * scale) %.2f" % ratio.max(),
          "rel-L2 %.2e" % rel_l2(got, ref))
    assert np.all(got[mask] == 0.0)
    assert ratio.max() <= 64.0


@pytest.mark.parametrize("name", sorted(FLOWS))
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_step_sequence_matches_oracle(name, prec, tol):
    flow, K, H, Hm = FLOWS[name]
    w = synth.xavier_weights(K, H, Hm, 1234)
    g = GpuRunner(make_gpu_flow(flow, K, H, Hm, 1e-3, w, prec))
    o = make_oracle_flow(flow, K, H, Hm, 1e-3, w)
    nsteps = 10 if name == "unit16_k1" else 5
    worst = {}
    for n in range(nsteps):
        v, p = flow.fields(n)
        got = g.step(v, p)
        ref = o.step(v, p, want=("Dbar", "bL", "dpatch"))
        merge_worst(worst, step_errors(got, ref, o.h, flow.nx, flow.ny, K, flow.dirichlet))
    print("step errors", name, prec, worst)
    assert_step_errors(worst, tol, 1e-5 if prec == "fp32" else tol)


@pytest.mark.parametrize("name", ["unit16_k1", "ragged13x7_k2_perturbed", "stretched5x3_k3"])
def test_rhs_restrict_stage_fp64(name):
    """b_L = P^T (1/dt) M_f (P v + dbar) for seeded v and dbar: FP64 on both sides."""
    import torch
    flow, K, H, Hm = FLOWS[name]
    w = synth.xavier_weights(K, H, Hm, 1234)
    g = make_gpu_flow(flow, K, H, Hm, 1e-3, w)
    s = g.s
    v, _ = flow.fields(1)
    dbar = (0.3 * synth.SplitMix64(5).uniform(2 * s["Fn"], -1.0, 1.0)).astype(np.float32)
    b = torch.empty(2 * s["Nc"], dtype=torch.float64, device="cuda")
    g.rhs_restrict(to_dev(v.reshape(-1)), to_dev(dbar), b)
    torch.cuda.synchronize()
    ref = oracle.rhs_restrict(flow.nx, flow.ny, K, flow.cxy.reshape(-1, 2), v.astype(np.float64),
                              dbar.astype(np.float64).reshape(-1, 2), flow.dt)
    err = rel_max(b.cpu().numpy().reshape(-1, 2), ref)
    print("rhs stage error", name, err)
    assert err < 1e-10


def test_state_read_back_and_round_trip():
    """The library keeps u_prev in rows padded to 16 nodes; get_state and
    set_state convert to and from the caller's NX+1 rows (NX+1 = 53 here).
    After two steps the corrected velocity read back matches the oracle's, and
    a state written with set_state reads back bit for bit."""
    import torch
    flow, K, H, Hm = FLOWS["ragged13x7_k2_perturbed"]
    w = synth.xavier_weights(K, H, Hm, 1234)
    g = GpuRunner(make_gpu_flow(flow, K, H, Hm, 1e-3, w))
    o = make_oracle_flow(flow, K, H, Hm, 1e-3, w)
    for n in range(2):
        v, p = flow.fields(n)
        g.step(v, p)
        o.step(v, p)
    s = g.g.s
    u = torch.empty(2 * s["Fn"], dtype=torch.float32, device="cuda")
    g.g.get_state(None, u)
    torch.cuda.synchronize()
    err = rel_l2(u.cpu().numpy().reshape(-1, 2), o.uprev)
    print("u_prev read back vs oracle", err)
    assert err < 1e-5
    rng = np.random.default_rng(11)
    hh = rng.standard_normal(s["P"] * H).astype(np.float32)
    uu = rng.standard_normal(2 * s["Fn"]).astype(np.float32)
    g.g.set_state(to_dev(hh), to_dev(uu), steps=2)
    h2 = torch.empty(s["P"] * H, dtype=torch.float32, device="cuda")
    u2 = torch.empty(2 * s["Fn"], dtype=torch.float32, device="cuda")
    g.g.get_state(h2, u2)
    torch.cuda.synchronize()
    assert np.array_equal(h2.cpu().numpy(), hh) and np.array_equal(u2.cpu().numpy(), uu)


def zero_weight_bl_bound(flow, K, v):
    """Per coarse node, the bound on |b_L - oracle| when d = 0.  The step forms
    b_L in FP64 from the stored FP32 corrected velocity u = P v: P v at a node
    takes two row interpolations (a difference and a fused multiply-add
    each), their difference and one fused multiply-add across, so
    |fl(P v) - P v| <= 12 * 2^-24 max|v| to first order (16 taken); b_L sums
    the nodal values with the nonnegative weights of R (1/dt) M, whose row
    sums the oracle gives as R (1/dt) M 1.  Plus FP64 rounding."""
    s = oracle.sizes(flow.nx, flow.ny, K)
    ones = np.ones(((flow.nx + 1) * (flow.ny + 1), 2))
    w1 = oracle.rhs_restrict(flow.nx, flow.ny, K, flow.cxy.reshape(-1, 2), ones, np.zeros((s["Fn"], 2)), flow.dt)
    return 16 * 2.0 ** -24 * float(np.abs(v).max()) * np.abs(w1) + 1e-12 * np.abs(w1).max()


@pytest.mark.parametrize("name", ["ragged13x7_k2_perturbed", "stretched5x3_k3"])
def test_zero_weights(name):
    flow, K, H, Hm = FLOWS[name]
    w = np.zeros_like(synth.xavier_weights(K, H, Hm, 1234))
    g = GpuRunner(make_gpu_flow(flow, K, H, Hm, 1e-3, w))
    o = make_oracle_flow(flow, K, H, Hm, 1e-3, w)
    for n in range(3):
        v, p = flow.fields(n)
        got = g.step(v, p)
        ref = o.step(v, p, want=("bL",))
        assert np.all(got["Dbar"] == 0.0) and np.all(got["h"] == 0.0)
        err = np.abs(got["bL"] - ref["bL"])
        bound = zero_weight_bl_bound(flow, K, v)
        print("zero weights", name, n, "max err / bound %.3f" % float((err / bound).max()))
        assert np.all(err <= bound)


def test_call_order_errors():
    import torch
    import paper_2008_11520_amd as pam
    flow, K, H, Hm = FLOWS["unit16_k1"]
    g = make_gpu_flow(flow, K, H, Hm, 1e-3, synth.xavier_weights(K, H, Hm, 1))
    b = torch.empty(2 * g.s["Nc"], dtype=torch.float64, device="cuda")
    with pytest.raises(pam.DnnmgError) as e:
        g.restrict_rhs(b)
    assert e.value.code == pam.DNNMG_ESTATE
    d = torch.empty(g.s["P"] * g.s["nout"], dtype=torch.float32, device="cuda")
    with pytest.raises(pam.DnnmgError) as e:
        g.patch_output(d)
    assert e.value.code == pam.DNNMG_ESTATE


def test_inverted_element_is_rejected():
    import paper_2008_11520_amd as pam
    flow = synth.unit_square_flow(3, 3, 1, 0.01)
    cxy = flow.cxy.copy()
    cxy[1, 1] = cxy[2, 2] + 0.2      # fold an interior node across its neighbours
    cfg = pam.make_config(3, 3, 1, 32, 0, 0.01, 1e-3, "fp32", 15)
    with pytest.raises(pam.DnnmgError) as e:
        pam.DnnMG(cfg, cxy, synth.xavier_weights(1, 32, 0, 1))
    assert e.value.code == pam.DNNMG_EINVAL


def test_bitwise_determinism():
    flow, K, H, Hm = FLOWS["ragged13x7_k2_perturbed"]
    w = synth.xavier_weights(K, H, Hm, 1234)
    outs = []
    for _ in range(2):
        g = GpuRunner(make_gpu_flow(flow, K, H, Hm, 1e-3, w, "bf16"))
        res = [g.step(*flow.fields(n)) for n in range(3)]
        outs.append(res)
    for a, b in zip(*outs):
        for k in a:
            assert np.array_equal(a[k], b[k]), k


ONE_LAUNCH_MESHES = {
    # one ragged tile row, two tile columns (8 + 5 patches)
    "channel13x7": lambda: synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5),
    # 3 x 3 tiles, the last column and row ragged; Dirichlet on every side, so
    # the middle tile has neighbours on all sides and the mesh-end lines lie
    # inside the ragged tiles
    "square20x19": lambda: synth.unit_square_flow(20, 19, 4, 0.01),
    # 2 x 2 full tiles: the mesh ends on tile lines
    "channel16x16": lambda: synth.channel_flow(16, 16, 6, 0.005, perturb_seed=8),
}


@pytest.mark.parametrize("mesh", sorted(ONE_LAUNCH_MESHES))
@pytest.mark.parametrize("Hm", [64, 0])
def test_fused_step_equals_unfused_bitwise(Hm, mesh):
    """K=2, H=64, BF16: the one-launch defect + GRU + MLP + averaging inside
    the tiles (with and without the per-patch outputs kept) and the separate
    launches do the same arithmetic in the same order: correction, state, b_L
    and u_prev bit for bit, the kept per-patch outputs too."""
    import torch
    import paper_2008_11520_amd as pam
    flow = ONE_LAUNCH_MESHES[mesh]()
    K, H = 2, 64
    w = synth.xavier_weights(K, H, Hm, 1234)
    runs = []
    for flags in (0, pam.DNNMG_F_PATCH_OUTPUTS, pam.DNNMG_F_UNFUSED):
        cfg = pam.make_config(flow.nx, flow.ny, K, H, Hm, flow.dt, 1e-3, "bf16", flow.dirichlet, flags)
        g = GpuRunner(pam.DnnMG(cfg, flow.cxy, w))
        res = []
        for n in range(4):
            r = g.step(*flow.fields(n))
            u = torch.empty(2 * g.g.s["Fn"], dtype=torch.float32, device="cuda")
            g.g.get_state(None, u)
            torch.cuda.synchronize()
            r["uprev"] = u.cpu().numpy()
            res.append(r)
        runs.append((flags, res))
    assert "dpatch" not in runs[0][1][0] and "dpatch" in runs[1][1][0]
    ref = runs[2][1]
    for flags, res in runs[:2]:
        for a, b in zip(res, ref):
            for k in a:
                assert np.array_equal(a[k], b[k]), (flags, k)


def test_patch_output_refused_after_one_launch_step_without_the_flag():
    import torch
    import paper_2008_11520_amd as pam
    flow = synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5)
    w = synth.xavier_weights(2, 64, 64, 1)
    cfg = pam.make_config(flow.nx, flow.ny, 2, 64, 64, flow.dt, 1e-3, "bf16", flow.dirichlet, 0)
    g = pam.DnnMG(cfg, flow.cxy, w)
    v, p = flow.fields(0)
    g.step(to_dev(v.reshape(-1)), to_dev(p))
    d = torch.empty(g.s["P"] * g.s["nout"], dtype=torch.float32, device="cuda")
    with pytest.raises(pam.DnnmgError) as e:
        g.patch_output(d)
    assert e.value.code == pam.DNNMG_ESTATE and "DNNMG_F_PATCH_OUTPUTS" in str(e.value)


def test_batched_step_equals_single_steps_bitwise():
    import torch
    import paper_2008_11520_amd as pam
    K, H, Hm = 2, 64, 64
    w = synth.xavier_weights(K, H, Hm, 1234)
    flows = [synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5), synth.channel_flow(32, 8, 4, 0.005),
             synth.channel_flow(5, 3, 9, 0.005)]
    for prec in ("fp32", "bf16"):
        single = [GpuRunner(make_gpu_flow(f, K, H, Hm, 1e-3, w, prec)) for f in flows]
        model = make_gpu_flow(flows[0], K, H, Hm, 1e-3, w, prec)
        batched = [make_gpu_flow(f, K, H, Hm, 1e-3, w, prec, share=model) for f in flows]
        runners = [GpuRunner(b) for b in batched]
        batch = pam.Batch(8)
        for n in range(3):
            fields = [f.fields(n) for f in flows]
            ref = [r.step(v, p) for r, (v, p) in zip(single, fields)]
            vs = [to_dev(v.reshape(-1)) for v, _ in fields]
            ps = [to_dev(p) for _, p in fields]
            batch.step(batched, vs, ps, [r.dbar for r in runners])
            for r, b, rf in zip(runners, batched, ref):
                b.restrict_rhs(r.bL)
                b.get_state(r.h, None)
                torch.cuda.synchronize()
                assert np.array_equal(r.dbar.cpu().numpy().reshape(-1, 2), rf["Dbar"])
                assert np.array_equal(r.bL.cpu().numpy().reshape(-1, 2), rf["bL"])
                assert np.array_equal(r.h.cpu().numpy().reshape(b.s["P"], -1), rf["h"])
        batch.close()


def test_batched_tile_frames_and_mixed_flags_bitwise():
    """The batched BF16 K=2 step with every flow's tile frame (flags 0: the
    per-patch outputs stay on chip), and with a mix in which one flow has no
    frame (DNNMG_F_UNFUSED: the whole batch stores and averages the per-patch
    outputs), equals the flows' own steps bit for bit; the per-patch outputs
    are refused exactly where the batched step kept them in the tiles."""
    import torch
    import paper_2008_11520_amd as pam
    K, H, Hm = 2, 64, 64
    w = synth.xavier_weights(K, H, Hm, 1234)
    flows = [synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5), synth.channel_flow(32, 8, 4, 0.005),
             synth.channel_flow(5, 3, 9, 0.005)]
    for flags in ([0, 0, 0], [0, pam.DNNMG_F_UNFUSED, pam.DNNMG_F_PATCH_OUTPUTS]):
        single = [GpuRunner(make_gpu_flow(f, K, H, Hm, 1e-3, w, "bf16", flags=fl)) for f, fl in zip(flows, flags)]
        model = make_gpu_flow(flows[0], K, H, Hm, 1e-3, w, "bf16")
        batched = [make_gpu_flow(f, K, H, Hm, 1e-3, w, "bf16", share=model, flags=fl) for f, fl in zip(flows, flags)]
        runners = [GpuRunner(b) for b in batched]
        batch = pam.Batch(8)
        for n in range(3):
            fields = [f.fields(n) for f in flows]
            ref = [r.step(v, p) for r, (v, p) in zip(single, fields)]
            vs = [to_dev(v.reshape(-1)) for v, _ in fields]
            ps = [to_dev(p) for _, p in fields]
            batch.step(batched, vs, ps, [r.dbar for r in runners])
            for r, b, rf in zip(runners, batched, ref):
                b.restrict_rhs(r.bL)
                b.get_state(r.h, None)
                torch.cuda.synchronize()
                assert np.array_equal(r.dbar.cpu().numpy().reshape(-1, 2), rf["Dbar"]), (flags, n)
                assert np.array_equal(r.bL.cpu().numpy().reshape(-1, 2), rf["bL"]), (flags, n)
                assert np.array_equal(r.h.cpu().numpy().reshape(b.s["P"], -1), rf["h"]), (flags, n)
        frames = not any(fl & pam.DNNMG_F_UNFUSED for fl in flags)
        for b, fl in zip(batched, flags):
            d = torch.empty(b.s["P"] * b.s["nout"], dtype=torch.float32, device="cuda")
            if frames and not fl & pam.DNNMG_F_PATCH_OUTPUTS:
                with pytest.raises(pam.DnnmgError) as e:
                    b.patch_output(d)
                assert e.value.code == pam.DNNMG_ESTATE
            else:
                b.patch_output(d)
        torch.cuda.synchronize()
        batch.close()


def test_channel_256x64_k2_full_size_100_steps():
    """The 256 x 64 channel (16384 patches), K=2, H=64, MLP 64-64-50, for
    the 100 steps of its configuration, FP32 and BF16 operands side by side
    against one FP64 oracle run: every step's correction, per-patch output,
    state and restricted rhs within the bounds (no drift beyond them), the
    worst error of every tenth step printed."""
    flow = synth.channel_flow(256, 64, 1, 0.005)
    K, H, Hm = 2, 64, 64
    w = synth.xavier_weights(K, H, Hm, 1234)
    runs = {prec: GpuRunner(make_gpu_flow(flow, K, H, Hm, 1e-3, w, prec)) for prec in ("fp32", "bf16")}
    tols = {"fp32": (1e-5, 1e-5), "bf16": (2e-2, 2e-2)}
    o = make_oracle_flow(flow, K, H, Hm, 1e-3, w)
    worst = {prec: {} for prec in runs}
    for n in range(100):
        v, p = flow.fields(n)
        ref = o.step(v, p, want=("Dbar", "bL", "dpatch"))
        for prec, g in runs.items():
            e = step_errors(g.step(v, p), ref, o.h, flow.nx, flow.ny, K, flow.dirichlet)
            merge_worst(worst[prec], e)
            assert_step_errors(e, *tols[prec])
            if n % 10 == 9:
                print("channel256x64 step %d %s Dbar %.2e (max %.2e) h %.2e (max %.2e) bL %.2e"
                      % (n + 1, prec, e["Dbar"], e["Dbar_max"], e["h"], e["h_max"], e["bL"]), flush=True)
    print("channel256x64 worst over 100 steps", worst)


def test_channel_1024x256_perturbed_steps_sampled_windows():
    """Full size (262144 patches), the launch configuration the benchmark
    times, for 5 steps, so the previous corrected velocity (mass term) and
    the GRU state carried between steps run at full size: after every step,
    windows the oracle steps alongside (the same 5 steps on the window's own
    data) are compared away from their edges.  Each step moves the reach of
    a window edge's missing neighbours inwards by about one patch (the
    defect reads one fine element beyond a patch, the averaging its
    neighbours' outputs), so the margin is steps + 2 patches; windows that
    touch the domain's boundary keep it there.  Relative L2 and max-relative
    of the correction and of b_L, per step."""
    flow = synth.channel_flow(1024, 256, 1, 0.005, perturb_seed=7)
    K, H, Hm = 2, 64, 64
    w = synth.xavier_weights(K, H, Hm, 1234)
    n = 1 << K
    nsteps = 5
    wins = ((0, 0, 24, 20), (500, 118, 24, 20), (1024 - 24, 256 - 20, 24, 20), (700, 0, 24, 20))
    for prec, tol in (("fp32", 1e-5), ("bf16", 2e-2)):
        g = GpuRunner(make_gpu_flow(flow, K, H, Hm, 1e-3, w, prec))
        subs = []
        for (i0, j0, wx, wy) in wins:
            i1, j1 = min(i0 + wx, 1024), min(j0 + wy, 256)
            sub = window(flow, i0, i1, j0, j1)
            subs.append((i0, j0, i1, j1, sub, make_oracle_flow(sub, K, H, Hm, 1e-3, w)))
        for step in range(nsteps):
            got = g.step(*flow.fields(step))
            Dg = got["Dbar"].reshape(flow.ny * n + 1, flow.nx * n + 1, 2)
            bg = got["bL"].reshape(flow.ny + 1, flow.nx + 1, 2)
            m = step + 2
            for (i0, j0, i1, j1, sub, o) in subs:
                ref = o.step(*window_fields(flow, step, i0, i1, j0, j1), want=("Dbar", "bL"))
                Dr = ref["Dbar"].reshape(sub.ny * n + 1, sub.nx * n + 1, 2)
                br = ref["bL"].reshape(sub.ny + 1, sub.nx + 1, 2)
                # interior region of the window (or up to the true boundary)
                a0 = 0 if i0 == 0 else m
                a1 = sub.nx if i1 == flow.nx else sub.nx - m
                c0 = 0 if j0 == 0 else m
                c1 = sub.ny if j1 == flow.ny else sub.ny - m
                dg = Dg[(j0 + c0) * n:(j0 + c1) * n + 1, (i0 + a0) * n:(i0 + a1) * n + 1]
                dr = Dr[c0 * n:c1 * n + 1, a0 * n:a1 * n + 1]
                bgw, brw = bg[j0 + c0 + 1:j0 + c1, i0 + a0 + 1:i0 + a1], br[c0 + 1:c1, a0 + 1:a1]
                e = dict(Dbar=rel_l2(dg, dr), Dbar_max=rel_max(dg, dr), bL=rel_l2(bgw, brw), bL_max=rel_max(bgw, brw))
                print("window", prec, "step", step, (i0, j0), {k: "%.2e" % x for k, x in e.items()}, flush=True)
                assert e["Dbar"] < tol and e["Dbar_max"] < tol
                assert max(e["bL"], e["bL_max"]) < (1e-5 if prec == "fp32" else tol)


def test_channel_1024x256_perturbed_200_steps_whole_field():
    """Full size (262144 patches) for the 200 steps of the configuration,
    whole fields against one FP64 oracle run: the BF16 step in the launch
    configuration the benchmark times (one launch, no per-patch outputs
    kept) and the FP32 step side by side.  Every step: the correction and
    b_L, relative L2 and max-relative; every twentieth step and the last,
    also the tile-edge and Dirichlet checks of the correction and the state
    h.  The GRU state and the previous corrected velocity are carried over
    all 200 steps, so this measures the drift at full length."""
    flow = synth.channel_flow(1024, 256, 1, 0.005, perturb_seed=7)
    K, H, Hm = 2, 64, 64
    w = synth.xavier_weights(K, H, Hm, 1234)
    runs = {prec: GpuRunner(make_gpu_flow(flow, K, H, Hm, 1e-3, w, prec, flags=0)) for prec in ("fp32", "bf16")}
    tols = {"fp32": 1e-5, "bf16": 2e-2}
    o = make_oracle_flow(flow, K, H, Hm, 1e-3, w)
    worst = {prec: {} for prec in runs}
    nsteps = 200
    for n in range(nsteps):
        v, p = flow.fields(n)
        ref = o.step(v, p, want=("Dbar", "bL"))
        full = n % 20 == 19 or n == nsteps - 1
        for prec, g in runs.items():
            got = g.step(v, p)
            if full:
                e = step_errors(got, ref, o.h, flow.nx, flow.ny, K, flow.dirichlet)
            else:
                e = dict(Dbar=rel_l2(got["Dbar"], ref["Dbar"]), Dbar_max=rel_max(got["Dbar"], ref["Dbar"]),
                         bL=rel_l2(got["bL"], ref["bL"]), bL_max=rel_max(got["bL"], ref["bL"]),
                         Dbar_dirichlet_nonzero=0)
            merge_worst(worst[prec], e)
            assert_step_errors(e, tols[prec], tols[prec])
            if full:
                print("channel1024x256 step %d %s Dbar %.2e (max %.2e, edge %.2e) h %.2e (max %.2e) bL %.2e (max %.2e)"
                      % (n + 1, prec, e["Dbar"], e["Dbar_max"], e["Dbar_edge_max"], e["h"], e["h_max"],
                         e["bL"], e["bL_max"]), flush=True)
    print("channel1024x256 worst over %d steps" % nsteps, worst)


def test_channel_1024x256_zero_weights_full_size():
    flow = synth.channel_flow(1024, 256, 1, 0.005, perturb_seed=7)
    K, H, Hm = 2, 64, 64
    w = np.zeros_like(synth.xavier_weights(K, H, Hm, 1))
    g = GpuRunner(make_gpu_flow(flow, K, H, Hm, 1e-3, w, "bf16"))
    v, p = flow.fields(0)
    got = g.step(v, p)
    assert np.all(got["Dbar"] == 0.0)
    s = oracle.sizes(flow.nx, flow.ny, K)
    ref = oracle.rhs_restrict(flow.nx, flow.ny, K, flow.cxy.reshape(-1, 2), v.astype(np.float64),
                              np.zeros((s["Fn"], 2)), flow.dt)
    err = np.abs(got["bL"] - ref)
    bound = zero_weight_bl_bound(flow, K, v)
    print("zero weights 1024x256: max err / bound %.3f" % float((err / bound).max()))
    assert np.all(err <= bound)
