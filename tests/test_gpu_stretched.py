"""The stretched-mesh workload at full size: 64 concurrent flows of 128 x 128
coarse elements on [0, s_f] x [0, 1] (s_f ~ U[1, 8], all-Dirichlet), K = 3,
H = 128, MLP 128-128-162, stepped together through one batched, graph-
captured launch in FP32, BF16 and FP8 E4M3.  Sampled flows are checked on
windows the oracle computes in seconds (outputs more than 3 patches from a
window edge depend on window data only): FP32 against the FP64 step (1e-5),
BF16 against it (2e-2), FP8 against the oracle's FP8 form (2e-2, see
test_gpu_fp8), each in relative L2 and in max |error| over max |oracle|.
FP8's max-relative bound is 0.1: there the largest node errors come from
single E4M3 code flips (the matrix cores' FP8 products carry ~1e-4 relative
error, enough to move a value of the hidden layer across a rounding
boundary), and one flip moves a patch's output by one code step of the
flipped value, up to 2^-3 of it, times its output weights.  The BF16 step
is also run for the configuration's 100 steps and checked on the whole
field of two flows."""
import numpy as np
import pytest

from paper_2008_11520_amd import synth

from gpu_common import make_gpu_flow, make_oracle_flow, rel_l2, rel_max, to_dev, window, window_fields

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2008_11520_amd as pam
    pam.lib()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 2e-2), ("fp8", 2e-2)])
def test_stretched_64_flows_k3_batched_sampled_windows(prec, tol):
    import torch
    import paper_2008_11520_amd as pam
    wl = synth.workload("stretched64x128x128_k3")
    K, H, Hm = wl.K, wl.H, wl.Hm
    w = synth.xavier_weights(K, H, Hm, wl.weight_seed)
    n = 1 << K
    model = make_gpu_flow(wl.flows[0], K, H, Hm, wl.nu, w, prec)
    ctxs = [make_gpu_flow(f, K, H, Hm, wl.nu, w, prec, share=model) for f in wl.flows]
    s = ctxs[0].s
    dbar = [torch.empty(2 * s["Fn"], dtype=torch.float32, device="cuda") for _ in ctxs]
    bL = [torch.empty(2 * s["Nc"], dtype=torch.float64, device="cuda") for _ in ctxs]
    batch = pam.Batch(64)
    st = torch.cuda.Stream()
    fields = [f.fields(0) for f in wl.flows]
    with torch.cuda.stream(st):
        vs = [to_dev(v.reshape(-1)) for v, _ in fields]
        ps = [to_dev(p) for _, p in fields]
        batch.prepare(ctxs, vs, ps, dbar, bL, stream=st)
        batch.launch(graph=True, stream=st)
    st.synchronize()
    m = 3
    for fi, (i0, j0) in ((0, (0, 0)), (17, (60, 50)), (63, (116, 116)), (40, (0, 100))):
        flow = wl.flows[fi]
        i1, j1 = min(i0 + 12, flow.nx), min(j0 + 12, flow.ny)
        sub = window(flow, i0, i1, j0, j1)
        o = oracle.OracleFlow(sub.nx, sub.ny, K, H, Hm, sub.dt, wl.nu, sub.dirichlet, sub.cxy,
                              w.astype(np.float64), fp8=(prec == "fp8"))
        ref = o.step(*window_fields(flow, 0, i0, i1, j0, j1), want=("Dbar", "bL"))
        Dg = dbar[fi].cpu().numpy().reshape(flow.ny * n + 1, flow.nx * n + 1, 2)
        bg = bL[fi].cpu().numpy().reshape(flow.ny + 1, flow.nx + 1, 2)
        Dr = ref["Dbar"].reshape(sub.ny * n + 1, sub.nx * n + 1, 2)
        br = ref["bL"].reshape(sub.ny + 1, sub.nx + 1, 2)
        a0 = 0 if i0 == 0 else m
        a1 = sub.nx if i1 == flow.nx else sub.nx - m
        c0 = 0 if j0 == 0 else m
        c1 = sub.ny if j1 == flow.ny else sub.ny - m
        dg = Dg[(j0 + c0) * n:(j0 + c1) * n + 1, (i0 + a0) * n:(i0 + a1) * n + 1]
        dr = Dr[c0 * n:c1 * n + 1, a0 * n:a1 * n + 1]
        bgw, brw = bg[j0 + c0 + 1:j0 + c1, i0 + a0 + 1:i0 + a1], br[c0 + 1:c1, a0 + 1:a1]
        e = [rel_l2(dg, dr), rel_max(dg, dr), rel_l2(bgw, brw), rel_max(bgw, brw)]
        print("stretched", prec, fi, (i0, j0), "Dbar %.2e (max %.2e) bL %.2e (max %.2e)" % tuple(e))
        max_tol = 0.1 if prec == "fp8" else tol
        assert e[0] < tol and e[2] < tol and e[1] < max_tol and e[3] < max_tol
    batch.close()
    for c in ctxs:
        c.close()
    model.close()


def test_stretched_64_flows_k3_bf16_100_steps_whole_field():
    """The 100 steps of the stretched workload: all 64 flows stepped
    together by replaying the captured batched launch, every flow with its
    own field sequence (copied into the launch's input buffers, then the
    step described and the captured graph replayed), BF16 operands as the
    benchmark times them.  Two flows, the shortest and the longest domain
    (the extremes of the stretch factor), are checked on
    the whole field against an FP64 oracle run of their own: every step the
    correction and b_L, relative L2 and max-relative; every twentieth step
    also the tile-edge and Dirichlet checks and the GRU state.  The state and
    the previous corrected velocity are carried over all 100 steps."""
    import torch
    import paper_2008_11520_amd as pam
    from gpu_common import assert_step_errors, merge_worst, step_errors
    wl = synth.workload("stretched64x128x128_k3")
    K, H, Hm = wl.K, wl.H, wl.Hm
    w = synth.xavier_weights(K, H, Hm, wl.weight_seed)
    model = make_gpu_flow(wl.flows[0], K, H, Hm, wl.nu, w, "bf16", flags=0)
    ctxs = [make_gpu_flow(f, K, H, Hm, wl.nu, w, "bf16", share=model, flags=0) for f in wl.flows]
    s = ctxs[0].s
    dbar = [torch.empty(2 * s["Fn"], dtype=torch.float32, device="cuda") for _ in ctxs]
    bL = [torch.empty(2 * s["Nc"], dtype=torch.float64, device="cuda") for _ in ctxs]
    hs = torch.empty(s["P"] * H, dtype=torch.float32, device="cuda")
    vs = [torch.empty(2 * s["Nc"], dtype=torch.float32, device="cuda") for _ in ctxs]
    ps = [torch.empty(s["Nc"], dtype=torch.float32, device="cuda") for _ in ctxs]
    lengths = [float(np.max(f.cxy[..., 0])) for f in wl.flows]
    checked = (int(np.argmin(lengths)), int(np.argmax(lengths)))
    orc = {fi: make_oracle_flow(wl.flows[fi], K, H, Hm, wl.nu, w) for fi in checked}
    batch = pam.Batch(64)
    st = torch.cuda.Stream()
    worst = {}
    nsteps = 100
    for n in range(nsteps):
        fields = [f.fields(n) for f in wl.flows]
        with torch.cuda.stream(st):
            for (v, p), vd, pd in zip(fields, vs, ps):
                vd.copy_(torch.from_numpy(np.ascontiguousarray(v.reshape(-1), dtype=np.float32)))
                pd.copy_(torch.from_numpy(np.ascontiguousarray(p.reshape(-1), dtype=np.float32)))
            batch.prepare(ctxs, vs, ps, dbar, bL, stream=st)
            batch.launch(graph=True, stream=st)
        st.synchronize()
        full = n % 20 == 19 or n == nsteps - 1
        for fi in checked:
            flow = wl.flows[fi]
            ref = orc[fi].step(*fields[fi], want=("Dbar", "bL"))
            got = dict(Dbar=dbar[fi].cpu().numpy().reshape(-1, 2), bL=bL[fi].cpu().numpy().reshape(-1, 2))
            if full:
                with torch.cuda.stream(st):
                    ctxs[fi].get_state(hs, None, stream=st)
                st.synchronize()
                got["h"] = hs.cpu().numpy().reshape(s["P"], H)
                e = step_errors(got, ref, orc[fi].h, flow.nx, flow.ny, K, flow.dirichlet)
                print("stretched flow %d step %d Dbar %.2e (max %.2e, edge %.2e) h %.2e (max %.2e) bL %.2e (max %.2e)"
                      % (fi, n + 1, e["Dbar"], e["Dbar_max"], e["Dbar_edge_max"], e["h"], e["h_max"],
                         e["bL"], e["bL_max"]), flush=True)
            else:
                e = dict(Dbar=rel_l2(got["Dbar"], ref["Dbar"]), Dbar_max=rel_max(got["Dbar"], ref["Dbar"]),
                         bL=rel_l2(got["bL"], ref["bL"]), bL_max=rel_max(got["bL"], ref["bL"]),
                         Dbar_dirichlet_nonzero=0)
            merge_worst(worst, e)
            assert_step_errors(e, 2e-2, 2e-2)
    print("stretched worst over %d steps" % nsteps, worst)
    assert batch.captures == 1
    batch.close()
    for c in ctxs:
        c.close()
    model.close()
