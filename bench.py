#!/usr/bin/env python3
"""Throughput of the fine-level DNN-MG step on one MI355X.

A step is one pass of the whole hot path over one flow's patches: prolongation,
defect, network input, GRU + MLP, averaging, corrected velocity, FP64
right-hand side and restriction (dnnmg_step + dnnmg_restrict_rhs).  Inputs
(coarse v, p of every timed step) are resident in HBM before the timed region.

Prints one JSON line: patch-steps/s for the BF16-operand form (value), the
FP32-operand form beside it, the roofline of the dominant kernel measured
with HIP events recorded by the library on the launch stream, and the FP64
oracle timed on a bounded sample on the host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp8": 5000.0}
PEAK_FP32_VECTOR_TFLOPS = 157.3      # published: packed (two-wide) FP32 FMA on every lane
PEAK_FP64_VECTOR_TFLOPS = 78.6       # published FP64 vector rate
# the vector FP32 rate this build can reach: packed FP32 instructions are kept
# out of the generated code, so one FMA per lane per cycle: 256 CUs x 4 SIMDs x
# 16 lanes x 2 FLOP x 2.4 GHz (reported beside the published-peak fraction)
PEAK_FP32_VALU_TFLOPS = 78.6
STAGES = ["prolong_defect", "gru_mlp", "avg_rhs_fp64", "restrict_gather"]
# kernel source files per stage (their hash guards the stored traffic counters)
STAGE_SOURCES = {0: ["defect.hip"], 1: ["net.hip"], 2: ["rhs.hip"], 3: ["rhs.hip"]}
STAGE_KERNELS = {0: "k_defect", 1: "k_net", 2: "k_rhs", 3: "k_gather"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def per_patch_gemm_flop(K, H, Hm):
    from paper_2008_11520_amd import synth
    nin, nout, shapes = synth.net_shapes(K, H, Hm)
    return 2 * sum(o * i for o, i in shapes)


def per_patch_step_bytes(K, H):
    """Minimum HBM bytes per patch-step the method must move (intermediates
    excluded): coarse v (8) + p (4) + geometry (8) per coarse node, the
    previous corrected velocity read and the new one written ((2^K)^2 fine
    nodes x 8 B each way), h read + written (2 H x 4 B), b_L written (16 B)."""
    n = 1 << K
    return 8 + 4 + 8 + 2 * n * n * 8 + 2 * H * 4 + 16


def stencil_flop_per_patch(K):
    """Defect FLOP per patch with general bilinear geometry: about 760 per fine
    element (the figure the measurement plan uses), n^2 fine elements per patch."""
    n = 1 << K
    return 760 * n * n


def fused_bytes_per_patch(K, H):
    """Algorithmic HBM bytes per patch of the one-launch defect + GRU + MLP
    (its share of the step's minimum bytes): coarse v, p and geometry (20 B),
    the previous corrected velocity read (n^2 fine nodes x 8 B), h read and
    written (2 H x 4 B).  Intermediates (the network input, the per-patch
    outputs) are not counted."""
    n = 1 << K
    return 20 + n * n * 8 + 2 * H * 4


def is_fused(wl, precision, flags=0):
    """The library runs defect + GRU + MLP as one launch for these shapes."""
    return precision == "bf16" and wl.K == 2 and wl.H == 64 and wl.Hm in (0, 64) and not flags


def rhs_bytes_per_patch(K):
    """Averaging/rhs kernel interface bytes per patch: per-patch outputs read
    (2 (n+1)^2 FP32), corrected velocity written (n^2 fine nodes x 8 B), corner
    partials written (4 x 16 B), coarse v read (8 B)."""
    n = 1 << K
    return 2 * (n + 1) ** 2 * 4 + n * n * 8 + 64 + 8


def source_hash(stage):
    import hashlib
    h = hashlib.sha256()
    for name in STAGE_SOURCES[stage] + ["internal.h", "device.h", "element.h", "fp8.h"]:
        with open(os.path.join(ROOT, "paper_2008_11520_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(stage, workload, precision, fused=False):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs in
    profiles/traffic.json, scaled by the copy-kernel factor; None if absent or
    if the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        e = t["kernels"][workload][precision]["k_defect_net" if fused else STAGE_KERNELS[stage]]
    except (OSError, KeyError, ValueError):
        return None
    if e.get("source_hash") != source_hash(stage):
        return None
    return (e["fetch_kib"] * t["copy_factor_fetch"] + e["write_kib"] * t["copy_factor_write"]) * 1024.0


def calibrate_copy(mib):
    """Plain device-to-device copy of a known size (for scaling the HBM
    counters): three copies of `mib` MiB."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n * 4, "launches": 3}))


def make_flow_leg(wl, precision, flags=0, copies=1, H=None):
    """A single-flow leg: `copies` contexts of the workload's flow and its
    coarse fields of 16 distinct steps, resident on the device.  With
    DNNMG_F_PAPER_NET in flags: the paper's network (hidden size H, no MLP)."""
    import torch
    import paper_2008_11520_amd as pam
    from paper_2008_11520_amd import synth
    flow = wl.flows[0]
    paper = bool(flags & pam.DNNMG_F_PAPER_NET)
    H = wl.H if H is None else H
    Hm = 0 if paper else wl.Hm
    w = synth.paper_net_weights(wl.K, H, wl.weight_seed) if paper else synth.xavier_weights(wl.K, H, Hm, wl.weight_seed)
    cfg = pam.make_config(flow.nx, flow.ny, wl.K, H, Hm, flow.dt, wl.nu, precision, flow.dirichlet, flags)
    ctxs = [pam.DnnMG(cfg, flow.cxy, w) for _ in range(copies)]
    s = ctxs[0].s
    vs, ps = [], []
    for n in range(16):
        v, p = flow.fields(n)
        vs.append(torch.from_numpy(v.reshape(-1)).cuda())
        ps.append(torch.from_numpy(p).cuda())
    bs = [torch.empty(2 * s["Nc"], dtype=torch.float64, device="cuda") for _ in ctxs]
    return dict(precision=precision, flags=flags, ctxs=ctxs, vs=vs, ps=ps, bs=bs, P=s["P"], n=0,
                fused=is_fused(wl, precision, flags))


def step_leg(leg, count):
    """Enqueue `count` steps (+ restriction), the contexts in turn."""
    ctxs, vs, ps, bs = leg["ctxs"], leg["vs"], leg["ps"], leg["bs"]
    for _ in range(count):
        k = leg["n"]
        c = k % len(ctxs)
        ctxs[c].step(vs[k % 16], ps[k % 16])
        ctxs[c].restrict_rhs(bs[c])
        leg["n"] = k + 1


def time_leg(leg, steps, warmup):
    """Enqueue warmup untimed steps, then `steps` steps bracketed by events
    with no events between the kernels (an event record puts a few
    microseconds of idle time on the stream).  Returns the two events; the
    caller synchronises once after all legs, so the GPU never waits for the
    host between legs."""
    import torch
    stream = torch.cuda.current_stream()
    step_leg(leg, warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    step_leg(leg, steps)
    e1.record(stream)
    return e0, e1


def profile_leg(leg, nprof=50):
    """The same steps with the library's per-stage HIP events on the launch
    stream: the kernels' own durations (roofline, stage breakdown)."""
    import torch
    g = leg["ctxs"][0]
    g.profile_enable(nprof)
    for _ in range(nprof):
        k = leg["n"]
        g.step(leg["vs"][k % 16], leg["ps"][k % 16])
        g.restrict_rhs(leg["bs"][0])
        leg["n"] = k + 1
    torch.cuda.synchronize()
    stage_ms, stage_n = g.profile_read()
    g.profile_enable(0)
    return stage_ms, stage_n


def close_leg(leg):
    import torch
    ok = all(bool(torch.isfinite(b).all().item()) for b in leg["bs"])
    for c in leg["ctxs"]:
        c.close()
    return ok


def run_gpu_batch(wl, precision, steps, warmup):
    """A multi-flow workload: every flow stepped together by one batched,
    graph-captured launch per step (with the restriction)."""
    import torch
    import paper_2008_11520_amd as pam
    from paper_2008_11520_amd import synth
    w = synth.xavier_weights(wl.K, wl.H, wl.Hm, wl.weight_seed)
    cfg0 = lambda f: pam.make_config(f.nx, f.ny, wl.K, wl.H, wl.Hm, f.dt, wl.nu, precision, f.dirichlet)
    model = pam.DnnMG(cfg0(wl.flows[0]), wl.flows[0].cxy, w)
    ctxs = [pam.DnnMG(cfg0(f), f.cxy, share=model) for f in wl.flows]
    nfield = min(warmup + steps, 4)
    vs = [[torch.from_numpy(f.fields(n)[0].reshape(-1)).cuda() for f in wl.flows] for n in range(nfield)]
    ps = [[torch.from_numpy(f.fields(n)[1]).cuda() for f in wl.flows] for n in range(nfield)]
    bs = [torch.empty(2 * c.s["Nc"], dtype=torch.float64, device="cuda") for c in ctxs]
    batch = pam.Batch(len(ctxs))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for n in range(warmup):
            batch.prepare(ctxs, vs[n % nfield], ps[n % nfield], None, bs, stream=st)
            batch.launch(graph=True, stream=st)
    st.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    with torch.cuda.stream(st):
        e0.record(st)
        for n in range(steps):
            k = (warmup + n) % nfield
            batch.prepare(ctxs, vs[k], ps[k], None, bs, stream=st)
            batch.launch(graph=True, stream=st)
        e1.record(st)
    st.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ok = all(bool(torch.isfinite(b).all().item()) for b in bs)
    P = sum(c.s["P"] for c in ctxs)
    batch.close()
    for c in ctxs:
        c.close()
    model.close()
    return dict(ms_total=ms, wall_s=wall, P=P, stage_ms=None, stage_n=None, finite=ok)


def run_umesh_leg(precision, steps, warmup, m=110, K=2, H=64, Hm=64):
    """The step on an unstructured mesh: the channel around a circular
    obstacle (O-grid ring with curved edges, five-element vertices), m
    elements per box side (m = 110: 272 470 patches, about the channel
    workload's 262 144), K = 2, H = 64, MLP 64-64-50.  Timed like the
    single-flow legs; per-stage HIP events for the stage breakdown."""
    import torch
    import paper_2008_11520_amd as pam
    from paper_2008_11520_amd import synth
    flow = synth.cylinder_channel_flow(m)
    w = synth.xavier_weights(K, H, Hm, 1234)
    g = pam.UDnnMG(K, H, Hm, flow.dt, 1e-3, flow.mesh, w, precision)
    vs, ps = [], []
    for n in range(8):
        v, p = flow.fields(n)
        vs.append(torch.from_numpy(v.reshape(-1)).cuda())
        ps.append(torch.from_numpy(p).cuda())
    b = torch.empty(2 * g.s["Nc"], dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for n in range(warmup):
        g.step(vs[n % 8], ps[n % 8])
        g.restrict_rhs(b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for n in range(steps):
        g.step(vs[n % 8], ps[n % 8])
        g.restrict_rhs(b)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    g.profile_enable(50)
    for n in range(50):
        g.step(vs[n % 8], ps[n % 8])
        g.restrict_rhs(b)
    torch.cuda.synchronize()
    stage_ms, stage_n = g.profile_read()
    ok = bool(torch.isfinite(b).all().item())
    P = g.s["P"]
    g.close()
    return {"workload": "cylinder channel, unstructured: %d elements (%d nodes, %d fine nodes), K=%d H=%d Hm=%d %s"
                        % (P, g.s["Nc"], g.s["Fn"], K, H, Hm, precision),
            "patches": P, "ms_per_step": ms, "patch_steps_per_s": P / (ms / 1e3),
            "stage_us": {STAGES[k]: stage_ms[k] / max(stage_n[k], 1) * 1e3 for k in range(4)}, "finite": ok}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, sample_steps=2):
    """The FP64 oracle (plain C, OpenMP over independent loops; results do not
    depend on the thread count) timed on this host: on all the threads the
    OpenMP runtime gives it (OMP_NUM_THREADS, else every core) and on one."""
    import oracle
    from paper_2008_11520_amd import synth
    flow = wl.flows[0]
    w = synth.xavier_weights(wl.K, wl.H, wl.Hm, wl.weight_seed)
    fields = [flow.fields(n) for n in range(sample_steps)]
    P = flow.nx * flow.ny
    threads_all = oracle.get_threads()

    def timed(threads):
        oracle.set_threads(threads)
        o = oracle.OracleFlow(flow.nx, flow.ny, wl.K, wl.H, wl.Hm, flow.dt, wl.nu, flow.dirichlet, flow.cxy, w)
        t0 = time.perf_counter()
        for v, p in fields:
            o.step(v, p, want=("bL",))
        return time.perf_counter() - t0

    t_all = timed(threads_all)
    t_one = timed(1) if threads_all > 1 else t_all
    oracle.set_threads(threads_all)
    return {"value": P * sample_steps / t_all, "unit": "patch-steps/s", "cores": threads_all, "kind": "oracle",
            "sample": "%d full steps of the %dx%d mesh (%d patches), FP64 C oracle: %.2f s on %d threads, "
                      "%.2f s on 1" % (sample_steps, flow.nx, flow.ny, P, t_all, threads_all, t_one),
            "single_thread_value": P * sample_steps / t_one,
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def run_serving(time_scales, n_requests=256, rate=20.0, hbm_budget=None, use_graph=True):
    """The serving mix: seeded Poisson arrivals of channel requests of mixed
    mesh sizes, continuous batching with HBM-budget admission (see serve.py).
    time_scale 1 is the offered rate; 1e9 puts every arrival at t = 0."""
    from paper_2008_11520_amd import synth
    from paper_2008_11520_amd.serve import Server
    reqs = synth.serving_requests(n_requests, rate, 11)
    out = []
    for scale in time_scales:
        srv = Server(max_flows=256, ring=8, use_graph=use_graph, hbm_budget=hbm_budget)
        st = srv.run(reqs, time_scale=scale)
        srv.close()
        st["offered_rate_per_s"] = rate * scale if scale < 1e6 else "all at t=0"
        out.append(st)
        print("bench: serving x%g: %.3g patch-steps/s, p50 %.3f ms, p99 %.3f ms, mean concurrency %.2f"
              % (scale, st["patch_steps_per_s"], st["p50_step_latency_ms"], st["p99_step_latency_ms"],
                 st["mean_concurrency"]), file=sys.stderr, flush=True)
    return out


def run_closed_loop(steps=5, fine_steps=2):
    """The closed DNN-MG loop (coarse Newton solve on level L, then the fine
    step on the GPU) against the same Newton solver run on level L+K (the
    fine solve DNN-MG replaces), per time step, on two flows."""
    import numpy as np
    from paper_2008_11520_amd import loop, synth
    cases = [("unit16x16_k1", synth.unit_square_flow(16, 16, 1, 0.01), 1, 32, 0, "fp32"),
             ("channel64x16_k2", synth.channel_flow(64, 16, 1, 0.005), 2, 64, 64, "bf16")]
    out = []
    nu = 1e-3
    for name, flow, K, H, Hm, prec in cases:
        w = synth.xavier_weights(K, H, Hm, 1234)
        fine = loop.GpuFineStep(flow, K, H, Hm, w, nu, prec)
        loop.run(flow, nu, 1, fine=fine)                      # first use of the kernels and solver paths
        fine.seconds = 0.0
        t0 = time.perf_counter()
        r = loop.run(flow, nu, steps, fine=fine)
        wall = time.perf_counter() - t0
        fine.close()
        n = 1 << K
        fflow = synth.Flow(flow.nx * n, flow.ny * n,
                           synth.rect_mesh(flow.nx * n, flow.ny * n, flow.cxy[-1, -1, 0], flow.cxy[-1, -1, 1]),
                           flow.dirichlet, flow.dt, flow.fourier, inflow_max=flow.inflow_max)
        t0 = time.perf_counter()
        f = loop.run(fflow, nu, fine_steps)
        fine_wall = time.perf_counter() - t0
        res = {"case": name, "K": K, "precision": prec, "steps": steps, "fine_steps": fine_steps,
               "dnnmg_ms_per_step": wall / steps * 1e3,
               "coarse_solve_ms_per_step": r["coarse_s"] / steps * 1e3,
               "fine_step_ms_per_step": fine.seconds / steps * 1e3,
               "fine_solve_ms_per_step": fine_wall / fine_steps * 1e3,
               "fine_over_dnnmg": (fine_wall / fine_steps) / (wall / steps),
               "coarse_unknowns": 3 * (flow.nx + 1) * (flow.ny + 1),
               "fine_unknowns": 3 * (fflow.nx + 1) * (fflow.ny + 1),
               "newton_steps": r["newton"], "fine_newton_steps": f["newton"]}
        out.append(res)
        print("bench: closed loop %s: DNN-MG %.1f ms/step (coarse %.1f, fine step %.2f), fine solve %.1f ms/step"
              % (name, res["dnnmg_ms_per_step"], res["coarse_solve_ms_per_step"], res["fine_step_ms_per_step"],
                 res["fine_solve_ms_per_step"]), file=sys.stderr, flush=True)
    return out


def cn_rhs_flop_per_patch(K):
    """FP64 FLOP per patch of the Crank-Nicolson explicit term in the rhs
    kernel (the transport of u = P v + d against the four coarse hats), as
    the formula is written: per fine-element Gauss point, the map's Jacobian
    and determinant (11), u and its reference gradient (38), the cofactor
    gradients (12), u . grad u (6), nu / det (1), the coarse hats (12), and
    per corner the cofactor gradient of the hat (6) and the weighted sums of
    both components (16); 4 Gauss points on each of the n^2 fine elements."""
    n = 1 << K
    per_point = 11 + 38 + 12 + 6 + 1 + 12 + 4 * (6 + 16)
    return 4 * n * n * per_point


def roofline(wl, flow, P, main_r, precision):
    """Roofline of the dominant stage: per-launch algorithmic work over the
    stage's average launch time from the library's HIP events on the launch
    stream."""
    avg = [main_r["stage_ms"][k] / max(main_r["stage_n"][k], 1) for k in range(4)]
    dom = int(np.argmax(avg))
    t_s = avg[dom] / 1e3
    if dom == 0 and main_r.get("fused"):
        # one launch with vector work (defect), matrix-core work (GRU, MLP) and
        # HBM traffic: the roofline is the largest of the three lower bounds at
        # the published peaks, reported in that bound's unit.  attainable_frac
        # takes the vector bound at the rate without packed FP32 instructions.
        vflop, mflop = stencil_flop_per_patch(wl.K), per_patch_gemm_flop(wl.K, wl.H, wl.Hm)
        hbm_bytes = fused_bytes_per_patch(wl.K, wl.H)
        bounds = {"alu": vflop * P / (PEAK_FP32_VECTOR_TFLOPS * 1e12),
                  "mfma": mflop * P / (PEAK_TFLOPS[precision] * 1e12),
                  "hbm": hbm_bytes * P / (PEAK_HBM_GBS * 1e9)}
        bound = max(bounds, key=bounds.get)
        per_unit, peak, unit, scale = {"alu": (vflop, PEAK_FP32_VECTOR_TFLOPS, "TFLOP/s", 1e12),
                                       "mfma": (mflop, PEAK_TFLOPS[precision], "TFLOP/s", 1e12),
                                       "hbm": (hbm_bytes, PEAK_HBM_GBS, "GB/s", 1e9)}[bound]
        achieved = per_unit * P / t_s / scale
        attainable = dict(bounds, alu=vflop * P / (PEAK_FP32_VALU_TFLOPS * 1e12))
        roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                "lower_bounds_us": {k: v * 1e6 for k, v in bounds.items()},
                "attainable_frac": max(attainable.values()) / t_s,
                "attainable_bound": max(attainable, key=attainable.get),
                "attainable_lower_bounds_us": {k: v * 1e6 for k, v in attainable.items()},
                "hbm_GBs": hbm_bytes * P / t_s / 1e9, "vector_tflops": vflop * P / t_s / 1e12,
                "mfma_tflops": mflop * P / t_s / 1e12}
        roof.update({"traffic": stored_traffic(dom, wl.name, precision, fused=True),
                     "kernel": "defect_gru_mlp (one launch)", "avg_launch_us": avg[dom] * 1e3,
                     "algorithmic_per_patch": per_unit, "hbm_bytes_per_patch": hbm_bytes,
                     "units_per_launch": P})
        return roof
    if dom == 0:
        unit_work = stencil_flop_per_patch(wl.K)
        achieved = unit_work * P / t_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "attainable_frac": achieved / PEAK_FP32_VALU_TFLOPS}
    elif dom == 1:
        unit_work = per_patch_gemm_flop(wl.K, wl.H, wl.Hm)
        peak = PEAK_TFLOPS[precision]
        achieved = unit_work * P / t_s / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak}
    else:
        unit_work = rhs_bytes_per_patch(wl.K) if dom == 2 else 5 * 16 * (flow.nx + 1) * (flow.ny + 1) / P
        achieved = unit_work * P / t_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS}
    roof.update({"traffic": stored_traffic(dom, wl.name, precision), "kernel": STAGES[dom],
                 "avg_launch_us": avg[dom] * 1e3, "algorithmic_per_patch": unit_work,
                 "units_per_launch": P})
    return roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    # (after the GPU has idled, its clocks take ~0.1 s of work to come up:
    # the single-flow legs run back to back after a two-context leg of at
    # least 600 steps, and each leg also takes `warmup` untimed steps)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="channel1024x256_k2_perturbed")
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32", "fp8"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-closed-loop", action="store_true")
    ap.add_argument("--no-umesh", action="store_true", help="skip the unstructured-mesh leg")
    ap.add_argument("--cpu-sample-steps", type=int, default=2)
    ap.add_argument("--serving", default="offered,all", metavar="LIST",
                    help="serving runs after the throughput legs: comma list of offered (20/s), x10, x100, "
                         "all (every arrival at t=0), or none")
    ap.add_argument("--serve-budget-mib", type=int, default=0, help="HBM budget of the serving runs (0: 80%% free)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each box has one MI355X); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2008_11520_amd import synth
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    wl = synth.workload(args.workload)
    flow = wl.flows[0]
    print("bench: workload %s, %d patches, precision %s, %d steps" % (wl.name, flow.nx * flow.ny, args.precision,
                                                                     args.steps), file=sys.stderr, flush=True)

    forms = {}
    batched = len(wl.flows) > 1
    rotated = None
    busy_before_ms = None
    if batched:
        for prec in ([p for p in ("fp32", "fp8", "bf16") if p != args.precision] + [args.precision]):
            r = run_gpu_batch(wl, prec, args.steps, args.warmup)
            forms[prec] = r
            print("bench: %s %.3f ms/step" % (prec, r["ms_total"] / args.steps), file=sys.stderr, flush=True)
    else:
        import paper_2008_11520_amd as pam
        # Every context and input is made first, so that the timed legs run
        # back to back with the GPU busy: its clocks come up from idle over
        # the first ~0.1 s of work and drop again after a fraction of a second
        # without it.  The two-context (last-level-cache-rotated) leg runs
        # first, for at least 600 steps; the headline form is timed last.
        order = [p for p in ("fp32", "fp8", "bf16") if p != args.precision]
        legs = {p: make_flow_leg(wl, p) for p in order}
        if args.precision == "bf16":
            legs["bf16_unfused"] = make_flow_leg(wl, "bf16", flags=pam.DNNMG_F_UNFUSED)
            order.append("bf16_unfused")
        # the Crank-Nicolson scheme (separate launches; FP64 explicit term in the rhs)
        cn = args.precision + "_crank_nicolson"
        legs[cn] = make_flow_leg(wl, args.precision, flags=pam.DNNMG_F_CRANK_NICOLSON)
        order.append(cn)
        # the paper's network (inputs with continuity rows, Peclet numbers and
        # twelve geometry values; dense + convolutional head), N_GRU = 96 at
        # K = 2 as in the paper's two-level network
        if args.precision != "fp8":
            pn = args.precision + "_paper_net_h96"
            legs[pn] = make_flow_leg(wl, args.precision, flags=pam.DNNMG_F_PAPER_NET, H=96)
            order.append(pn)
        legs[args.precision] = make_flow_leg(wl, args.precision)
        order.append(args.precision)
        rot = make_flow_leg(wl, args.precision, copies=2)
        torch.cuda.synchronize()
        rot_steps = max(args.steps, 600)
        start = torch.cuda.Event(enable_timing=True)
        start.record(torch.cuda.current_stream())
        ev_rot = time_leg(rot, rot_steps, args.warmup)
        ev = {name: time_leg(legs[name], args.steps, args.warmup) for name in order}
        torch.cuda.synchronize()
        ms_rot = ev_rot[0].elapsed_time(ev_rot[1]) / rot_steps
        rotated = {"contexts": 2, "steps": rot_steps, "ms_per_step": ms_rot,
                   "patch_steps_per_s": rot["P"] / (ms_rot / 1e3)}
        print("bench: %s, two contexts in turn %.3f ms/step" % (args.precision, ms_rot), file=sys.stderr, flush=True)
        ms = {name: e0.elapsed_time(e1) for name, (e0, e1) in ev.items()}
        busy_before_ms = start.elapsed_time(ev[args.precision][0])
        for name in order:
            stage_ms, stage_n = profile_leg(legs[name])
            forms[name] = dict(ms_total=ms[name], P=legs[name]["P"], stage_ms=stage_ms, stage_n=stage_n,
                               fused=legs[name]["fused"], finite=close_leg(legs[name]))
            print("bench: %s %.3f ms/step" % (name, ms[name] / args.steps), file=sys.stderr, flush=True)
        close_leg(rot)

    main_r = forms[args.precision]
    P = main_r["P"]
    ms_step = main_r["ms_total"] / args.steps
    value = P * args.steps / (main_r["ms_total"] / 1e3)

    # dominant kernel and its roofline (per-launch algorithmic work / average
    # launch time from the library's HIP events on the launch stream)
    roof = None
    if main_r["stage_ms"] is not None:
        roof = roofline(wl, flow, P, main_r, args.precision)
    step_bytes = per_patch_step_bytes(wl.K, wl.H) * P
    cn_roof = None
    cn_r = forms.get(args.precision + "_crank_nicolson")
    if cn_r is not None and cn_r["stage_ms"] is not None:
        # the rhs kernel of the Crank-Nicolson form: FP64 vector arithmetic
        t_s = cn_r["stage_ms"][2] / max(cn_r["stage_n"][2], 1) / 1e3
        fl = cn_rhs_flop_per_patch(wl.K)
        cn_roof = {"kernel": "avg_rhs_fp64 with the explicit transport term", "bound": "alu",
                   "achieved": fl * P / t_s / 1e12, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                   "frac": fl * P / t_s / 1e12 / PEAK_FP64_VECTOR_TFLOPS, "algorithmic_per_patch": fl,
                   "avg_launch_us": t_s * 1e6, "units_per_launch": P}
    out = {
        "metric": "patch-steps/sec of fine DNN-MG step (BF16 vs FP32); serving p50/p99 step latency",
        "value": value,
        "unit": "patch-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic (seeded meshes, Fourier-mode coarse fields, Xavier weights)",
        "config": {"workload": wl.name, "patches": P, "K": wl.K, "H": wl.H, "Hm": wl.Hm,
                   "gemm_operands": args.precision, "defect": "f32", "rhs_restriction": "f64"},
        "forms": {p: {"patch_steps_per_s": P * args.steps / (r["ms_total"] / 1e3),
                      "ms_per_step": r["ms_total"] / args.steps,
                      "stage_us": ({STAGES[k]: r["stage_ms"][k] / max(r["stage_n"][k], 1) * 1e3 for k in range(4)}
                                   if r["stage_ms"] is not None else None)}
                  for p, r in forms.items()},
        "step_hbm": {"algorithmic_bytes_per_patch": per_patch_step_bytes(wl.K, wl.H),
                     "achieved_GBs": step_bytes / (ms_step / 1e3) / 1e9,
                     "frac": step_bytes / (ms_step / 1e3) / 1e9 / PEAK_HBM_GBS},
        "roofline": roof,
        "crank_nicolson_rhs_roofline": cn_roof,
        "cache_rotated": rotated,
        "gpu_busy_before_timed_ms": busy_before_ms,
        "finite": main_r["finite"],
    }
    scales = {"offered": 1.0, "x10": 10.0, "x100": 100.0, "all": 1e9}
    runs = [r for r in args.serving.split(",") if r and r != "none"]
    if runs:
        budget = args.serve_budget_mib << 20 if args.serve_budget_mib else None
        res = run_serving([scales[r] for r in runs], hbm_budget=budget)
        out["serving"] = {"workload": "256 requests, Poisson 20/s, channel meshes 32x8..512x128, 50-500 steps, "
                                      "K=2 H=64 bf16, hipGraph",
                          "runs": dict(zip(runs, res))}
    if not batched and args.precision != "fp8" and not args.no_umesh:
        print("bench: unstructured mesh leg", file=sys.stderr, flush=True)
        out["unstructured"] = run_umesh_leg(args.precision, args.steps, args.warmup)
        print("bench: unstructured %.3f ms/step" % out["unstructured"]["ms_per_step"], file=sys.stderr, flush=True)
    if not args.no_closed_loop:
        out["closed_loop"] = {"note": "coarse Newton solve (host, sparse LU) + fine step (GPU) per time step, "
                                      "against the same Newton solver on level L+K",
                              "runs": run_closed_loop()}
    if not args.no_cpu_baseline:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
