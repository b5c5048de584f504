"""FP8 E4M3 operand form on the GPU against the oracle's FP8 form.

The activation quantiser takes the same FP32 decisions on both sides, so its
codes and scales must agree bit for bit.  The whole step is compared with
the oracle's FP8 step (same quantisation rule, exact accumulation).  The two
differ by FP32 accumulation and the matrix cores' internal alignment (about
1e-4 relative per product, measured), which moves h' by ~1e-4; a fraction
f ~ 16 * 1e-4 of the next layer's codes then lands on the other side of a
rounding boundary, each flip moving one patch's output by ~1/8 / sqrt(H) of
its size, so the correction differs by ~sqrt(f) / 8 ~ 5e-3 per step of
state drift.  Bounds: 2e-2 relative L2 on the correction and the per-patch
output, 5e-3 on the state, over four steps -- and the GPU must be several
times closer to the FP8 oracle than to the FP64 step (6e-2 away), which a
different rounding rule or scale would not be.  The distance to the FP64
step is printed as the form's accuracy."""
import numpy as np
import pytest

import oracle
from paper_2008_11520_amd import synth

from gpu_common import GpuRunner, make_gpu_flow, rel_l2, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2008_11520_amd as pam
    pam.lib()


@pytest.mark.parametrize("rows,cols", [(37, 104), (5, 1000), (1, 1), (300, 64)])
def test_quantiser_codes_and_scales_bitwise(rows, cols):
    import torch
    import paper_2008_11520_amd as pam
    rng = np.random.default_rng(rows * 1000 + cols)
    a = (rng.standard_normal((rows, cols)) * np.exp(rng.uniform(-20, 20, (rows, 1)))).astype(np.float32)
    if rows > 2:
        a[1] = 0.0
        a[2, : cols // 2] = 448.0 * 2.0 ** rng.integers(-12, 12)        # ties of the scale
    ad = to_dev(a)
    q = torch.empty((rows, cols), dtype=torch.uint8, device="cuda")
    s = torch.empty(rows, dtype=torch.float32, device="cuda")
    pam.quantize_e4m3(ad, q, s)
    torch.cuda.synchronize()
    qr, sr = oracle.quantize_rows(a)
    assert np.array_equal(s.cpu().numpy(), sr)
    assert np.array_equal(q.cpu().numpy(), qr)


def _flows():
    return {
        "ragged13x7_k2_perturbed": (synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5), 2, 64, 64),
        "stretched5x3_k3": (synth.stretched_flow(5, 3, 3.7, 4, 0.01), 3, 128, 128),
        "unit16_k1": (synth.unit_square_flow(16, 16, 1, 0.01), 1, 32, 0),
        "strip9x1_k1": (synth.channel_flow(9, 1, 6, 0.005), 1, 64, 0),
    }


FLOWS = _flows()


@pytest.mark.parametrize("name", sorted(FLOWS))
def test_fp8_step_matches_fp8_oracle(name):
    flow, K, H, Hm = FLOWS[name]
    w = synth.xavier_weights(K, H, Hm, 1234)
    g = GpuRunner(make_gpu_flow(flow, K, H, Hm, 1e-3, w, "fp8"))
    o8 = oracle.OracleFlow(flow.nx, flow.ny, K, H, Hm, flow.dt, 1e-3, flow.dirichlet, flow.cxy,
                           w.astype(np.float64), fp8=True)
    o64 = oracle.OracleFlow(flow.nx, flow.ny, K, H, Hm, flow.dt, 1e-3, flow.dirichlet, flow.cxy,
                            w.astype(np.float64))
    for n in range(4):
        v, p = flow.fields(n)
        got = g.step(v, p)
        r8 = o8.step(v, p, want=("Dbar", "bL", "dpatch"))
        r64 = o64.step(v, p, want=("Dbar",))
        e = dict(Dbar=rel_l2(got["Dbar"], r8["Dbar"]), dpatch=rel_l2(got["dpatch"], r8["dpatch"]),
                 h=rel_l2(got["h"], o8.h), bL=rel_l2(got["bL"], r8["bL"]),
                 Dbar_vs_fp64=rel_l2(got["Dbar"], r64["Dbar"]), oracle_fp8_vs_fp64=rel_l2(r8["Dbar"], r64["Dbar"]))
        print(name, n, {k: "%.2e" % v for k, v in e.items()})
        assert e["Dbar"] < 2e-2 and e["dpatch"] < 2e-2 and e["h"] < 5e-3, e
        assert e["Dbar"] < 0.4 * e["Dbar_vs_fp64"], e


def test_fp8_zero_weights_give_zero_correction():
    flow, K, H, Hm = FLOWS["ragged13x7_k2_perturbed"]
    w = np.zeros_like(synth.xavier_weights(K, H, Hm, 1))
    g = GpuRunner(make_gpu_flow(flow, K, H, Hm, 1e-3, w, "fp8"))
    for n in range(2):
        got = g.step(*flow.fields(n))
        assert np.all(got["Dbar"] == 0.0) and np.all(got["h"] == 0.0)


def test_fp8_batched_equals_single_bitwise():
    import torch
    import paper_2008_11520_amd as pam
    K, H, Hm = 3, 128, 128
    w = synth.xavier_weights(K, H, Hm, 77)
    flows = [synth.stretched_flow(5, 3, 2.5, 1, 0.01), synth.stretched_flow(4, 4, 6.0, 2, 0.01)]
    single = [GpuRunner(make_gpu_flow(f, K, H, Hm, 1e-3, w, "fp8")) for f in flows]
    model = make_gpu_flow(flows[0], K, H, Hm, 1e-3, w, "fp8")
    ctxs = [make_gpu_flow(f, K, H, Hm, 1e-3, w, "fp8", share=model) for f in flows]
    runners = [GpuRunner(c) for c in ctxs]
    b = pam.Batch(4)
    st = torch.cuda.Stream()
    for n in range(3):
        fields = [f.fields(n) for f in flows]
        ref = [r.step(v, p) for r, (v, p) in zip(single, fields)]
        with torch.cuda.stream(st):
            vs = [to_dev(v.reshape(-1)) for v, _ in fields]
            ps = [to_dev(p) for _, p in fields]
            b.prepare(ctxs, vs, ps, [r.dbar for r in runners], [r.bL for r in runners], stream=st)
            b.launch(graph=(n > 0), stream=st)
        st.synchronize()
        for r, c, rf in zip(runners, ctxs, ref):
            c.get_state(r.h, None)
            torch.cuda.synchronize()
            assert np.array_equal(r.dbar.cpu().numpy().reshape(-1, 2), rf["Dbar"])
            assert np.array_equal(r.bL.cpu().numpy().reshape(-1, 2), rf["bL"])
            assert np.array_equal(r.h.cpu().numpy().reshape(c.s["P"], -1), rf["h"])
    b.close()
