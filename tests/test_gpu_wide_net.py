"""The BF16 network on 128-patch tiles (H = 128, or K = 3): each tile is a
pair of 64-patch row tiles, and in a batch the two halves of a pair may
belong to different flows.  Step sequences against the FP64 oracle for the
shapes the stretched workload does not use (ragged last tiles, a pair with an
empty half), and batched steps against single-flow steps, bit for bit, for
flows with odd numbers of 64-patch row tiles, so that pairs straddle flows."""
import numpy as np
import pytest

from paper_2008_11520_amd import synth

from gpu_common import GpuRunner, assert_step_errors, make_gpu_flow, make_oracle_flow, merge_worst, step_errors, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2008_11520_amd as pam
    pam.lib()


# (flow, K, H, Hm): patch counts 77 (64 + 13 rows), 153 (64 + 64 + 25), 143,
# and single tiles whose first half has fewer than 64 rows and whose second
# half is empty: 15, 35, 12, 1
SHAPES = {
    "k3_h128_linear_11x7": (synth.stretched_flow(11, 7, 2.5, 6, 0.01), 3, 128, 0),
    "k3_h64_mlp_11x7": (synth.channel_flow(11, 7, 7, 0.005, perturb_seed=3), 3, 64, 64),
    "k2_h128_mlp_17x9": (synth.channel_flow(17, 9, 2, 0.005, perturb_seed=4), 2, 128, 128),
    "k1_h128_linear_13x11": (synth.unit_square_flow(13, 11, 1, 0.01), 1, 128, 0),
    "k3_h128_linear_5x3": (synth.stretched_flow(5, 3, 3.7, 4, 0.01), 3, 128, 0),
    "k3_h128_mlp_5x3": (synth.stretched_flow(5, 3, 1.5, 8, 0.01), 3, 128, 128),
    "k2_h128_mlp_7x5": (synth.channel_flow(7, 5, 5, 0.005, perturb_seed=6), 2, 128, 128),
    "k3_h64_mlp_4x3": (synth.channel_flow(4, 3, 2, 0.005, perturb_seed=9), 3, 64, 64),
    "k3_h128_mlp_1x1": (synth.unit_square_flow(1, 1, 3, 0.01), 3, 128, 128),
}


@pytest.mark.parametrize("name", sorted(SHAPES))
def test_wide_bf16_step_sequence_matches_oracle(name):
    flow, K, H, Hm = SHAPES[name]
    w = synth.xavier_weights(K, H, Hm, 77)
    g = GpuRunner(make_gpu_flow(flow, K, H, Hm, 1e-3, w, "bf16"))
    o = make_oracle_flow(flow, K, H, Hm, 1e-3, w)
    worst = {}
    for n in range(4):
        v, p = flow.fields(n)
        got = g.step(v, p)
        ref = o.step(v, p, want=("Dbar", "bL", "dpatch"))
        merge_worst(worst, step_errors(got, ref, o.h, flow.nx, flow.ny, K, flow.dirichlet))
    print("wide bf16", name, worst)
    assert_step_errors(worst, 2e-2, 2e-2)


@pytest.mark.parametrize("K,H,Hm", [(2, 128, 128), (3, 128, 0)])
def test_wide_bf16_batched_pairs_straddle_flows_bitwise(K, H, Hm):
    import torch
    import paper_2008_11520_amd as pam
    w = synth.xavier_weights(K, H, Hm, 5)
    # 64-patch row tiles per flow: 1, 3, 2, 1 (prefix 0, 1, 4, 6): the pairs
    # (0, 1) and (6, -) cross or end a flow
    flows = [synth.channel_flow(9, 7, 3, 0.005), synth.channel_flow(13, 11, 4, 0.005, perturb_seed=8),
             synth.unit_square_flow(10, 10, 2, 0.01), synth.channel_flow(5, 3, 9, 0.005)]
    single = [GpuRunner(make_gpu_flow(f, K, H, Hm, 1e-3, w, "bf16")) for f in flows]
    model = make_gpu_flow(flows[0], K, H, Hm, 1e-3, w, "bf16")
    batched = [make_gpu_flow(f, K, H, Hm, 1e-3, w, "bf16", share=model) for f in flows]
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
    for x in batched + [model] + [r.g for r in single]:
        x.close()
