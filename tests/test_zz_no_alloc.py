"""The allocation-free rhs + restriction (dnnmg_rhs_restrict_noalloc, scratch
in one static device array) against the context entry point
dnnmg_rhs_restrict on the same inputs: three calls in a row on one GPU, each
on a smaller mesh than the one before (so the array holds a larger call's
leftovers), each equal to the context's result bit for bit and within the
FP64 stage bound (1e-10) of the oracle."""
import numpy as np
import pytest

import oracle
from paper_2008_11520_amd import synth

from gpu_common import make_gpu_flow, rel_max, to_dev

pytestmark = pytest.mark.gpu


def test_noalloc_rhs_restrict_equals_context_entry_point():
    import torch
    import paper_2008_11520_amd as pam
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    cases = [(synth.channel_flow(37, 23, 3, 0.005, perturb_seed=5), 2),
             (synth.stretched_flow(9, 5, 2.5, 4, 0.01), 3),
             (synth.unit_square_flow(4, 3, 1, 0.01), 1)]
    for flow, K in cases:
        print("noalloc rhs: %dx%d K=%d" % (flow.nx, flow.ny, K), flush=True)
        g = make_gpu_flow(flow, K, 32, 0, 1e-3, synth.xavier_weights(K, 32, 0, 1))
        s = g.s
        v, _ = flow.fields(1)
        dbar = (0.3 * synth.SplitMix64(5 + K).uniform(2 * s["Fn"], -1.0, 1.0)).astype(np.float32)
        vd, dd = to_dev(v.reshape(-1)), to_dev(dbar)
        b_ctx = torch.empty(2 * s["Nc"], dtype=torch.float64, device="cuda")
        b_na = torch.full_like(b_ctx, float("nan"))
        g.rhs_restrict(vd, dd, b_ctx)
        pam.rhs_restrict_noalloc(flow.nx, flow.ny, K, flow.dt, to_dev(flow.cxy.reshape(-1)), vd, dd, b_na)
        torch.cuda.synchronize()
        assert torch.equal(b_na, b_ctx)
        ref = oracle.rhs_restrict(flow.nx, flow.ny, K, flow.cxy.reshape(-1, 2), v.astype(np.float64),
                                  dbar.astype(np.float64).reshape(-1, 2), flow.dt)
        err = rel_max(b_na.cpu().numpy().reshape(-1, 2), ref)
        print("  max-rel vs oracle %.2e" % err)
        assert err < 1e-10
        g.close()
