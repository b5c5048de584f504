"""The paper's network form (DNNMG_F_PAPER_NET: residual with continuity rows,
corner velocities, Peclet numbers and twelve geometry values in; dense layer
and two convolutional blocks out), the GRU with the reset gate after U_h
(DNNMG_F_GRU_RESET_AFTER) and H = 96, on the GPU against the oracle's
orc_step_form.  Bounds as the other step sequences: 1e-5 with FP32 operands,
2e-2 with BF16, on rel-L2 and max-rel of the correction, the per-patch
output and the state, b_L 1e-5 / 2e-2 -- except the max-rel checks with
BF16 operands in the paper's form: its inputs are not normalised (Peclet
numbers reach ~100), so one gate pre-activation a = W x + U h carries a
BF16 rounding error up to 2^-8 S, S = sum |W_i x_i| + sum |U_m h_m|, which
can be far above 2e-2 of max |h|.  There the element-wise checks follow the
running-error scale instead (rel-L2 stays at 2e-2):
  state      |dh| <= hb = 16 * 2^-8 (1 + S), S the largest of the entry's
             three gate sums at that step (16: the gates' three products
             and the error carried through four steps);
  output     |dd| <= |A| hb + 2^-8 |A| |h| per entry, |A| the head with
             every weight in absolute value (an upper bound of the folded
             dense + convolution map), the second term the head's own BF16
             operand rounding;
  D-bar      |dD| <= the duplicate average of those output bounds;
with S, h and the head from the oracle.  The head is also checked on its
own, tightly: the GPU's output against the oracle's head applied to the
GPU's own state, |d - A h_gpu| <= 2^-7 |A| |h_gpu| (BF16 rounding of the
folded weights and of h, 2^-9 each, and FP32 accumulation, with a factor 2)."""
import numpy as np
import pytest

import oracle
from paper_2008_11520_amd import synth

from gpu_common import GpuRunner, assert_step_errors, merge_worst, step_errors, to_dev

pytestmark = pytest.mark.gpu
NU = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2008_11520_amd as pam
    pam.lib()


# name: (flow, K, H, Hm, paper form, reset after, theta)
CASES = {
    # the paper's networks: 51 -> 32 -> 18 at K = 1, 99 -> 96 -> 50 at K = 2
    "paper_unit16_k1_h32": (synth.unit_square_flow(16, 16, 1, 0.01), 1, 32, 0, True, False, 1.0),
    "paper_channel24x8_k2_h96": (synth.channel_flow(24, 8, 3, 0.005, perturb_seed=4), 2, 96, 0, True, False, 1.0),
    "paper_reset_after_channel24x8_k2_h96": (synth.channel_flow(24, 8, 3, 0.005, perturb_seed=4), 2, 96, 0, True,
                                             True, 1.0),
    # other shapes: K = 2, H = 64 (rows as wide as the standard form's: the
    # persistent kernel), K = 3 (generic kernel), a ragged mesh, and with
    # Crank-Nicolson
    "paper_ragged13x7_k2_h64": (synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5), 2, 64, 0, True, False, 1.0),
    "paper_stretched5x3_k3_h64": (synth.stretched_flow(5, 3, 3.7, 4, 0.01), 3, 64, 0, True, False, 1.0),
    "paper_cn_unit16_k1_h32": (synth.unit_square_flow(16, 16, 1, 0.01), 1, 32, 0, True, True, 0.5),
    # the workloads' form with the reset gate after U_h, and with H = 96
    "reset_after_ragged13x7_k2_h64_mlp": (synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5), 2, 64, 64, False,
                                          True, 1.0),
    "h96_ragged13x7_k2_mlp": (synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5), 2, 96, 64, False, False, 1.0),
}


def _make(name, prec):
    import paper_2008_11520_amd as pam
    flow, K, H, Hm, paper, ra, theta = CASES[name]
    flags = (pam.DNNMG_F_PAPER_NET if paper else 0) | (pam.DNNMG_F_GRU_RESET_AFTER if ra else 0) | \
        (pam.DNNMG_F_CRANK_NICOLSON if theta != 1.0 else 0)
    w = synth.paper_net_weights(K, H, 1234) if paper else synth.xavier_weights(K, H, Hm, 1234)
    cfg = pam.make_config(flow.nx, flow.ny, K, H, Hm, flow.dt, NU, prec, flow.dirichlet, flags)
    g = pam.DnnMG(cfg, flow.cxy, w)
    o = oracle.OracleFlow(flow.nx, flow.ny, K, H, Hm, flow.dt, NU, flow.dirichlet, flow.cxy, w.astype(np.float64),
                          theta=theta, form=1 if paper else 0, reset_after=ra)
    return flow, K, g, o


def _gate_scale(o, X, h_prev):
    """Per (patch, unit): the largest over the three gates of
    sum_i |W_ki x_i| + sum_m |U_km h_m| (the oracle's weights, input, state)."""
    H, nin = o.H, X.shape[1]
    w = o.w
    S = None
    for g in range(3):
        W = np.abs(w[g * H * nin:(g + 1) * H * nin].reshape(H, nin))
        U = np.abs(w[3 * H * nin + g * H * H:3 * H * nin + (g + 1) * H * H].reshape(H, H))
        Sg = np.abs(X) @ W.T + np.abs(h_prev) @ U.T
        S = Sg if S is None else np.maximum(S, Sg)
    return S


def _head_abs(o, K, x):
    """|A| x for the paper head A (every weight in absolute value)."""
    H, nf = o.H, (2 ** K + 1) ** 2
    nin, nout = 3 * nf + 24, 2 * nf
    w = np.abs(o.w)
    off = 3 * H * nin + 3 * H * H
    M = w[off:off + nout * H].reshape(nout, H)
    WV, WS, wf = w[off + nout * H:off + nout * H + 36], w[off + nout * H + 36:off + nout * H + 72], w[-nout:]
    return oracle.conv_head(K, x, M, WV, WS, wf)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_step_sequence_matches_oracle(name, prec, tol):
    flow, K, g, o = _make(name, prec)
    paper_bf16 = CASES[name][4] and prec == "bf16"
    r = GpuRunner(g)
    worst, ratio = {}, {"h": 0.0, "dpatch": 0.0, "Dbar": 0.0, "head": 0.0}
    for n in range(4):
        v, p = flow.fields(n)
        h_prev = o.h.copy()
        got = r.step(v, p)
        ref = o.step(v, p, want=("Dbar", "bL", "dpatch", "X"))
        merge_worst(worst, step_errors(got, ref, o.h, flow.nx, flow.ny, K, flow.dirichlet))
        if paper_bf16:
            hb = 16.0 * 2.0 ** -8 * (1.0 + _gate_scale(o, ref["X"], h_prev))
            db = _head_abs(o, K, hb) + 2.0 ** -8 * _head_abs(o, K, np.abs(o.h))
            Db = oracle.average(flow.nx, flow.ny, K, db, flow.dirichlet)
            H, nf = o.H, (2 ** K + 1) ** 2
            nin, nout = 3 * nf + 24, 2 * nf
            off = 3 * H * nin + 3 * H * H
            w = o.w
            head = oracle.conv_head(K, got["h"].astype(np.float64), w[off:off + nout * H].reshape(nout, H),
                                    w[off + nout * H:off + nout * H + 36], w[off + nout * H + 36:off + nout * H + 72],
                                    w[-nout:])
            hdb = 2.0 ** -7 * _head_abs(o, K, np.abs(got["h"].astype(np.float64)))
            for k, err, bound in (("h", got["h"] - o.h, hb), ("dpatch", got["dpatch"] - ref["dpatch"], db),
                                  ("Dbar", got["Dbar"] - ref["Dbar"], Db), ("head", got["dpatch"] - head, hdb)):
                ratio[k] = max(ratio[k], float((np.abs(err) / (bound + 1e-300)).max()))
    print("paper-form step errors", name, prec, worst, "error / running-error bound", ratio)
    if paper_bf16:
        assert max(ratio.values()) <= 1.0, ratio
        for k in ("h_max", "dpatch_max", "Dbar_max", "Dbar_edge_max"):
            worst[k] = 0.0        # judged element-wise by the bounds above
    assert_step_errors(worst, tol, 1e-5 if prec == "fp32" else tol)


def test_paper_weights_change_the_correction():
    """The head's convolutional blocks and output weights are used: other
    block weights give another correction (GPU and oracle agree on both)."""
    import paper_2008_11520_amd as pam
    flow, K, H = synth.unit_square_flow(8, 8, 1, 0.01), 1, 32
    outs = []
    for seed in (1, 2):
        w = synth.paper_net_weights(K, H, 1234)
        w[-(72 + 18):-18] = synth.paper_net_weights(K, H, seed)[-(72 + 18):-18]
        cfg = pam.make_config(flow.nx, flow.ny, K, H, 0, flow.dt, NU, "fp32", flow.dirichlet, pam.DNNMG_F_PAPER_NET)
        r = GpuRunner(pam.DnnMG(cfg, flow.cxy, w))
        v, p = flow.fields(0)
        outs.append(r.step(v, p)["dpatch"])
    assert np.abs(outs[0] - outs[1]).max() > 1e-3 * np.abs(outs[0]).max()


def test_batched_step_rejects_paper_form_contexts():
    import paper_2008_11520_amd as pam
    flow, K, H = synth.unit_square_flow(8, 8, 1, 0.01), 1, 32
    cfg = pam.make_config(flow.nx, flow.ny, K, H, 0, flow.dt, NU, "fp32", flow.dirichlet, pam.DNNMG_F_PAPER_NET)
    a = pam.DnnMG(cfg, flow.cxy, synth.paper_net_weights(K, H, 1))
    b = pam.DnnMG(cfg, flow.cxy, share=a)
    v, p = flow.fields(0)
    vd, pd = to_dev(v.reshape(-1)), to_dev(p)
    with pytest.raises(pam.DnnmgError) as e:
        pam.Batch(2).step([a, b], [vd, vd], [pd, pd])
    assert e.value.code == pam.DNNMG_EINVAL and "PAPER_NET" in str(e.value)
