"""Crank-Nicolson (DNNMG_F_CRANK_NICOLSON, theta = 1/2 of Eq.
(4cranknicholson3)) on the GPU against the oracle's theta scheme.

Bounds:
  D (defect, given u_prev)   rel-L2 1e-5 and, node by node, 64 eps32 of the
                             running-error scale: defect_abs of the new level
                             (mass, convection, diffusion, pressure of P v)
                             plus defect_abs of the old level's transport
                             (u_prev with 1/dt = 0 and no pressure)
  first-step defect          the implicit-Euler context's within 4 eps32 of
                             the scale (u_prev = P v: both schemes take the
                             same elements), and the oracle's within 64
  b_L stage                  1e-10 max-rel (FP64 on both sides), also with a
                             large time step where the explicit transport term
                             dominates the mass term
  steps                      as the implicit-Euler step sequences: 1e-5 FP32,
                             2e-2 BF16, on rel-L2 and max-rel
"""
import numpy as np
import pytest

import oracle
from paper_2008_11520_amd import loop, synth

from gpu_common import (EPS32, GpuRunner, OracleFineStep, assert_step_errors, make_gpu_flow, make_oracle_flow,
                        merge_worst, rel_l2, rel_max, step_errors, to_dev)

pytestmark = pytest.mark.gpu
CN = 4   # DNNMG_F_CRANK_NICOLSON


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2008_11520_amd as pam
    assert pam.DNNMG_F_CRANK_NICOLSON == CN
    pam.lib()


def _flows():
    return {
        "unit16_k1": (synth.unit_square_flow(16, 16, 1, 0.01), 1, 32, 0),
        "ragged13x7_k2_perturbed": (synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5), 2, 64, 64),
        "stretched5x3_k3": (synth.stretched_flow(5, 3, 3.7, 4, 0.01), 3, 128, 128),
        "single1x1_k2": (synth.unit_square_flow(1, 1, 2, 0.01), 2, 32, 32),
        "channel40x9_k2_perturbed": (synth.channel_flow(40, 9, 2, 0.005, perturb_seed=8), 2, 64, 64),
    }


FLOWS = _flows()
NU = 1e-3


@pytest.mark.parametrize("name", sorted(FLOWS))
def test_defect_with_given_previous_velocity(name):
    import torch
    flow, K, H, Hm = FLOWS[name]
    w = synth.xavier_weights(K, H, Hm, 1234)
    g = make_gpu_flow(flow, K, H, Hm, NU, w, flags=CN)
    s = g.s
    # a smooth previous velocity (the flow's field two steps on, prolongated)
    # plus a seeded rough part, so that its transport term is not small
    u_prev = oracle.prolong(flow.nx, flow.ny, K, flow.fields(5)[0].astype(np.float64))
    u_prev = (u_prev + 0.1 * synth.SplitMix64(77).uniform(2 * s["Fn"], -1.0, 1.0).reshape(-1, 2)).astype(np.float32)
    g.set_state(None, to_dev(u_prev.reshape(-1)), steps=1)
    v, p = flow.fields(3)
    D = torch.empty(2 * s["Fn"], dtype=torch.float32, device="cuda")
    g.defect(to_dev(v.reshape(-1)), to_dev(p), D)
    torch.cuda.synchronize()
    cxy = flow.cxy.reshape(-1, 2)
    pv = oracle.prolong(flow.nx, flow.ny, K, v.astype(np.float64))
    pp = oracle.prolong(flow.nx, flow.ny, K, p.astype(np.float64))
    u64 = u_prev.astype(np.float64)
    ref = oracle.defect_theta(flow.nx, flow.ny, K, cxy, pv, pp, u64, flow.dt, NU, 0.5, flow.dirichlet)
    ie = oracle.defect(flow.nx, flow.ny, K, cxy, pv, pp, u64, flow.dt, NU, flow.dirichlet)
    S = oracle.defect_abs(flow.nx, flow.ny, K, cxy, pv, pp, u64, 1.0 / flow.dt, NU) + \
        oracle.defect_abs(flow.nx, flow.ny, K, cxy, u64, np.zeros_like(pp), u64, 0.0, NU)
    got = D.cpu().numpy().reshape(-1, 2)
    mask = oracle.dirichlet_mask(flow.nx, flow.ny, K, flow.dirichlet)
    ratio = np.abs(got - ref) / (EPS32 * S + 1e-300)
    err = rel_l2(got, ref)
    print("CN defect", name, "rel-L2 %.2e" % err, "max error / (eps32 * scale) %.2f" % ratio.max(),
          "CN vs IE oracle rel-L2 %.2e" % rel_l2(ref, ie))
    # the schemes differ by far more than the bound (the test sees the theta terms)
    assert rel_l2(ref, ie) > 100 * max(err, 1e-7)
    assert np.all(got[mask] == 0.0)
    assert err < 1e-5
    assert ratio.max() <= 64.0


@pytest.mark.parametrize("name", ["ragged13x7_k2_perturbed", "stretched5x3_k3"])
def test_first_step_defect_takes_the_implicit_euler_elements(name):
    """Before the first step u_prev = P v: the Crank-Nicolson kernel takes
    the implicit-Euler elements with 1/dt = 0 (the same source in another
    kernel, so equal up to the compiler's choice of fused multiply-adds:
    within 4 eps32 of the running-error scale) and matches the oracle."""
    import torch
    flow, K, H, Hm = FLOWS[name]
    w = synth.xavier_weights(K, H, Hm, 1234)
    v, p = flow.fields(2)
    out = []
    for flags in (0, CN):
        g = make_gpu_flow(flow, K, H, Hm, NU, w, flags=flags)
        D = torch.empty(2 * g.s["Fn"], dtype=torch.float32, device="cuda")
        g.defect(to_dev(v.reshape(-1)), to_dev(p), D)
        torch.cuda.synchronize()
        out.append(D.cpu().numpy().reshape(-1, 2))
    cxy = flow.cxy.reshape(-1, 2)
    pv = oracle.prolong(flow.nx, flow.ny, K, v.astype(np.float64))
    pp = oracle.prolong(flow.nx, flow.ny, K, p.astype(np.float64))
    ref = oracle.defect_theta(flow.nx, flow.ny, K, cxy, pv, pp, pv, flow.dt, NU, 0.5, flow.dirichlet)
    S = oracle.defect_abs(flow.nx, flow.ny, K, cxy, pv, pp, pv, 0.0, NU)
    print("first step: CN vs IE kernel bitwise equal:", np.array_equal(out[0], out[1]))
    assert np.all(np.abs(out[1] - out[0]) <= 4 * EPS32 * S)
    assert np.all(np.abs(out[1] - ref) <= 64 * EPS32 * S)


@pytest.mark.parametrize("name,dt", [("unit16_k1", None), ("ragged13x7_k2_perturbed", None),
                                     ("stretched5x3_k3", None), ("ragged13x7_k2_perturbed", 1e3),
                                     ("stretched5x3_k3", 1e3)])
def test_rhs_restrict_stage_fp64(name, dt):
    """b_L = R [(1/dt) M_f u - (1/2) T(u)], u = P v + dbar, for seeded v and
    dbar.  dt = 1e3 makes the explicit transport term the larger part."""
    import torch
    import paper_2008_11520_amd as pam
    flow, K, H, Hm = FLOWS[name]
    dt = flow.dt if dt is None else dt
    w = synth.xavier_weights(K, H, Hm, 1234)
    cfg = pam.make_config(flow.nx, flow.ny, K, H, Hm, dt, NU, "fp32", flow.dirichlet, CN)
    g = pam.DnnMG(cfg, flow.cxy, w)
    s = g.s
    v, _ = flow.fields(1)
    dbar = (0.3 * synth.SplitMix64(5).uniform(2 * s["Fn"], -1.0, 1.0)).astype(np.float32)
    b = torch.empty(2 * s["Nc"], dtype=torch.float64, device="cuda")
    g.rhs_restrict(to_dev(v.reshape(-1)), to_dev(dbar), b)
    torch.cuda.synchronize()
    cxy = flow.cxy.reshape(-1, 2)
    v64, d64 = v.astype(np.float64), dbar.astype(np.float64).reshape(-1, 2)
    ref = oracle.rhs_restrict_theta(flow.nx, flow.ny, K, cxy, v64, d64, dt, NU, 0.5)
    mass = oracle.rhs_restrict(flow.nx, flow.ny, K, cxy, v64, d64, dt)
    got = b.cpu().numpy().reshape(-1, 2)
    err = rel_max(got, ref)
    share = np.abs(ref - mass).max() / np.abs(ref).max()
    print("CN rhs stage", name, "dt", dt, "max-rel %.2e" % err, "explicit share %.2e" % share)
    if dt > 1.0:
        assert share > 0.5
    assert err < 1e-10


@pytest.mark.parametrize("name", sorted(FLOWS))
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_step_sequence_matches_oracle(name, prec, tol):
    flow, K, H, Hm = FLOWS[name]
    w = synth.xavier_weights(K, H, Hm, 1234)
    g = GpuRunner(make_gpu_flow(flow, K, H, Hm, NU, w, prec, flags=CN))
    o = make_oracle_flow(flow, K, H, Hm, NU, w, theta=0.5)
    worst = {}
    for n in range(5):
        v, p = flow.fields(n)
        got = g.step(v, p)
        ref = o.step(v, p, want=("Dbar", "bL", "dpatch"))
        merge_worst(worst, step_errors(got, ref, o.h, flow.nx, flow.ny, K, flow.dirichlet))
    print("CN step errors", name, prec, worst)
    assert_step_errors(worst, tol, 1e-5 if prec == "fp32" else tol)


def test_batched_step_rejects_crank_nicolson_contexts():
    import torch
    import paper_2008_11520_amd as pam
    flow, K, H, Hm = FLOWS["ragged13x7_k2_perturbed"]
    w = synth.xavier_weights(K, H, Hm, 1234)
    a = make_gpu_flow(flow, K, H, Hm, NU, w, "bf16")
    b = make_gpu_flow(flow, K, H, Hm, NU, None, "bf16", share=a, flags=CN)
    v, p = flow.fields(0)
    vd, pd = to_dev(v.reshape(-1)), to_dev(p)
    batch = pam.Batch(2)
    with pytest.raises(pam.DnnmgError) as e:
        batch.step([a, b], [vd, vd], [pd, pd])
    assert e.value.code == pam.DNNMG_EINVAL and "CRANK_NICOLSON" in str(e.value)
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_closed_loop_gpu_step_matches_oracle_step(prec, tol):
    """The closed loop of Alg. 2 with Crank-Nicolson on both levels: the GPU
    fine step against the oracle's, 8 steps of the unit-square configuration."""
    flow, K, H, Hm = synth.unit_square_flow(16, 16, 1, 0.01), 1, 32, 0
    w = synth.xavier_weights(K, H, Hm, 1234)
    gpu = loop.GpuFineStep(flow, K, H, Hm, w, NU, prec, theta=0.5)
    a = loop.run(flow, NU, 8, fine=gpu, theta=0.5)
    b = loop.run(flow, NU, 8, fine=OracleFineStep(flow, K, H, Hm, w, NU, theta=0.5), theta=0.5)
    gpu.close()
    scale = np.abs(b["v"]).max()
    errs = [float(np.abs(a["v"][n] - b["v"][n]).max() / scale) for n in range(8)]
    print("CN closed loop", prec, ["%.1e" % e for e in errs])
    assert max(errs) < tol
