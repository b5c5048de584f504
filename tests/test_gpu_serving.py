"""Serving form on the GPU: batched prepare/launch, eager and graph-replayed,
against single-flow steps, and the request loop alone versus in a mix.

All comparisons are bitwise: every flow's kernels do the same arithmetic in
the same order whether it runs alone, in a batch, eagerly or from a graph."""
import numpy as np
import pytest

from paper_2008_11520_amd import synth

from gpu_common import GpuRunner, make_gpu_flow, to_dev

pytestmark = pytest.mark.gpu

K, H, Hm = 2, 64, 64


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2008_11520_amd as pam
    pam.lib()


def _eager_noise(stream):
    """Unrelated torch work on the serving stream between launches."""
    import torch
    with torch.cuda.stream(stream):
        x = torch.randn(1 << 18, device="cuda")
        y = (x * 2.0).cumsum(0)
        return float(y[-1].item()) + float(x.sum().item())


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_batch_graph_replays_equal_eager_and_single(prec):
    import torch
    import paper_2008_11520_amd as pam
    w = synth.xavier_weights(K, H, Hm, 1234)
    flows = [synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5), synth.channel_flow(32, 8, 4, 0.005),
             synth.channel_flow(5, 3, 9, 0.005)]
    # ticks: who steps.  Flows leave, return and change order; one graph
    # serves them all.
    schedule = [[0, 1, 2], [0, 1, 2], [0, 2], [0, 2], [0, 1, 2], [2, 0, 1], [1, 2, 0]]
    st = torch.cuda.Stream()
    single = [GpuRunner(make_gpu_flow(f, K, H, Hm, 1e-3, w, prec)) for f in flows]
    sets = {}
    for mode in ("eager", "graph"):
        model = make_gpu_flow(flows[0], K, H, Hm, 1e-3, w, prec)
        ctxs = [make_gpu_flow(f, K, H, Hm, 1e-3, w, prec, share=model) for f in flows]
        sets[mode] = dict(model=model, ctxs=ctxs, runners=[GpuRunner(c) for c in ctxs], batch=pam.Batch(4))
    nstep = [0] * len(flows)
    for tick, members in enumerate(schedule):
        fields = {i: flows[i].fields(nstep[i]) for i in members}
        ref = {i: single[i].step(*fields[i]) for i in members}
        torch.cuda.synchronize()
        for mode, S in sets.items():
            with torch.cuda.stream(st):
                vs = [to_dev(fields[i][0].reshape(-1)) for i in members]
                ps = [to_dev(fields[i][1]) for i in members]
                S["batch"].prepare([S["ctxs"][i] for i in members], vs, ps,
                                   [S["runners"][i].dbar for i in members],
                                   [S["runners"][i].bL for i in members], stream=st)
                S["batch"].launch(graph=(mode == "graph"), stream=st)
            _eager_noise(st)
            st.synchronize()
            for i in members:
                r, c = S["runners"][i], S["ctxs"][i]
                c.get_state(r.h, None)
                torch.cuda.synchronize()
                s = c.s
                for key, got in (("Dbar", r.dbar.cpu().numpy().reshape(s["Fn"], 2)),
                                 ("bL", r.bL.cpu().numpy().reshape(s["Nc"], 2)),
                                 ("h", r.h.cpu().numpy().reshape(s["P"], -1))):
                    assert np.array_equal(got, ref[i][key]), (mode, tick, i, key)
                assert c.steps == nstep[i] + 1
        for i in members:
            nstep[i] += 1
    assert sets["eager"]["batch"].captures == 0
    assert sets["graph"]["batch"].captures == 1
    for S in sets.values():
        S["batch"].close()


def test_graph_grows_with_the_membership():
    """The one-launch tiles run one per block from the graph's captured grid
    (at least 8 blocks per CU, twice the tiles it was captured for): a
    membership with more tiles than that captures the graph again, a smaller
    one replays it (its extra blocks return); every tick equals the eager
    launch, bit for bit."""
    import torch
    import paper_2008_11520_amd as pam
    w = synth.xavier_weights(K, H, Hm, 1234)
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    big_nx = 8 * (2 * ncu + 8)                     # (2 ncu + 8) tiles of 8 x 8 patches per row, 4 rows: > 8 per CU
    flows = [synth.channel_flow(13, 7, 3, 0.005, perturb_seed=5), synth.channel_flow(big_nx, 32, 4, 0.005)]
    schedule = [[0], [0, 1], [0], [1, 0]]
    st = torch.cuda.Stream()
    sets = {}
    for mode in ("eager", "graph"):
        model = make_gpu_flow(flows[0], K, H, Hm, 1e-3, w, "bf16")
        ctxs = [make_gpu_flow(f, K, H, Hm, 1e-3, w, "bf16", share=model) for f in flows]
        sets[mode] = dict(model=model, ctxs=ctxs, runners=[GpuRunner(c) for c in ctxs], batch=pam.Batch(4))
    nstep = [0] * len(flows)
    for tick, members in enumerate(schedule):
        fields = {i: flows[i].fields(nstep[i]) for i in members}
        got = {}
        for mode, S in sets.items():
            with torch.cuda.stream(st):
                vs = [to_dev(fields[i][0].reshape(-1)) for i in members]
                ps = [to_dev(fields[i][1]) for i in members]
                S["batch"].prepare([S["ctxs"][i] for i in members], vs, ps,
                                   [S["runners"][i].dbar for i in members],
                                   [S["runners"][i].bL for i in members], stream=st)
                S["batch"].launch(graph=(mode == "graph"), stream=st)
            st.synchronize()
            got[mode] = {i: (S["runners"][i].dbar.cpu().numpy().copy(), S["runners"][i].bL.cpu().numpy().copy())
                         for i in members}
        for i in members:
            assert np.array_equal(got["graph"][i][0], got["eager"][i][0]), (tick, i)
            assert np.array_equal(got["graph"][i][1], got["eager"][i][1]), (tick, i)
            nstep[i] += 1
    assert sets["eager"]["batch"].captures == 0
    assert sets["graph"]["batch"].captures == 2
    for S in sets.values():
        S["batch"].close()


def test_graph_launch_rejects_default_stream():
    import torch
    import paper_2008_11520_amd as pam
    w = synth.xavier_weights(K, H, Hm, 1234)
    f = synth.channel_flow(8, 2, 1, 0.005)
    ctx = make_gpu_flow(f, K, H, Hm, 1e-3, w, "bf16")
    b = pam.Batch(2)
    with pytest.raises(pam.DnnmgError) as e:
        b.launch(graph=True, stream=None)
    assert e.value.code == pam.DNNMG_ESTATE
    v, p = f.fields(0)
    b.prepare([ctx], [to_dev(v.reshape(-1))], [to_dev(p)], stream=torch.cuda.default_stream())
    with pytest.raises(pam.DnnmgError) as e:
        b.launch(graph=True, stream=torch.cuda.default_stream())
    assert e.value.code == pam.DNNMG_EINVAL
    torch.cuda.synchronize()
    b.close()


def test_server_mix_equals_alone():
    """A small request mix under an HBM budget that holds two of the larger
    flows, so requests queue; every request's final GRU state, corrected
    velocity and last restricted rhs equal those of the same request served
    alone, bit for bit."""
    from paper_2008_11520_amd.serve import Server
    # arrivals 0.1 ms apart and 20-36 steps each, so that requests overlap on
    # the GPU and later ones queue behind the budget
    meshes = [(16, 4), (32, 8), (8, 2), (16, 4), (32, 8), (4, 1)]
    reqs = [dict(id=i, arrival=1e-4 * i, nx=nx, ny=ny, steps=20 + 4 * ((i * 2) % 5), field_seed=500 + i)
            for i, (nx, ny) in enumerate(meshes)]
    probe = Server(max_flows=8, ring=4)
    budget = 2 * probe.flow_bytes(32, 8) + probe.flow_bytes(4, 1)
    probe.close()
    srv = Server(max_flows=8, ring=4, hbm_budget=budget)
    mix = {}
    stats = srv.run(reqs, results=mix)
    srv.close()
    print("serve mix:", stats)
    assert stats["requests"] == len(reqs)
    assert stats["steps"] == sum(r["steps"] for r in reqs)
    assert max(m["queue_delay"] for m in mix.values()) > 0.0
    assert stats["max_concurrency"] >= 2
    for r in reqs:
        solo_srv = Server(max_flows=8, ring=4)
        solo = {}
        st = solo_srv.run([dict(r, arrival=0.0)], results=solo)
        solo_srv.close()
        assert st["requests"] == 1 and solo[r["id"]]["steps"] == r["steps"]
        for key in ("h", "u", "bL"):
            assert np.array_equal(mix[r["id"]][key], solo[r["id"]][key]), (r["id"], key)
