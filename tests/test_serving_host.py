"""Host logic of the serving form: admission policy and the device-side input
evaluators (run here on CPU tensors)."""
import numpy as np
import pytest

from paper_2008_11520_amd import synth
from paper_2008_11520_amd.serve import Scheduler


def _reqs(costs):
    return [dict(id=i, cost=c) for i, c in enumerate(costs)]


def test_scheduler_fcfs_within_budget():
    s = Scheduler(budget=100, max_flows=8, cost=lambda r: r["cost"])
    for r in _reqs([40, 40, 30, 10]):
        s.arrive(r)
    got = [r["id"] for r in s.admissible()]
    assert got == [0, 1]            # the 30 does not fit; the 10 behind it waits too (no overtaking)
    assert s.used == 80 and s.running == 2 and [r["id"] for r in s.queue] == [2, 3]
    s.release(dict(id=0, cost=40))
    assert [r["id"] for r in s.admissible()] == [2, 3]
    assert s.used == 80 and s.running == 3 and not s.queue


def test_scheduler_slot_limit():
    s = Scheduler(budget=10 ** 9, max_flows=2, cost=lambda r: r["cost"])
    for r in _reqs([1, 1, 1]):
        s.arrive(r)
    assert [r["id"] for r in s.admissible()] == [0, 1]
    assert s.admissible() == []
    s.release(dict(id=1, cost=1))
    assert [r["id"] for r in s.admissible()] == [2]


def test_scheduler_refuses_request_larger_than_budget():
    s = Scheduler(budget=50, max_flows=4, cost=lambda r: r["cost"])
    with pytest.raises(ValueError):
        s.arrive(dict(id=7, cost=51))
    s.arrive(dict(id=8, cost=50))
    assert [r["id"] for r in s.admissible()] == [8]


def test_serving_requests_recipe():
    reqs = synth.serving_requests(256, 20.0, 11)
    assert len(reqs) == 256
    arr = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(arr) > 0)
    # Poisson arrivals at 20/s: the mean gap is 1/20 s within sampling error
    assert abs(np.diff(arr).mean() - 0.05) < 0.01
    assert all(50 <= r["steps"] <= 500 for r in reqs)
    assert {(r["nx"], r["ny"]) for r in reqs} <= set(synth.SERVE_MESHES)


@pytest.mark.parametrize("inflow", [0.0, 1.5])
def test_torch_fields_match_numpy_fields(inflow):
    import torch
    nx, ny = 12, 5
    cxy = synth.perturb_interior(synth.rect_mesh(nx, ny, synth.CHANNEL_LX, synth.CHANNEL_LY), 0.1, 3)
    ff = synth.FourierField(synth.CHANNEL_LX, synth.CHANNEL_LY, 42).calibrate(cxy)
    flow = synth.Flow(nx, ny, cxy, synth.DIR_CHANNEL, 0.005, ff, inflow_max=inflow)
    xy = torch.from_numpy(cxy.reshape(-1, 2).copy())
    ff2 = synth.FourierField(synth.CHANNEL_LX, synth.CHANNEL_LY, 42).calibrate_torch(xy)
    assert ff2.vscale == pytest.approx(ff.vscale, rel=1e-13)
    assert ff2.pscale == pytest.approx(ff.pscale, rel=1e-13)
    v, p = ff2.fields_torch(xy, [n * 0.005 for n in range(4)], inflow_max=inflow, height=synth.CHANNEL_LY)
    for n in range(4):
        vn, pn = flow.fields(n)
        np.testing.assert_allclose(v[n].numpy().astype(np.float32), vn, rtol=0, atol=2e-6)
        np.testing.assert_allclose(p[n].numpy().astype(np.float32), pn, rtol=0, atol=2e-6)


@pytest.mark.parametrize("inflow", [0.0, 1.5])
def test_device_calibrated_fields_match_numpy_fields(inflow):
    """The serving loop's field evaluation with the calibration kept on the
    device (no host read-back) gives the numpy fields."""
    import torch
    nx, ny = 12, 5
    cxy = synth.rect_mesh(nx, ny, synth.CHANNEL_LX, synth.CHANNEL_LY)
    ff = synth.FourierField(synth.CHANNEL_LX, synth.CHANNEL_LY, 7).calibrate(cxy)
    flow = synth.Flow(nx, ny, cxy, synth.DIR_CHANNEL, 0.005, ff, inflow_max=inflow)
    xy = torch.from_numpy(cxy.reshape(-1, 2).copy())
    v, p = synth.fields_torch_calibrated(synth.FourierField(synth.CHANNEL_LX, synth.CHANNEL_LY, 7), xy,
                                         [n * 0.005 for n in range(3)], inflow_max=inflow, height=synth.CHANNEL_LY)
    for n in range(3):
        vn, pn = flow.fields(n)
        np.testing.assert_allclose(v[n].numpy().astype(np.float32), vn, rtol=0, atol=2e-6)
        np.testing.assert_allclose(p[n].numpy().astype(np.float32), pn, rtol=0, atol=2e-6)


@pytest.mark.parametrize("inflow", [0.0, 1.5])
def test_grouped_field_rings_match_numpy_fields(inflow):
    """The serving loop's field rings, evaluated for a group of flows at once,
    give each flow's numpy fields, and a flow's values are those it gets when
    evaluated alone."""
    import torch
    meshes = [(12, 5), (4, 1), (9, 3)]
    seeds = [7, 8, 9]
    times = [n * 0.005 for n in range(3)]
    mk = lambda: [synth.FourierField(synth.CHANNEL_LX, synth.CHANNEL_LY, s) for s in seeds]
    v, p, offs = synth.channel_rings_torch(mk(), meshes, times, synth.CHANNEL_LX, synth.CHANNEL_LY, inflow,
                                           synth.CHANNEL_LY, "cpu")
    assert v.shape == (3, offs[-1], 2) and p.shape == (3, offs[-1])
    for f, ((nx, ny), s) in enumerate(zip(meshes, seeds)):
        cxy = synth.rect_mesh(nx, ny, synth.CHANNEL_LX, synth.CHANNEL_LY)
        ff = synth.FourierField(synth.CHANNEL_LX, synth.CHANNEL_LY, s).calibrate(cxy)
        flow = synth.Flow(nx, ny, cxy, synth.DIR_CHANNEL, 0.005, ff, inflow_max=inflow)
        a, b = offs[f], offs[f + 1]
        v1, p1, o1 = synth.channel_rings_torch(mk()[f:f + 1], meshes[f:f + 1], times, synth.CHANNEL_LX,
                                               synth.CHANNEL_LY, inflow, synth.CHANNEL_LY, "cpu")
        np.testing.assert_allclose(v[:, a:b].numpy(), v1.numpy(), rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(p[:, a:b].numpy(), p1.numpy(), rtol=1e-14, atol=1e-15)
        for n in range(3):
            vn, pn = flow.fields(n)
            np.testing.assert_allclose(v[n, a:b].numpy().astype(np.float32), vn, rtol=0, atol=2e-6)
            np.testing.assert_allclose(p[n, a:b].numpy().astype(np.float32), pn, rtol=0, atol=2e-6)


def test_device_mesh_equals_numpy_mesh():
    import torch
    for nx, ny in ((32, 8), (512, 128), (3, 1)):
        a = synth.rect_mesh(nx, ny, synth.CHANNEL_LX, synth.CHANNEL_LY).reshape(-1, 2)
        b = synth.rect_mesh_torch(nx, ny, synth.CHANNEL_LX, synth.CHANNEL_LY, "cpu").numpy()
        assert np.array_equal(a, b)


def test_scheduler_admission_limit():
    s = Scheduler(budget=100, max_flows=8, cost=lambda r: r["cost"])
    for r in _reqs([10, 10, 10, 10]):
        s.arrive(r)
    assert [r["id"] for r in s.admissible(limit=2)] == [0, 1]
    assert [r["id"] for r in s.admissible(limit=0)] == []
    assert [r["id"] for r in s.admissible()] == [2, 3]
    s.requeue(dict(id=3, cost=10))
    assert s.used == 30 and s.running == 3 and [r["id"] for r in s.queue] == [3]
