"""Serving form on the GPU: continuous batching gives each request the result it gets alone."""
import numpy as np
import pytest

from workloads import robots
from workloads.requests import NAMES, DeviceSource, Request

pytestmark = pytest.mark.gpu

MIXED = [Request(0, "humanoid", 40, 45, 11, 0), Request(1, "quadruped", 100, 30, 12, 0),
         Request(2, "arm_box", 24, 50, 13, 3), Request(3, "chain3", 16, 25, 14, 7),
         Request(4, "humanoid", 17, 21, 15, 10), Request(5, "quadruped", 33, 60, 16, 22),
         Request(6, "arm_box", 5, 41, 17, 40), Request(7, "chain3", 64, 33, 18, 41)]


def _server(**kw):
    from paper_2601_22074_amd.serve import Server
    src = DeviceSource({k: robots.by_name(k) for k in NAMES})
    return Server(src, capacity={k: 256 for k in NAMES}, **kw)


def _run(reqs, **kw):
    s = _server(**kw)
    res = s.run_script(reqs)
    out = {rid: (r.qpos.cpu().numpy(), r.qvel.cpu().numpy(), r.status.cpu().numpy()) for rid, r in res.items()}
    peak, budget = s.sched.peak, s.sched.budget
    s.close()
    return out, peak, budget


def test_alone_equals_mix_bitwise():
    mix, _, _ = _run(MIXED)
    assert sorted(mix) == [r.rid for r in MIXED]
    for r in MIXED:
        alone, _, _ = _run([Request(r.rid, r.name, r.n, r.horizon, r.seed, 0)])
        for a, b in zip(alone[r.rid], mix[r.rid]):
            np.testing.assert_array_equal(a, b)
        assert np.all(np.isfinite(mix[r.rid][0])) and np.all(mix[r.rid][2] & 1 == 0)


def test_small_budget_serialises_admission():
    """A budget that holds about one request at a time: requests wait for memory, never
    exceed it, and still get the same results."""
    from paper_2601_22074_amd import rbstep
    from paper_2601_22074_amd.serve import bytes_per_world
    import torch  # noqa: F401
    free, _, _ = _run(MIXED)
    m = rbstep.Model(robots.by_name("quadruped"))
    budget = bytes_per_world(m, 0) * 110
    m.close()
    tight, peak, b = _run(MIXED, budget=budget)
    assert b == budget and peak <= budget
    for rid in free:
        for a, c in zip(free[rid], tight[rid]):
            np.testing.assert_array_equal(a, c)


def test_served_request_matches_plain_steps():
    """The served result of one request equals plain rb_step launches over the same inputs
    (drawn from the request's generator in the same order)."""
    import torch
    import paper_2601_22074_amd as rb
    req = Request(0, "quadruped", 48, 47, 99, 0)
    served, _, _ = _run([req])
    src = DeviceSource({"quadruped": robots.by_name("quadruped")})
    M = rb.Model(robots.by_name("quadruped"))
    B = rb.Batch(M, req.n)
    g = src.generator(req.seed)
    q = torch.zeros(req.n, M.nq, device="cuda")
    v = torch.zeros(req.n, M.nv, device="cuda")
    u = torch.zeros(req.n, M.nu, device="cuda")
    src.initial("quadruped", req.n, g, q, v)
    fr, ms = src.params("quadruped", req.n, g)
    assert fr is None and ms is None
    src.ctrl("quadruped", g, u)
    for k in range(req.horizon):
        B.step(u, q, v)
        if (k + 1) % 20 == 0:
            src.ctrl("quadruped", g, u)
    torch.cuda.synchronize()
    np.testing.assert_allclose(q.cpu().numpy(), served[0][0], rtol=0, atol=0)
    np.testing.assert_allclose(v.cpu().numpy(), served[0][1], rtol=0, atol=0)
    B.close()
    M.close()


def test_timed_run_reports_latency():
    from paper_2601_22074_amd.serve import Server
    from workloads.requests import poisson_requests
    src = DeviceSource({k: robots.by_name(k) for k in NAMES})
    s = Server(src, budget=256 << 20)
    reqs = poisson_requests(20.0, 2.0, seed=3, wmax=256, hmax=100)
    out = s.run_timed(reqs)
    s.close()
    assert out["finished"] == len(reqs) and out["queued_at_end"] == 0
    assert 0 < out["p50_latency_s"] <= out["p99_latency_s"] < out["wall_s"]
    assert out["env_steps"] == sum(r.n * r.horizon for r in reqs)


def test_plain_launch_server_same_results():
    """The plain-launch baseline (one rb_step launch per live request per tick) serves the same
    trace to the same bits as the fused server, with one launch per request-tick."""
    from paper_2601_22074_amd.serve import PlainServer
    fused, _, _ = _run(MIXED)
    src = DeviceSource({k: robots.by_name(k) for k in NAMES})
    s = PlainServer(src, capacity={k: 256 for k in NAMES})
    res = s.run_script(MIXED)
    launches = s.launches
    plain = {rid: (r.qpos.cpu().numpy(), r.qvel.cpu().numpy(), r.status.cpu().numpy()) for rid, r in res.items()}
    s.close()
    assert launches == sum(r.horizon for r in MIXED)
    for rid in fused:
        for a, b in zip(fused[rid], plain[rid]):
            np.testing.assert_array_equal(a, b)


def test_default_budget_is_free_device_memory():
    """Without a configured budget the server admits against the device's free memory (less a
    reserve), read through hipMemGetInfo, and re-reads it at each admission."""
    import torch
    from paper_2601_22074_amd.serve import DEVICE_RESERVE, Server
    src = DeviceSource({k: robots.by_name(k) for k in NAMES})
    free0 = torch.cuda.mem_get_info()[0]
    calls = []

    def probe():
        calls.append(1)
        return torch.cuda.mem_get_info()[0]

    s = Server(src, capacity={k: 256 for k in NAMES}, free_probe=probe)
    assert abs(s.sched.budget - (free0 - DEVICE_RESERVE)) <= 64 << 20
    n0 = len(calls)
    s.run_script(MIXED[:3])
    s.close()
    assert len(calls) - n0 >= 3
