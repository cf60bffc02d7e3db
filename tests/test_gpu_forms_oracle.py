"""The batching and serving forms against the FP64 oracle directly (needs an MI355X).

Both forms run every world through the same per-world code as the plain launch, so each test
checks two links: the form's result equals the plain launch bit for bit, and the plain launch
matches the oracle one env step at a time (StepTally: the step tolerance wherever the work
records of both paths agree)."""
import numpy as np
import pytest

from gpu_common import (RTOL_ROLLOUT, StepTally, band_worlds, by_name, fp32_floor, gpu_step_records,
                        oracle_step_records, rel_err)
from workloads import inputs, robots
from workloads.requests import DeviceSource, Request

pytestmark = pytest.mark.gpu

# the mixed batch of the batching workload: model, worlds
MIX = [("chain3", 512), ("quadruped", 4096), ("humanoid", 2048), ("arm_box", 1024)]


def _advanced(name, n, idx, start, o):
    """Inputs of n worlds of a workload with the sampled worlds idx advanced `start` env steps by
    the oracle (FP64, rounded to FP32); the other worlds keep their initial states."""
    W = inputs.workload(name, n, start + 1)
    q, v = W["qpos"].copy(), W["qvel"].copy()
    ws = np.zeros((n, o.nv), np.float32)
    fr, ms = W["friction"], W["mass_scale"]
    sub = lambda a: None if a is None else a[idx].astype(np.float64)
    qq, vv, wd = q[idx].astype(np.float64), v[idx].astype(np.float64), np.zeros((len(idx), o.nv))
    st = np.zeros(len(idx), np.uint32)
    for s in range(start):
        o.step(W["ctrl"][s // inputs.CTRL_PERIOD][idx].astype(np.float64), qq, vv, wd, sub(fr), sub(ms), st)
    q[idx], v[idx], ws[idx] = qq.astype(np.float32), vv.astype(np.float32), wd.astype(np.float32)
    u = W["ctrl"][start // inputs.CTRL_PERIOD]
    return W["model"], q, v, u, ws, fr, ms


def test_fused_mixed_batch_against_oracle(oracle_mod):
    """The batching workload at its counts (chain 512, quadruped 4096, humanoid 2048, arm and
    cube 1024) in one fused launch: every world equals its plain launch bit for bit, and 64
    sampled worlds of each model (states 20 env steps into the oracle's trajectory, in contact)
    match the oracle's env step."""
    import torch
    import paper_2601_22074_amd as rb
    dev = torch.device("cuda:0")
    S = []
    for name, n in MIX:
        o = oracle_mod.Oracle(by_name(name))
        idx = np.arange(0, n, n // 64)
        m, q, v, u, ws, fr, ms = _advanced(name, n, idx, 0 if name == "chain3" else 20, o)
        M = rb.Model(m)
        B = rb.Batch(M, n)
        if fr is not None:
            B.set_params(rb.PARAM_FRICTION, torch.tensor(fr, device=dev))
        if ms is not None:
            B.set_params(rb.PARAM_MASS_SCALE, torch.tensor(ms, device=dev))
        B.reset(torch.arange(n, dtype=torch.int32, device=dev), torch.tensor(ws, device=dev))
        x = dict(name=name, n=n, idx=idx, o=o, m=m, q=q, v=v, u=u, ws=ws, fr=fr, ms=ms, M=M, B=B,
                 qt=torch.tensor(q, device=dev), vt=torch.tensor(v, device=dev),
                 ut=torch.tensor(u if M.nu else np.zeros((n, 1), np.float32), device=dev),
                 st=torch.zeros(n, dtype=torch.int32, device=dev))
        x["con"] = B.contacts(n)
        S.append(x)
    plan = rb.Multi([x["B"] for x in S])
    try:
        for i, x in enumerate(S):
            plan.bind(i, x["ut"] if x["M"].nu else None, x["qt"], x["vt"], x["con"], x["st"])
        plan.set_schedule(rb.ORDER_HEAVY_FIRST, 0)
        plan.step()
        torch.cuda.synchronize()
        for x in S:
            g = gpu_step_records(x["m"], x["q"], x["v"], x["u"], x["ws"], x["fr"], x["ms"])
            np.testing.assert_array_equal(x["qt"].cpu().numpy(), g["qpos"])
            np.testing.assert_array_equal(x["vt"].cpu().numpy(), g["qvel"])
            for k in ("ncon", "geom", "feature", "dist", "pos", "frame", "force"):
                np.testing.assert_array_equal(getattr(x["con"], k).cpu().numpy(), g["contacts"][k])
            idx, o, m = x["idx"], x["o"], x["m"]
            sub = lambda a: None if a is None else a[idx]
            args = (x["q"][idx], x["v"][idx], x["u"][idx], x["ws"][idx], sub(x["fr"]), sub(x["ms"]))
            r = oracle_step_records(o, *args)
            band = band_worlds(oracle_mod, m, *args)
            T = StepTally(f"fused {x['name']} x{x['n']}")
            for j, w in enumerate(idx):
                T.add(g, r, w, j, band[j], (x["name"], int(w)), floor=lambda j=j: fp32_floor(o, m, *args, j))
            T.finish()
    finally:
        plan.close()
        for x in S:
            x["B"].close()
            x["M"].close()


def _request_inputs(req, m):
    """A request's inputs as the server draws them from its generator (device Philox, in the
    server's order): initial state, per-world parameters and the control table (segment j is
    held for ticks [20 j, 20 j + 20))."""
    import torch
    src = DeviceSource({req.name: m})
    g = src.generator(req.seed)
    nq = len(robots.qpos0(m))
    nv = sum(6 if j["type"] == "free" else 1 for j in m["joints"])
    nu = len(m["actuators"])
    q = torch.zeros(req.n, nq, device="cuda")
    v = torch.zeros(req.n, nv, device="cuda")
    src.initial(req.name, req.n, g, q, v)
    fr, ms = src.params(req.name, req.n, g)
    ctab = []
    for _ in range(0, req.horizon, inputs.CTRL_PERIOD):
        u = torch.zeros(req.n, nu, device="cuda")
        if nu:
            src.ctrl(req.name, g, u)
        ctab.append(u.cpu().numpy())
    c = lambda t: None if t is None else t.cpu().numpy()
    return q.cpu().numpy(), v.cpu().numpy(), c(fr), c(ms), ctab


def _oracle_path(o, q, v, fr, ms, ctab, horizon):
    """The oracle's own trajectory from the request's initial state: (qpos, qvel, warm start) in
    FP64 before every tick and after the last."""
    qq, vv, ws = q.astype(np.float64), v.astype(np.float64), np.zeros((q.shape[0], o.nv))
    f64 = lambda a: None if a is None else a.astype(np.float64)
    st = np.zeros(q.shape[0], np.uint32)
    out = [(qq.copy(), vv.copy(), ws.copy())]
    for k in range(horizon):
        o.step(ctab[k // inputs.CTRL_PERIOD].astype(np.float64), qq, vv, ws, f64(fr), f64(ms), st)
        out.append((qq.copy(), vv.copy(), ws.copy()))
    return out


def _serve_forced(req, forced):
    """Serve one request alone; before each tick in `forced`, its state (qpos, qvel, warm start)
    is overwritten with the given FP32 values.  Returns the state found at the start of every
    tick (before any overwrite) and after the last: the served results."""
    import torch
    from paper_2601_22074_amd.serve import Server
    src = DeviceSource({req.name: robots.by_name(req.name)})
    n = req.n
    snaps = []

    class Forced(Server):
        def _snap(self):
            p = self.pools[0]
            snaps.append((p["q"][:n].clone(), p["v"][:n].clone()))

        def _tick(self):
            self._snap()
            k = self.nticks
            if k in forced:
                p = self.pools[0]
                q32, v32, w32 = forced[k]
                p["q"][:n].copy_(torch.tensor(q32, device=self.dev))
                p["v"][:n].copy_(torch.tensor(v32, device=self.dev))
                p["batch"].reset(torch.arange(n, dtype=torch.int32, device=self.dev), torch.tensor(w32, device=self.dev))
            super()._tick()

    s = Forced(src, capacity={req.name: n})
    s.run_script([req])
    s._snap()
    torch.cuda.synchronize()
    out = [(q.cpu().numpy(), v.cpu().numpy()) for q, v in snaps]
    s.close()
    return out


@pytest.mark.parametrize("name,n,horizon", [("humanoid", 32, 60), ("quadruped", 32, 60), ("arm_box", 16, 60)])
def test_served_request_against_oracle(oracle_mod, name, n, horizon):
    """One served request, teacher-forced from the oracle's own trajectory (inputs drawn as the
    server draws them): every 3rd tick the served state is replaced by the oracle's (rounded to
    FP32) and the served next state is compared with one oracle env step from it (StepTally;
    the work records come from the plain launch on the same inputs, which must give the served
    bits)."""
    m = by_name(name)
    req = Request(0, name, n, horizon, 777, 0)
    q0, v0, fr, ms, ctab = _request_inputs(req, m)
    o = oracle_mod.Oracle(m)
    path = _oracle_path(o, q0, v0, fr, ms, ctab, horizon)
    ticks = list(range(0, horizon, 3))
    forced = {k: tuple(x.astype(np.float32) for x in path[k]) for k in ticks}
    served = _serve_forced(req, forced)
    assert len(served) == horizon + 1
    T = StepTally(f"served {name} x{n}")
    for k in ticks:
        q, v, ws = forced[k]
        u = ctab[k // inputs.CTRL_PERIOD]
        g = gpu_step_records(m, q, v, u, ws, fr, ms)
        np.testing.assert_array_equal(g["qpos"], served[k + 1][0])
        np.testing.assert_array_equal(g["qvel"], served[k + 1][1])
        r = oracle_step_records(o, q, v, u, ws, fr, ms)
        band = band_worlds(oracle_mod, m, q, v, u, ws, fr, ms)
        for w in range(n):
            T.add(g, r, w, w, band[w], (name, k, w), floor=lambda w=w: fp32_floor(o, m, q, v, u, ws, fr, ms, w))
    T.finish()


def test_served_chain_windows_against_oracle(oracle_mod):
    """A served chain request (contact-free), forced onto the oracle's own trajectory every 10
    ticks: each 10-tick window of served steps against the oracle's 10 env steps from the same
    FP32 state (rollout tolerance)."""
    m = by_name("chain3")
    req = Request(0, "chain3", 64, 100, 31, 0)
    q0, v0, fr, ms, ctab = _request_inputs(req, m)
    o = oracle_mod.Oracle(m)
    path = _oracle_path(o, q0, v0, fr, ms, ctab, 100)
    forced = {k: tuple(x.astype(np.float32) for x in path[k]) for k in range(0, 100, 10)}
    served = _serve_forced(req, forced)
    for k, (q32, v32, _) in forced.items():
        q, v, ws = q32.astype(np.float64), v32.astype(np.float64), np.zeros((64, o.nv))
        for _ in range(10):
            o.step(np.zeros((64, 0)), q, v, ws)
        assert rel_err(served[k + 10][0], q) <= RTOL_ROLLOUT
        assert rel_err(served[k + 10][1], v) <= RTOL_ROLLOUT
