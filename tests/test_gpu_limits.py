"""Joint limits on the HIP path against the FP64 oracle (needs an MI355X)."""
import numpy as np
import pytest

from gpu_common import StepTally, band_worlds, by_name, fp32_floor, gpu_step_records, oracle_step_records
from helpers import lever, lever_rest_angle
from workloads import inputs

pytestmark = pytest.mark.gpu

LIMITED = ["chain3_lim", "quadruped_lim", "humanoid_lim"]


def _hinge_qadr(m):
    out, adr = [], 0
    for j in m["joints"]:
        if j["type"] == "hinge":
            out.append(adr)
            adr += 1
        else:
            adr += 7
    return out


@pytest.mark.parametrize("name", LIMITED)
def test_single_step_outside_limits(oracle_mod, name):
    """States with hinges up to 0.1 rad past their bounds (and moving): one env step against
    the oracle (StepTally: the step tolerance wherever the work records of both paths agree)."""
    m = by_name(name)
    n = 64
    worlds = range(n)
    q, v = inputs.initial_state(m, name, worlds)
    u = inputs.ctrl_table(m, name, worlds, 1)[0]
    fr, ms = inputs.world_params(m, name, worlds)
    rng = np.random.default_rng(11)
    hq = _hinge_qadr(m)
    lo, hi = m["joints"][-1]["range"]
    q = q.copy()
    q[:, hq] = rng.uniform(lo - 0.1, hi + 0.1, (n, len(hq))).astype(np.float32)
    v = (v + rng.normal(0, 0.5, v.shape)).astype(np.float32)
    o = oracle_mod.Oracle(m)
    ws = np.zeros((n, o.nv), np.float32)
    g = gpu_step_records(m, q, v, u, ws, fr, ms)
    r = oracle_step_records(o, q, v, u, ws, fr, ms)
    band = band_worlds(oracle_mod, m, q, v, u, ws, fr, ms)
    T = StepTally(f"{name} outside its limits")
    for w in range(n):
        T.add(g, r, w, w, band[w], (name, w), floor=lambda w=w: fp32_floor(o, m, q, v, u, ws, fr, ms, w))
    T.finish()
    assert np.all(g["status"] & 1 == 0)


def test_lever_rests_at_the_soft_equilibrium_gpu():
    """The HIP path settles the lever on its bound at the closed-form soft equilibrium (FP32:
    the rest angle to 1e-4 of its value)."""
    import torch
    import paper_2601_22074_amd as rb
    l, mass, r = 0.5, 2.0, 0.02
    m = lever([-1.0, 0.0], l=l, m=mass, r=r)
    M = rb.Model(m)
    B = rb.Batch(M, 4)
    dev = torch.device("cuda:0")
    q = torch.zeros(4, 1, device=dev)
    v = torch.zeros(4, 1, device=dev)
    u = torch.zeros(4, 0, device=dev)
    for _ in range(4000):
        B.step(u, q, v)
    torch.cuda.synchronize()
    qa = q.cpu().numpy()[:, 0]
    B.close()
    M.close()
    ref = lever_rest_angle(l, mass, r)
    assert np.all(np.abs(qa - ref) <= 1e-4 * ref), (qa, ref)


def test_fused_equals_separate_with_limits():
    """A fused launch over limited and unlimited models reproduces their plain launches bit
    for bit."""
    import torch
    import paper_2601_22074_amd as rb
    dev = torch.device("cuda:0")
    plan_models = [("chain3_lim", 64), ("quadruped", 128), ("humanoid_lim", 96)]
    runs = []
    for fused in (False, True):
        S = []
        for name, n in plan_models:
            m = by_name(name)
            q, v = inputs.initial_state(m, name, range(n))
            fr, ms = inputs.world_params(m, name, range(n))
            ctab = inputs.ctrl_table(m, name, range(n), 3)
            M = rb.Model(m)
            B = rb.Batch(M, n)
            if fr is not None:
                B.set_params(rb.PARAM_FRICTION, torch.tensor(fr, device=dev))
            if ms is not None:
                B.set_params(rb.PARAM_MASS_SCALE, torch.tensor(ms, device=dev))
            nu = max(M.nu, 1)
            ct = torch.zeros(3, n, nu, device=dev)
            if M.nu:
                ct[:, :, :M.nu] = torch.tensor(ctab, device=dev)
            S.append(dict(M=M, B=B, q=torch.tensor(q, device=dev), v=torch.tensor(v, device=dev), ct=ct,
                          u=ct[0].clone(), st=torch.zeros(n, dtype=torch.int32, device=dev)))
        plan = None
        if fused:
            plan = rb.Multi([x["B"] for x in S])
            for i, x in enumerate(S):
                plan.bind(i, x["u"], x["q"], x["v"], None, x["st"])
            with pytest.raises(rb.RbError):
                plan.step()          # no work list yet
            plan.set_schedule(rb.ORDER_HEAVY_FIRST, 0)
        for s in range(60):
            for x in S:
                x["u"].copy_(x["ct"][s // 20])
            if fused:
                plan.step()
            else:
                for x in S:
                    x["B"].step(x["u"], x["q"], x["v"], None, x["st"])
        torch.cuda.synchronize()
        runs.append([(x["q"].cpu().numpy(), x["v"].cpu().numpy(), x["st"].cpu().numpy()) for x in S])
        if plan is not None:
            plan.close()
        for x in S:
            x["B"].close()
            x["M"].close()
    for a, b in zip(runs[0], runs[1]):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
