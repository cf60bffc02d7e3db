"""Joint damping (implicit) on the HIP path against the FP64 oracle and its closed form
(needs an MI355X)."""
import numpy as np
import pytest

from gpu_common import RTOL_ROLLOUT, RTOL_STEP, by_name, gpu_run, oracle_run, rel_err
from helpers import DT_LEVER, lever
from workloads import inputs

pytestmark = pytest.mark.gpu


def test_damped_lever_geometric_decay_gpu():
    """Without gravity the damped lever's velocity falls by M / (M + dt B) per step (FP32)."""
    import torch
    import paper_2601_22074_amd as rb
    b, l, mass, r = 0.3, 0.5, 2.0, 0.02
    m = lever(None, gravity=(0, 0, 0), l=l, m=mass, r=r)
    m["joints"][0]["damping"] = b
    I = mass * l * l + 0.4 * mass * r * r
    M = rb.Model(m)
    B = rb.Batch(M, 4)
    q = torch.zeros(4, 1, device="cuda")
    v = torch.ones(4, 1, device="cuda")
    u = torch.zeros(4, 0, device="cuda")
    got = []
    for _ in range(50):
        B.step(u, q, v)
        got.append(v[0, 0].item())
    B.close()
    M.close()
    ref = (I / (I + DT_LEVER * b)) ** np.arange(1, 51)
    np.testing.assert_allclose(got, ref, rtol=2e-6)


@pytest.mark.parametrize("name", ["chain3_damp", "humanoid_damp"])
def test_single_step_damped(oracle_mod, name):
    m = by_name(name)
    n = 64
    q, v = inputs.initial_state(m, name, range(n))
    u = inputs.ctrl_table(m, name, range(n), 1)[0]
    fr, ms = inputs.world_params(m, name, range(n))
    g = gpu_run(m, q, v, u, friction=fr, mass_scale=ms)
    r = oracle_run(oracle_mod.Oracle(m), q, v, u, None, fr, ms)
    assert rel_err(g["qpos"], r["qpos"]) <= RTOL_STEP
    assert rel_err(g["qvel"], r["qvel"]) <= RTOL_STEP
    assert np.all(g["status"] & 1 == 0)


def test_ten_steps_damped_chain(oracle_mod):
    m = by_name("chain3_damp")
    q, v = inputs.initial_state(m, "chain3_damp", range(32))
    g = gpu_run(m, q, v, nsteps=10)
    r = oracle_run(oracle_mod.Oracle(m), q, v, nsteps=10)
    assert rel_err(g["qpos"], r["qpos"]) <= RTOL_ROLLOUT
    assert rel_err(g["qvel"], r["qvel"]) <= RTOL_ROLLOUT


def test_fused_equals_separate_with_damping():
    """A fused launch over damped and undamped models reproduces their plain launches bit for
    bit."""
    import torch
    import paper_2601_22074_amd as rb
    dev = torch.device("cuda:0")
    plan_models = [("chain3_damp", 64), ("humanoid_damp", 96), ("quadruped", 64)]
    runs = []
    for fused in (False, True):
        S = []
        for name, n in plan_models:
            m = by_name(name)
            q, v = inputs.initial_state(m, name, range(n))
            fr, ms = inputs.world_params(m, name, range(n))
            ctab = inputs.ctrl_table(m, name, range(n), 2)
            M = rb.Model(m)
            B = rb.Batch(M, n)
            if fr is not None:
                B.set_params(rb.PARAM_FRICTION, torch.tensor(fr, device=dev))
                B.set_params(rb.PARAM_MASS_SCALE, torch.tensor(ms, device=dev))
            ct = torch.zeros(2, n, max(M.nu, 1), device=dev)
            if M.nu:
                ct[:, :, :M.nu] = torch.tensor(ctab, device=dev)
            S.append(dict(M=M, B=B, q=torch.tensor(q, device=dev), v=torch.tensor(v, device=dev), ct=ct,
                          u=ct[0].clone(), st=torch.zeros(n, dtype=torch.int32, device=dev)))
        plan = None
        if fused:
            plan = rb.Multi([x["B"] for x in S])
            for i, x in enumerate(S):
                plan.bind(i, x["u"], x["q"], x["v"], None, x["st"])
            plan.set_schedule(rb.ORDER_INTERLEAVE, 0)
        for s in range(40):
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
