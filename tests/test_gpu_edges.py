"""Edge cases of the step on the HIP path: no worlds, part of a batch, ragged world counts, a
fused plan with an empty batch (needs an MI355X)."""
import numpy as np
import pytest

from gpu_common import RTOL_STEP, by_name, gpu_run, oracle_run, rel_err
from workloads import inputs

pytestmark = pytest.mark.gpu


def _batch(rb, torch, name, cap):
    m = by_name(name)
    M = rb.Model(m)
    B = rb.Batch(M, cap)
    fr, ms = inputs.world_params(m, name, range(cap))
    if fr is not None:
        B.set_params(rb.PARAM_FRICTION, torch.tensor(fr, device="cuda"))
        B.set_params(rb.PARAM_MASS_SCALE, torch.tensor(ms, device="cuda"))
    return m, M, B


def test_zero_worlds_is_a_no_op():
    import torch
    import paper_2601_22074_amd as rb
    m, M, B = _batch(rb, torch, "quadruped", 8)
    q = torch.zeros(0, M.nq, device="cuda")
    v = torch.zeros(0, M.nv, device="cuda")
    u = torch.zeros(0, M.nu, device="cuda")
    B.step(u, q, v)
    ws = torch.ones(8, M.nv, device="cuda")
    st = torch.ones(8, dtype=torch.int32, device="cuda")
    B.get_state(8, ws, st)
    torch.cuda.synchronize()
    assert float(ws.abs().max()) == 0.0 and int(st.abs().max()) == 0
    B.close()
    M.close()


def test_part_of_a_batch_leaves_the_rest_untouched():
    """Stepping the first 10 of 64 slots changes only their warm starts and status."""
    import torch
    import paper_2601_22074_amd as rb
    m, M, B = _batch(rb, torch, "humanoid", 64)
    q, v = inputs.initial_state(m, "humanoid", range(10))
    u = inputs.ctrl_table(m, "humanoid", range(10), 1)[0]
    qt, vt = torch.tensor(q, device="cuda"), torch.tensor(v, device="cuda")
    for _ in range(5):
        B.step(torch.tensor(u, device="cuda"), qt, vt)
    ws = torch.zeros(64, M.nv, device="cuda")
    B.get_state(64, ws, None)
    torch.cuda.synchronize()
    w = ws.cpu().numpy()
    assert np.abs(w[:10]).max() > 0 and np.abs(w[10:]).max() == 0.0
    B.close()
    M.close()


@pytest.mark.parametrize("n", [1, 37, 257])
def test_ragged_world_counts(oracle_mod, n):
    """World counts that fill no round of the grid evenly step like the oracle."""
    m = by_name("humanoid")
    q, v = inputs.initial_state(m, "humanoid", range(n))
    u = inputs.ctrl_table(m, "humanoid", range(n), 1)[0]
    fr, ms = inputs.world_params(m, "humanoid", range(n))
    g = gpu_run(m, q, v, u, friction=fr, mass_scale=ms)
    r = oracle_run(oracle_mod.Oracle(m), q, v, u, None, fr, ms)
    assert rel_err(g["qpos"], r["qpos"]) <= RTOL_STEP
    assert rel_err(g["qvel"], r["qvel"]) <= RTOL_STEP


def test_fused_plan_with_an_empty_batch():
    """A fused plan where one batch is bound with no worlds steps the other exactly as its
    plain launch does."""
    import torch
    import paper_2601_22074_amd as rb
    out = []
    for fused in (False, True):
        ma, Ma, Ba = _batch(rb, torch, "quadruped", 32)
        mb, Mb, Bb = _batch(rb, torch, "chain3", 8)
        q, v = inputs.initial_state(ma, "quadruped", range(32))
        u = torch.tensor(inputs.ctrl_table(ma, "quadruped", range(32), 1)[0], device="cuda")
        qt, vt = torch.tensor(q, device="cuda"), torch.tensor(v, device="cuda")
        if fused:
            plan = rb.Multi([Ba, Bb])
            plan.bind(0, u, qt, vt)
            plan.bind(1, torch.zeros(0, 1, device="cuda"), torch.zeros(0, Mb.nq, device="cuda"),
                      torch.zeros(0, Mb.nv, device="cuda"))
            plan.set_schedule(rb.ORDER_HEAVY_FIRST, 0)
            for _ in range(10):
                plan.step()
            plan.close()
        else:
            for _ in range(10):
                Ba.step(u, qt, vt)
        torch.cuda.synchronize()
        out.append((qt.cpu().numpy(), vt.cpu().numpy()))
        for x in (Ba, Bb, Ma, Mb):
            x.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_plain_step_in_a_captured_graph():
    """The plain step records into a HIP graph (torch.cuda.graph); every replay, with eager
    work between them, matches the eager steps bit for bit."""
    import torch
    import paper_2601_22074_amd as rb
    m, M, B = _batch(rb, torch, "humanoid", 128)
    q0, v0 = inputs.initial_state(m, "humanoid", range(128))
    u = torch.tensor(inputs.ctrl_table(m, "humanoid", range(128), 1)[0], device="cuda")
    # eager reference: 4 steps, state after each
    qe, ve = torch.tensor(q0, device="cuda"), torch.tensor(v0, device="cuda")
    ws0 = torch.zeros(128, M.nv, device="cuda")
    ref = []
    for _ in range(4):
        B.step(u, qe, ve)
        ref.append((qe.cpu().numpy(), ve.cpu().numpy()))
    # the same from the same start, replayed from a graph of one step
    B.reset(torch.arange(128, dtype=torch.int32, device="cuda"), ws0)
    qg, vg = torch.tensor(q0, device="cuda"), torch.tensor(v0, device="cuda")
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    # capture records without running, so the graph starts from the same state
    with torch.cuda.graph(graph, stream=side):
        B.step(u, qg, vg)
    torch.cuda.synchronize()
    for k in range(4):
        graph.replay()
        torch.cuda.synchronize()
        _ = float(qg.sum())                       # eager work between replays
        np.testing.assert_array_equal(qg.cpu().numpy(), ref[k][0])
        np.testing.assert_array_equal(vg.cpu().numpy(), ref[k][1])
    B.close()
    M.close()
