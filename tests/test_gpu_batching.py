"""Mixed-model batching: one fused launch over several batches (needs an MI355X)."""
import numpy as np
import pytest

from workloads import inputs

pytestmark = pytest.mark.gpu

MIX = [("chain3", 48), ("quadruped", 96), ("humanoid", 64), ("arm_box", 40)]


def _setup(rb, torch, mix=MIX, first=0):
    dev = torch.device("cuda:0")
    out = []
    for name, n in mix:
        W = inputs.workload(name, n, 40, first_world=first)
        model = rb.Model(W["model"])
        b = rb.Batch(model, n)
        if W["friction"] is not None:
            b.set_params(rb.PARAM_FRICTION, torch.tensor(W["friction"], device=dev))
        if W["mass_scale"] is not None:
            b.set_params(rb.PARAM_MASS_SCALE, torch.tensor(W["mass_scale"], device=dev))
        u = torch.tensor(W["ctrl"][0], device=dev).contiguous()
        if u.numel() == 0:
            u = torch.zeros(n, 0, device=dev)
        out.append(dict(model=model, batch=b, u=u, q=torch.tensor(W["qpos"], device=dev),
                        v=torch.tensor(W["qvel"], device=dev)))
    return out


def _run_separate(rb, torch, steps, mix=MIX):
    S = _setup(rb, torch, mix)
    for _ in range(steps):
        for s in S:
            s["batch"].step(s["u"], s["q"], s["v"])
    torch.cuda.synchronize()
    return [(s["q"].cpu().numpy(), s["v"].cpu().numpy()) for s in S]


@pytest.mark.parametrize("order,grid", [(0, 0), (1, 0), (2, 0), (1, 64), (2, 100)])
def test_fused_equals_separate(order, grid):
    import torch
    import paper_2601_22074_amd as rb
    ref = _run_separate(rb, torch, 3)
    S = _setup(rb, torch)
    plan = rb.Multi([s["batch"] for s in S])
    for i, s in enumerate(S):
        plan.bind(i, s["u"], s["q"], s["v"])
    plan.set_schedule(order, grid)
    for _ in range(3):
        plan.step()
    torch.cuda.synchronize()
    for (q, v), s in zip(ref, S):
        np.testing.assert_array_equal(s["q"].cpu().numpy(), q)
        np.testing.assert_array_equal(s["v"].cpu().numpy(), v)


@pytest.mark.parametrize("occ", [1, 2, 4])
def test_fused_with_occupancy_cap_equals_separate(occ):
    import torch
    import paper_2601_22074_amd as rb
    ref = _run_separate(rb, torch, 3)
    S = _setup(rb, torch)
    plan = rb.Multi([s["batch"] for s in S])
    for i, s in enumerate(S):
        plan.bind(i, s["u"], s["q"], s["v"])
    plan.set_schedule(rb.ORDER_HEAVY_FIRST, 0)
    plan.set_occupancy(occ)
    for _ in range(3):
        plan.step()
    torch.cuda.synchronize()
    for (q, v), s in zip(ref, S):
        np.testing.assert_array_equal(s["q"].cpu().numpy(), q)
        np.testing.assert_array_equal(s["v"].cpu().numpy(), v)


ODD_MIX = [("chain3", 47), ("quadruped", 95), ("humanoid", 63), ("arm_box", 41)]
LEVEL_MIX = [("pincer_cube", 21), ("humanoid_weld", 19), ("quadruped_elliptic", 30), ("quadruped_lim", 33),
             ("quadruped_elliptic6", 17)]


@pytest.mark.parametrize("mix,wpg,order,grid,occ", [
    ("odd", 2, 0, 0, 0), ("odd", 4, 1, 0, 0), ("odd", 4, 2, 100, 0), ("odd", 2, 1, 62, 2), ("odd", 4, 0, 0, 2),
    ("odd", 4, 1, 0, 4), ("levels", 2, 1, 0, 0), ("levels", 4, 0, 0, 0), ("levels", 4, 2, 30, 0)])
def test_fused_worlds_per_workgroup_equals_separate(mix, wpg, order, grid, occ):
    """2 or 4 worlds per workgroup (one wave each, a partial last workgroup, persistent grids that
    are not a multiple of the group, occupancy caps, models of every level of extended code):
    every world ends bitwise where its plain launch puts it."""
    import torch
    import paper_2601_22074_amd as rb
    mx = ODD_MIX if mix == "odd" else LEVEL_MIX
    ref = _run_separate(rb, torch, 3, mx)
    S = _setup(rb, torch, mx)
    plan = rb.Multi([s["batch"] for s in S])
    for i, s in enumerate(S):
        plan.bind(i, s["u"], s["q"], s["v"])
    plan.set_schedule(order, grid)
    if occ == 4 and mix == "levels":
        pytest.skip("the level mix does not fit 4 waves per SIMD")
    plan.set_occupancy(occ)
    plan.set_group(wpg)
    for _ in range(3):
        plan.step()
    torch.cuda.synchronize()
    for (q, v), s in zip(ref, S):
        np.testing.assert_array_equal(s["q"].cpu().numpy(), q)
        np.testing.assert_array_equal(s["v"].cpu().numpy(), v)
    with pytest.raises(rb.RbError):
        plan.set_group(3)
    plan.close()


def test_fused_equals_separate_long_rollout():
    """300 env steps of contact-rich worlds: any rounding difference between the fused and the
    plain instantiations would have grown into visible divergence by then."""
    import torch
    import paper_2601_22074_amd as rb
    mix = [("chain3", 64), ("quadruped", 256), ("humanoid", 256), ("arm_box", 128)]
    ref = _run_separate(rb, torch, 300, mix)
    S = _setup(rb, torch, mix)
    plan = rb.Multi([s["batch"] for s in S])
    for i, s in enumerate(S):
        plan.bind(i, s["u"], s["q"], s["v"])
    plan.set_schedule(rb.ORDER_INTERLEAVE, 0)
    for _ in range(300):
        plan.step()
    torch.cuda.synchronize()
    for (q, v), s in zip(ref, S):
        np.testing.assert_array_equal(s["q"].cpu().numpy(), q)
        np.testing.assert_array_equal(s["v"].cpu().numpy(), v)


@pytest.mark.parametrize("wpg", [1, 2])
def test_graph_replay_equals_eager(wpg):
    """Three replays of a captured control period (2 fused steps each, with eager work between
    them), one or two worlds per workgroup: every world ends where 6 plain steps put it."""
    import torch
    import paper_2601_22074_amd as rb
    ref = _run_separate(rb, torch, 6)
    S = _setup(rb, torch)
    plan = rb.Multi([s["batch"] for s in S])
    for i, s in enumerate(S):
        plan.bind(i, s["u"], s["q"], s["v"])
    plan.set_schedule(1, 0)
    plan.set_group(wpg)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    plan.graph_capture(2, side)
    torch.cuda.synchronize()
    seen = []
    for r in range(3):
        plan.graph_launch(side)
        side.synchronize()
        seen.append(S[2]["q"].sum().item())          # eager work between replays
    torch.cuda.synchronize()
    for (q, v), s in zip(ref, S):
        np.testing.assert_array_equal(s["q"].cpu().numpy(), q)
        np.testing.assert_array_equal(s["v"].cpu().numpy(), v)
    assert len(set(seen)) == 3


def test_autotune_leaves_state_untouched(tmp_path, monkeypatch):
    import torch
    import paper_2601_22074_amd as rb
    from paper_2601_22074_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    ref = _run_separate(rb, torch, 2)
    S = _setup(rb, torch)
    plan = rb.Multi([s["batch"] for s in S])
    choice, timings = autotune.tune(plan, [(s["u"], s["q"], s["v"]) for s in S], reps=1, resident=64, advance=3)
    assert choice[0] in ("separate", "fused") and len(timings) >= 4
    # dimensions: dispatch order, grid, occupancy cap and worlds per workgroup
    assert all(len(k.split("/")) == 5 for k in timings)
    assert {k.split("/")[4] for k in timings if k.startswith("fused")} == {"1", "2", "4"}
    for _ in range(2):
        if choice[0] == "fused":
            plan.step()
        else:
            for s in S:
                s["batch"].step(s["u"], s["q"], s["v"])
    torch.cuda.synchronize()
    for (q, v), s in zip(ref, S):
        np.testing.assert_array_equal(s["q"].cpu().numpy(), q)
        np.testing.assert_array_equal(s["v"].cpu().numpy(), v)
    # a second tuning of the same configuration comes from the cache
    choice2, timings2 = autotune.tune(plan, [(s["u"], s["q"], s["v"]) for s in S], reps=1, resident=64)
    assert choice2 == choice and timings2 == {}
