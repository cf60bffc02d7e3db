"""Torsional and rolling friction (condim 4 and 6) on the HIP path: a spinning ball's decay
against the oracle's from the same rest state, spin and roll kept or lost by condim, the normal
force summing every row, and the fused launch equal to the plain one.  Teacher-forced parity of
the quadruped_condim6 and humanoid_condim4 workloads runs with the other workloads in the parity
tests."""
import numpy as np
import pytest

from gpu_common import gpu_run, oracle_run
from workloads import inputs, robots

pytestmark = pytest.mark.gpu


def _ball(condim, spin=0.002, roll=0.0005, mass=1.0):
    m = robots.free_body("sphere", size=(0.1,), mass=mass, pos=(0, 0, 0.1), timestep=0.002)
    for g in m["geoms"]:
        g.update(condim=condim, friction_spin=spin, friction_roll=roll)
    return m


def _rest(oracle_mod, m, n):
    """n balls at the oracle's rest state (FP64 settled, rounded to FP32)."""
    r = oracle_run(oracle_mod.Oracle(m), np.tile([[0, 0, 0.1, 1, 0, 0, 0]], (1, 1)).astype(np.float32),
                   np.zeros((1, 6), np.float32), nsteps=1500)
    q = np.tile(r["qpos"].astype(np.float32), (n, 1))
    return q, r["qacc_ws"]


def test_spin_decay_against_oracle(oracle_mod):
    """Balls spinning at 0.25-1 rad/s on a plane with torsional friction: after 1, 10 and 100
    steps the spin equals the oracle's (both from the same FP32 states) to 1e-4 relative."""
    m = _ball(4)
    n = 16
    q, _ = _rest(oracle_mod, m, n)
    v = np.zeros((n, 6), np.float32)
    v[:, 5] = np.linspace(0.25, 1.0, n, dtype=np.float32)
    o = oracle_mod.Oracle(m)
    for steps in (1, 10, 100):
        g = gpu_run(m, q, v, nsteps=steps)
        r = oracle_run(o, q, v, nsteps=steps)
        err = np.abs(g["qvel"][:, 5] - r["qvel"][:, 5]) / np.abs(r["qvel"][:, 5])
        assert err.max() < 1e-4, (steps, err.max())
        assert np.all(g["qvel"][:, 5] < v[:, 5])


@pytest.mark.parametrize("condim,keeps_spin,keeps_roll", [(3, True, True), (4, False, True), (6, False, False)])
def test_spin_and_roll_losses_by_condim(oracle_mod, condim, keeps_spin, keeps_roll):
    """Over 4 s a spinning ball keeps its spin and a rolling ball its speed (to 0.1 %) unless the
    contact has torsional (condim 4, 6) or rolling (condim 6) friction, which take at least 10 %."""
    m = _ball(condim)
    q, _ = _rest(oracle_mod, m, 2)
    v = np.zeros((2, 6), np.float32)
    v[0, 5] = 1.0
    v[1, 0], v[1, 4] = 0.5, 5.0
    g = gpu_run(m, q, v, nsteps=2000)
    assert (abs(g["qvel"][0, 5] - 1.0) < 1e-3) == keeps_spin and (g["qvel"][0, 5] < 0.9) != keeps_spin
    assert (abs(g["qvel"][1, 0] - 0.5) < 5e-4) == keeps_roll and (g["qvel"][1, 0] < 0.45) != keeps_roll


def test_normal_force_sums_every_row(oracle_mod):
    """A ball at rest with condim 6: the returned normal force (all ten rows) carries its weight,
    as the oracle's does, to 1e-4 relative."""
    m = _ball(6, 0.003, 0.001, mass=1.7)
    q, _ = _rest(oracle_mod, m, 4)
    v = np.zeros((4, 6), np.float32)
    g = gpu_run(m, q, v, nsteps=200, contacts=True)
    c = g["contacts"]
    assert np.all(c["ncon"] == 1)
    np.testing.assert_allclose(c["force"][:, 0, 0], 1.7 * 9.81, rtol=1e-4)


@pytest.mark.parametrize("name", ["quadruped_condim6", "humanoid_condim4"])
def test_fused_equals_plain(name):
    """The fused launch of a condim-4/6 model beside a plain model computes the same bits as the
    model's own plain launch."""
    import torch
    import paper_2601_22074_amd as rb
    dev = torch.device("cuda:0")
    out = {}
    for fused in (False, True):
        Ms = [rb.Model(robots.by_name(name)), rb.Model(robots.by_name("quadruped"))]
        Bs, ins = [], []
        for M, nm, nw in zip(Ms, (name, "quadruped"), (96, 64)):
            W = inputs.workload(nm, nw, 20)
            B = rb.Batch(M, nw)
            if W["friction"] is not None:
                B.set_params(rb.PARAM_FRICTION, torch.tensor(W["friction"], device=dev))
            if W["mass_scale"] is not None:
                B.set_params(rb.PARAM_MASS_SCALE, torch.tensor(W["mass_scale"], device=dev))
            t = lambda a: torch.tensor(a, device=dev).contiguous()
            ins.append((t(W["ctrl"][0]), t(W["qpos"]), t(W["qvel"]), torch.zeros(nw, dtype=torch.int32, device=dev)))
            Bs.append(B)
        if fused:
            plan = rb.Multi(Bs)
            for i, (u, q, v, st) in enumerate(ins):
                plan.bind(i, u, q, v, None, st)
            plan.set_schedule(rb.ORDER_HEAVY_FIRST, 0)
            for _ in range(20):
                plan.step()
        else:
            u, q, v, st = ins[0]
            for _ in range(20):
                Bs[0].step(u, q, v, None, st)
        torch.cuda.synchronize()
        out[fused] = (ins[0][1].cpu().numpy(), ins[0][2].cpu().numpy())
        if fused:
            plan.close()
        for B in Bs:
            B.close()
        for M in Ms:
            M.close()
    assert np.array_equal(out[False][0], out[True][0]) and np.array_equal(out[False][1], out[True][1])
