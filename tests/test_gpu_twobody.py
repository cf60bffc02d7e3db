"""Contacts between two moving bodies on the HIP path (level-3 code: rows of the relative
motion, A-hat over both chains, a dense Newton Hessian): linear momentum conserved through a
collision of two free boxes in zero gravity, single steps of colliding boxes against the oracle,
a resting stack's floor and box-box forces carrying the weights, and the fused launch equal to
the plain one.  Teacher-forced parity of the cube_stack workload runs with the other workloads
in the parity tests."""
import numpy as np
import pytest

from gpu_common import RTOL_STEP, gpu_run, oracle_run, rel_err
from workloads import inputs, robots

pytestmark = pytest.mark.gpu


def _two_boxes(gravity=(0, 0, 0), floor=False, h=0.05, mass=(1.0, 2.0), dt=0.002):
    mb = robots.ModelBuilder("two_boxes", timestep=dt, nsubsteps=1, gravity=list(gravity))
    if floor:
        mb.geom(0, "plane", [0, 0, 0], contype=0, conaffinity=1)
    for i, (z, m) in enumerate(zip((h, 3 * h + 0.001), mass)):
        b = mb.body(f"box{i}", 0, (0, 0, z), m, robots.box_inertia(m, 0.1, 0.1, h))
        mb.joint(b, "free")
        mb.geom(b, "box", [0.1, 0.1, h], contype=1, conaffinity=1)
    return mb.build()


def _throws(n, seed):
    """Two boxes thrown at each other off-centre with random spins."""
    rng = np.random.default_rng(seed)
    q = np.zeros((n, 14), np.float32); v = np.zeros((n, 12), np.float32)
    for w in range(n):
        a = rng.normal(size=4); a /= np.linalg.norm(a)
        q[w] = [-0.25, rng.uniform(-0.05, 0.05), rng.uniform(-0.03, 0.03), 1, 0, 0, 0,
                0.25, rng.uniform(-0.05, 0.05), rng.uniform(-0.03, 0.03), *a]
        v[w, :3] = [1.0, 0, 0]
        v[w, 6:9] = [-0.8, 0, 0]
        v[w, 3:6] = rng.normal(0, 1.0, 3)
        v[w, 9:12] = rng.normal(0, 1.0, 3)
    return q, v


def test_collision_conserves_linear_momentum():
    """64 pairs of boxes colliding in zero gravity over 300 steps: the total linear momentum
    stays at its initial value to FP32 resolution (1e-5 of its size)."""
    m = _two_boxes()
    q, v = _throws(64, 3)
    P0 = 1.0 * v[:, :3].astype(np.float64) + 2.0 * v[:, 6:9].astype(np.float64)
    g = gpu_run(m, q, v, nsteps=300, contacts=True)
    assert np.all(g["status"] & 1 == 0)
    P = 1.0 * g["qvel"][:, :3].astype(np.float64) + 2.0 * g["qvel"][:, 6:9].astype(np.float64)
    assert np.abs(P - P0).max() <= 1e-5 * np.abs(P0).max()
    # they did collide: the lighter box bounced
    assert np.all(g["qvel"][:, 0] < 0.5)


def test_colliding_steps_against_oracle(oracle_mod):
    """Single steps of the colliding boxes from the oracle's own states in contact (after 100
    steps): qpos and qvel at the step tolerance, contact keys exact."""
    m = _two_boxes()
    q, v = _throws(32, 4)
    o = oracle_mod.Oracle(m)
    r0 = oracle_run(o, q, v, nsteps=120)
    q1, v1, w1 = (r0[k].astype(np.float32) for k in ("qpos", "qvel", "qacc_ws"))
    g = gpu_run(m, q1, v1, None, w1, contacts=True)
    r = oracle_run(o, q1, v1, None, w1, contacts=True)
    touching = 0
    for w in range(32):
        nc = int(r["contacts"]["ncon"][w])
        touching += nc > 0
        assert int(g["contacts"]["ncon"][w]) == nc
        err = max(rel_err(g["qpos"][w], r["qpos"][w]), rel_err(g["qvel"][w], r["qvel"][w]))
        assert err <= RTOL_STEP, (w, err)
    assert touching >= 8


def test_stack_forces_carry_the_weights(oracle_mod):
    """cube_stack settled (the oracle's state after 1500 steps): per world, the returned floor
    contacts' resultant and that of the contacts between cubes 0 and 1 equal the oracle's on the
    same state to 1e-4 of the weight, and where the oracle's stack is at rest (its floor resultant
    equals the three cubes' weight to 1e-4) they carry 0.6 g and 0.3 g."""
    m = robots.cube_stack()
    W = inputs.workload("cube_stack", 8, 1)
    o = oracle_mod.Oracle(m)
    r0 = oracle_run(o, W["qpos"], W["qvel"], nsteps=1500)
    q1, v1, w1 = (r0[k].astype(np.float32) for k in ("qpos", "qvel", "qacc_ws"))
    g = gpu_run(m, q1, v1, None, w1, nsteps=1, contacts=True)
    r = oracle_run(o, q1, v1, None, w1, nsteps=1, contacts=True)

    def sums(c, w, cast):
        floor = np.zeros(3); mid = np.zeros(3)
        for k in range(c["ncon"][w]):
            f = cast(c["force"][w, k]) @ cast(c["frame"][w, k]).reshape(3, 3)
            g1, g2 = c["geom"][w, k]
            if g1 == 0:
                floor += f
            elif {int(g1), int(g2)} == {1, 2}:
                mid += f    # on g2's body (cube 1)
        return floor, mid

    rest = 0
    for w in range(8):
        gf, gm = sums(g["contacts"], w, lambda a: np.asarray(a, np.float64))
        of, om = sums(r["contacts"], w, lambda a: np.asarray(a, np.float64))
        np.testing.assert_allclose(gf, of, atol=1e-4 * 0.6 * 9.81)
        np.testing.assert_allclose(gm, om, atol=1e-4 * 0.6 * 9.81)
        if np.abs(of - [0, 0, 0.6 * 9.81]).max() < 1e-4 * 0.6 * 9.81:
            rest += 1
            np.testing.assert_allclose(gf, [0, 0, 0.6 * 9.81], atol=1e-4 * 0.6 * 9.81)
            np.testing.assert_allclose(gm, [0, 0, 0.3 * 9.81], atol=1e-4 * 0.6 * 9.81)
    assert rest >= 6


def test_pincer_holds_the_cube():
    """pincer_cube with the palm held still (targets 0) for 2 s: the fingers' friction carries the
    cube, which stays between the fingertips (above 0.2 m), on both paths."""
    import copy
    m = robots.pincer_cube()
    W = inputs.workload("pincer_cube", 16, 1)
    u = np.tile(np.array([[0.0, -0.2, 0.2]], np.float32), (16, 1))
    g = gpu_run(m, W["qpos"], W["qvel"], u, nsteps=250)
    assert np.all(g["status"] & 1 == 0)
    assert g["qpos"][:, 5].min() > 0.2, g["qpos"][:, 5]


def test_fused_equals_plain():
    """cube_stack in a fused launch beside the quadruped computes the same bits as its own plain
    launch."""
    import torch
    import paper_2601_22074_amd as rb
    dev = torch.device("cuda:0")
    out = {}
    for fused in (False, True):
        Ms = [rb.Model(robots.by_name("cube_stack")), rb.Model(robots.by_name("quadruped"))]
        Bs, ins = [], []
        for M, nm, nw in zip(Ms, ("cube_stack", "quadruped"), (96, 64)):
            W = inputs.workload(nm, nw, 20)
            B = rb.Batch(M, nw)
            t = lambda a: torch.tensor(a, device=dev).contiguous()
            ins.append((t(W["ctrl"][0]) if M.nu else None, t(W["qpos"]), t(W["qvel"]),
                        torch.zeros(nw, dtype=torch.int32, device=dev)))
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
