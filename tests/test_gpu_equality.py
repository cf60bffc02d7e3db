"""Equality constraints (connect, weld with the world) on the HIP path: rest states against the
closed-form soft sag and the oracle's, a closed-loop chain's full-size rollout against the oracle's,
and the fused launch equal to the plain one.  Teacher-forced parity of the chain3_loop and
humanoid_weld workloads runs with the other workloads in the parity tests."""
import math

import numpy as np
import pytest

from gpu_common import gpu_run, oracle_run
from helpers import rot, soft_sag
from workloads import inputs, robots

pytestmark = pytest.mark.gpu

DT = 0.002


def _hanging(kind, anchor=(0.0, 0.0, 0.0), mass=2.0, r=0.05, target=(0.0, 0.0, 1.0), quat=(1.0, 0, 0, 0)):
    mb = robots.ModelBuilder("hang", timestep=DT, nsubsteps=1)
    b = mb.body("ball", 0, (0, 0, 1), mass, robots.sphere_inertia(mass, r))
    mb.joint(b, "free")
    mb.equality(kind, b, anchor, target, quat)
    return mb.build()


def _ball_states(n, rng, spread=0.01):
    """Balls near the held pose: small offsets, tilts and speeds."""
    q = np.zeros((n, 7)); v = rng.normal(0.0, 0.05, (n, 6))
    for i in range(n):
        ax = rng.normal(size=3); ax /= np.linalg.norm(ax)
        th = rng.uniform(0, 0.05)
        q[i, :3] = [0.0, 0.0, 1.0] + rng.uniform(-spread, spread, 3)
        q[i, 3:] = [math.cos(th / 2), *(math.sin(th / 2) * ax)]
    return q.astype(np.float32), v.astype(np.float32)


def test_connect_settles_at_the_closed_form_sag():
    """Balls connected at their centres, released near the point, come to rest below it by the
    closed-form soft sag (0.37 mm; 1e-4 of it plus a few FP32 ulps of the height)."""
    m = _hanging("connect")
    q, v = _ball_states(64, np.random.default_rng(4))
    g = gpu_run(m, q, v, nsteps=3000)
    assert np.all(g["status"] & 1 == 0)
    sag = soft_sag(2.0)
    err = np.abs(g["qpos"][:, 2].astype(np.float64) - (1.0 + sag))
    assert err.max() <= 1e-4 * abs(sag) + 4 * 2.0 ** -23, err.max()
    assert np.abs(g["qpos"][:, :2]).max() < 1e-6
    # the connect holds the centre only: the balls keep spinning at their initial rates.  Their
    # centres rest to within the speed at which an FP32 height near 1 stops moving in one step,
    # ulp(1) / (2 dt) = 3e-5 m/s, below which the position update rounds to nothing
    assert np.abs(g["qvel"][:, :3]).max() < 2.0 ** -24 / DT


def test_weld_rest_pose_equals_oracle(oracle_mod):
    """A ball welded at a point 10 cm beside its centre: the rest pose (soft sag and tilt under the
    weight's moment) equals the oracle's, both reached from the same releases."""
    m = _hanging("weld", (0.1, 0.0, 0.0), target=(0.1, 0.0, 1.0))
    q, v = _ball_states(32, np.random.default_rng(5))
    g = gpu_run(m, q, v, nsteps=3000)
    r = oracle_run(oracle_mod.Oracle(m), q, v, nsteps=3000)
    assert np.all(g["status"] & 1 == 0)
    # the rest pose is an attractor: both paths land on it to FP32 resolution
    np.testing.assert_allclose(g["qpos"], r["qpos"], atol=2e-6)
    tilt = 2 * np.arccos(np.minimum(1.0, np.abs(g["qpos"][:, 3])))
    assert np.all((tilt > 0.005) & (tilt < 0.05))


def _tip(q):
    a = np.cumsum(q, axis=1)
    return 0.5 * np.stack([-np.sin(a).sum(1), -np.cos(a).sum(1)], 1)


def test_loop_rollout_full_size(oracle_mod):
    """chain3_loop at 8192 worlds, 400 env steps in the launch bench.py times, against the
    oracle's rollout of every world: the closed loop is a one-degree-of-freedom mechanism, whose
    final state moves by under 1e-4 rad for a 1e-6 rad change of the initial angles, so the
    FP32 rounding of 400 steps stays well inside 2e-3 rad per angle; the tips' largest distance
    from the held point (the soft rows' stretch under the swing, 16 mm) agrees to 1e-4 m."""
    n, steps = 8192, 400
    W = inputs.workload("chain3_loop", n, steps)
    g = gpu_run(W["model"], W["qpos"], W["qvel"], nsteps=steps)
    assert np.all(g["status"] & 1 == 0)
    r = oracle_run(oracle_mod.Oracle(W["model"]), W["qpos"], W["qvel"], nsteps=steps)
    err = np.abs(g["qpos"].astype(np.float64) - r["qpos"]).max(1)
    assert err.max() < 2e-3, (err.max(), int(err.argmax()))
    P = np.array([robots.LOOP_POINT[0], robots.LOOP_POINT[2]])
    dg = np.abs(_tip(g["qpos"].astype(np.float64)) - P).max()
    dr = np.abs(_tip(r["qpos"]) - P).max()
    assert abs(dg - dr) < 1e-4, (dg, dr)


@pytest.mark.parametrize("name", ["chain3_loop", "humanoid_weld"])
def test_fused_equals_plain(name):
    """The fused launch of an equality model beside a model without equality rows computes the
    same bits as the model's own plain launch."""
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
