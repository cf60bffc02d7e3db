"""Elliptic friction cones on the HIP path: contact forces inside the friction cone, a plate
sliding down an incline at the oracle's rate, a sliding ball's friction antiparallel to its
velocity, and the fused launch equal to the plain one.  Teacher-forced parity of the
quadruped_elliptic and humanoid_elliptic workloads runs with the other workloads in the parity
tests."""
import math

import numpy as np
import pytest

from gpu_common import gpu_run, oracle_run
from helpers import rot
from workloads import inputs, robots

pytestmark = pytest.mark.gpu


def _elliptic(m, impratio=1.0):
    m["opt"]["cone"] = "elliptic"
    m["opt"]["impratio"] = impratio
    return m


def test_forces_inside_the_cone():
    """quadruped_elliptic and humanoid_elliptic after 40 steps: every returned contact force
    lies in its cone, |f_t| <= mu f_n (to FP32 rounding), and some lie on its surface."""
    for name in ("quadruped_elliptic", "humanoid_elliptic"):
        W = inputs.workload(name, 256, 40)
        m = W["model"]
        g = gpu_run(m, W["qpos"], W["qvel"], W["ctrl"][0], None, W["friction"], W["mass_scale"], nsteps=40,
                    contacts=True)
        c = g["contacts"]
        mu = W["friction"] if W["friction"] is not None else np.ones(256, np.float32)
        surface = 0
        for w in range(256):
            for k in range(c["ncon"][w]):
                fn, f1, f2 = c["force"][w, k].astype(np.float64)
                ft = math.hypot(f1, f2)
                assert fn >= 0 and ft <= mu[w] * fn * (1 + 1e-5) + 1e-6, (name, w, k, fn, ft)
                surface += fn > 1e-3 and ft > mu[w] * fn * (1 - 1e-4)
        assert surface > 0


def test_incline_slide_against_oracle(oracle_mod):
    """Plates sliding down a 30 degree incline (mu 0.3): after 400 steps their speed equals the
    oracle's from the same settled states to 1e-3 relative; both average the Coulomb rate."""
    theta, mu, h = math.radians(30), 0.3, 0.005
    qg = robots.quat_axis_angle((1, 0, 0), theta)
    n = rot(qg)[:, 2]
    m = _elliptic(robots.free_body("box", size=(0.1, 0.1, h), mass=1.0, ground_quat=qg, friction=mu,
                                   timestep=0.002))
    o = oracle_mod.Oracle(m)
    r0 = oracle_run(o, np.concatenate([n * (h - 2e-4), qg])[None].astype(np.float32),
                    np.zeros((1, 6), np.float32), nsteps=100)
    q = np.tile(r0["qpos"].astype(np.float32), (4, 1))
    v = np.tile(r0["qvel"].astype(np.float32), (4, 1))
    g = gpu_run(m, q, v, nsteps=400)
    r = oracle_run(o, q, v, nsteps=400)
    down = np.cross(n, np.cross([0, 0, -1.0], n))
    down /= np.linalg.norm(down)
    vg, vr, v0 = g["qvel"][:, :3] @ down, r["qvel"][:, :3] @ down, v[0, :3] @ down
    assert np.abs(vg - vr).max() < 1e-3 * np.abs(vr).max()
    acc = (vg.mean() - v0) / 0.8
    assert abs(acc / (9.81 * (math.sin(theta) - mu * math.cos(theta))) - 1) < 5e-3


def test_sliding_ball_friction_opposes_velocity(oracle_mod):
    """Balls sliding without spin in 8 directions: each loaded contact's friction is antiparallel
    to the ball's horizontal velocity within 1e-4 rad (FP32)."""
    m = _elliptic(robots.free_body("sphere", size=(0.05,), mass=0.5, friction=0.4, timestep=0.002))
    r0 = oracle_run(oracle_mod.Oracle(m), np.array([[0, 0, 0.05, 1, 0, 0, 0]], np.float32),
                    np.zeros((1, 6), np.float32), nsteps=300)
    q = np.tile(r0["qpos"].astype(np.float32), (8, 1))
    v = np.tile(r0["qvel"].astype(np.float32), (8, 1))
    ang = np.arange(8) * (2 * math.pi / 8) + 0.3
    v[:, 0], v[:, 1] = 2.0 * np.cos(ang), 2.0 * np.sin(ang)
    loaded = 0
    for steps in (1, 2, 3, 5, 8):
        g = gpu_run(m, q, v, nsteps=steps, contacts=True)
        c = g["contacts"]
        for w in range(8):
            if c["ncon"][w] and c["force"][w, 0, 0] > 1e-3:
                loaded += 1
                F = c["force"][w, 0].astype(np.float64) @ c["frame"][w, 0].reshape(3, 3).astype(np.float64)
                vt = g["qvel"][w, :2].astype(np.float64)
                vt /= np.linalg.norm(vt)
                a = math.atan2(F[0] * vt[1] - F[1] * vt[0], -(F[0] * vt[0] + F[1] * vt[1]))
                assert abs(a) < 1e-4, (steps, w, a)
    assert loaded >= 8


@pytest.mark.parametrize("name", ["quadruped_elliptic", "humanoid_elliptic"])
def test_fused_equals_plain(name):
    """The fused launch of an elliptic-cone model beside a pyramidal one computes the same bits as
    the model's own plain launch."""
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


@pytest.mark.parametrize("iters", [1, 2, 4])
def test_stiff_tangential_solve_against_oracle(oracle_mod, iters):
    """The humanoid with elliptic cones and impratio 10 (tangential rows ten times stiffer), on
    the oracle's own states after 124 env steps: one substep's solved acceleration (stage tap)
    with a budget of 1, 2 and 4 Newton updates equals the oracle's at the step tolerance."""
    import copy
    from gpu_common import RTOL_STEP, substeps1
    m = robots.with_elliptic(robots.humanoid(), 10.0, "humanoid_impratio10")
    n, step = 32, 124
    q, v = inputs.initial_state(m, "humanoid_elliptic", range(n))
    fr, ms = inputs.world_params(m, "humanoid_elliptic", range(n))
    ctab = inputs.ctrl_table(m, "humanoid_elliptic", range(n), step // 20 + 2)
    o = oracle_mod.Oracle(m)
    qq, vv = q.astype(np.float64), v.astype(np.float64)
    ws, st = np.zeros((n, o.nv)), np.zeros(n, np.uint32)
    for s in range(step):
        o.step(ctab[s // 20].astype(np.float64), qq, vv, ws, fr.astype(np.float64), ms.astype(np.float64), st)
    q32, v32, w32 = (x.astype(np.float32) for x in (qq, vv, ws))
    u32 = ctab[step // 20]
    mi = substeps1(copy.deepcopy(m))
    mi["opt"]["iterations"] = iters
    g = gpu_run(mi, q32, v32, u32, w32, fr, ms, taps=True)
    oi = oracle_mod.Oracle(mi)
    for w in range(n):
        t = oi.forward(q32[w], v32[w], u32[w], w32[w], fr[w], ms[w])
        assert int(g["stats"][w, 2]) == t["niter"]
        err = np.abs(g["qacc"][w] - t["qacc"]).max() / max(np.abs(t["qacc"]).max(), 1.0)
        assert err <= RTOL_STEP, (w, err)
