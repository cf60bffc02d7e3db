"""Elliptic cones with torsional and rolling friction (condim 4 and 6) on the HIP path: a
spinning ball's step against the oracle's from the same settled states (spins from well inside
the cone to far on its surface), a spinning and rolling ball's step under condim 6, a slow
spin's decay over 50 steps against the oracle and the closed form, rolling kept by condim 4 and
lost by condim 6, the workloads' returned contact forces inside the cone, and the fused launch
equal to the plain one.  Teacher-forced parity of quadruped_elliptic4, humanoid_elliptic4 and
quadruped_elliptic6 runs with the other workloads in the parity tests."""
import math

import numpy as np
import pytest

from gpu_common import RTOL_STEP, gpu_run, oracle_run, rel_err
from helpers import impedance
from workloads import inputs, robots

pytestmark = pytest.mark.gpu


def _ball(mus=0.02, impratio=1.0, condim=4, mur=0.002):
    m = robots.free_body("sphere", size=(0.1,), mass=1.0, pos=(0, 0, 0.1), friction=0.8, timestep=0.002)
    m["opt"]["cone"] = "elliptic"
    m["opt"]["impratio"] = impratio
    for g in m["geoms"]:
        g.update(condim=condim, friction_spin=mus, friction_roll=mur)
    return m


def _settled(oracle_mod, m, spins):
    """The ball settled on the plane by the oracle (500 steps), then given each spin: FP32
    states and warm starts, and the FP64 ones."""
    o = oracle_mod.Oracle(m)
    n = len(spins)
    q = np.tile([0, 0, 0.1, 1, 0, 0, 0.0], (n, 1))
    v = np.zeros((n, 6))
    ws = np.zeros((n, 6))
    for _ in range(500):
        o.step(np.zeros((n, 0)), q, v, ws)
    v[:, 5] = spins
    return o, q.astype(np.float32), v.astype(np.float32), ws.astype(np.float32)


@pytest.mark.parametrize("impratio", [1.0, 4.0])
def test_spinning_ball_step_against_oracle(oracle_mod, impratio):
    """32 spins from 0.01 to 20 rad/s (inside the cone, then on its surface): one env step of the
    HIP path equals the oracle's from the same FP32 state at the step tolerance, and both move
    the spin the same way."""
    m = _ball(impratio=impratio)
    spins = np.geomspace(0.01, 20.0, 32)
    o, q, v, ws = _settled(oracle_mod, m, spins)
    g = gpu_run(m, q, v, None, ws)
    r = oracle_run(o, q, v, None, ws)
    for w in range(len(spins)):
        assert rel_err(g["qpos"][w], r["qpos"][w]) <= RTOL_STEP, (w, spins[w])
        assert rel_err(g["qvel"][w], r["qvel"][w]) <= RTOL_STEP, (w, spins[w])
        assert g["qvel"][w, 5] < spins[w]


@pytest.mark.parametrize("impratio", [1.0, 4.0])
def test_spinning_rolling_ball_step_against_oracle(oracle_mod, impratio):
    """condim 6: 32 balls spinning (0.01 to 20 rad/s about the vertical) and rolling (0.02 to 2 m/s
    along x, with the matching spin about y): one env step of the HIP path equals the oracle's
    from the same FP32 state at the step tolerance."""
    m = _ball(impratio=impratio, condim=6)
    spins = np.geomspace(0.01, 20.0, 32)
    o, q, v, ws = _settled(oracle_mod, m, spins)
    roll = np.geomspace(0.02, 2.0, 32)[::-1]
    v[:, 0] = roll
    v[:, 4] = roll / 0.1
    g = gpu_run(m, q, v, None, ws)
    r = oracle_run(o, q, v, None, ws)
    for w in range(len(spins)):
        assert rel_err(g["qpos"][w], r["qpos"][w]) <= RTOL_STEP, (w, spins[w], roll[w])
        assert rel_err(g["qvel"][w], r["qvel"][w]) <= RTOL_STEP, (w, spins[w], roll[w])


@pytest.mark.parametrize("condim,keeps_roll", [(4, True), (6, False)])
def test_rolling_kept_or_lost_by_condim(oracle_mod, condim, keeps_roll):
    """A ball rolling at 0.5 m/s for 4 s on the HIP path keeps its speed to 0.1 % with condim 4 and
    loses at least 10 % of it with condim 6 (mu_roll 0.002), as the oracle's does."""
    m = _ball(mus=0.002, condim=condim)
    o, q, v, ws = _settled(oracle_mod, m, [0.0])
    v[0, 0], v[0, 4] = 0.5, 5.0
    g = gpu_run(m, q, v, None, ws, nsteps=2000)
    vx = float(g["qvel"][0, 0])
    assert (abs(vx - 0.5) < 5e-4) == keeps_roll and (vx < 0.45) != keeps_roll, vx


def test_slow_spin_decay_against_oracle(oracle_mod):
    """A slow spin (0.05 rad/s, inside the cone) over 50 steps: the HIP path's spin follows the
    oracle's to 1e-4 of the initial spin and both follow the closed-form geometric decay of the
    cone's quadratic zone, 1 - dt D_s b / (I + D_s) per step (within 1 % of the spin lost)."""
    m = _ball()
    o, q, v, ws = _settled(oracle_mod, m, [0.05] * 4)
    g = gpu_run(m, q, v, None, ws, nsteps=50)
    r = oracle_run(o, q, v, None, ws, nsteps=50)
    w0 = 0.05
    np.testing.assert_allclose(g["qvel"][:, 5], r["qvel"][:, 5], rtol=0, atol=1e-4 * w0)
    imp = impedance(0.1 - float(q[0, 2]))
    Ds = imp / (1 - imp) * (0.02 / 0.8) ** 2
    ratio = 1 - 0.002 * Ds * (2.0 / (0.95 * 0.02)) / (0.004 + Ds)
    lost = w0 - w0 * ratio ** 50
    assert abs((w0 - g["qvel"][0, 5]) / lost - 1) < 1e-2


@pytest.mark.parametrize("name", ["quadruped_elliptic4", "humanoid_elliptic4", "quadruped_elliptic6"])
def test_forces_inside_the_cone(name):
    """After 40 steps every returned contact force lies in its cone (the spin force takes its
    share, so |f_t| <= mu f_n a fortiori), to FP32 rounding, and some lie on the cone's surface
    or carry a spin force (|f_t| < mu f_n strictly while loaded)."""
    W = inputs.workload(name, 256, 40)
    m = W["model"]
    g = gpu_run(m, W["qpos"], W["qvel"], W["ctrl"][0], None, W["friction"], W["mass_scale"], nsteps=40,
                contacts=True)
    c = g["contacts"]
    mu = W["friction"] if W["friction"] is not None else np.ones(256, np.float32)
    loaded = 0
    for w in range(256):
        for k in range(c["ncon"][w]):
            fn, f1, f2 = c["force"][w, k].astype(np.float64)
            ft = math.hypot(f1, f2)
            assert fn >= 0 and ft <= mu[w] * fn * (1 + 1e-5) + 1e-6, (name, w, k, fn, ft)
            loaded += fn > 1e-3
    assert loaded > 0


@pytest.mark.parametrize("name", ["quadruped_elliptic4", "humanoid_elliptic4", "quadruped_elliptic6"])
def test_fused_equals_plain(name):
    """The fused launch of a condim-4 elliptic model beside a pyramidal one computes the same bits
    as the model's own plain launch."""
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
