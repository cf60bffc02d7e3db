"""Pins of the oracle's per-world model fields (geom size, body position, actuator gains):
each world steps exactly as a model whose description carries its values, and a PD-actuated
hinge oscillates at the closed-form frequency of its own gain."""
import copy
import math

import numpy as np

from workloads import inputs, robots


def _per_world_models(m, n, edit):
    """n copies of model m with edit(copy, w) applied, and the per-world field arrays."""
    out = []
    for w in range(n):
        mw = copy.deepcopy(m)
        edit(mw, w)
        out.append(mw)
    f = dict(geom_size=np.array([[g["size"] for g in mw["geoms"]] for mw in out]),
             body_pos=np.array([[b["pos"] for b in mw["bodies"]] for mw in out]),
             act_kp=np.array([[a["kp"] for a in mw["actuators"]] for mw in out]).reshape(n, -1),
             act_kd=np.array([[a["kd"] for a in mw["actuators"]] for mw in out]).reshape(n, -1))
    return out, f


def _check_equivalent(oracle_mod, name, edit, fields, nsteps=8, n=6):
    m = robots.by_name(name)
    models, f = _per_world_models(m, n, edit)
    q, v = inputs.initial_state(m, name, range(n))
    fr, ms = inputs.world_params(m, name, range(n))
    u = inputs.ctrl_table(m, name, range(n), 1)[0].astype(np.float64)
    o = oracle_mod.Oracle(m)
    qq, vv, ws = q.astype(np.float64), v.astype(np.float64), np.zeros((n, o.nv))
    f64 = lambda a: None if a is None else a.astype(np.float64)
    for _ in range(nsteps):
        _, c = o.step(u, qq, vv, ws, f64(fr), f64(ms), contacts=True, fields={k: f[k] for k in fields})
    for w in range(n):
        ow = oracle_mod.Oracle(models[w])
        sl = slice(w, w + 1)
        q1, v1, w1 = q[sl].astype(np.float64), v[sl].astype(np.float64), np.zeros((1, o.nv))
        for _ in range(nsteps):
            _, c1 = ow.step(u[sl], q1, v1, w1, None if fr is None else f64(fr)[sl], None if ms is None else f64(ms)[sl],
                            contacts=True)
        np.testing.assert_array_equal(qq[w], q1[0])
        np.testing.assert_array_equal(vv[w], v1[0])
        np.testing.assert_array_equal(c["force"][w], c1["force"][0])
    return c


def test_geom_size_per_world_equals_description(oracle_mod):
    """Humanoid feet and shins sized per world (boxes and capsules up to +-20 %)."""
    rng = np.random.default_rng(4)
    scale = rng.uniform(0.8, 1.2, (6, 3))

    def edit(mw, w):
        for g in mw["geoms"]:
            if g["type"] == "box":
                g["size"] = [s * scale[w, 0] for s in g["size"]]
            elif g["type"] == "capsule":
                g["size"] = [g["size"][0] * scale[w, 1], g["size"][1] * scale[w, 2], 0.0]
    c = _check_equivalent(oracle_mod, "humanoid", edit, ["geom_size"], nsteps=30)
    assert c["ncon"].sum() > 0


def test_body_pos_per_world_equals_description(oracle_mod):
    """Chain links of per-world length (the joint positions of links 2 and 3) and quadruped hips
    moved per world."""
    rng = np.random.default_rng(5)

    def edit_chain(mw, w):
        for b in mw["bodies"][2:]:
            b["pos"] = [b["pos"][0], b["pos"][1], b["pos"][2] * rng.uniform(0.7, 1.3)]
    _check_equivalent(oracle_mod, "chain3", edit_chain, ["body_pos"], nsteps=50)

    def edit_quad(mw, w):
        for b in mw["bodies"][2:]:
            b["pos"] = [x + rng.uniform(-0.01, 0.01) for x in b["pos"]]
    _check_equivalent(oracle_mod, "quadruped", edit_quad, ["body_pos"], nsteps=30)


def test_actuator_gains_per_world_equal_description(oracle_mod):
    rng = np.random.default_rng(6)

    def edit(mw, w):
        for a in mw["actuators"]:
            a["kp"] = a["kp"] * rng.uniform(0.5, 2.0)
            a["kd"] = a["kd"] * rng.uniform(0.5, 2.0)
    _check_equivalent(oracle_mod, "quadruped", edit, ["act_kp", "act_kd"], nsteps=30)


def test_pd_gain_per_world_sets_the_oscillation_frequency(oracle_mod):
    """A hinge at zero gravity driven by a position actuator with gain kp (kd = 0) towards 0
    oscillates at omega = sqrt(kp / I) about its axis (I: the rotor's inertia plus armature);
    each world has its own kp."""
    dt = 5e-4
    mb = robots.ModelBuilder("rotor", timestep=dt, nsubsteps=1, gravity=[0, 0, 0])
    I = 0.02
    b = mb.body("rotor", 0, (0, 0, 0), 1.0, [I, I, I])
    j = mb.joint(b, "hinge", axis=(0, 0, 1), armature=0.01)
    mb.actuator(j, "position", kp=1.0, kd=0.0)
    m = mb.build()
    kps = np.array([0.5, 2.0, 8.0, 30.0])
    n = len(kps)
    o = oracle_mod.Oracle(m)
    q = np.full((n, 1), 0.01)
    v = np.zeros((n, 1))
    ws = np.zeros((n, 1))
    u = np.zeros((n, 1))
    f = dict(act_kp=kps[:, None], act_kd=np.zeros((n, 1)))
    prev = q[:, 0].copy()
    crossings = [[] for _ in range(n)]
    T = int(4 * 2 * math.pi * math.sqrt((I + 0.01) / kps.min()) / dt) + 10
    for s in range(1, T):
        o.step(u, q, v, ws, fields=f)
        for w in range(n):
            if prev[w] > 0 >= q[w, 0]:
                # linear interpolation of the downward zero crossing
                crossings[w].append((s - 1 + prev[w] / (prev[w] - q[w, 0])) * dt)
        prev = q[:, 0].copy()
    for w in range(n):
        period = np.diff(crossings[w]).mean()
        ref = 2 * math.pi * math.sqrt((I + 0.01) / kps[w])
        assert abs(period / ref - 1) < 2e-3, (kps[w], period, ref)
