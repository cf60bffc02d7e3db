"""Pins of the FP64 oracle's kinematics and smooth dynamics against closed forms and
definitions that share nothing with the oracle's code (runs on the CPU)."""
import math

import numpy as np
import pytest

from helpers import joint_layout, q_plus, rot, vee
from workloads import robots


def fixed_humanoid():
    """The humanoid with its pelvis welded to the world: a 29-hinge branched tree."""
    m = robots.humanoid()
    m["joints"] = [j for j in m["joints"] if j["type"] != "free"]
    m["actuators"] = []
    m["per_world"] = {"friction": False, "mass_scale": False}
    return m


# ---------------------------------------------------------------- kinematics
def test_chain_fk_closed_form(oracle_mod):
    m = robots.chain3()
    o = oracle_mod.Oracle(m)
    rng = np.random.default_rng(0)
    for _ in range(20):
        th = rng.uniform(-math.pi, math.pi, 3)
        t = o.forward(th, np.zeros(3))
        phi = np.cumsum(th)
        # body origins: link1 at the base, link i+1 at the tip of link i
        exp = [np.zeros(3)]
        for i in range(2):
            exp.append(exp[-1] + 0.5 * np.array([-math.sin(phi[i]), 0, -math.cos(phi[i])]))
        for i in range(3):
            np.testing.assert_allclose(t["xpos"][i + 1], exp[i], atol=1e-14)
            Ry = np.array([[math.cos(phi[i]), 0, math.sin(phi[i])], [0, 1, 0], [-math.sin(phi[i]), 0, math.cos(phi[i])]])
            np.testing.assert_allclose(t["xmat"][i + 1], Ry, atol=1e-14)
        tip = t["xpos"][3] + t["xmat"][3] @ np.array([0, 0, -0.5])
        exp_tip = sum(0.5 * np.array([-math.sin(p), 0, -math.cos(p)]) for p in phi)
        np.testing.assert_allclose(tip, exp_tip, atol=1e-14)
        # centre of mass at the middle of each link
        np.testing.assert_allclose(t["com"][1], 0.25 * np.array([-math.sin(phi[0]), 0, -math.cos(phi[0])]), atol=1e-14)


def test_free_body_fk_is_qpos(oracle_mod):
    m = robots.free_body("box", size=(0.2, 0.1, 0.05), ground=False)
    o = oracle_mod.Oracle(m)
    rng = np.random.default_rng(1)
    for _ in range(10):
        q = np.concatenate([rng.normal(size=3), rng.normal(size=4) * 3.0])
        t = o.forward(q, np.zeros(6))
        np.testing.assert_allclose(t["xpos"][1], q[:3], atol=1e-15)
        qn = q[3:] / np.linalg.norm(q[3:])
        np.testing.assert_allclose(t["xquat"][1], qn, atol=1e-15)
        np.testing.assert_allclose(t["xmat"][1], rot(qn), atol=1e-14)
        np.testing.assert_allclose(t["gmat"][0], rot(qn), atol=1e-14)


@pytest.mark.parametrize("name", ["quadruped", "humanoid"])
def test_fk_rotations_orthonormal(oracle_mod, name):
    m = robots.by_name(name)
    o = oracle_mod.Oracle(m)
    rng = np.random.default_rng(2)
    q = robots.qpos0(m)
    q[7:] = rng.uniform(-1, 1, len(q) - 7)
    t = o.forward(q, np.zeros(o.nv))
    for R in t["xmat"]:
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14
    np.testing.assert_allclose(np.linalg.norm(t["xquat"], axis=1), 1.0, atol=1e-15)


# ---------------------------------------------------------------- inertia of solids
def test_capsule_inertia_monte_carlo():
    rng = np.random.default_rng(3)
    r, L, m = 0.05, 0.5, 1.0
    n = 2_000_000
    pts = rng.uniform([-r, -r, -L / 2 - r], [r, r, L / 2 + r], size=(n, 3))
    zc = np.clip(pts[:, 2], -L / 2, L / 2)
    inside = pts[:, 0] ** 2 + pts[:, 1] ** 2 + (pts[:, 2] - zc) ** 2 <= r * r
    p = pts[inside]
    ixx = m * np.mean(p[:, 1] ** 2 + p[:, 2] ** 2)
    izz = m * np.mean(p[:, 0] ** 2 + p[:, 1] ** 2)
    I = robots.capsule_inertia(m, r, L)
    assert abs(I[0] / ixx - 1) < 3e-3
    assert abs(I[2] / izz - 1) < 3e-3
    # published values for the 0.5 m, r = 0.05, 1 kg link
    assert abs(I[0] - 0.0275074) < 5e-8 and abs(I[2] - 0.00122059) < 5e-9


def test_box_and_sphere_inertia():
    np.testing.assert_allclose(robots.box_inertia(3.0, 0.1, 0.2, 0.3), [3 / 3 * (0.04 + 0.09), 3 / 3 * (0.01 + 0.09),
                                                                        3 / 3 * (0.01 + 0.04)], rtol=1e-15)
    np.testing.assert_allclose(robots.sphere_inertia(2.0, 0.1), [0.008] * 3, rtol=1e-15)


# ---------------------------------------------------------------- mass matrix
def kinetic_energy_fd(o, model, q, v, eps=1e-5):
    """0.5 * sum(m |com_dot|^2 + w' I w) with body velocities from central differences of FK."""
    tp = o.forward(q_plus(model, q, eps * v), np.zeros(o.nv))
    tm = o.forward(q_plus(model, q, -eps * v), np.zeros(o.nv))
    t0 = o.forward(q, np.zeros(o.nv))
    T = 0.0
    for b in range(1, len(model["bodies"])):
        body = model["bodies"][b]
        cd = (tp["com"][b] - tm["com"][b]) / (2 * eps)
        w = vee((tp["xmat"][b] - tm["xmat"][b]) / (2 * eps) @ t0["xmat"][b].T)
        Rl = t0["xmat"][b] @ rot(body["iquat"])
        I = Rl @ np.diag(body["inertia"]) @ Rl.T
        T += 0.5 * body["mass"] * cd @ cd + 0.5 * w @ I @ w
    for (jt, _, da), j in zip(joint_layout(model), model["joints"]):
        if jt == "hinge":
            T += 0.5 * j["armature"] * v[da] ** 2
    return T


@pytest.mark.parametrize("name", ["chain3", "quadruped", "humanoid", "free_offset"])
def test_mass_matrix_is_kinetic_energy_hessian(oracle_mod, name):
    m = robots.free_offset() if name == "free_offset" else robots.by_name(name)
    o = oracle_mod.Oracle(m)
    rng = np.random.default_rng(4)
    q = robots.qpos0(m)
    off = 7 if name != "chain3" else 0
    q[off:] = rng.uniform(-1.0, 1.0, len(q) - off)
    if off:
        q[3:7] = rng.normal(size=4)
        q[3:7] /= np.linalg.norm(q[3:7])
    M = o.forward(q, np.zeros(o.nv))["M"]
    np.testing.assert_allclose(M, M.T, atol=1e-14 * np.abs(M).max())
    assert np.linalg.eigvalsh(M).min() > 0
    nv = o.nv
    E = np.eye(nv)
    Ti = [kinetic_energy_fd(o, m, q, E[i]) for i in range(nv)]
    idx = list(range(nv)) if nv <= 18 else list(rng.choice(nv, 12, replace=False))
    for i in idx:
        assert abs(2 * Ti[i] - M[i, i]) <= 1e-6 * max(abs(M[i, i]), 1e-3)
        for j in idx:
            if j <= i:
                continue
            Tij = kinetic_energy_fd(o, m, q, E[i] + E[j])
            assert abs((Tij - Ti[i] - Ti[j]) - M[i, j]) <= 1e-6 * max(abs(M[i, i]), abs(M[j, j]))


def test_double_pendulum_mass_matrix_closed_form(oracle_mod):
    m = robots.chain(2)
    o = oracle_mod.Oracle(m)
    Ic = robots.capsule_inertia(1.0, 0.05, 0.5)[0]
    d, L = 0.25, 0.5
    for t2 in np.linspace(-3, 3, 13):
        M = o.forward(np.array([0.3, t2]), np.zeros(2))["M"]
        c = math.cos(t2)
        M11 = 2 * Ic + d * d + (L * L + d * d + 2 * L * d * c)
        M12 = Ic + d * d + L * d * c
        M22 = Ic + d * d
        np.testing.assert_allclose(M, [[M11, M12], [M12, M22]], rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- bias forces
def lagrangian_bias(o, q, v, eps=1e-5):
    """c_i = sum_jk (dM_ij/dq_k - 0.5 dM_jk/dq_i) v_j v_k + dV/dq_i for a hinge-only tree."""
    n = len(q)
    dM = np.zeros((n, n, n))
    dV = np.zeros(n)
    for k in range(n):
        e = np.zeros(n); e[k] = eps
        dM[:, :, k] = (o.forward(q + e, np.zeros(n))["M"] - o.forward(q - e, np.zeros(n))["M"]) / (2 * eps)
        dV[k] = (o.energy(q + e, np.zeros(n))[1] - o.energy(q - e, np.zeros(n))[1]) / (2 * eps)
    c = np.einsum("ijk,j,k->i", dM, v, v) - 0.5 * np.einsum("jki,j,k->i", dM, v, v) + dV
    return c


@pytest.mark.parametrize("which", ["chain3", "fixed_humanoid"])
def test_bias_matches_lagrangian(oracle_mod, which):
    m = robots.chain3() if which == "chain3" else fixed_humanoid()
    o = oracle_mod.Oracle(m)
    rng = np.random.default_rng(5)
    q = rng.uniform(-1, 1, o.nq)
    v = rng.normal(0, 1.0, o.nv)
    c = o.forward(q, v)["bias"]
    cl = lagrangian_bias(o, q, v)
    np.testing.assert_allclose(c, cl, rtol=1e-6, atol=1e-6 * np.abs(cl).max())
    # v = 0: pure gravity torque
    c0 = o.forward(q, np.zeros(o.nv))["bias"]
    np.testing.assert_allclose(c0, lagrangian_bias(o, q, np.zeros(o.nv)), rtol=1e-6, atol=1e-8)


def test_free_body_bias_closed_form(oracle_mod):
    m = robots.free_box_asym(gravity=(0, 0, -9.81))
    o = oracle_mod.Oracle(m)
    I = np.array(m["bodies"][1]["inertia"])
    rng = np.random.default_rng(6)
    for _ in range(5):
        q = np.concatenate([rng.normal(size=3), rng.normal(size=4)])
        v = rng.normal(size=6)
        c = o.forward(q, v)["bias"]
        w = v[3:]
        np.testing.assert_allclose(c[:3], [0, 0, 2.0 * 9.81], atol=1e-13)
        np.testing.assert_allclose(c[3:], np.cross(w, I * w), atol=1e-13)
