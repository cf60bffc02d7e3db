"""Pins of the oracle's time stepping against closed forms and conservation laws (CPU)."""
import math

import numpy as np
import pytest

from helpers import q_plus, quat_exp, quat_mul, rot
from workloads import robots


def test_small_angle_pendulum_period(oracle_mod):
    """Single 0.5 m capsule link, theta0 = 0.01 rad, dt = 2 ms: T0 = 2 pi sqrt(I_O / (m g d))."""
    m = robots.chain(1)
    o = oracle_mod.Oracle(m)
    I_O = robots.capsule_inertia(1.0, 0.05, 0.5)[0] + 0.25 ** 2
    T0 = 2 * math.pi * math.sqrt(I_O / (9.81 * 0.25))
    assert abs(T0 - 1.203689) < 1e-6
    q, v = np.array([[0.01]]), np.zeros((1, 1))
    ws = np.zeros((1, 1))
    dt = m["opt"]["timestep"]
    th = [q[0, 0]]
    for _ in range(int(10.5 * T0 / dt)):
        o.step(np.zeros((1, 0)), q, v, ws)
        th.append(q[0, 0])
    th = np.array(th)
    # downward zero crossings, linearly interpolated
    idx = np.where((th[:-1] > 0) & (th[1:] <= 0))[0]
    tc = (idx + th[idx] / (th[idx] - th[idx + 1])) * dt
    T = (tc[-1] - tc[0]) / (len(tc) - 1)
    assert len(tc) >= 10
    assert abs(T / T0 - 1) < 1e-4


def _rk4_energy_drift(o, model, q, v, dt, t_end):
    """Classical RK4 on the oracle's accelerations (configuration update through q_plus)."""
    def acc(q, v):
        return o.forward(q, v)["qacc"]

    E0 = sum(o.energy(q, v))
    drift = 0.0
    for _ in range(int(round(t_end / dt))):
        k1v, k1a = v, acc(q, v)
        q2, v2 = q_plus(model, q, 0.5 * dt * k1v), v + 0.5 * dt * k1a
        k2v, k2a = v2, acc(q2, v2)
        q3, v3 = q_plus(model, q, 0.5 * dt * k2v), v + 0.5 * dt * k2a
        k3v, k3a = v3, acc(q3, v3)
        q4, v4 = q_plus(model, q, dt * k3v), v + dt * k3a
        k4v, k4a = v4, acc(q4, v4)
        q = q_plus(model, q, dt / 6 * (k1v + 2 * k2v + 2 * k3v + k4v))
        v = v + dt / 6 * (k1a + 2 * k2a + 2 * k3a + k4a)
        drift = max(drift, abs(sum(o.energy(q, v)) - E0))
    return drift


def test_energy_conserved_contact_free_chain_rk4(oracle_mod):
    m = robots.chain3()
    o = oracle_mod.Oracle(m)
    q = np.array([1.0, -0.5, 2.0])
    v = np.array([0.5, -0.3, 0.8])
    scale = 3 * 1.0 * 9.81 * 1.5
    drift = _rk4_energy_drift(o, m, q, v, 5e-4, 1.0)
    assert drift / scale < 1e-7


def test_energy_conserved_floating_quadruped_rk4(oracle_mod):
    """Zero gravity, no actuators, no ground: kinetic energy of the free-floating tree is conserved."""
    m = robots.quadruped()
    m["opt"]["gravity"] = [0.0, 0.0, 0.0]
    m["actuators"] = []
    m["geoms"] = [g for g in m["geoms"] if g["type"] != "plane"]
    o = oracle_mod.Oracle(m)
    rng = np.random.default_rng(7)
    q = robots.qpos0(m)
    q[7:] = rng.uniform(-0.5, 0.5, 12)
    v = rng.normal(0, 1.0, 18)
    E = sum(o.energy(q, v))
    drift = _rk4_energy_drift(o, m, q, v, 2.5e-4, 0.25)
    assert drift / E < 1e-7


def test_energy_conserved_free_body_offset_com_rk4(oracle_mod):
    """Zero gravity free body whose centre of mass is off its frame origin: energy conserved."""
    m = robots.free_offset(gravity=(0, 0, 0))
    o = oracle_mod.Oracle(m)
    q = np.concatenate([[0.1, 0.2, 0.3], robots.quat_axis_angle((0.3, -1, 0.5), 1.1)])
    v = np.array([0.3, -0.4, 0.2, 1.5, -2.0, 0.7])
    E = sum(o.energy(q, v))
    assert _rk4_energy_drift(o, m, q, v, 2.5e-4, 0.25) / E < 1e-7


def test_semi_implicit_euler_energy_drift_first_order(oracle_mod):
    drifts = []
    for dt in (0.002, 0.001):
        m = robots.chain(3, timestep=dt)
        o = oracle_mod.Oracle(m)
        q = np.array([[0.4, -0.3, 0.2]])
        v = np.zeros((1, 3))
        ws = np.zeros((1, 3))
        E0 = sum(o.energy(q[0], v[0]))
        d = 0.0
        for _ in range(int(round(1.0 / dt))):
            o.step(np.zeros((1, 0)), q, v, ws)
            d = max(d, abs(sum(o.energy(q[0], v[0])) - E0))
        drifts.append(d)
    assert 1.6 < drifts[0] / drifts[1] < 2.4


def test_free_body_momentum_and_spin(oracle_mod):
    m = robots.free_box_asym(gravity=(0, 0, 0), timestep=0.005)
    o = oracle_mod.Oracle(m)
    # linear momentum exact, spin about a principal axis exact
    q = np.array([[0.1, 0.2, 0.3, 1, 0, 0, 0]], float)
    v = np.array([[0.3, -0.2, 0.5, 0, 0, 2.0]])
    ws = np.zeros((1, 6))
    for _ in range(200):
        o.step(np.zeros((1, 0)), q, v, ws)
    np.testing.assert_allclose(v[0], [0.3, -0.2, 0.5, 0, 0, 2.0], atol=1e-13)
    np.testing.assert_allclose(q[0, :3], [0.1 + 0.3, 0.2 - 0.2, 0.3 + 0.5], atol=1e-12)
    # quaternion follows the exponential map exactly for a constant body rate
    np.testing.assert_allclose(q[0, 3:], quat_mul([1, 0, 0, 0], quat_exp([0, 0, 2.0 * 1.0])), atol=1e-12)


def test_free_body_angular_momentum_first_order(oracle_mod):
    I = np.array(robots.free_box_asym()["bodies"][1]["inertia"])
    errs = []
    for dt in (0.002, 0.001):
        m = robots.free_box_asym(gravity=(0, 0, 0), timestep=dt)
        o = oracle_mod.Oracle(m)
        q = np.array([[0, 0, 0, 1, 0, 0, 0]], float)
        w0 = np.array([1.0, 2.0, 0.5])
        v = np.concatenate([[0, 0, 0], w0])[None]
        ws = np.zeros((1, 6))
        L0 = rot(q[0, 3:]) @ (I * w0)
        e = 0.0
        for _ in range(int(round(0.5 / dt))):
            o.step(np.zeros((1, 0)), q, v, ws)
            L = rot(q[0, 3:]) @ (I * v[0, 3:])
            e = max(e, np.linalg.norm(L - L0))
        errs.append(e)
    assert errs[1] < errs[0]
    assert 1.6 < errs[0] / errs[1] < 2.4


def test_floating_quadruped_linear_momentum(oracle_mod):
    """Zero-g floating quadruped: total linear momentum P = M[0:3] v drifts first order in dt."""
    errs = []
    for dt in (0.002, 0.001):
        m = robots.quadruped()
        m["opt"].update(gravity=[0.0, 0.0, 0.0], timestep=dt, nsubsteps=1)
        m["actuators"] = []
        m["geoms"] = [g for g in m["geoms"] if g["type"] != "plane"]
        o = oracle_mod.Oracle(m)
        rng = np.random.default_rng(8)
        q = robots.qpos0(m)[None].copy()
        q[0, 7:] = rng.uniform(-0.5, 0.5, 12)
        v = rng.normal(0, 1.0, (1, 18))
        ws = np.zeros((1, 18))
        P0 = o.forward(q[0], v[0])["M"][:3] @ v[0]
        e = 0.0
        for _ in range(int(round(0.2 / dt))):
            o.step(np.zeros((1, 0)), q, v, ws)
            P = o.forward(q[0], v[0])["M"][:3] @ v[0]
            e = max(e, np.linalg.norm(P - P0))
        errs.append(e)
    assert errs[1] < errs[0] and 1.5 < errs[0] / errs[1] < 2.5
    assert errs[0] < 1e-2 * 10.0


def test_integrate_step_formula(oracle_mod):
    m = robots.quadruped()
    o = oracle_mod.Oracle(m)
    rng = np.random.default_rng(9)
    q = robots.qpos0(m)
    q[3:7] = rng.normal(size=4); q[3:7] /= np.linalg.norm(q[3:7])
    v = rng.normal(size=18)
    a = rng.normal(size=18)
    qo, vo = o.integrate(q, v, a)
    dt = m["opt"]["timestep"]
    np.testing.assert_allclose(vo, v + dt * a, rtol=1e-15)
    np.testing.assert_allclose(qo[:3], q[:3] + dt * vo[:3], rtol=1e-15)
    np.testing.assert_allclose(qo[7:], q[7:] + dt * vo[6:], rtol=1e-15)
    np.testing.assert_allclose(qo[3:7], quat_mul(q[3:7], quat_exp(dt * vo[3:6])), atol=1e-15)
