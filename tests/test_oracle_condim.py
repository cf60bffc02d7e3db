"""Pins of the oracle's torsional and rolling friction (condim 4 and 6, pyramidal): the extra
pyramid rows are the normal row plus / minus mu times the contact frame's components of the
body's angular velocity, a slowly spinning ball loses its spin at the rate the soft pyramid's
quadratic cost fixes in closed form, spin and roll are lost by the condims that have them and
kept by the others, the converged solution minimises the cost, and the normal force sums every
row."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from helpers import impedance, q_plus
from workloads import robots


def _set(m, condim, spin=None, roll=None):
    for g in m["geoms"]:
        g["condim"] = condim
        if spin is not None:
            g["friction_spin"] = spin
        if roll is not None:
            g["friction_roll"] = roll
    return m


def _omega(o, m, q, v, eps=1e-6):
    """World angular velocity of body 1 from finite differences of its rotation."""
    Rp = o.forward(q_plus(m, q, eps * v), np.zeros(len(v)))["xmat"][1]
    Rm = o.forward(q_plus(m, q, -eps * v), np.zeros(len(v)))["xmat"][1]
    R = o.forward(q, np.zeros(len(v)))["xmat"][1]
    W = (Rp - Rm) / (2 * eps) @ R.T
    return np.array([W[2, 1], W[0, 2], W[1, 0]])


@pytest.mark.parametrize("condim", [4, 6])
def test_rows_are_pyramids_of_point_and_angular_velocity(oracle_mod, condim):
    """A tilted box touching the plane: rows 0..3 of each contact are the sliding pyramid, rows
    4, 5 the normal row +- mu_spin n.omega, rows 6..9 (condim 6) +- mu_roll t1.omega, t2.omega."""
    m = _set(robots.free_body("box", size=(0.1, 0.1, 0.1), friction=0.7), condim, spin=0.03, roll=0.02)
    o = oracle_mod.Oracle(m)
    q = np.concatenate([[0, 0, 0.05], robots.quat_axis_angle((1, 2, 3), 0.3)])
    v = np.random.default_rng(12).normal(size=6)
    t = o.forward(q, v)
    assert t["ncon"] >= 1
    nr = 2 * (condim - 1)
    assert t["J"].shape[0] == nr * t["ncon"]
    w = _omega(o, m, q, v)
    eps = 1e-6
    tp = o.forward(q_plus(m, q, eps * v), np.zeros(6))
    tm = o.forward(q_plus(m, q, -eps * v), np.zeros(6))
    for ci in range(t["ncon"]):
        p = t["pos"][ci]
        local = t["xmat"][1].T @ (p - t["xpos"][1])
        vel = ((tp["xpos"][1] + tp["xmat"][1] @ local) - (tm["xpos"][1] + tm["xmat"][1] @ local)) / (2 * eps)
        F = t["frame"][ci]
        lin, ang = F @ vel, F @ w
        exp = [lin[0] + 0.7 * lin[1], lin[0] - 0.7 * lin[1], lin[0] + 0.7 * lin[2], lin[0] - 0.7 * lin[2],
               lin[0] + 0.03 * ang[0], lin[0] - 0.03 * ang[0]]
        if condim == 6:
            exp += [lin[0] + 0.02 * ang[1], lin[0] - 0.02 * ang[1], lin[0] + 0.02 * ang[2], lin[0] - 0.02 * ang[2]]
        np.testing.assert_allclose(t["J"][nr * ci:nr * ci + nr] @ v, exp, rtol=1e-7, atol=1e-8)


def test_pair_takes_the_larger_spin_and_roll(oracle_mod):
    m = _set(robots.free_body("sphere", size=(0.1,)), 6, spin=0.001, roll=0.0002)
    m["geoms"][0]["friction_spin"] = 0.004   # the plane
    m["geoms"][1]["friction_roll"] = 0.0007  # the ball
    o = oracle_mod.Oracle(m)
    q = np.array([0, 0, 0.0999, 1, 0, 0, 0.0])
    J = o.forward(q, np.zeros(6))["J"]
    # free-joint angular dofs are body-local, the world axes at the identity pose; the frame of
    # the normal +z is t1 = +x, t2 = +y
    np.testing.assert_allclose(J[4:10, 3:], [[0, 0, 0.004], [0, 0, -0.004], [0.0007, 0, 0], [-0.0007, 0, 0],
                                             [0, 0.0007, 0], [0, -0.0007, 0]], atol=1e-15)


def _rest_sphere(oracle_mod, m, steps=500):
    o = oracle_mod.Oracle(m)
    q = np.array([[0, 0, 0.1, 1, 0, 0, 0.0]]); v = np.zeros((1, 6)); ws = np.zeros((1, 6))
    for _ in range(steps):
        o.step(np.zeros((1, 0)), q, v, ws)
    return o, q, v, ws


def test_spin_decay_closed_form(oracle_mod):
    """A ball resting on a plane (condim 4) spinning slowly about the vertical: both spin rows
    stay active (b mu w below the depth term k imp |r|), the rows' depth terms cancel in the
    spin equation and the sliding rows do not touch it, so the quadratic cost gives
    I a_w = -2 D mu^2 (a_w + b w), D = imp / ((1 - imp) A-hat), A-hat = 1/m + mu^2 / I: one step
    scales w by 1 - dt 2 D mu^2 b / (I + 2 D mu^2), imp taken at the ball's penetration."""
    mass, r, mu, dt = 1.0, 0.1, 0.002, 0.002
    m = _set(robots.free_body("sphere", size=(r,), mass=mass, pos=(0, 0, r), timestep=dt), 4, spin=mu)
    o, q, v, ws = _rest_sphere(oracle_mod, m)
    v[0, 5] = 1.0
    I = 0.4 * mass * r * r
    b = 2.0 / (0.95 * 0.02)
    for _ in range(200):
        imp = impedance(r - q[0, 2])
        D = imp / ((1 - imp) * (1 / mass + mu * mu / I))
        ratio = 1 - dt * 2 * D * mu * mu * b / (I + 2 * D * mu * mu)
        w0 = v[0, 5]
        o.step(np.zeros((1, 0)), q, v, ws)
        assert abs(v[0, 5] - ratio * w0) < 1e-9 * abs(w0)
    assert 0.4 < v[0, 5] < 0.9


@pytest.mark.parametrize("condim,keeps_spin,keeps_roll", [(3, True, True), (4, False, True), (6, False, False)])
def test_spin_and_roll_losses_by_condim(oracle_mod, condim, keeps_spin, keeps_roll):
    """Over 4 s a spinning ball keeps its spin and a rolling ball its speed, to 0.1 %, unless the
    contact has torsional (condim 4, 6) or rolling (condim 6) friction, which take away at least
    10 % of them."""
    m = _set(robots.free_body("sphere", size=(0.1,), pos=(0, 0, 0.1), timestep=0.002), condim, 0.002, 0.0005)
    o, q, v, ws = _rest_sphere(oracle_mod, m)
    v[0, 5] = 1.0
    for _ in range(2000):
        o.step(np.zeros((1, 0)), q, v, ws)
    assert (abs(v[0, 5] - 1.0) < 1e-3) == keeps_spin and (v[0, 5] < 0.9) != keeps_spin
    o, q, v, ws = _rest_sphere(oracle_mod, m)
    v[0, 0], v[0, 4] = 0.5, 5.0
    for _ in range(2000):
        o.step(np.zeros((1, 0)), q, v, ws)
    assert (abs(v[0, 0] - 0.5) < 5e-4) == keeps_roll and (v[0, 0] < 0.45) != keeps_roll


def test_resting_normal_force_sums_every_row(oracle_mod):
    """A ball at rest with condim 6: the reported normal force (the sum of all ten rows' forces)
    carries its weight."""
    m = _set(robots.free_body("sphere", size=(0.1,), mass=1.7, pos=(0, 0, 0.1), timestep=0.002), 6, 0.003, 0.001)
    o, q, v, ws = _rest_sphere(oracle_mod, m, 1500)
    t = o.forward(q[0], v[0], None, ws[0])
    assert t["ncon"] == 1 and t["J"].shape[0] == 10
    np.testing.assert_allclose(t["cforce"][0], [1.7 * 9.81, 0, 0], atol=1e-6)
    assert np.count_nonzero(t["efc_force"][4:]) > 0


def _problem(t):
    M, a0, J, aref, D = t["M"], t["a0"], t["J"], t["aref"], t["D"]

    def f(a):
        jar = J @ a - aref
        return 0.5 * (a - a0) @ M @ (a - a0) + 0.5 * np.sum(D * np.minimum(jar, 0) ** 2)

    def g(a):
        jar = J @ a - aref
        return M @ (a - a0) + J.T @ (D * np.minimum(jar, 0))

    return f, g


@pytest.mark.parametrize("seed", range(3))
def test_condim6_converged_matches_scipy(oracle_mod, seed):
    rng = np.random.default_rng(200 + seed)
    m = _set(robots.free_body("box", size=(0.1, 0.07, 0.05), mass=1.3, friction=0.8), 6, 0.02, 0.01)
    o = oracle_mod.Oracle(m)
    o.set_mode("converged")
    qb = rng.normal(size=4); qb /= np.linalg.norm(qb)
    q = np.concatenate([[0, 0, 0.05], qb])
    v = rng.normal(0, 0.5, 6)
    t = o.forward(q, v)
    assert t["ncon"] >= 1
    f, g = _problem(t)
    res = minimize(f, t["a0"], jac=g, method="BFGS", options={"gtol": 1e-12, "maxiter": 10000})
    scale = np.abs(res.x).max() + 1
    np.testing.assert_allclose(t["qacc"], res.x, atol=1e-6 * scale)
    assert f(t["qacc"]) <= f(res.x) + 1e-9 * abs(f(res.x))
