"""Pins of the oracle's equality constraints (connect, weld): their rows are the anchor's
finite-differenced velocity and the body's angular velocity, a body hanging from a connect
settles at the closed-form soft sag with the constraint carrying its weight, and a weld with the
anchor away from the centre of mass carries the weight's moment."""
import math

import numpy as np

from helpers import rot, soft_sag
from workloads import robots

DT = 0.002


def _hanging(kind, anchor=(0.0, 0.0, 0.0), mass=2.0, r=0.05, target=(0.0, 0.0, 1.0), quat=(1.0, 0, 0, 0)):
    mb = robots.ModelBuilder("hang", timestep=DT, nsubsteps=1)
    b = mb.body("ball", 0, (0, 0, 1), mass, robots.sphere_inertia(mass, r))
    mb.joint(b, "free")
    mb.equality(kind, b, anchor, target, quat)
    return mb.build()


def _settle(oracle_mod, m, q0, steps=4000):
    o = oracle_mod.Oracle(m)
    q = np.array(q0, float)[None]; v = np.zeros((1, 6)); ws = np.zeros((1, 6))
    for _ in range(steps):
        o.step(np.zeros((1, 0)), q, v, ws)
    return o, q, v, ws


def test_connect_rows_are_the_anchor_velocity(oracle_mod):
    """Rows of a connect at a random state: J v = world velocity of the anchor point, by finite
    differences of its position along the motion."""
    from helpers import q_plus
    anchor = (0.03, -0.02, 0.04)
    m = _hanging("connect", anchor)
    rng = np.random.default_rng(1)
    qq = rng.normal(size=4); qq /= np.linalg.norm(qq)
    q = np.concatenate([[0.1, 0.0, 0.95], qq])
    v = rng.normal(size=6)
    t = oracle_mod.Oracle(m).forward(q, v)
    assert t["J"].shape[0] == 3
    pt = lambda qx: qx[:3] + rot(qx[3:]) @ np.array(anchor)
    h = 1e-6
    fd = (pt(q_plus(m, q, h * v)) - pt(q_plus(m, q, -h * v))) / (2 * h)
    np.testing.assert_allclose(t["J"] @ v, fd, atol=1e-8)


def test_weld_rows_add_the_angular_velocity(oracle_mod):
    m = _hanging("weld", (0.0, 0.0, 0.02))
    rng = np.random.default_rng(2)
    qq = rng.normal(size=4); qq /= np.linalg.norm(qq)
    q = np.concatenate([[0.0, 0.1, 1.0], qq])
    v = rng.normal(size=6)
    t = oracle_mod.Oracle(m).forward(q, v)
    assert t["J"].shape[0] == 6
    # free-joint angular velocity is body-local: world omega = R w
    np.testing.assert_allclose(t["J"][3:] @ v, rot(qq) @ v[3:], atol=1e-12)


def test_connect_at_the_centre_of_mass_sags_by_the_closed_form(oracle_mod):
    """A ball connected at its centre to a world point settles below it by the soft sag, the
    three rows' forces summing to (0, 0, m g)."""
    mass = 2.0
    m = _hanging("connect", mass=mass)
    o, q, v, ws = _settle(oracle_mod, m, [0.0, 0.0, 1.0, 1.0, 0, 0, 0])
    t = o.forward(q[0], v[0], None, ws[0])
    assert abs(q[0, 2] - 1.0 - soft_sag(mass)) < 1e-6 * abs(soft_sag(mass))
    np.testing.assert_allclose(t["efc_force"], [0.0, 0.0, mass * 9.81], atol=1e-6)
    assert np.abs(v).max() < 1e-8


def test_weld_off_the_centre_carries_the_moment(oracle_mod):
    """A ball welded at a point 10 cm beside its centre: at rest the translational rows carry the
    weight and the rotational rows its moment about the anchor, (anchor - centre) x (0, 0, m g)
    in the world frame; the soft rotational rows let the body tip by a small angle about the
    horizontal axis normal to the anchor offset."""
    mass = 2.0
    anchor = np.array([0.1, 0.0, 0.0])
    m = _hanging("weld", tuple(anchor), mass=mass, target=(0.1, 0.0, 1.0))
    o, q, v, ws = _settle(oracle_mod, m, [0.0, 0.0, 1.0, 1.0, 0, 0, 0])
    t = o.forward(q[0], v[0], None, ws[0])
    f = t["efc_force"]
    np.testing.assert_allclose(f[:3], [0.0, 0.0, mass * 9.81], atol=1e-6)
    R = rot(q[0, 3:])
    moment = np.cross(R @ anchor, [0.0, 0.0, mass * 9.81])   # about the centre: the anchor force's
    np.testing.assert_allclose(f[3:], -moment, atol=1e-6)
    assert np.abs(v).max() < 1e-8
    ang = 2 * math.acos(min(1.0, abs(q[0, 3])))
    assert 0 < ang < 0.05
    np.testing.assert_allclose(np.abs(q[0, 4:]) / np.linalg.norm(q[0, 4:]), [0, 1, 0], atol=1e-9)


def _chain_tip(mb_kind="connect"):
    m = robots.chain(3, "chain3_eq")
    m["equality"] = [dict(type=mb_kind, body=3, anchor=[0.0, 0.0, -0.5], target=[0.0, 0.0, -1.5])]
    if mb_kind == "weld":
        m["equality"][0]["quat"] = [1.0, 0.0, 0.0, 0.0]
    return m


def _chain_pose(q):
    """World position of the chain's tip and rotation of its last link (planar chain, y hinges)."""
    R = np.eye(3); p = np.zeros(3)
    for i in range(3):
        if i:
            p = p + R @ np.array([0.0, 0.0, -0.5])
        c, s = math.cos(q[i]), math.sin(q[i])
        R = R @ np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return p + R @ np.array([0.0, 0.0, -0.5]), R


def test_chain_rows_are_the_tip_velocity(oracle_mod):
    """Rows of a connect and a weld on the last link of a hinge chain: the tip's velocity and the
    link's angular velocity by finite differences of its pose."""
    rng = np.random.default_rng(3)
    q = rng.uniform(-1, 1, 3); v = rng.normal(size=3)
    h = 1e-6
    for kind in ("connect", "weld"):
        t = oracle_mod.Oracle(_chain_tip(kind)).forward(q, v)
        (pa, Ra), (pb, Rb) = _chain_pose(q + h * v), _chain_pose(q - h * v)
        np.testing.assert_allclose(t["J"][:3] @ v, (pa - pb) / (2 * h), atol=1e-8)
        if kind == "weld":
            W = (Ra - Rb) / (2 * h) @ _chain_pose(q)[1].T
            np.testing.assert_allclose(t["J"][3:] @ v, [W[2, 1], W[0, 2], W[1, 0]], atol=1e-8)


def test_pinned_chain_at_rest_carries_no_force(oracle_mod):
    """A hanging chain whose tip is connected at its own rest point: nothing moves and the
    constraint carries no force (the free chain is already in equilibrium there)."""
    o = oracle_mod.Oracle(_chain_tip())
    q = np.zeros((1, 3)); v = np.zeros((1, 3)); ws = np.zeros((1, 3))
    for _ in range(50):
        o.step(np.zeros((1, 0)), q, v, ws)
    assert np.abs(q).max() < 1e-12 and np.abs(v).max() < 1e-12
    np.testing.assert_allclose(o.forward(q[0], v[0], None, ws[0])["efc_force"], 0.0, atol=1e-9)


def test_connect_pendulum_period(oracle_mod):
    """A ball hung by a connect 0.3 m above its centre swings as a compound pendulum about the
    world point: small-angle period 2 pi sqrt((I + m L^2) / (m g L)).  The soft rows reach only a
    fraction (the impedance, about 0.9) of the reference acceleration each step, the rest of the
    pivot's acceleration being what it would be unconstrained, which lengthens the period by a few
    percent; the pivot stays within a millimetre of the world point."""
    mass, r, L = 1.0, 0.05, 0.3
    m = _hanging("connect", anchor=(0.0, 0.0, L), mass=mass, r=r, target=(0.0, 0.0, 1.0 + L))
    o = oracle_mod.Oracle(m)
    th = 0.05
    qq = [math.cos(th / 2), 0.0, math.sin(th / 2), 0.0]
    c = np.array([0.0, 0.0, 1.0 + L]) - rot(qq) @ np.array([0.0, 0.0, L])
    q = np.concatenate([c, qq])[None]; v = np.zeros((1, 6)); ws = np.zeros((1, 6))
    I = 0.4 * mass * r * r
    T = 2 * math.pi * math.sqrt((I + mass * L * L) / (mass * 9.81 * L))
    xs, drift = [], 0.0
    for _ in range(int(2.5 * T / DT)):
        o.step(np.zeros((1, 0)), q, v, ws)
        xs.append(q[0, 0])
        pivot = q[0, :3] + rot(q[0, 3:]) @ np.array([0.0, 0.0, L])
        drift = max(drift, np.linalg.norm(pivot - [0.0, 0.0, 1.0 + L]))
    xs = np.array(xs)
    # times of the upward zero crossings of x, linearly interpolated
    k = np.nonzero((xs[:-1] < 0) & (xs[1:] >= 0))[0]
    tz = (k + 1 - xs[k + 1] / (xs[k + 1] - xs[k])) * DT + DT
    assert len(tz) >= 2
    assert T < tz[1] - tz[0] < 1.05 * T
    assert drift < 1e-3
