"""Pins of the oracle's contacts between two moving bodies: two free boxes colliding in zero
gravity conserve linear momentum and angular momentum about the origin exactly (the contact
forces act at one point, equal and opposite, since the rows use the difference of the two
bodies' point Jacobians), a box resting on a free box carries its weight into the lower box's
floor contacts, and contact rows equal the frame times the relative velocity of the two bodies'
points at the contact."""
import numpy as np

from helpers import q_plus, rot
from workloads import robots


def _two_boxes(gravity=(0, 0, 0), floor=False, h=0.05, mass=(1.0, 2.0), dt=0.002):
    mb = robots.ModelBuilder("two_boxes", timestep=dt, nsubsteps=1, gravity=list(gravity))
    if floor:
        mb.geom(0, "plane", [0, 0, 0], contype=0, conaffinity=1)
    ids = []
    for i, (z, m) in enumerate(zip((h, 3 * h + 0.001), mass)):
        b = mb.body(f"box{i}", 0, (0, 0, z), m, robots.box_inertia(m, 0.1, 0.1, h))
        mb.joint(b, "free")
        mb.geom(b, "box", [0.1, 0.1, h], contype=1, conaffinity=1)
        ids.append(b)
    return mb.build()


def _momenta(o, m, q, v):
    """Linear momentum and angular momentum about the origin of the two free boxes."""
    P = np.zeros(3); L = np.zeros(3)
    t = o.forward(q, v)
    for k, b in enumerate((1, 2)):
        mass = m["bodies"][b]["mass"]
        I = np.diag(m["bodies"][b]["inertia"])
        vb = v[6 * k:6 * k + 3]
        R = t["xmat"][b]
        w = R @ v[6 * k + 3:6 * k + 6]
        x = t["xpos"][b]
        P += mass * vb
        L += mass * np.cross(x, vb) + R @ I @ R.T @ w
    return P, L


def test_collision_conserves_momentum(oracle_mod):
    """Two boxes thrown at each other off-centre, spinning, in zero gravity: through the whole
    collision the total linear momentum stays constant to 1e-10 relative (the contact forces are
    equal and opposite), and the angular momentum about the origin to 2e-3 (the contact forces
    act at one point; what moves it is the integrator's own first-order drift of free spinning
    bodies)."""
    m = _two_boxes()
    o = oracle_mod.Oracle(m)
    q = np.array([[-0.25, 0.03, 0.0, 1, 0, 0, 0, 0.25, -0.02, 0.01] + list(robots.quat_axis_angle((1, 2, 3), 0.3))])
    v = np.array([[1.0, 0.0, 0.1, 0.5, -0.3, 2.0, -0.8, 0.2, 0.0, -1.0, 0.7, 0.4]])
    ws = np.zeros((1, 12))
    P0, L0 = _momenta(o, m, q[0], v[0])
    touched = 0
    for _ in range(300):
        o.step(np.zeros((1, 0)), q, v, ws)
        t = o.forward(q[0], v[0])
        touched += t["ncon"] > 0
        P, L = _momenta(o, m, q[0], v[0])
        np.testing.assert_allclose(P, P0, rtol=0, atol=1e-10 * np.abs(P0).max())
        np.testing.assert_allclose(L, L0, rtol=0, atol=2e-3 * np.abs(L0).max())
    assert touched >= 5


def test_rows_are_relative_point_velocities(oracle_mod):
    """Rows of a contact between two moving boxes: the frame times the difference of the two
    boxes' point velocities at the contact, by finite differences."""
    m = _two_boxes()
    o = oracle_mod.Oracle(m)
    q = np.array([0, 0, 0.05, 1, 0, 0, 0, 0.02, 0.01, 0.149] + list(robots.quat_axis_angle((0, 0, 1), 0.2)))
    v = np.random.default_rng(7).normal(size=12)
    t = o.forward(q, v)
    assert t["ncon"] >= 1
    eps = 1e-6
    tp = o.forward(q_plus(m, q, eps * v), np.zeros(12))
    tm = o.forward(q_plus(m, q, -eps * v), np.zeros(12))
    for ci in range(t["ncon"]):
        p = t["pos"][ci]
        vel = []
        for b in (1, 2):
            loc = t["xmat"][b].T @ (p - t["xpos"][b])
            vel.append(((tp["xpos"][b] + tp["xmat"][b] @ loc) - (tm["xpos"][b] + tm["xmat"][b] @ loc)) / (2 * eps))
        g1, g2 = t["geom"][ci]
        b1, b2 = m["geoms"][g1]["body"], m["geoms"][g2]["body"]
        rel = vel[b2 - 1] - vel[b1 - 1]
        F, mu = t["frame"][ci], t["mu"][ci]
        lin = F @ rel
        exp = [lin[0] + mu * lin[1], lin[0] - mu * lin[1], lin[0] + mu * lin[2], lin[0] - mu * lin[2]]
        np.testing.assert_allclose(t["J"][4 * ci:4 * ci + 4] @ v, exp, rtol=1e-7, atol=1e-8)


def test_stack_carries_both_weights(oracle_mod):
    """A 2 kg box resting on a 1 kg free box on the floor: at rest the box-box contacts carry
    2 g and the floor contacts 3 g, each set's forces summing to a vertical resultant."""
    m = _two_boxes(gravity=(0, 0, -9.81), floor=True)
    o = oracle_mod.Oracle(m)
    q = np.array([[0, 0, 0.05, 1, 0, 0, 0, 0, 0, 0.15, 1, 0, 0, 0]], float)
    v = np.zeros((1, 12)); ws = np.zeros((1, 12))
    for _ in range(2000):
        o.step(np.zeros((1, 0)), q, v, ws)
    t = o.forward(q[0], v[0], qacc_ws=ws[0])
    assert np.abs(v).max() < 1e-8
    floor = np.zeros(3); mid = np.zeros(3)
    for ci in range(t["ncon"]):
        f = t["cforce"][ci] @ t["frame"][ci]
        g1, g2 = t["geom"][ci]
        if m["geoms"][g1]["type"] == "plane" or m["geoms"][g2]["type"] == "plane":
            floor += f
        else:
            # force on g2's body; the upper box is body 2
            b2 = m["geoms"][g2]["body"]
            mid += f if b2 == 2 else -f
    np.testing.assert_allclose(floor, [0, 0, 3 * 9.81], atol=1e-6)
    np.testing.assert_allclose(mid, [0, 0, 2 * 9.81], atol=1e-6)
