"""Pins of the oracle's collision, soft-constraint and Newton stages (CPU)."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq, minimize

from helpers import q_plus, quat_mul, rot
from workloads import robots

K_REF = 1.0 / (0.95 ** 2 * 0.02 ** 2)      # stiffness of the default solref/solimp, 1/s^2
B_REF = 2.0 / (0.95 * 0.02)                 # damping, 1/s


def imp_ref(r, dmin=0.9, dmax=0.95, width=0.001, mid=0.5, p=2.0):
    x = min(abs(r) / width, 1.0)
    y = x ** p / mid ** (p - 1) if x <= mid else 1 - (1 - x) ** p / (1 - mid) ** (p - 1)
    return dmin + y * (dmax - dmin)


def test_reference_coefficients():
    assert abs(K_REF - 2770.083) < 1e-3 and abs(B_REF - 105.263) < 1e-3


# ---------------------------------------------------------------- collision
def test_sphere_plane(oracle_mod):
    m = robots.free_body("sphere", size=(0.05,), ground_quat=robots.quat_axis_angle((1, 0, 0), 0.3))
    o = oracle_mod.Oracle(m)
    n = rot(m["geoms"][0]["quat"])[:, 2]
    for h in (0.06, 0.05, 0.049, 0.03):
        c = n * h + np.array([0.0, 0.0, 0.0])
        c = c + np.cross(n, [1, 0, 0]) * 0.7       # slide along the plane: distance unchanged
        q = np.concatenate([c, [1, 0, 0, 0]])
        t = o.forward(q, np.zeros(6))
        d = h - 0.05
        if d < 0:
            assert t["ncon"] == 1
            assert abs(t["dist"][0] - d) < 1e-15
            np.testing.assert_allclose(t["pos"][0], c - n * (0.05 + d / 2), atol=1e-15)
            np.testing.assert_allclose(t["frame"][0][0], n, atol=1e-15)
            F = t["frame"][0]
            np.testing.assert_allclose(F @ F.T, np.eye(3), atol=1e-15)
            assert abs(np.linalg.det(F) - 1) < 1e-14
            assert tuple(t["geom"][0]) == (0, 1) and t["feature"][0] == 0
        else:
            assert t["ncon"] == 0   # d == 0 is not a contact (strict inequality)


def test_tangent_frame_rule(oracle_mod):
    m = robots.free_body("sphere", size=(0.05,))
    o = oracle_mod.Oracle(m)
    t = o.forward(np.array([0, 0, 0.04, 1, 0, 0, 0]), np.zeros(6))
    # rows (n, t1, t2): n = z -> t1 = x, t2 = y
    np.testing.assert_allclose(t["frame"][0], [[0, 0, 1], [1, 0, 0], [0, 1, 0]], atol=1e-15)
    # tilted plane: t1 = normalise(e_k - (e_k . n) n) with k = argmin |n_k|
    qg = robots.quat_axis_angle((0.3, 1.0, 0.2), 0.7)
    m = robots.free_body("sphere", size=(0.05,), ground_quat=qg)
    o = oracle_mod.Oracle(m)
    n = rot(qg)[:, 2]
    t = o.forward(np.concatenate([n * 0.04, [1, 0, 0, 0]]), np.zeros(6))
    k = int(np.argmin(np.abs(n)))
    e = np.eye(3)[k]
    t1 = e - e.dot(n) * n
    t1 /= np.linalg.norm(t1)
    np.testing.assert_allclose(t["frame"][0], np.stack([n, t1, np.cross(n, t1)]), atol=1e-15)


def test_capsule_plane_ends(oracle_mod):
    qc = robots.quat_axis_angle((1, 0, 0), 0.4)
    m = robots.free_body("capsule", size=(0.03, 0.2), ground=True)
    o = oracle_mod.Oracle(m)
    R = rot(qc)
    x = np.array([0.1, -0.2, 0.09])
    t = o.forward(np.concatenate([x, qc]), np.zeros(6))
    ends = [x - 0.2 * R[:, 2], x + 0.2 * R[:, 2]]
    exp = [(f, e[2] - 0.03) for f, e in enumerate(ends) if e[2] - 0.03 < 0]
    assert t["ncon"] == len(exp) == 1
    for i, (f, d) in enumerate(exp):
        assert t["feature"][i] == f
        assert abs(t["dist"][i] - d) < 1e-15
        np.testing.assert_allclose(t["pos"][i], ends[f] - np.array([0, 0, 1]) * (0.03 + d / 2), atol=1e-15)


def test_box_plane_vertices(oracle_mod):
    m = robots.free_body("box", size=(0.1, 0.2, 0.3))
    o = oracle_mod.Oracle(m)
    rng = np.random.default_rng(10)
    for _ in range(20):
        qb = rng.normal(size=4); qb /= np.linalg.norm(qb)
        R = rot(qb)
        x = np.array([0.0, 0.0, rng.uniform(0.0, 0.3)])
        t = o.forward(np.concatenate([x, qb]), np.zeros(6))
        exp = []
        for k in range(8):
            s = np.array([0.1 if k & 4 else -0.1, 0.2 if k & 2 else -0.2, 0.3 if k & 1 else -0.3])
            vk = x + R @ s
            if vk[2] < 0:
                exp.append((k, vk[2], vk - np.array([0, 0, vk[2] / 2])))
        assert t["ncon"] == len(exp)
        for i, (k, d, p) in enumerate(exp):
            assert t["feature"][i] == k
            assert abs(t["dist"][i] - d) < 1e-15
            np.testing.assert_allclose(t["pos"][i], p, atol=1e-15)


def test_pair_filters(oracle_mod):
    mb = robots.ModelBuilder("filters", timestep=0.005, nsubsteps=1)
    mb.geom(0, "plane", [0, 0, 0], contype=1, conaffinity=1)
    a = mb.body("a", 0, (0, 0, 0.5), 1.0, robots.sphere_inertia(1.0, 0.1))
    mb.joint(a, "free")
    mb.geom(a, "sphere", [0.1], contype=1, conaffinity=1)
    b = mb.body("b", a, (0, 0, 0), 1.0, robots.sphere_inertia(1.0, 0.1))
    mb.joint(b, "hinge", (0, 1, 0))
    mb.geom(b, "sphere", [0.1], contype=2, conaffinity=2)      # (2 & 1) | (1 & 2) = 0 with the plane
    m = mb.build()
    o = oracle_mod.Oracle(m)
    assert o.npair == 1 and o.maxcon == 1        # plane-a only: a-b is parent-child, plane-b masked
    t = o.forward(np.array([0, 0, 0.05, 1, 0, 0, 0, 0.0]), np.zeros(7))
    assert t["ncon"] == 1 and tuple(t["geom"][0]) == (0, 1)


def test_humanoid_contacts_sorted_and_bounded(oracle_mod):
    m = robots.humanoid()
    o = oracle_mod.Oracle(m)
    assert o.maxcon == 32 * 2 + 8 * 8 and o.npair == 40
    q = robots.qpos0(m)
    q[2] = 0.05                                   # pelvis dropped into the floor
    t = o.forward(q, np.zeros(o.nv))
    keys = [(g[0], g[1], f) for g, f in zip(t["geom"], t["feature"])]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    assert np.all(t["dist"] < 0)


# ---------------------------------------------------------------- constraint rows
def test_jacobian_rows_are_point_velocities(oracle_mod):
    """J_c v equals the contact frame times the velocity of the body point at the contact."""
    m = robots.free_body("box", size=(0.1, 0.1, 0.1))
    o = oracle_mod.Oracle(m)
    qb = robots.quat_axis_angle((1, 2, 3), 0.3)
    q = np.concatenate([[0, 0, 0.05], qb])
    rng = np.random.default_rng(11)
    v = rng.normal(size=6)
    t = o.forward(q, v)
    eps = 1e-6
    tp = o.forward(q_plus(m, q, eps * v), np.zeros(6))
    tm = o.forward(q_plus(m, q, -eps * v), np.zeros(6))
    for ci in range(t["ncon"]):
        p = t["pos"][ci]
        local = t["xmat"][1].T @ (p - t["xpos"][1])
        vel = ((tp["xpos"][1] + tp["xmat"][1] @ local) - (tm["xpos"][1] + tm["xmat"][1] @ local)) / (2 * eps)
        F, mu = t["frame"][ci], t["mu"][ci]
        Jc_v = F @ vel
        rows = t["J"][4 * ci:4 * ci + 4] @ v
        exp = [Jc_v[0] + mu * Jc_v[1], Jc_v[0] - mu * Jc_v[1], Jc_v[0] + mu * Jc_v[2], Jc_v[0] - mu * Jc_v[2]]
        np.testing.assert_allclose(rows, exp, rtol=1e-7, atol=1e-8)


def test_impedance_reference_and_regulariser(oracle_mod):
    m = robots.free_body("sphere", size=(0.05,), friction=0.7)
    o = oracle_mod.Oracle(m)
    for depth, vz in ((2e-4, -0.3), (8e-4, 0.1), (3e-3, 0.0)):
        q = np.array([0, 0, 0.05 - depth, 1, 0, 0, 0.0])
        v = np.array([0.2, 0, vz, 0, 0.5, 0])
        t = o.forward(q, v)
        r = t["dist"][0]
        imp = imp_ref(r)
        Minv = np.linalg.inv(t["M"])
        for e in range(4):
            J = t["J"][e]
            A = J @ Minv @ J
            assert abs(t["Ahat"][e] - A) < 1e-13 * A
            np.testing.assert_allclose(t["aref"][e], -B_REF * (J @ v) - K_REF * imp * r, rtol=1e-12)
            np.testing.assert_allclose(t["D"][e], imp / ((1 - imp) * A), rtol=1e-12)


def test_single_row_closed_form(oracle_mod):
    """Frictionless contact: the four pyramid rows coincide, so the solve reduces to one row
    with regulariser R/4: a = a0 + M^-1 Jn' f, f = max(0, (aref - Jn a0) / (A + R/4))."""
    m = robots.free_body("sphere", size=(0.05,), friction=0.0, iterations=4)
    o = oracle_mod.Oracle(m)
    q = np.array([0, 0, 0.0496, 1, 0, 0, 0.0])
    for vz in (-0.5, -0.05, 0.0, 0.3):
        v = np.array([0, 0, vz, 0, 0, 0.0])
        t = o.forward(q, v)
        Jn = t["J"][0]
        Minv = np.linalg.inv(t["M"])
        A = Jn @ Minv @ Jn
        R = 1.0 / t["D"][0]
        f = max(0.0, (t["aref"][0] - Jn @ t["a0"]) / (A + R / 4))
        np.testing.assert_allclose(t["qacc"], t["a0"] + Minv @ Jn * f, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(t["efc_force"].sum(), f, rtol=1e-10, atol=1e-12)


def _settle(o, m, q, steps, friction=None):
    q = np.array(q, float)[None].copy()
    v = np.zeros((1, o.nv)); ws = np.zeros((1, o.nv))
    fr = None if friction is None else np.array([friction])
    for _ in range(steps):
        o.step(np.zeros((1, o.nu)), q, v, ws, friction=fr)
    return q[0], v[0], ws[0]


def test_resting_sphere_penetration_closed_form(oracle_mod):
    """Steady state: 4 imp^2 k |r| / ((1 - imp) A) = m g, A = 1/m + mu^2 (1/m + rho^2 / I),
    rho = radius + dist/2 the lever arm of the mid-surface contact point."""
    m = robots.free_body("sphere", size=(0.05,), mass=1.0, pos=(0, 0, 0.05))
    o = oracle_mod.Oracle(m)
    q, v, ws = _settle(o, m, robots.qpos0(m), 400)
    I = 0.4 * 1.0 * 0.05 ** 2

    def resid(r):
        imp = imp_ref(r)
        A = 1.0 + (1.0 + (0.05 - r / 2) ** 2 / I)
        return 4 * imp ** 2 * K_REF * r / ((1 - imp) * A) - 9.81

    r_star = brentq(resid, 1e-6, 9e-4, xtol=1e-18)
    assert abs(r_star - 3.98e-4) < 1e-6
    assert abs((0.05 - q[2]) / r_star - 1) < 1e-6
    assert np.abs(v).max() < 1e-9


def test_resting_box_forces(oracle_mod):
    m = robots.free_body("box", size=(0.1, 0.1, 0.1), mass=1.0, pos=(0, 0, 0.1))
    o = oracle_mod.Oracle(m)
    q, v, ws = _settle(o, m, robots.qpos0(m), 400)
    t = o.forward(q, v, qacc_ws=ws)
    assert t["ncon"] == 4
    fn = t["cforce"][:, 0]
    assert abs(fn.sum() / 9.81 - 1) < 1e-6
    np.testing.assert_allclose(fn, fn.mean(), rtol=1e-6)
    # tangential forces cancel (they need not vanish per corner: each pyramid edge row has its own A)
    ft_world = sum(t["cforce"][i, 1] * t["frame"][i][1] + t["cforce"][i, 2] * t["frame"][i][2] for i in range(4))
    assert np.linalg.norm(ft_world) < 1e-6
    assert np.abs(v).max() < 1e-9


@pytest.mark.parametrize("theta,mu,slides,h", [(math.radians(30), 1.0, False, 0.05),
                                               (math.radians(30), 0.3, True, 0.005)])
def test_inclined_plane_friction(oracle_mod, theta, mu, slides, h):
    """Sticking cube (tan theta < mu) and sliding thin plate (tan theta > mu; thin so that the
    friction torque about the centre of mass cannot rock it): a = g (sin theta - mu cos theta)."""
    qg = robots.quat_axis_angle((1, 0, 0), theta)
    n = rot(qg)[:, 2]
    m = robots.free_body("box", size=(0.05 if not slides else 0.1, 0.05 if not slides else 0.1, h), mass=1.0,
                         ground_quat=qg, friction=mu)
    o = oracle_mod.Oracle(m)
    x = n * (h - 2e-4)
    q0 = np.concatenate([x, qg])
    q, v, ws = _settle(o, m, q0, 100)
    down = np.cross(n, np.cross([0, 0, -1.0], n))
    down /= np.linalg.norm(down)
    s0, v0 = q[:3] @ down, v[:3] @ down
    dt = m["opt"]["timestep"]
    q, v, ws = q[None].copy(), v[None].copy(), ws[None].copy()
    for _ in range(100):
        o.step(np.zeros((1, 0)), q, v, ws)
    v1 = v[0, :3] @ down
    if slides:
        acc = (v1 - v0) / (100 * dt)
        exp = 9.81 * (math.sin(theta) - mu * math.cos(theta))
        assert abs(acc / exp - 1) < 0.02
    else:
        # the soft friction rows act through aref = -b v, so a sticking box creeps at a small
        # constant speed while the contact forces exactly balance gravity
        assert abs(v1 - v0) < 1e-7 and 0 <= v1 < 1e-2
        t = o.forward(q[0], v[0], qacc_ws=ws[0])
        F = sum(t["cforce"][i] @ t["frame"][i] for i in range(t["ncon"]))
        np.testing.assert_allclose(F, [0, 0, 9.81], atol=1e-6 * 9.81)


# ---------------------------------------------------------------- Newton solver
def _problem(t):
    M, a0, J, aref, D = t["M"], t["a0"], t["J"], t["aref"], t["D"]

    def f(a):
        jar = J @ a - aref
        return 0.5 * (a - a0) @ M @ (a - a0) + 0.5 * np.sum(D * np.minimum(jar, 0) ** 2)

    def g(a):
        jar = J @ a - aref
        return M @ (a - a0) + J.T @ (D * np.minimum(jar, 0))

    return f, g


@pytest.mark.parametrize("seed", range(4))
def test_newton_converged_matches_scipy(oracle_mod, seed):
    rng = np.random.default_rng(100 + seed)
    m = robots.free_body("box", size=(0.1, 0.07, 0.05), mass=1.3, friction=0.8)
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
    assert np.linalg.norm(g(t["qacc"])) < 1e-8 * o.meaninertia * o.nv * 10
    assert np.all(t["efc_force"] >= 0)
    # mirror mode with at most 4 iterations never does worse than its starting point
    o.set_mode("mirror")
    t4 = o.forward(q, v)
    assert t4["niter"] <= 4 and f(t4["qacc"]) <= f(t4["a0"]) + 1e-12


def test_warm_start_at_optimum_is_kept(oracle_mod):
    m = robots.free_body("box", size=(0.1, 0.07, 0.05), mass=1.3, friction=0.8)
    o = oracle_mod.Oracle(m)
    o.set_mode("converged")
    q = np.concatenate([[0, 0, 0.04], robots.quat_axis_angle((1, 1, 0), 0.2)])
    v = np.array([0.1, 0, -0.2, 0, 0.3, 0])
    t = o.forward(q, v)
    o.set_mode("mirror")
    t2 = o.forward(q, v, qacc_ws=t["qacc"])
    assert t2["niter"] == 0
    np.testing.assert_allclose(t2["qacc"], t["qacc"], rtol=0, atol=0)


def test_no_contact_means_smooth_acceleration(oracle_mod):
    m = robots.quadruped()
    o = oracle_mod.Oracle(m)
    q = robots.qpos0(m); q[2] = 2.0
    t = o.forward(q, np.ones(18) * 0.1, ctrl=np.full(12, 0.3))
    assert t["ncon"] == 0
    np.testing.assert_array_equal(t["qacc"], t["a0"])
    np.testing.assert_allclose(t["M"] @ t["a0"], t["tau"] - t["bias"], rtol=1e-12, atol=1e-12)
    # position actuators: tau = kp (ctrl - q) - kd v on each driven hinge
    np.testing.assert_allclose(t["tau"][6:], 20 * (0.3 - q[7:]) - 0.5 * 0.1, rtol=1e-15)


# ---------------------------------------------------------------- box-box
def _table_cube(cube_pos, cube_quat=(1, 0, 0, 0), table_half=(0.3, 0.3, 0.2), h=0.025):
    mb = robots.ModelBuilder("table_cube", timestep=0.005, nsubsteps=1)
    mb.geom(0, "box", list(table_half), pos=(0, 0, table_half[2]), contype=0, conaffinity=1)
    b = mb.body("cube", 0, (0, 0, 1), 0.1, robots.box_inertia(0.1, h, h, h))
    mb.joint(b, "free")
    mb.geom(b, "box", [h, h, h], contype=1, conaffinity=0)
    m = mb.build()
    q = np.concatenate([cube_pos, cube_quat])
    return m, q


def test_box_box_resting_cube_corners(oracle_mod):
    dz = 2e-4
    m, q = _table_cube([0.1, -0.05, 0.4 + 0.025 - dz])
    o = oracle_mod.Oracle(m)
    assert o.maxcon == 8
    t = o.forward(q, np.zeros(6))
    assert t["ncon"] == 4
    np.testing.assert_allclose(t["frame"][:, 0], np.tile([0, 0, 1.0], (4, 1)), atol=1e-15)
    np.testing.assert_allclose(t["dist"], -dz, atol=1e-12)
    exp = {(0.1 + sx * 0.025, -0.05 + sy * 0.025) for sx in (-1, 1) for sy in (-1, 1)}
    got = {(round(p[0], 12), round(p[1], 12)) for p in t["pos"]}
    assert got == {(round(a, 12), round(b, 12)) for a, b in exp}
    np.testing.assert_allclose(t["pos"][:, 2], 0.4 - dz / 2, atol=1e-12)
    assert list(t["feature"]) == [0, 1, 2, 3]


def test_box_box_overhanging_cube_clipped(oracle_mod):
    dz = 1e-4
    x = 0.3 - 0.01       # cube spans x in [0.265, 0.315]: clipped at the table edge x = 0.3
    m, q = _table_cube([x, 0.0, 0.4 + 0.025 - dz])
    o = oracle_mod.Oracle(m)
    t = o.forward(q, np.zeros(6))
    assert t["ncon"] == 4
    xs = sorted(set(np.round(t["pos"][:, 0], 12)))
    np.testing.assert_allclose(xs, [x - 0.025, 0.3], atol=1e-12)
    ys = sorted(set(np.round(t["pos"][:, 1], 12)))
    np.testing.assert_allclose(ys, [-0.025, 0.025], atol=1e-12)
    np.testing.assert_allclose(t["dist"], -dz, atol=1e-12)


def test_box_box_rotated_cube(oracle_mod):
    dz = 3e-4
    qz = robots.quat_axis_angle((0, 0, 1), math.pi / 4)
    m, q = _table_cube([0.0, 0.0, 0.4 + 0.025 - dz], qz)
    t = oracle_mod.Oracle(m).forward(q, np.zeros(6))
    assert t["ncon"] == 4
    r = 0.025 * math.sqrt(2)
    pts = {(round(p[0], 10), round(p[1], 10)) for p in t["pos"]}
    assert pts == {(round(a, 10), round(b, 10)) for a, b in [(r, 0), (-r, 0), (0, r), (0, -r)]}


def test_box_box_separated_and_touching(oracle_mod):
    m, q = _table_cube([0.0, 0.0, 0.4 + 0.025 + 1e-4])
    assert oracle_mod.Oracle(m).forward(q, np.zeros(6))["ncon"] == 0
    m, q = _table_cube([0.0, 0.0, 0.4 + 0.025])            # exactly touching: dist 0 is not < 0
    assert oracle_mod.Oracle(m).forward(q, np.zeros(6))["ncon"] == 0


@pytest.mark.parametrize("dx,dy", [(0.0, 0.0), (0.01, 0.1), (-0.015, -0.2)])
def test_box_box_edge_edge(oracle_mod, dx, dy):
    """A table edge (along y) pressed by a cube edge crossing it at right angles: one contact
    at the crossing, depth = the edge-edge overlap.  Offsets move the crossing away from
    both edges' midpoints."""
    qt = robots.quat_axis_angle((0, 1, 0), math.pi / 4)        # table turned: its top edge ridge along y
    mb = robots.ModelBuilder("edges", timestep=0.005, nsubsteps=1)
    mb.geom(0, "box", [0.3, 0.3, 0.3], pos=(0, 0, 0), quat=qt, contype=0, conaffinity=1)
    b = mb.body("cube", 0, (0, 0, 1), 0.1, robots.box_inertia(0.1, 0.025, 0.025, 0.025))
    mb.joint(b, "free")
    mb.geom(b, "box", [0.025, 0.025, 0.025], contype=1, conaffinity=0)
    m = mb.build()
    qc = robots.quat_axis_angle((1, 0, 0), math.pi / 4)        # cube turned: its bottom edge along x
    ridge = 0.3 * math.sqrt(2)
    pen = 1e-3
    zc = ridge + 0.025 * math.sqrt(2) - pen
    t = oracle_mod.Oracle(m).forward(np.concatenate([[dx, dy, zc], qc]), np.zeros(6))
    assert t["ncon"] == 1 and t["feature"][0] == 0
    np.testing.assert_allclose(t["dist"][0], -pen, atol=1e-12)
    np.testing.assert_allclose(t["frame"][0][0], [0, 0, 1], atol=1e-12)
    np.testing.assert_allclose(t["pos"][0], [0, dy, ridge - pen / 2], atol=1e-12)


def _box_vertices(center, R, half):
    s = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], float)
    return center + (s * half) @ R.T


def _overlap(va, vb, u):
    pa, pb = va @ u, vb @ u
    return min(pa.max() - pb.min(), pb.max() - pa.min())


def test_box_box_depth_is_minimal_overlap(oracle_mod):
    """Random orientations: the reported normal carries the smallest projection overlap of the
    two boxes over all directions (checked against a dense direction sample), and no contact is
    deeper than that overlap."""
    rng = np.random.default_rng(7)
    k = np.arange(40000) + 0.5
    phi = np.arccos(1 - 2 * k / len(k))
    th = math.pi * (1 + 5 ** 0.5) * k
    dirs = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    half_t = np.array([0.3, 0.3, 0.2])
    half_c = np.array([0.025, 0.025, 0.025])
    seen = 0
    for _ in range(12):
        qc = rng.normal(size=4)
        qc /= np.linalg.norm(qc)
        Rc = rot(qc)
        zext = np.abs(Rc[2]) @ half_c
        pen = rng.uniform(1e-4, 4e-3)
        c = np.array([rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), 0.4 + zext - pen])
        m, q = _table_cube(c, qc)
        t = oracle_mod.Oracle(m).forward(q, np.zeros(6))
        assert t["ncon"] >= 1
        vt = _box_vertices(np.array([0, 0, 0.2]), np.eye(3), half_t)
        vc = _box_vertices(c, Rc, half_c)
        n = t["frame"][0, 0]
        ov = _overlap(vt, vc, n)
        ovs = np.array([_overlap(vt, vc, d) for d in dirs])
        best, u = ovs.min(), dirs[ovs.argmin()]
        for r in (0.03, 3e-3, 3e-4):            # refine around the best direction found so far
            cap = u + r * rng.normal(size=(4000, 3))
            cap /= np.linalg.norm(cap, axis=1, keepdims=True)
            o2 = np.array([_overlap(vt, vc, d) for d in cap])
            if o2.min() < best:
                best, u = o2.min(), cap[o2.argmin()]
        assert ov <= best + 1e-9
        assert ov >= best - 2e-5
        assert np.all(-t["dist"][: t["ncon"]] <= ov + 1e-12)
        seen += t["ncon"]
    assert seen > 12


def test_box_box_cube_settles_on_table(oracle_mod):
    """The arm-and-cube scene: the cube dropped 1 mm onto the static table comes to rest on four
    corner contacts that together carry exactly its weight."""
    m = robots.arm_box()
    o = oracle_mod.Oracle(m)
    q = np.array([robots.qpos0(m)], np.float64)
    v = np.zeros((1, o.nv))
    ws = np.zeros((1, o.nv))
    st = np.zeros(1, np.uint32)
    for _ in range(60):
        _, c = o.step(np.zeros((1, o.nu)), q, v, ws, status=st, contacts=True)
    n = c["ncon"][0]
    assert st[0] == 0 and n == 4
    assert all(tuple(g) == (1, len(m["geoms"]) - 1) for g in c["geom"][0, :n])
    np.testing.assert_allclose(c["force"][0, :n, 0].sum(), 0.1 * 9.81, rtol=1e-6)
    assert np.abs(v[0, -6:]).max() < 1e-6
    assert abs(q[0, -7] - 0.5) < 1e-12 and 0.4 + 0.025 - 1e-3 < q[0, -5] < 0.4 + 0.025


def test_newton_iteration_cap_status(oracle_mod):
    """Status bit 1 reports a Newton loop stopped by the iteration cap: set with a single
    iteration on a contact-rich state, clear when the loop may converge."""
    import copy
    m = robots.humanoid()
    q = np.array([robots.qpos0(m)], np.float64)
    q[0, 2] -= 0.02                      # pressed into the floor: many active rows
    v = np.zeros((1, len(q[0]) - 1))
    m1 = copy.deepcopy(m)
    m1["opt"]["iterations"] = 1
    o1 = oracle_mod.Oracle(m1)
    st = np.zeros(1, np.uint32)
    o1.step(np.zeros((1, o1.nu)), q.copy(), v.copy(), np.zeros((1, o1.nv)), status=st)
    assert st[0] & 2
    m50 = copy.deepcopy(m)
    m50["opt"]["iterations"] = 50
    o50 = oracle_mod.Oracle(m50)
    st = np.array([2], np.uint32)        # cleared at the start of the step
    o50.step(np.zeros((1, o50.nu)), q.copy(), v.copy(), np.zeros((1, o50.nv)), status=st)
    assert st[0] == 0


# ---------------------------------------------------------------- sphere vs static box
def _box_ball(ball_pos, box_quat=(1, 0, 0, 0), box_half=(0.3, 0.2, 0.1), box_pos=(0.0, 0.0, 0.1), r=0.05,
              gravity=(0, 0, -9.81), mass=0.5):
    """A free ball (radius r) and a static box on the world body."""
    mb = robots.ModelBuilder("box_ball", timestep=0.005, nsubsteps=1, gravity=list(gravity))
    mb.geom(0, "box", list(box_half), pos=box_pos, quat=box_quat, contype=0, conaffinity=1)
    b = mb.body("ball", 0, (0, 0, 1), mass, robots.sphere_inertia(mass, r))
    mb.joint(b, "free")
    mb.geom(b, "sphere", [r], contype=1, conaffinity=0)
    m = mb.build()
    return m, np.concatenate([ball_pos, [1.0, 0, 0, 0]])


def _box_surface_points(box_pos, box_quat, half, n=121):
    """Dense grid on the box's six faces, world frame (brute-force closest point)."""
    g = np.linspace(-1, 1, n)
    A, B = np.meshgrid(g, g)
    pts = []
    for ax in range(3):
        o1, o2 = [i for i in range(3) if i != ax]
        for sgn in (-1, 1):
            P = np.zeros((A.size, 3))
            P[:, ax] = sgn * half[ax]
            P[:, o1] = A.ravel() * half[o1]
            P[:, o2] = B.ravel() * half[o2]
            pts.append(P)
    P = np.concatenate(pts)
    return P @ rot(box_quat).T + np.asarray(box_pos)


def test_sphere_on_box_face(oracle_mod):
    """A ball 1e-4 into the top face: one contact, normal from the ball down into the box, the
    point halfway between the surfaces."""
    dz = 1e-4
    m, q = _box_ball([0.1, -0.05, 0.2 + 0.05 - dz])
    t = oracle_mod.Oracle(m).forward(q, np.zeros(6))
    assert t["ncon"] == 1 and tuple(t["geom"][0]) == (1, 0)
    np.testing.assert_allclose(t["frame"][0, 0], [0, 0, -1.0], atol=1e-15)
    assert abs(t["dist"][0] + dz) < 1e-12
    np.testing.assert_allclose(t["pos"][0], [0.1, -0.05, 0.2 - dz / 2], atol=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_sphere_box_distance_brute_force(oracle_mod, seed):
    """Ball near a rotated box (centre outside or inside): the signed distance and contact
    normal against the closest point of a dense sampling of the box surface (the grid's
    spacing bounds the difference)."""
    rng = np.random.default_rng(seed)
    ax = rng.normal(size=3)
    quat = robots.quat_axis_angle(ax / np.linalg.norm(ax), rng.uniform(0, np.pi))
    half = (0.3, 0.2, 0.1)
    box_pos = (0.0, 0.0, 0.5)
    r = 0.05
    # a direction away from the box; place the ball just within the margin band
    while True:
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = np.asarray(box_pos) + d * rng.uniform(0.2, 0.45)
        P = _box_surface_points(box_pos, quat, half)
        dist = np.linalg.norm(P - c, axis=1)
        k = np.argmin(dist)
        if dist[k] - r < 0.03 and dist[k] > r * 0.5:
            break
    mb = robots.ModelBuilder("box_ball", timestep=0.005, nsubsteps=1)
    mb.geom(0, "box", list(half), pos=box_pos, quat=quat, contype=0, conaffinity=1)
    b = mb.body("ball", 0, (0, 0, 1), 0.5, robots.sphere_inertia(0.5, r))
    mb.joint(b, "free")
    mb.geom(b, "sphere", [r], contype=1, conaffinity=0, margin=0.05)
    m = mb.build()
    t = oracle_mod.Oracle(m).forward(np.concatenate([c, [1.0, 0, 0, 0]]), np.zeros(6))
    assert t["ncon"] == 1
    spacing = 2 * max(half) / 120
    inside = np.all(np.abs(rot(quat).T @ (c - np.asarray(box_pos))) <= np.asarray(half))
    sgn = -1.0 if inside else 1.0        # a centre inside is -(depth to the nearest face) from it
    assert abs(t["dist"][0] - (sgn * dist[k] - r)) <= spacing
    n_bf = sgn * (P[k] - c) / dist[k]    # from the ball towards the box
    assert np.dot(t["frame"][0, 0], n_bf) > 1 - 5 * spacing / dist[k]
    # the point lies on the segment from the centre along the normal, halfway into the gap
    np.testing.assert_allclose(t["pos"][0], c + t["frame"][0, 0] * (r + t["dist"][0] / 2), atol=1e-12)


def test_sphere_center_inside_box(oracle_mod):
    """Centre inside the box: the nearest face wins, depth = r + distance to that face."""
    m, q = _box_ball([0.25, 0.0, 0.12])          # x face 0.05 away, z top 0.08 away
    t = oracle_mod.Oracle(m).forward(q, np.zeros(6))
    assert t["ncon"] == 1
    np.testing.assert_allclose(t["frame"][0, 0], [-1.0, 0, 0], atol=1e-15)
    assert abs(t["dist"][0] + (0.05 + 0.05)) < 1e-12


def test_sphere_box_separated(oracle_mod):
    m, q = _box_ball([0.0, 0.0, 0.2 + 0.05 + 1e-3])
    assert oracle_mod.Oracle(m).forward(q, np.zeros(6))["ncon"] == 0


def test_ball_rests_on_box(oracle_mod):
    """Dropped on the box, the ball comes to rest on the face with its contact carrying its
    weight (normal force = m g, no tangential force)."""
    o = oracle_mod.Oracle(_box_ball([0.05, 0.02, 0.3])[0])
    q = np.array([[0.05, 0.02, 0.3, 1.0, 0, 0, 0]]); v = np.zeros((1, 6)); ws = np.zeros((1, 6))
    for _ in range(600):
        o.step(np.zeros((1, 0)), q, v, ws)
    t = o.forward(q[0], v[0], None, ws[0])
    assert t["ncon"] == 1
    assert abs(t["cforce"][0, 0] - 0.5 * 9.81) < 1e-6 * 0.5 * 9.81
    assert np.abs(t["cforce"][0, 1:]).max() < 1e-9
    assert np.abs(v).max() < 1e-6
    assert 0.2 + 0.05 - 1e-3 < q[0, 2] < 0.2 + 0.05


# ---------------------------------------------------------------- frictionless contacts (condim 1)
def _incline_box(theta, box_condim, plane_condim=1, h=0.05):
    """A free box resting on a plane tilted by theta about +y (downhill along the plane's +x)."""
    mb = robots.ModelBuilder("incline", timestep=0.002, nsubsteps=1)
    mb.geom(0, "plane", [0, 0, 0], quat=robots.quat_axis_angle([0, 1, 0], theta), contype=0, conaffinity=1)
    mb.geoms[-1]["condim"] = plane_condim
    b = mb.body("box", 0, (0, 0, 1), 1.0, robots.box_inertia(1.0, h, h, h))
    mb.joint(b, "free")
    mb.geom(b, "box", [h, h, h], contype=1, conaffinity=0)
    mb.geoms[-1]["condim"] = box_condim
    m = mb.build()
    R = rot(robots.quat_axis_angle([0, 1, 0], theta))
    n = R[:, 2]
    q = np.concatenate([n * (h - 1e-4), robots.quat_axis_angle([0, 1, 0], theta)])
    return m, q, R


def _slide(oracle_mod, m, q, steps):
    o = oracle_mod.Oracle(m)
    qq = q[None].copy(); v = np.zeros((1, 6)); ws = np.zeros((1, 6))
    vs = []
    for _ in range(steps):
        o.step(np.zeros((1, 0)), qq, v, ws)
        vs.append(v[0, :3].copy())
    return o, qq, v, np.array(vs)


def test_frictionless_box_slides_at_g_sin_theta(oracle_mod):
    """On a 0.3 rad incline a frictionless box (pair condim 1: one normal row per contact)
    accelerates downhill at g sin(theta) once the normal transient has settled."""
    th = 0.3
    m, q, R = _incline_box(th, 1)
    o, qq, v, vs = _slide(oracle_mod, m, q, 600)
    downhill = R[:, 0]                       # rotated about +y, the plane's +x axis points down the slope
    a = np.diff(vs @ downhill)[-100:] / 0.002
    np.testing.assert_allclose(a, 9.81 * np.sin(th), rtol=1e-6)
    t = o.forward(qq[0], v[0])
    assert t["ncon"] == 4 and t["J"].shape[0] == 4          # one row per contact
    assert np.abs(t["cforce"][:, 1:]).max() == 0.0
    assert abs(t["cforce"][:, 0].sum() - 9.81 * np.cos(th)) < 1e-6


def test_pair_condim_is_the_larger(oracle_mod):
    """A condim-1 box on a condim-3 plane keeps friction (the pair takes the larger), and with
    mu = 1 > tan(0.3) it stays nearly at rest where the frictionless box slides."""
    m, q, R = _incline_box(0.3, 1, plane_condim=3)
    o, qq, v, vs = _slide(oracle_mod, m, q, 600)
    t = o.forward(qq[0], v[0])
    assert t["J"].shape[0] == 4 * t["ncon"]
    assert np.abs(vs[-1]).max() < 0.05 * 9.81 * np.sin(0.3) * 600 * 0.002


def test_invalid_condim_rejected(oracle_mod):
    m, q, R = _incline_box(0.3, 2)
    with pytest.raises(Exception):
        oracle_mod.Oracle(m)


# ---------------------------------------------------------------- capsule against box
def _box_capsule(pos, quat=(1.0, 0, 0, 0), r=0.04, half_len=0.15, margin=0.0, box_quat=(1.0, 0, 0, 0)):
    """A static box (half sizes 0.3, 0.2, 0.1, top at z = 0.2) and a free capsule (radius r,
    segment half-length half_len along its z) at pos / quat."""
    mb = robots.ModelBuilder("box_capsule", timestep=0.002, nsubsteps=1)
    mb.geom(0, "box", [0.3, 0.2, 0.1], pos=(0.0, 0.0, 0.1), quat=box_quat, contype=0, conaffinity=1)
    b = mb.body("capsule", 0, (0, 0, 1), 0.8, robots.capsule_inertia(0.8, r, 2 * half_len))
    mb.joint(b, "free")
    mb.geom(b, "capsule", [r, half_len], contype=1, conaffinity=0, margin=margin)
    return mb.build(), np.concatenate([pos, quat])


def test_capsule_lying_on_box_face(oracle_mod):
    """A capsule lying along x, 1e-4 into the top face: two contacts (its ends, features 0 and
    1), each normal from the capsule down into the box, points halfway between the surfaces."""
    dz, r, hl = 1e-4, 0.04, 0.15
    quat = robots.quat_axis_angle([0, 1, 0], np.pi / 2)      # capsule z along world x
    m, q = _box_capsule([0.05, 0.02, 0.2 + r - dz], quat, r, hl)
    t = oracle_mod.Oracle(m).forward(q, np.zeros(6))
    assert t["ncon"] == 2 and list(t["feature"]) == [0, 1]
    ends = [np.array([0.05, 0.02, 0.2 + r - dz]) + s * hl * rot(quat)[:, 2] for s in (-1, 1)]
    for i in range(2):
        np.testing.assert_allclose(t["frame"][i, 0], [0, 0, -1.0], atol=1e-12)
        assert abs(t["dist"][i] + dz) < 1e-12
        np.testing.assert_allclose(t["pos"][i], ends[i] - [0, 0, r - dz / 2], atol=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_capsule_box_ends_brute_force(oracle_mod, seed):
    """A capsule at a random pose near a rotated box: each end listed exactly when its sphere's
    signed distance to the box (brute force over a dense sampling of the box surface) is within
    the margin, with that distance and normal."""
    rng = np.random.default_rng(100 + seed)
    ax = rng.normal(size=3)
    box_quat = robots.quat_axis_angle(ax / np.linalg.norm(ax), rng.uniform(0, np.pi))
    half, box_pos, r, hl, margin = (0.3, 0.2, 0.1), np.array([0.0, 0.0, 0.1]), 0.04, 0.15, 0.05
    cq = rng.normal(size=4)
    cq /= np.linalg.norm(cq)
    P = _box_surface_points(box_pos, box_quat, half)
    Rb = rot(box_quat)
    while True:
        d = rng.normal(size=3)
        c = box_pos + d / np.linalg.norm(d) * rng.uniform(0.15, 0.5)
        ends = [c + s * hl * rot(cq)[:, 2] for s in (-1, 1)]
        sd = []
        for e in ends:
            dist = np.linalg.norm(P - e, axis=1)
            k = np.argmin(dist)
            inside = np.all(np.abs(Rb.T @ (e - box_pos)) <= np.asarray(half))
            sd.append(((-1.0 if inside else 1.0) * dist[k] - r, P[k], inside, dist[k]))
        if any(x[0] < margin - 0.01 for x in sd) and all(abs(x[0] - margin) > 0.01 for x in sd):
            break
    mb = robots.ModelBuilder("box_capsule", timestep=0.005, nsubsteps=1)
    mb.geom(0, "box", list(half), pos=box_pos, quat=box_quat, contype=0, conaffinity=1)
    b = mb.body("capsule", 0, (0, 0, 1), 0.8, robots.capsule_inertia(0.8, r, 2 * hl))
    mb.joint(b, "free")
    mb.geom(b, "capsule", [r, hl], contype=1, conaffinity=0, margin=margin)
    t = oracle_mod.Oracle(mb.build()).forward(np.concatenate([c, cq]), np.zeros(6))
    spacing = 2 * max(half) / 120
    listed = [f for f in range(2) if sd[f][0] < margin]
    assert list(t["feature"]) == listed
    for i, f in enumerate(listed):
        dist_bf, Pk, inside, dk = sd[f]
        assert abs(t["dist"][i] - dist_bf) <= spacing
        n_bf = (-1.0 if inside else 1.0) * (Pk - ends[f]) / dk
        assert np.dot(t["frame"][i, 0], n_bf) > 1 - 5 * spacing / dk
        np.testing.assert_allclose(t["pos"][i], ends[f] + t["frame"][i, 0] * (r + t["dist"][i] / 2), atol=1e-12)


def test_capsule_rests_on_box(oracle_mod):
    """Dropped flat onto the box, the capsule comes to rest on its two ends, whose normal forces
    carry its weight (each half, by symmetry); their tangential forces cancel in total (as the
    corners of a resting box's do, not each one: R31)."""
    r, hl, mass = 0.04, 0.15, 0.8
    quat = robots.quat_axis_angle([0, 1, 0], np.pi / 2)
    m, q0 = _box_capsule([0.0, 0.0, 0.2 + r + 0.01], quat, r, hl)
    o = oracle_mod.Oracle(m)
    q = q0[None].copy(); v = np.zeros((1, 6)); ws = np.zeros((1, 6))
    for _ in range(1500):
        o.step(np.zeros((1, 0)), q, v, ws)
    t = o.forward(q[0], v[0], None, ws[0])
    assert t["ncon"] == 2
    np.testing.assert_allclose(t["cforce"][:, 0], [mass * 9.81 / 2] * 2, rtol=1e-5)
    np.testing.assert_allclose(t["frame"][0], t["frame"][1], atol=1e-9)
    assert np.abs(t["cforce"][:, 1:].sum(0)).max() < 1e-6
    assert np.abs(v).max() < 1e-6
