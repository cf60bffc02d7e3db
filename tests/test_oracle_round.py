"""Pins of the oracle's sphere and capsule pairs (self-collision of limbs): the contact of two
spheres in closed form, capsule-capsule and sphere-capsule distances, points and normals against
a bounded numerical minimisation over the two segments' parameters, and a capsule resting
crosswise on a static capsule carrying its weight on one contact."""
import numpy as np
from scipy.optimize import minimize

from helpers import rot
from workloads import robots


def _pair(kind1, size1, kind2, size2, pose1, pose2, moving=(True, True)):
    mb = robots.ModelBuilder("round", timestep=0.002, nsubsteps=1, gravity=[0, 0, 0])
    for k, (kind, size, (pos, quat), mov) in enumerate(zip((kind1, kind2), (size1, size2), (pose1, pose2), moving)):
        if mov:
            b = mb.body(f"b{k}", 0, pos, 1.0, [0.01, 0.01, 0.01], quat=quat)
            mb.joint(b, "free")
            mb.geom(b, kind, size, contype=1, conaffinity=1)
        else:
            mb.geom(0, kind, size, pos=pos, quat=quat, contype=1, conaffinity=1)
    return mb.build()


def _segment(kind, size, pos, quat):
    h = size[1] if kind == "capsule" else 0.0
    ax = rot(quat)[:, 2]
    return np.asarray(pos) - h * ax, np.asarray(pos) + h * ax


def _brute(seg1, seg2):
    """min over s, t in [0, 1] of |p1(s) - p2(t)|: grid start, then bounded quasi-Newton."""
    (a1, b1), (a2, b2) = seg1, seg2
    f = lambda z: np.sum((a1 + z[0] * (b1 - a1) - a2 - z[1] * (b2 - a2)) ** 2)
    g = np.linspace(0, 1, 41)
    z0 = min(((s, t) for s in g for t in g), key=f)
    r = minimize(f, z0, method="L-BFGS-B", bounds=[(0, 1), (0, 1)], options={"ftol": 1e-20, "gtol": 1e-14})
    s, t = r.x
    return a1 + s * (b1 - a1), a2 + t * (b2 - a2)


def _state(m):
    q = np.concatenate([np.concatenate([b["pos"], b["quat"]]) for b in m["bodies"][1:]]) if len(m["bodies"]) > 1 else np.zeros(0)
    return q


def test_sphere_sphere_closed_form(oracle_mod):
    rng = np.random.default_rng(5)
    for _ in range(20):
        c1, c2 = rng.normal(0, 0.05, 3), rng.normal(0, 0.05, 3)
        m = _pair("sphere", [0.04], "sphere", [0.03], (c1, [1, 0, 0, 0]), (c2, [1, 0, 0, 0]))
        t = oracle_mod.Oracle(m).forward(_state(m), np.zeros(12))
        dvec = c2 - c1
        dist = np.linalg.norm(dvec) - 0.07
        if dist >= 0:
            assert t["ncon"] == 0
            continue
        n = dvec / np.linalg.norm(dvec)
        assert t["ncon"] == 1
        np.testing.assert_allclose(t["dist"][0], dist, atol=1e-12)
        np.testing.assert_allclose(t["frame"][0][0], n, atol=1e-12)
        np.testing.assert_allclose(t["pos"][0], c1 + n * (0.04 + dist / 2), atol=1e-12)


def test_capsule_pairs_against_brute_force(oracle_mod):
    """Capsule-capsule and sphere-capsule at random poses near each other: the contact's distance
    to 1e-9, its normal and point to 1e-6, against a numerical minimisation over the segments."""
    rng = np.random.default_rng(6)
    checked = 0
    for trial in range(60):
        kinds = ("capsule", "capsule") if trial % 2 == 0 else ("sphere", "capsule")
        sizes = ([0.03, 0.1], [0.04, 0.08]) if kinds[0] == "capsule" else ([0.05], [0.04, 0.08])
        poses = []
        for k in range(2):
            qq = rng.normal(size=4); qq /= np.linalg.norm(qq)
            poses.append((rng.normal(0, 0.06, 3), qq))
        m = _pair(kinds[0], sizes[0], kinds[1], sizes[1], poses[0], poses[1])
        t = oracle_mod.Oracle(m).forward(_state(m), np.zeros(12))
        s1, s2 = _segment(kinds[0], sizes[0], *poses[0]), _segment(kinds[1], sizes[1], *poses[1])
        c1, c2 = _brute(s1, s2)
        r1, r2 = sizes[0][0], sizes[1][0]
        dist = np.linalg.norm(c2 - c1) - r1 - r2
        if dist >= -1e-9 or np.linalg.norm(c2 - c1) < 1e-3:
            continue
        checked += 1
        assert t["ncon"] == 1
        n = (c2 - c1) / np.linalg.norm(c2 - c1)
        np.testing.assert_allclose(t["dist"][0], dist, atol=1e-9)
        np.testing.assert_allclose(t["frame"][0][0], n, atol=1e-6)
        np.testing.assert_allclose(t["pos"][0], c1 + n * (r1 + dist / 2), atol=1e-6)
    assert checked >= 20


def test_capsule_rests_across_a_capsule(oracle_mod):
    """A 0.5 kg capsule lying crosswise on a static horizontal capsule (gravity on): one contact
    whose normal force is m g at rest."""
    qx = robots.quat_axis_angle((0, 1, 0), np.pi / 2)     # capsule along world x
    qy = robots.quat_axis_angle((1, 0, 0), np.pi / 2)     # capsule along world y
    mb = robots.ModelBuilder("cross", timestep=0.002, nsubsteps=1)
    mb.geom(0, "capsule", [0.03, 0.2], pos=(0, 0, 0.1), quat=qx, contype=1, conaffinity=1)
    b = mb.body("bar", 0, (0, 0, 0.1 + 0.06), 0.5, robots.capsule_inertia(0.5, 0.03, 0.3), quat=qy)
    mb.joint(b, "free")
    mb.geom(b, "capsule", [0.03, 0.15], contype=1, conaffinity=1)
    m = mb.build()
    o = oracle_mod.Oracle(m)
    q = _state(m)[None].copy(); v = np.zeros((1, 6)); ws = np.zeros((1, 6))
    for _ in range(1500):
        o.step(np.zeros((1, 0)), q, v, ws)
    t = o.forward(q[0], v[0], qacc_ws=ws[0])
    assert t["ncon"] == 1 and np.abs(v).max() < 1e-8
    np.testing.assert_allclose(t["cforce"][0] @ t["frame"][0], [0, 0, 0.5 * 9.81], atol=1e-6)
