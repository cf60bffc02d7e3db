"""Pins of the oracle's height-field contacts: a flat grid is the plane, a planar sloped grid is
the tilted plane, the triangle under a point is the one an exhaustive search finds, points
off the grid make no contact, and a ball rests on a slope with its weight carried."""
import numpy as np
import pytest

from helpers import rot
from workloads import robots

SX, SY = 1.0, 0.8          # half extents of the grid


def _scene(heights, other="sphere", size=(0.05,), pos=(0, 0, 1), quat=(1, 0, 0, 0), plane_quat=None, plane_z=0.0,
           margin=0.0):
    """A free geom over a height field (heights [nrow, ncol]), or over a plane when heights is None."""
    mb = robots.ModelBuilder("hf", timestep=0.002, nsubsteps=1)
    if heights is None:
        mb.geom(0, "plane", [0, 0, 0], pos=(0, 0, plane_z), quat=plane_quat or (1, 0, 0, 0), contype=0, conaffinity=1)
    else:
        mb.hfield(heights)
        mb.geom(0, "hfield", [SX, SY, 0], contype=0, conaffinity=1)
    inertia = {"sphere": lambda: robots.sphere_inertia(1.0, size[0]),
               "capsule": lambda: robots.capsule_inertia(1.0, size[0], 2 * size[1]),
               "box": lambda: robots.box_inertia(1.0, *size)}[other]()
    b = mb.body("b", 0, (0, 0, 1), 1.0, inertia)
    mb.joint(b, "free")
    mb.geom(b, other, list(size), contype=1, conaffinity=0, margin=margin)
    return mb.build(), np.concatenate([pos, quat])


SHAPES = [("sphere", (0.05,)), ("capsule", (0.04, 0.12)), ("box", (0.06, 0.04, 0.03))]


@pytest.mark.parametrize("other,size", SHAPES)
def test_flat_grid_is_the_plane(oracle_mod, other, size):
    rng = np.random.default_rng(1)
    flat = np.zeros((7, 9))
    for _ in range(10):
        q = rng.normal(size=4); q /= np.linalg.norm(q)
        pos = [rng.uniform(-0.6, 0.6), rng.uniform(-0.5, 0.5), rng.uniform(0.0, 0.08)]
        mh, qq = _scene(flat, other, size, pos, q)
        mp, _ = _scene(None, other, size, pos, q)
        th = oracle_mod.Oracle(mh).forward(qq, np.zeros(6))
        tp = oracle_mod.Oracle(mp).forward(qq, np.zeros(6))
        assert th["ncon"] == tp["ncon"]
        assert list(th["feature"]) == list(tp["feature"])
        for k in ("dist", "pos", "frame"):
            np.testing.assert_allclose(th[k], tp[k], atol=1e-12)


@pytest.mark.parametrize("other,size", SHAPES)
def test_planar_sloped_grid_is_the_tilted_plane(oracle_mod, other, size):
    """Heights a x + b y + c sampled on the grid: every triangle lies in that plane, so the
    contacts are those of a plane through (0, 0, c) with normal (-a, -b, 1) / norm."""
    a, b, c = 0.2, -0.1, 0.03
    xs = np.linspace(-SX, SX, 9)
    ys = np.linspace(-SY, SY, 7)
    H = a * xs[None, :] + b * ys[:, None] + c
    n = np.array([-a, -b, 1.0]) / np.linalg.norm([-a, -b, 1.0])
    # the plane geom's rotation takes +z to n (about the axis z x n)
    ax = np.cross([0, 0, 1.0], n)
    qp = robots.quat_axis_angle(ax / np.linalg.norm(ax), np.arccos(n[2]))
    rng = np.random.default_rng(2)
    for _ in range(10):
        q = rng.normal(size=4); q /= np.linalg.norm(q)
        x, y = rng.uniform(-0.6, 0.6), rng.uniform(-0.5, 0.5)
        pos = [x, y, a * x + b * y + c + rng.uniform(0.0, 0.08)]
        mh, qq = _scene(H, other, size, pos, q)
        mp, _ = _scene(None, other, size, pos, q, plane_quat=qp, plane_z=c)
        th = oracle_mod.Oracle(mh).forward(qq, np.zeros(6))
        tp = oracle_mod.Oracle(mp).forward(qq, np.zeros(6))
        assert th["ncon"] == tp["ncon"]
        for k in ("dist", "pos", "frame"):
            np.testing.assert_allclose(th[k], tp[k], atol=1e-12)


def _exhaustive_triangle_plane(H, p):
    """The plane (unit normal with positive z, a vertex) of the grid triangle containing the
    horizontal point p, found by testing every triangle's barycentric coordinates."""
    nr, nc = H.shape
    xs = np.linspace(-SX, SX, nc)
    ys = np.linspace(-SY, SY, nr)
    V = lambda i, j: np.array([xs[j], ys[i], H[i, j]])
    for i in range(nr - 1):
        for j in range(nc - 1):
            for tri in ((V(i, j), V(i, j + 1), V(i + 1, j + 1)), (V(i, j), V(i + 1, j + 1), V(i + 1, j))):
                A = np.array([[tri[1][0] - tri[0][0], tri[2][0] - tri[0][0]],
                              [tri[1][1] - tri[0][1], tri[2][1] - tri[0][1]]])
                l1, l2 = np.linalg.solve(A, p[:2] - tri[0][:2])
                if l1 >= -1e-12 and l2 >= -1e-12 and l1 + l2 <= 1 + 1e-12:
                    nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
                    return nrm / np.linalg.norm(nrm), tri[0]
    return None


def test_triangle_under_a_point_by_exhaustive_search(oracle_mod):
    """Random grid, ball centres at random points: the contact is against the plane of the
    triangle that an exhaustive barycentric search finds under the centre."""
    rng = np.random.default_rng(3)
    H = rng.uniform(-0.03, 0.03, (6, 8))
    r = 0.05
    for _ in range(40):
        x, y = rng.uniform(-SX, SX), rng.uniform(-SY, SY)
        pos = np.array([x, y, rng.uniform(0.0, 0.06)])
        m, qq = _scene(H, "sphere", (r,), pos, margin=0.2)
        t = oracle_mod.Oracle(m).forward(qq, np.zeros(6))
        nrm, p0 = _exhaustive_triangle_plane(H, pos)
        assert t["ncon"] == 1
        np.testing.assert_allclose(t["frame"][0, 0], nrm, atol=1e-12)
        assert abs(t["dist"][0] - (nrm @ (pos - p0) - r)) < 1e-12


def test_off_the_grid_no_contact(oracle_mod):
    m, qq = _scene(np.zeros((4, 4)), "sphere", (0.05,), (SX + 0.01, 0.0, 0.0), margin=0.5)
    assert oracle_mod.Oracle(m).forward(qq, np.zeros(6))["ncon"] == 0


def test_box_rests_on_a_slope(oracle_mod):
    """A box on a planar grid sloped by theta = atan(0.2) (mu = 1 > tan theta) comes to rest on
    four corners whose normal forces sum to m g cos(theta) and whose friction sums to
    m g sin(theta) up the slope."""
    a = 0.2
    xs = np.linspace(-SX, SX, 5)
    H = np.tile(a * xs, (4, 1))
    th = np.arctan(a)
    hz = 0.03
    n = np.array([-np.sin(th), 0.0, np.cos(th)])
    quat = robots.quat_axis_angle([0, 1, 0], -th)
    m, q0 = _scene(H, "box", (0.06, 0.04, hz), n * (hz + 1e-3), quat)
    o = oracle_mod.Oracle(m)
    q = q0[None].copy(); v = np.zeros((1, 6)); ws = np.zeros((1, 6))
    for _ in range(1500):
        o.step(np.zeros((1, 0)), q, v, ws)
    t = o.forward(q[0], v[0], None, ws[0])
    assert t["ncon"] == 4
    # world-frame resultant of the contact forces (rows of the frame: normal, t1, t2)
    F = sum(t["cforce"][i] @ t["frame"][i] for i in range(4))
    np.testing.assert_allclose(F @ n, 9.81 * np.cos(th), rtol=1e-4)
    np.testing.assert_allclose(F, [0.0, 0.0, 9.81], atol=1e-3 * 9.81)
