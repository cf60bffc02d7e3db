"""Pins of the oracle's elliptic friction cones: each contact's force is the projection of
-D jar onto the friction cone {f_n >= |f_t| / mu} in the metric of R = D^-1 (computed here by a
general constrained minimiser), the converged acceleration is stationary for the cost those
forces derive from, a sliding plate slides at the Coulomb rate g (sin theta - mu cos theta), a
sliding puck's friction opposes its velocity exactly (which the pyramid does not), and
frictionless contacts do not depend on the cone."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from helpers import rot
from workloads import robots


def _elliptic(m, impratio=1.0):
    m["opt"]["cone"] = "elliptic"
    m["opt"]["impratio"] = impratio
    return m


def _states(m, n, seed, height):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        qb = rng.normal(size=4); qb /= np.linalg.norm(qb)
        q = np.concatenate([[0, 0, height], qb])
        out.append((q, rng.normal(0, 0.7, 6)))
    return out


@pytest.mark.parametrize("impratio", [1.0, 3.0])
def test_contact_forces_are_the_cone_projection(oracle_mod, impratio):
    """Tilted boxes touching the plane at random velocities, Newton run to convergence: every
    contact's three row forces f are the projection of y = -D jar onto the cone
    K = {|f_t| <= mu f_n} in the metric R = D^-1, by the conditions that define it (f in K, the
    residual w = R (y - f) in the polar cone {w_n <= -mu |w_t|}, w.f = 0), all three zones
    (f = 0, f = y, f on the surface) occur, and the acceleration is stationary: M (a - a0) = J' f."""
    mu = 0.6
    m = _elliptic(robots.free_body("box", size=(0.1, 0.07, 0.05), mass=1.3, friction=mu), impratio)
    o = oracle_mod.Oracle(m)
    o.set_mode("converged")
    zones = set()
    for q, v in _states(m, 16, 31, 0.06):
        t = o.forward(q, v)
        if t["ncon"] == 0:
            continue
        J, D, f = t["J"], t["D"], t["efc_force"]
        assert J.shape[0] == 3 * t["ncon"]
        jar = J @ t["qacc"] - t["aref"]
        for c in range(t["ncon"]):
            r = slice(3 * c, 3 * c + 3)
            np.testing.assert_allclose(D[3 * c + 1:3 * c + 3], impratio * D[3 * c], rtol=1e-12)
            y = -D[r] * jar[r]
            fc = f[r]
            w = (y - fc) / D[r]
            sf = max(np.abs(y).max(), 1e-12)
            sw = max(np.abs(y / D[r]).max(), 1e-12)
            assert np.hypot(fc[1], fc[2]) <= mu * fc[0] + 1e-10 * sf
            assert w[0] + mu * np.hypot(w[1], w[2]) <= 1e-10 * sw
            assert abs(w @ fc) <= 1e-10 * sf * sw
            fz, wz = np.abs(fc).max() <= 1e-12 * sf, np.abs(w).max() <= 1e-12 * sw
            zones.add(0 if fz else (2 if wz else 1))
        g = t["M"] @ (t["qacc"] - t["a0"]) - J.T @ f
        assert np.abs(g).max() < 1e-9 * max(1.0, np.abs(J.T @ f).max())
    assert zones == {0, 1, 2}


def _slide(oracle_mod, m, q0, n):
    o = oracle_mod.Oracle(m)
    q = np.array(q0, float)[None]; v = np.zeros((1, 6)); ws = np.zeros((1, 6))
    for _ in range(n):
        o.step(np.zeros((1, 0)), q, v, ws)
    return o, q, v, ws


@pytest.mark.parametrize("theta,mu,slides", [(math.radians(30), 1.0, False), (math.radians(30), 0.3, True)])
def test_incline_coulomb(oracle_mod, theta, mu, slides):
    """A thin plate on an incline: sticks with the contact forces balancing gravity when
    tan theta < mu; else slides at a = g (sin theta - mu cos theta) on average over 0.8 s, within
    0.5 % (the soft contact chatters while sliding, so shorter windows vary by several percent),
    with every loaded contact's force on the cone's surface, |f_t| = mu f_n."""
    qg = robots.quat_axis_angle((1, 0, 0), theta)
    n = rot(qg)[:, 2]
    h = 0.005
    m = _elliptic(robots.free_body("box", size=(0.1, 0.1, h), mass=1.0, ground_quat=qg, friction=mu,
                                   timestep=0.002))
    q0 = np.concatenate([n * (h - 2e-4), qg])
    o, q, v, ws = _slide(oracle_mod, m, q0, 100)
    down = np.cross(n, np.cross([0, 0, -1.0], n))
    down /= np.linalg.norm(down)
    v0 = v[0, :3] @ down
    loaded = 0
    for k in range(400):
        if slides and k % 10 == 0:
            t = o.forward(q[0], v[0], qacc_ws=ws[0])
            for fc in t["cforce"]:
                if fc[0] > 1e-3:
                    loaded += 1
                    assert abs(np.hypot(fc[1], fc[2]) - mu * fc[0]) < 1e-9 * fc[0]
        o.step(np.zeros((1, 0)), q, v, ws)
    v1 = v[0, :3] @ down
    if slides:
        acc = (v1 - v0) / (400 * 0.002)
        exp = 9.81 * (math.sin(theta) - mu * math.cos(theta))
        assert abs(acc / exp - 1) < 5e-3
        assert loaded >= 40
    else:
        t = o.forward(q[0], v[0], qacc_ws=ws[0])
        assert abs(v1 - v0) < 1e-6 and 0 <= v1 < 1e-2
        F = sum(t["cforce"][i] @ t["frame"][i] for i in range(t["ncon"]))
        np.testing.assert_allclose(F, [0, 0, 9.81], atol=1e-6 * 9.81)


@pytest.mark.parametrize("cone", ["elliptic", "pyramidal"])
def test_friction_opposes_the_sliding_velocity(oracle_mod, cone):
    """A ball sliding without spin diagonally across a flat plane (one contact, whose point slides
    along the ball's velocity): with the elliptic cone the friction force is antiparallel to the
    velocity (within 1e-6 rad) at every loaded step; the pyramid's is not (its four edges favour
    the frame axes)."""
    m = robots.free_body("sphere", size=(0.05,), mass=0.5, friction=0.4, timestep=0.002)
    if cone == "elliptic":
        _elliptic(m)
    o, q, v, ws = _slide(oracle_mod, m, [0, 0, 0.05, 1, 0, 0, 0], 300)
    v[0, :2] = [2.0, 0.7]
    worst, loaded = 0.0, 0
    for _ in range(100):
        t = o.forward(q[0], v[0], qacc_ws=ws[0])
        if t["ncon"] and t["cforce"][0, 0] > 1e-3:
            loaded += 1
            F = t["cforce"][0] @ t["frame"][0]
            vt = v[0, :2] / np.linalg.norm(v[0, :2])
            worst = max(worst, abs(math.atan2(F[0] * vt[1] - F[1] * vt[0], -(F[0] * vt[0] + F[1] * vt[1]))))
        o.step(np.zeros((1, 0)), q, v, ws)
    assert loaded >= 10
    if cone == "elliptic":
        assert worst < 1e-6
    else:
        assert worst > 1e-3


def test_frictionless_contacts_ignore_the_cone(oracle_mod):
    """condim-1 contacts have the normal row only: pyramidal and elliptic steps are identical."""
    res = []
    for cone in ("pyramidal", "elliptic"):
        m = robots.free_body("box", size=(0.1, 0.07, 0.05), friction=0.5)
        for g in m["geoms"]:
            g["condim"] = 1
        if cone == "elliptic":
            _elliptic(m)
        o = oracle_mod.Oracle(m)
        q = np.concatenate([[0, 0, 0.06], robots.quat_axis_angle((1, 1, 0), 0.4)])[None]
        v = np.full((1, 6), 0.3); ws = np.zeros((1, 6))
        for _ in range(20):
            o.step(np.zeros((1, 0)), q, v, ws)
        res.append((q.copy(), v.copy()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


def test_elliptic_takes_condim_1_3_4_and_6(oracle_mod):
    m = _elliptic(robots.free_body("sphere", size=(0.1,)))
    for cd in (1, 3, 4, 6):
        m["geoms"][1]["condim"] = cd
        oracle_mod.Oracle(m)
    m["geoms"][1]["condim"] = 5
    with pytest.raises(Exception):
        oracle_mod.Oracle(m)
    m = robots.free_body("sphere", size=(0.1,))
    m["opt"]["impratio"] = 0.0
    with pytest.raises(Exception):
        oracle_mod.Oracle(m)
