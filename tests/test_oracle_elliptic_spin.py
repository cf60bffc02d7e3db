"""Pins of the oracle's elliptic cones with torsional and rolling friction (condim 4 and 6):
the contact's row forces (normal, two tangents, spin about the normal, rolling about the
tangents) are the projection of -D jar onto the cone {sum_i (f_i / mu_i)^2 <= f_n^2} in the
metric of R = D^-1 (checked by the conditions that define a projection onto a closed convex
cone), friction row i's regulariser is the normal's times mu^2 / (mu_i^2 impratio), a contact
without torsional (rolling) friction steps exactly as its condim-3 (condim-4) cone, a rolling
ball keeps its speed with condim 4 and loses it with condim 6, a slowly spinning ball loses its spin at the rate the cone's quadratic zone fixes
in closed form, and a fast-spinning one has its spin force on the cone's surface."""
import numpy as np
import pytest

from helpers import impedance
from workloads import robots


def _elliptic4(m, mu_spin, impratio=1.0, condim=4):
    m["opt"]["cone"] = "elliptic"
    m["opt"]["impratio"] = impratio
    for g in m["geoms"]:
        g["condim"] = condim
        g["friction_spin"] = mu_spin
    return m


def _states(n, seed, height):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        qb = rng.normal(size=4)
        qb /= np.linalg.norm(qb)
        out.append((np.concatenate([[0, 0, height], qb]), rng.normal(0, 0.7, 6)))
    return out


@pytest.mark.parametrize("condim,impratio", [(4, 1.0), (4, 4.0), (6, 1.0), (6, 4.0)])
def test_forces_are_the_anisotropic_cone_projection(oracle_mod, condim, impratio):
    """Tilted boxes touching the plane at random velocities, Newton run to convergence: per
    contact, D of the tangents is impratio D_n, of the spin impratio D_n (mu_spin / mu)^2 and of
    the rolling rows (condim 6) impratio D_n (mu_roll / mu)^2; the forces f lie in
    K = {f_n >= |(f_1 / mu, f_2 / mu, f_s / mu_spin, f_r1 / mu_roll, f_r2 / mu_roll)|}, the
    residual w = R (y - f) (y = -D jar) lies in K's polar cone
    {w_n <= -|(mu w_1, mu w_2, mu_spin w_s, mu_roll w_r1, mu_roll w_r2)|}, w . f = 0, all three
    zones occur, and M (a - a0) = J' f."""
    mu, mus, mur = 0.6, 0.05, 0.01
    m = _elliptic4(robots.free_body("box", size=(0.1, 0.07, 0.05), mass=1.3, friction=mu), mus, impratio, condim)
    for g in m["geoms"]:
        g["friction_roll"] = mur
    o = oracle_mod.Oracle(m)
    o.set_mode("converged")
    scale = np.array([1.0, mu, mu, mus, mur, mur])[:condim]
    zones = set()
    for q, v in _states(64, 37, 0.06):
        t = o.forward(q, v)
        if t["ncon"] == 0:
            continue
        J, D, f = t["J"], t["D"], t["efc_force"]
        assert J.shape[0] == condim * t["ncon"]
        jar = J @ t["qacc"] - t["aref"]
        for c in range(t["ncon"]):
            r = slice(condim * c, condim * c + condim)
            Dn = D[condim * c]
            np.testing.assert_allclose(D[r][1:], impratio * Dn * (scale[1:] / mu) ** 2, rtol=1e-12)
            y = -D[r] * jar[r]
            fc = f[r]
            w = (y - fc) / D[r]
            sf = max(np.abs(y).max(), 1e-12)
            sw = max(np.abs(y / D[r]).max(), 1e-12)
            assert np.linalg.norm(fc[1:] / scale[1:]) <= fc[0] + 1e-10 * sf / scale.min()
            assert w[0] + np.linalg.norm(w[1:] * scale[1:]) <= 1e-10 * sw
            assert abs(w @ fc) <= 1e-10 * sf * sw
            fz, wz = np.abs(fc).max() <= 1e-12 * sf, np.abs(w).max() <= 1e-12 * sw
            zones.add(0 if fz else (2 if wz else 1))
        g = t["M"] @ (t["qacc"] - t["a0"]) - J.T @ f
        assert np.abs(g).max() < 1e-9 * max(1.0, np.abs(J.T @ f).max())
    assert zones == {0, 1, 2}


def test_no_torsional_friction_steps_as_condim3(oracle_mod):
    """condim 4 with mu_spin = 0 gives the spin row D = 0, so its cone is the condim-3 cone: 30
    steps of a tumbling box agree with the condim-3 steps to 1e-12."""
    res = []
    for condim in (3, 4):
        m = _elliptic4(robots.free_body("box", size=(0.1, 0.07, 0.05), friction=0.5), 0.0, 2.0, condim)
        o = oracle_mod.Oracle(m)
        q = np.concatenate([[0, 0, 0.06], robots.quat_axis_angle((1, 1, 0), 0.4)])[None]
        v = np.full((1, 6), 0.3)
        ws = np.zeros((1, 6))
        for _ in range(30):
            o.step(np.zeros((1, 0)), q, v, ws)
        res.append((q.copy(), v.copy()))
    np.testing.assert_allclose(res[0][0], res[1][0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(res[0][1], res[1][1], rtol=0, atol=1e-12)


def test_no_rolling_friction_steps_as_condim4(oracle_mod):
    """condim 6 with mu_roll = 0 gives the rolling rows D = 0, so its cone is the condim-4 cone: 30
    steps of a tumbling box agree with the condim-4 steps to 1e-12."""
    res = []
    for condim in (4, 6):
        m = _elliptic4(robots.free_body("box", size=(0.1, 0.07, 0.05), friction=0.5), 0.03, 2.0, condim)
        for g in m["geoms"]:
            g["friction_roll"] = 0.0
        o = oracle_mod.Oracle(m)
        q = np.concatenate([[0, 0, 0.06], robots.quat_axis_angle((1, 1, 0), 0.4)])[None]
        v = np.full((1, 6), 0.3)
        ws = np.zeros((1, 6))
        for _ in range(30):
            o.step(np.zeros((1, 0)), q, v, ws)
        res.append((q.copy(), v.copy()))
    np.testing.assert_allclose(res[0][0], res[1][0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(res[0][1], res[1][1], rtol=0, atol=1e-12)


@pytest.mark.parametrize("condim,keeps_roll", [(4, True), (6, False)])
def test_rolling_kept_or_lost_by_condim(oracle_mod, condim, keeps_roll):
    """A ball rolling at 0.5 m/s on a plane with elliptic cones keeps its speed over 4 s to 0.1 %
    with condim 4 (no rolling friction) and loses at least 10 % of it with condim 6 (mu_roll
    0.002)."""
    m = _elliptic4(robots.free_body("sphere", size=(0.1,), pos=(0, 0, 0.1), timestep=0.002), 0.002, 1.0, condim)
    for g in m["geoms"]:
        g["friction_roll"] = 0.002
    o, q, v, ws = _rest_sphere(oracle_mod, m, 500)
    v[0, 0], v[0, 4] = 0.5, 5.0
    for _ in range(2000):
        o.step(np.zeros((1, 0)), q, v, ws)
    assert (abs(v[0, 0] - 0.5) < 5e-4) == keeps_roll and (v[0, 0] < 0.45) != keeps_roll


def _rest_sphere(oracle_mod, m, steps):
    o = oracle_mod.Oracle(m)
    q = np.array([[0, 0, 0.1, 1, 0, 0, 0.0]])
    v = np.zeros((1, 6))
    ws = np.zeros((1, 6))
    for _ in range(steps):
        o.step(np.zeros((1, 0)), q, v, ws)
    return o, q, v, ws


@pytest.mark.parametrize("impratio", [1.0, 4.0])
def test_slow_spin_decay_closed_form(oracle_mod, impratio):
    """A ball resting on a plane spinning slowly about the vertical: its contact stays inside the
    cone (every row active, cost |x|^2 / 2), the spin row decouples from the others (the ball's
    spin moves no contact point), and the quadratic cost gives I a_w = -D_s (a_w + b w) with
    D_s = impratio D_n (mu_spin / mu)^2, D_n = imp / ((1 - imp) A-hat_n), A-hat_n = 1 / m: one
    step scales w by 1 - dt D_s b / (I + D_s), imp taken at the ball's penetration."""
    mass, r, mu, mus, dt = 1.0, 0.1, 0.8, 0.02, 0.002
    m = _elliptic4(robots.free_body("sphere", size=(r,), mass=mass, pos=(0, 0, r), friction=mu,
                                    timestep=dt), mus, impratio)
    o, q, v, ws = _rest_sphere(oracle_mod, m, 500)
    v[0, 5] = 0.05
    I = 0.4 * mass * r * r
    b = 2.0 / (0.95 * 0.02)
    for _ in range(40):
        imp = impedance(r - q[0, 2])
        Ds = impratio * imp / ((1 - imp) / mass) * (mus / mu) ** 2
        ratio = 1 - dt * Ds * b / (I + Ds)
        w0 = v[0, 5]
        t = o.forward(q[0], v[0], qacc_ws=ws[0])
        o.step(np.zeros((1, 0)), q, v, ws)
        assert abs(v[0, 5] - ratio * w0) < 1e-9 * abs(w0)
        f = t["efc_force"]
        assert t["ncon"] == 1 and abs(f[3]) < mus * f[0]          # inside the cone
    assert 0 < v[0, 5] < 0.05 * 0.9


def test_fast_spin_force_on_the_cone_surface(oracle_mod):
    """Spun fast (10 rad/s), the ball's spin force stays in the cone, |f_s| <= mu_spin f_n, on its
    surface in many contact steps (inside it at the harder landings), with no tangential force
    (the ball does not slide), and the spin falls at every contact step.  (The soft cone's surface force also raises f_n above the weight -- the
    projection of y onto the cone moves y_n up by mu |y_t| / (1 + mu^2) in the scaled
    coordinates -- so the fast-spinning ball hops; the slow spin above stays inside the cone.)"""
    mass, r, mus, dt = 1.0, 0.1, 0.02, 0.002
    m = _elliptic4(robots.free_body("sphere", size=(r,), mass=mass, pos=(0, 0, r), friction=0.8,
                                    timestep=dt), mus)
    o, q, v, ws = _rest_sphere(oracle_mod, m, 500)
    v[0, 5] = 10.0
    touching = surface = 0
    for _ in range(200):
        t = o.forward(q[0], v[0], qacc_ws=ws[0])
        w0 = v[0, 5]
        o.step(np.zeros((1, 0)), q, v, ws)
        if t["ncon"] == 0:
            assert v[0, 5] == w0
            continue
        f = t["efc_force"]
        if f[0] > 1e-6:
            touching += 1
            assert abs(f[3]) <= mus * f[0] * (1 + 1e-9)
            surface += abs(abs(f[3]) - mus * f[0]) < 1e-9 * f[0]
            assert abs(f[1]) < 1e-9 * f[0] and abs(f[2]) < 1e-9 * f[0]
            assert v[0, 5] < w0
    assert touching >= 20 and surface >= 20 and v[0, 5] < 9.0
