"""Pins of the oracle's joint limits (one unilateral soft row per violated hinge bound),
against closed forms of the soft-constraint equilibrium, a dense inverse and the unlimited
model (runs on the CPU)."""
import math

import numpy as np
import pytest

from helpers import lever, lever_rest_angle
from workloads import robots


def settle(o, q, v, steps, ctrl=None):
    q = np.array(q, np.float64).reshape(1, -1)
    v = np.array(v, np.float64).reshape(1, -1)
    ws = np.zeros((1, o.nv))
    u = np.zeros((1, o.nu)) if ctrl is None else np.array(ctrl, np.float64).reshape(1, -1)
    for _ in range(steps):
        o.step(u, q, v, ws)
    return q[0], v[0]


def test_lever_rests_at_the_soft_equilibrium(oracle_mod):
    """Against the upper bound 0, at rest (a = 0, v = 0) the Newton optimum balances
    M a0 against the row force: with A-hat = 1/M, the penetration d = q - 0 solves
    k imp(d) d = a0(q) (1 - imp(d)) / imp(d), a scalar equation solved here by bisection."""
    l, mass, r = 0.5, 2.0, 0.02
    o = oracle_mod.Oracle(lever([-1.0, 0.0], l=l, m=mass, r=r))
    q, v = settle(o, 0.0, 0.0, 4000)
    lo = lever_rest_angle(l, mass, r)
    assert abs(v[0]) < 1e-9
    assert q[0] > 0
    assert abs(q[0] - lo) <= 1e-9 * max(lo, 1e-6) + 1e-12, (q[0], lo)


def test_motor_against_limit_force_equals_torque(oracle_mod):
    """Without gravity a motor torque u presses the lever on its upper bound; at rest the
    limit row carries exactly u (M a = u - f = 0)."""
    o = oracle_mod.Oracle(lever([-0.5, 0.3], gravity=(0, 0, 0), motor=True))
    q, v = settle(o, 0.25, 0.0, 3000, ctrl=[2.0])
    t = o.forward(q, v, ctrl=[2.0])
    assert t["ncon"] == 0 and t["J"].shape[0] == 1
    np.testing.assert_array_equal(t["J"][0], [-1.0])
    # the critically damped approach has not quite ended after 6 s
    assert abs(t["efc_force"][0] - 2.0) < 1e-7
    assert abs(t["qacc"][0]) < 1e-7
    assert q[0] > 0.3


def test_lower_bound_row_sign(oracle_mod):
    """Below the lower bound the row is +e_i and pushes the angle up."""
    o = oracle_mod.Oracle(lever([-0.2, 0.2], gravity=(0, 0, 0)))
    t = o.forward([-0.25], [0.0])
    np.testing.assert_array_equal(t["J"], [[1.0]])
    assert t["efc_force"][0] > 0 and t["qacc"][0] > 0
    t = o.forward([0.0], [0.0])
    assert t["J"].shape[0] == 0


def test_limit_rows_ahat_is_inverse_mass_diagonal(oracle_mod):
    """Limit rows come after the contact rows, one per violated bound, with Jacobian
    +-e_i and A-hat = (M^-1)_ii (here from a dense inverse)."""
    m = robots.quadruped_lim()
    o = oracle_mod.Oracle(m)
    q = robots.qpos0(m)
    rng = np.random.default_rng(3)
    hinge_q = [i for i in range(7, 19)]
    q[hinge_q] = rng.uniform(-0.4, 0.4, 12)
    t = o.forward(q, np.zeros(o.nv))
    nc = t["ncon"]
    lim = t["J"][4 * nc:]
    viol = [(k, -1.0 if q[7 + k] > 0.25 else 1.0) for k in range(12) if abs(q[7 + k]) > 0.25]
    assert len(lim) == len(viol) > 0
    Minv = np.linalg.inv(t["M"])
    for row, (k, sgn) in zip(range(len(lim)), viol):
        e = np.zeros(o.nv)
        e[6 + k] = sgn
        np.testing.assert_array_equal(lim[row], e)
        assert abs(t["Ahat"][4 * nc + row] - Minv[6 + k, 6 + k]) <= 1e-10 * Minv[6 + k, 6 + k]


def test_wide_limits_change_nothing(oracle_mod):
    """Bounds never reached leave the trajectory bit for bit unchanged."""
    a = oracle_mod.Oracle(robots.chain3())
    b = oracle_mod.Oracle(robots.with_limits(robots.chain3(), -20.0, 20.0))
    q0 = np.array([0.4, -0.3, 1.0]); v0 = np.array([0.5, -1.0, 0.2])
    qa, va = settle(a, q0, v0, 200)
    qb, vb = settle(b, q0, v0, 200)
    np.testing.assert_array_equal(qa, qb)
    np.testing.assert_array_equal(va, vb)


def test_limited_chain_stays_near_its_bounds(oracle_mod):
    """A fast chain under +-0.6 rad limits overshoots its bounds only by the soft penetration
    (a few hundredths of a radian), where the unlimited chain swings far past them."""
    o = oracle_mod.Oracle(robots.chain3_lim())
    q = np.array([[0.5, -0.5, 0.3]]); v = np.array([[4.0, -4.0, 3.0]]); ws = np.zeros((1, 3))
    worst = 0.0
    for _ in range(500):
        o.step(np.zeros((1, 0)), q, v, ws)
        worst = max(worst, float(np.max(np.abs(q))))
    assert 0.6 < worst < 0.7, worst
    u = oracle_mod.Oracle(robots.chain3())
    q = np.array([[0.5, -0.5, 0.3]]); v = np.array([[4.0, -4.0, 3.0]]); ws = np.zeros((1, 3))
    far = 0.0
    for _ in range(500):
        u.step(np.zeros((1, 0)), q, v, ws)
        far = max(far, float(np.max(np.abs(q))))
    assert far > 1.0


@pytest.mark.parametrize("case", ["free", "inverted", "nonfinite"])
def test_invalid_ranges_rejected(oracle_mod, case):
    m = robots.quadruped_lim()
    if case == "free":
        m["joints"][0]["range"] = [-1.0, 1.0]
    elif case == "inverted":
        m["joints"][1]["range"] = [0.5, -0.5]
    else:
        m["joints"][1]["range"] = [-math.inf, 0.5]
    with pytest.raises(Exception):
        oracle_mod.Oracle(m)
