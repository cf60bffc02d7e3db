"""Pins of the oracle's joint damping: a passive torque -B v integrated implicitly, the step
applying (M + dt B)^-1 M a (runs on the CPU)."""
import math

import numpy as np
import pytest

from helpers import DT_LEVER, lever
from workloads import robots


def damped_lever(b, l=0.5, m=2.0, r=0.02):
    mdl = lever(None, gravity=(0, 0, 0), l=l, m=m, r=r)
    mdl["joints"][0]["damping"] = float(b)
    return mdl, m * l * l + 0.4 * m * r * r


def run(o, q0, v0, steps):
    q = np.array([[q0]], np.float64); v = np.array([[v0]], np.float64); ws = np.zeros((1, 1))
    vs = []
    for _ in range(steps):
        o.step(np.zeros((1, 0)), q, v, ws)
        vs.append(v[0, 0])
    return np.array(vs)


def test_implicit_damping_geometric_decay(oracle_mod):
    """Without gravity a damped lever's velocity falls by M / (M + dt B) each step: the
    force -B v is taken at the end-of-step velocity."""
    b = 0.3
    mdl, I = damped_lever(b)
    vs = run(oracle_mod.Oracle(mdl), 0.0, 1.0, 50)
    ratio = I / (I + DT_LEVER * b)
    np.testing.assert_allclose(vs, ratio ** np.arange(1, 51), rtol=1e-12)


def test_stiff_damping_stays_stable(oracle_mod):
    """dt B / M = 10: explicit damping would flip and grow the velocity by -9 each step; the
    implicit step shrinks it by 1/11 without changing its sign."""
    mdl, I = damped_lever(0.0)
    b = 10 * I / DT_LEVER
    mdl["joints"][0]["damping"] = b
    vs = run(oracle_mod.Oracle(mdl), 0.0, 1.0, 10)
    np.testing.assert_allclose(vs, (1 / 11) ** np.arange(1, 11), rtol=1e-12)


def test_damping_torque_in_applied_forces(oracle_mod):
    """The passive torque joins the applied forces (the tau tap) as -B v."""
    mdl, _ = damped_lever(0.7)
    t = oracle_mod.Oracle(mdl).forward([0.2], [1.5])
    assert abs(t["tau"][0] + 0.7 * 1.5) < 1e-15


def test_zero_damping_changes_nothing(oracle_mod):
    a = oracle_mod.Oracle(robots.chain3())
    b = oracle_mod.Oracle(robots.with_damping(robots.chain3(), 0.0))
    q0 = np.array([[0.4, -0.3, 1.0]]); v0 = np.array([[0.5, -1.0, 0.2]])
    out = []
    for o in (a, b):
        q, v, ws = q0.copy(), v0.copy(), np.zeros((1, 3))
        for _ in range(100):
            o.step(np.zeros((1, 0)), q, v, ws)
        out.append((q, v))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_damped_chain_loses_energy(oracle_mod):
    """A damped chain dissipates: its energy above the hanging rest state falls at every
    checkpoint and ends below 2 % of the start after 6 s."""
    o = oracle_mod.Oracle(robots.chain3_damp())
    q = np.array([[1.0, -0.5, 0.8]]); v = np.zeros((1, 3)); ws = np.zeros((1, 3))
    Emin = sum(o.energy(np.zeros(3), np.zeros(3)))     # hanging at rest
    E = [sum(o.energy(q[0], v[0])) - Emin]
    for k in range(3000):
        o.step(np.zeros((1, 0)), q, v, ws)
        if k % 250 == 249:
            E.append(sum(o.energy(q[0], v[0])) - Emin)
    assert all(b < a for a, b in zip(E, E[1:])), E
    assert E[-1] < 0.02 * E[0]


@pytest.mark.parametrize("case", ["free", "negative", "nonfinite"])
def test_invalid_damping_rejected(oracle_mod, case):
    m = robots.humanoid_damp()
    if case == "free":
        m["joints"][0]["damping"] = 1.0
    elif case == "negative":
        m["joints"][1]["damping"] = -0.1
    else:
        m["joints"][1]["damping"] = math.nan
    with pytest.raises(Exception):
        oracle_mod.Oracle(m)
