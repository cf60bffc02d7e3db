"""Test-only helpers: configuration-space stepping and rotation utilities written for the pins.

These are independent of both the oracle and the HIP path (plain numpy).
"""
from __future__ import annotations

import numpy as np


def quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def quat_exp(theta):
    """Unit quaternion of the rotation vector ``theta``."""
    th = np.asarray(theta, float)
    a = np.linalg.norm(th)
    if a == 0:
        return np.array([1.0, 0, 0, 0])
    return np.concatenate([[np.cos(a / 2)], np.sin(a / 2) * th / a])


def rot(q):
    q = np.asarray(q, float) / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def joint_layout(model):
    """List of (type, qadr, dadr) per joint."""
    out, qa, da = [], 0, 0
    for j in model["joints"]:
        out.append((j["type"], qa, da))
        if j["type"] == "free":
            qa, da = qa + 7, da + 6
        else:
            qa, da = qa + 1, da + 1
    return out


def q_plus(model, q, dv):
    """Configuration reached from q by the velocity increment dv (free joints: world-frame
    translation, body-frame rotation vector)."""
    q = np.array(q, float)
    out = q.copy()
    for t, qa, da in joint_layout(model):
        if t == "hinge":
            out[qa] = q[qa] + dv[da]
        else:
            out[qa:qa + 3] = q[qa:qa + 3] + dv[da:da + 3]
            out[qa + 3:qa + 7] = quat_mul(q[qa + 3:qa + 7], quat_exp(dv[da + 3:da + 6]))
    return out


def vee(S):
    return np.array([S[2, 1] - S[1, 2], S[0, 2] - S[2, 0], S[1, 0] - S[0, 1]]) / 2.0


# ---------------------------------------------------------------- a lever against a joint limit
DT_LEVER = 0.002


def lever(range_, gravity=(0, 0, -9.81), motor=False, l=0.5, m=2.0, r=0.02):
    """One hinge about +y at the origin with a mass m on a massless lever of length l along +x
    (a small solid sphere of radius r).  Positive angles lower the mass."""
    from workloads import robots
    mb = robots.ModelBuilder("lever", timestep=DT_LEVER, nsubsteps=1, gravity=list(gravity))
    b = mb.body("lever", 0, (0, 0, 0), m, robots.sphere_inertia(m, r), ipos=(l, 0, 0))
    j = mb.joint(b, "hinge", axis=(0, 1, 0), range_=range_)
    if motor:
        mb.actuator(j, "motor", gear=1.0)
    return mb.build()


def impedance(r, solimp=(0.9, 0.95, 0.001, 0.5, 2.0)):
    """The soft-constraint impedance curve (dmin, dmax, width, midpoint, power)."""
    dmin, dmax, width, mid, p = solimp
    x = min(abs(r) / width, 1.0)
    y = x ** p / mid ** (p - 1) if x <= mid else 1 - (1 - x) ** p / (1 - mid) ** (p - 1)
    return min(max(dmin + y * (dmax - dmin), 1e-4), 0.9999)


def lever_rest_angle(l, mass, r, g=9.81, solref=(0.02, 1.0), dmax=0.95):
    """Resting angle of the lever on an upper bound at 0 under gravity.  At rest (a = 0, v = 0)
    the Newton optimum balances M a0 against the single row's force; with A-hat = 1/M the
    penetration d solves k imp(d) d = a0(d) (1 - imp(d)) / imp(d), solved by bisection."""
    import math
    I = mass * l * l + 0.4 * mass * r * r
    tc, zeta = max(solref[0], 2 * DT_LEVER), solref[1]
    k = 1.0 / (dmax * dmax * tc * tc * zeta * zeta)

    def resid(d):
        a0 = mass * g * l * math.cos(d) / I
        imp = impedance(d)
        return k * imp * d - a0 * (1 - imp) / imp

    lo, hi = 0.0, 0.1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if resid(mid) < 0 else (lo, mid)
    return lo


def soft_sag(mass, g=9.81, ahat=None, tc=0.02, dmax=0.95):
    """Closed-form sag r < 0 of a bilateral row holding a weight m g at rest: the row's force
    -D jar, jar = k imp(r) r, balances m g with D = imp / ((1 - imp) A-hat) and A-hat = 1/m for a
    point held at its body's centre of mass; solved by bisection."""
    k = 1.0 / (dmax * dmax * tc * tc)
    A = ahat if ahat is not None else 1.0 / mass

    def resid(d):
        imp = impedance(-d)
        return imp * imp * k * d / ((1 - imp) * A) - mass * g

    lo, hi = 0.0, 0.1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if resid(mid) < 0 else (lo, mid)
    return -lo
