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
