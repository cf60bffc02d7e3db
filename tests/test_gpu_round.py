"""Sphere and capsule pairs (limb self-collision) on the HIP path: contact keys, depths, points
and normals of free capsules and spheres at random poses around a static capsule against the
oracle on the same FP32 states, and a capsule resting across a static capsule carrying its
weight.  Teacher-forced parity of humanoid_self (its legs' capsules colliding with each other,
two branches below the pelvis) runs with the other workloads in the parity tests."""
import numpy as np
import pytest

from gpu_common import MARGIN_BAND, gpu_run
from helpers import rot
from workloads import robots

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["capsule", "sphere"])
def test_round_contacts_random_poses(oracle_mod, kind):
    n = 64
    quat = robots.quat_axis_angle([0.3, -0.5, 0.8], 0.7)
    mb = robots.ModelBuilder("round", timestep=0.002, nsubsteps=1)
    mb.geom(0, "capsule", [0.05, 0.2], pos=(0.0, 0.0, 0.5), quat=quat, contype=0, conaffinity=1)
    b = mb.body("free", 0, (0, 0, 1), 0.8, [0.01, 0.01, 0.01])
    mb.joint(b, "free")
    size = [0.04, 0.12] if kind == "capsule" else [0.06]
    mb.geom(b, kind, size, contype=1, conaffinity=0, margin=0.02)
    m = mb.build()
    rng = np.random.default_rng(16)
    ax = rot(quat)[:, 2]
    q = np.zeros((n, 7))
    for w in range(n):
        # the free geom's centre near a random point of the static segment, at a random distance
        # around contact (penetrating to outside the margin), at a random orientation
        s = rng.uniform(-0.25, 0.25)
        d = rng.normal(size=3)
        d -= (d @ ax) * ax
        d /= np.linalg.norm(d)
        gap = 0.05 + size[0] + rng.uniform(-0.03, 0.04)
        cq = rng.normal(size=4)
        cq /= np.linalg.norm(cq)
        q[w, :3] = np.array([0, 0, 0.5]) + s * ax + gap * d
        q[w, 3:] = cq
    q = q.astype(np.float32)
    v = np.zeros((n, 6), np.float32)
    g = gpu_run(m, q, v, contacts=True)
    c = g["contacts"]
    o = oracle_mod.Oracle(m)
    kinds = set()
    for w in range(n):
        t = o.forward(q[w], v[w])
        if any(abs(dd - 0.02) <= MARGIN_BAND for dd in t["dist"]):
            continue
        nc = t["ncon"]
        assert c["ncon"][w] == nc, f"world {w}"
        kinds.add(nc)
        if nc == 0:
            continue
        assert [tuple(x) for x in c["geom"][w, :nc]] == [tuple(x) for x in t["geom"]]
        assert np.abs(c["dist"][w, :nc] - t["dist"]).max() <= 2e-6, f"world {w}"
        assert np.abs(c["pos"][w, :nc] - t["pos"]).max() <= 2e-6, f"world {w}"
        assert np.abs(c["frame"][w, :nc].reshape(nc, 9) - t["frame"].reshape(nc, 9)).max() <= 2e-5, f"world {w}"
    assert {0, 1} <= kinds


def test_capsule_rests_across_a_capsule():
    """A 0.5 kg capsule dropped crosswise onto a static horizontal capsule comes to rest on one
    contact carrying its weight (HIP path, 3 s)."""
    qx = robots.quat_axis_angle((0, 1, 0), np.pi / 2)
    qy = robots.quat_axis_angle((1, 0, 0), np.pi / 2)
    mb = robots.ModelBuilder("cross", timestep=0.002, nsubsteps=1)
    mb.geom(0, "capsule", [0.03, 0.2], pos=(0, 0, 0.1), quat=qx, contype=1, conaffinity=1)
    b = mb.body("bar", 0, (0, 0, 0.1 + 0.06), 0.5, robots.capsule_inertia(0.5, 0.03, 0.3), quat=qy)
    mb.joint(b, "free")
    mb.geom(b, "capsule", [0.03, 0.15], contype=1, conaffinity=1)
    m = mb.build()
    q = np.tile(np.array([0, 0, 0.165, *qy], np.float32), (4, 1))
    q[:, 0] = [0.0, 0.01, -0.01, 0.02]
    v = np.zeros((4, 6), np.float32)
    g = gpu_run(m, q, v, nsteps=1500, contacts=True)
    c = g["contacts"]
    for w in range(4):
        assert c["ncon"][w] == 1
        f = c["force"][w, 0].astype(np.float64) @ c["frame"][w, 0].reshape(3, 3).astype(np.float64)
        np.testing.assert_allclose(f, [0, 0, 0.5 * 9.81], atol=1e-4 * 0.5 * 9.81 * 10)
    # at rest up to a slow roll about the bar's own axis that FP32 rounding starts on the
    # crosswise contact (the oracle's FP64 bar stays still)
    assert np.abs(g["qvel"][:, :3]).max() < 1e-3 and np.abs(g["qvel"]).max() < 1e-2
