"""Height-field terrain on the HIP path against the oracle (needs an MI355X)."""
import numpy as np
import pytest

from gpu_common import MARGIN_BAND, gpu_run, teacher_forced
from helpers import rot
from workloads import robots

pytestmark = pytest.mark.gpu

SX, SY = 1.0, 0.8


def _scene(H, other, size, margin=0.02):
    mb = robots.ModelBuilder("hf", timestep=0.002, nsubsteps=1)
    mb.hfield(H)
    mb.geom(0, "hfield", [SX, SY, 0], pos=(0.1, -0.05, 0.0), quat=robots.quat_axis_angle([0, 0, 1], 0.3),
            contype=0, conaffinity=1)
    inertia = {"sphere": lambda: robots.sphere_inertia(1.0, size[0]),
               "capsule": lambda: robots.capsule_inertia(1.0, size[0], 2 * size[1]),
               "box": lambda: robots.box_inertia(1.0, *size)}[other]()
    b = mb.body("b", 0, (0, 0, 1), 1.0, inertia)
    mb.joint(b, "free")
    mb.geom(b, other, list(size), contype=1, conaffinity=0, margin=margin)
    return mb.build()


@pytest.mark.parametrize("other,size", [("sphere", (0.05,)), ("capsule", (0.04, 0.12)), ("box", (0.06, 0.04, 0.03))])
def test_hfield_contacts_random_poses(oracle_mod, other, size):
    """Geoms at random poses over a random, rotated and shifted grid (some over its edge): contact
    keys, depths, points and normals against the oracle on the same FP32 state."""
    rng = np.random.default_rng({"sphere": 1, "capsule": 2, "box": 3}[other])
    H = rng.uniform(-0.04, 0.04, (9, 11))
    m = _scene(H, other, size)
    n = 128
    q = np.zeros((n, 7))
    for w in range(n):
        qq = rng.normal(size=4)
        q[w, 3:] = qq / np.linalg.norm(qq)
        q[w, :3] = [rng.uniform(-1.15, 1.15), rng.uniform(-0.95, 0.95), rng.uniform(-0.05, 0.1)]
    q = q.astype(np.float32)
    v = np.zeros((n, 6), np.float32)
    g = gpu_run(m, q, v, contacts=True)
    c = g["contacts"]
    o = oracle_mod.Oracle(m)
    counts = set()
    for w in range(n):
        t = o.forward(q[w], v[w])
        if any(abs(d - 0.02) <= MARGIN_BAND for d in t["dist"]):
            continue
        nc = t["ncon"]
        assert c["ncon"][w] == nc, f"world {w}"
        counts.add(nc)
        if nc == 0:
            continue
        assert [tuple(x) for x in c["geom"][w, :nc]] == [tuple(x) for x in t["geom"]]
        assert list(c["feature"][w, :nc]) == list(t["feature"])
        assert np.abs(c["dist"][w, :nc] - t["dist"]).max() <= 2e-6, f"world {w}"
        assert np.abs(c["pos"][w, :nc] - t["pos"]).max() <= 2e-6, f"world {w}"
        assert np.abs(c["frame"][w, :nc].reshape(nc, 9) - t["frame"].reshape(nc, 9)).max() <= 2e-5, f"world {w}"
    assert 0 in counts and len(counts) >= 2


def test_box_rests_on_a_sloped_grid_gpu():
    """A box on a planar grid sloped by atan(0.2) (mu = 1) comes to rest with its contact
    resultant balancing its weight (HIP path, 3 s)."""
    import torch
    import paper_2601_22074_amd as rb
    a = 0.2
    xs = np.linspace(-SX, SX, 5)
    H = np.tile(a * xs, (4, 1))
    th = np.arctan(a)
    hz = 0.03
    nrm = np.array([-np.sin(th), 0.0, np.cos(th)])
    mb = robots.ModelBuilder("hf", timestep=0.002, nsubsteps=1)
    mb.hfield(H)
    mb.geom(0, "hfield", [SX, SY, 0], contype=0, conaffinity=1)
    b = mb.body("b", 0, (0, 0, 1), 1.0, robots.box_inertia(1.0, 0.06, 0.04, hz))
    mb.joint(b, "free")
    mb.geom(b, "box", [0.06, 0.04, hz], contype=1, conaffinity=0)
    m = mb.build()
    q0 = np.concatenate([nrm * (hz + 1e-3), robots.quat_axis_angle([0, 1, 0], -th)])
    M = rb.Model(m)
    B = rb.Batch(M, 4)
    q = torch.tensor(np.tile(q0, (4, 1)), dtype=torch.float32, device="cuda")
    v = torch.zeros(4, 6, device="cuda")
    con = B.contacts(4)
    for _ in range(1500):
        B.step(torch.zeros(4, 0, device="cuda"), q, v, con)
    nc = int(con.ncon[0].item())
    f = con.force[0, :nc].cpu().numpy().astype(np.float64)
    fr = con.frame[0, :nc].cpu().numpy().astype(np.float64)
    B.close()
    M.close()
    assert nc == 4
    F = sum(f[i] @ fr[i] for i in range(nc))
    np.testing.assert_allclose(F, [0.0, 0.0, 9.81], atol=1e-3 * 9.81)


def test_quadruped_on_hfield_teacher_forced(oracle_mod):
    """The quadruped on height-field terrain, teacher-forced along the oracle's trajectory."""
    T = teacher_forced(oracle_mod, "quadruped_hfield", 200)
    assert T.nmatch >= 0.8 * T.n
