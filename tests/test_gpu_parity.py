"""Parity of the HIP path against the FP64 oracle (needs an MI355X)."""
import numpy as np
import pytest

from gpu_common import (CONV_TRUNC, DEPTH_TOL, MARGIN_BAND, RTOL_ROLLOUT, RTOL_STEP, by_name, contact_keys, gpu_run,
                        lifted, oracle_run, qacc_floor, rel_err, substeps1, teacher_forced, vec_err)
from helpers import rot
from workloads import inputs, robots

pytestmark = pytest.mark.gpu


def _wl(name, n, first=0):
    m = by_name(name)
    worlds = range(first, first + n)
    q, v = inputs.initial_state(m, name, worlds)
    u = inputs.ctrl_table(m, name, worlds, 1)[0]
    fr, ms = inputs.world_params(m, name, worlds)
    return m, q, v, u, fr, ms


# ------------------------------------------------------------------ stage taps
@pytest.mark.parametrize("name", ["chain3", "quadruped", "humanoid", "arm_box"])
def test_stage_taps_smooth_dynamics(oracle_mod, name):
    m, q, v, u, fr, ms = _wl(name, 16)
    rng = np.random.default_rng(1)
    if name != "chain3":
        q = lifted(m, q)
        v = rng.normal(0, 0.5, v.shape).astype(np.float32)
    g = gpu_run(m, q, v, u, friction=fr, mass_scale=ms, taps=True)
    o = oracle_mod.Oracle(m)
    for w in range(q.shape[0]):
        t = o.forward(q[w], v[w], u[w], None, None if fr is None else fr[w], None if ms is None else ms[w])
        scale = np.abs(t["M"]).max()
        assert np.abs(g["M"][w] - t["M"]).max() <= 2e-5 * scale, f"M world {w}"
        bscale = max(1.0, np.abs(t["bias"]).max())
        assert np.abs(g["bias"][w] - t["bias"]).max() <= 2e-5 * bscale, f"bias world {w}"
        # accelerations come out of a solve with M (condition ~1e4 for the humanoid), so their
        # FP32 error scales with the vector, not with each element
        assert vec_err(g["a0"][w], t["a0"]) <= RTOL_STEP, f"a0 world {w}"
        assert vec_err(g["qacc"][w], t["qacc"]) <= RTOL_STEP, f"qacc world {w}"


@pytest.mark.parametrize("name", ["quadruped", "humanoid", "arm_box"])
def test_stage_taps_contact_rows(oracle_mod, name):
    """One substep from states in contact: rows (aref, D, A-hat) and the solved acceleration."""
    m = substeps1(by_name(name))
    _, q, v, u, fr, ms = _wl(name, 16)
    # advance the oracle until the robots are on the ground, then tap one substep there
    o = oracle_mod.Oracle(m)
    r = oracle_run(o, q, v, u, None, fr, ms, nsteps=60)
    q1, v1, ws1 = r["qpos"].astype(np.float32), r["qvel"].astype(np.float32), r["qacc_ws"].astype(np.float32)
    g = gpu_run(m, q1, v1, u, ws1, fr, ms, taps=True, contacts=True)
    ncmp = nsame = nfloor = 0
    for w in range(q1.shape[0]):
        t = o.forward(q1[w], v1[w], u[w], ws1[w], None if fr is None else fr[w], None if ms is None else ms[w])
        nc = t["ncon"]
        assert g["contacts"]["ncon"][w] == min(nc, g["ncap"])
        keys = [(int(a), int(b), int(f)) for (a, b), f in zip(t["geom"], t["feature"])]
        gk = [(int(a), int(b), int(f)) for (a, b), f in zip(g["contacts"]["geom"][w, :nc], g["contacts"]["feature"][w, :nc])]
        if any(abs(d) <= MARGIN_BAND for d in t["dist"]):
            continue
        assert gk == keys
        efc = g["efc"][w, :nc]
        # penetration depths agree to FP32 rounding of body positions (~1 m scale)
        ddist = np.abs(g["contacts"]["dist"][w, :nc] - t["dist"]).max()
        assert ddist <= DEPTH_TOL
        np.testing.assert_allclose(efc[:, :, 2].reshape(-1), t["Ahat"], rtol=1e-4)
        np.testing.assert_allclose(efc[:, :, 1].reshape(-1), t["D"], rtol=2e-4)
        # aref = -b v - k imp r carries the stiffness k (~2770 / s^2) times the depth error
        kref = 1.0 / (0.95 ** 2 * 0.02 ** 2)
        np.testing.assert_allclose(efc[:, :, 0].reshape(-1), t["aref"], rtol=1e-4, atol=2 * kref * DEPTH_TOL + 1e-5)
        # the first substep's Newton updates and active rows (work record) against the oracle's:
        # where they agree the accelerations match at the step tolerance, or, where the oracle's
        # own accelerations move by more than that when the state carries single-precision
        # rounding, within that floor (qacc_floor)
        grec = g["stats"][w, 14:14 + 9]
        if grec[2] == t["niter"] and int(grec[3]) == int(np.sum(t["efc_force"] > 0)):
            err = vec_err(g["qacc"][w], t["qacc"])
            if err > RTOL_STEP:
                fl = qacc_floor(oracle_mod, m, q1[w], v1[w], u[w], ws1[w], None if fr is None else fr[w],
                                None if ms is None else ms[w])
                assert err <= fl, (f"qacc world {w}", err, fl)
                nfloor += 1
            nsame += 1
        ncmp += 1
    print(f"{name}: {ncmp} worlds compared, {nsame} on the same Newton path, {nfloor} of those above "
          f"RTOL_STEP within their FP32 floor")
    assert ncmp >= q1.shape[0] // 2
    assert nsame >= 0.9 * ncmp


# ------------------------------------------------------------------ single env step
@pytest.mark.parametrize("name", ["chain3", "quadruped", "humanoid", "arm_box"])
def test_single_step_from_initial_states(oracle_mod, name):
    m, q, v, u, fr, ms = _wl(name, 64)
    g = gpu_run(m, q, v, u, friction=fr, mass_scale=ms)
    r = oracle_run(oracle_mod.Oracle(m), q, v, u, None, fr, ms)
    assert rel_err(g["qpos"], r["qpos"]) <= RTOL_STEP
    assert rel_err(g["qvel"], r["qvel"]) <= RTOL_STEP
    assert np.all(g["status"] & 1 == 0)


@pytest.mark.parametrize("name,horizon", [("quadruped", 1000), ("humanoid", 1000), ("arm_box", 200),
                                          ("chain3_lim", 200), ("quadruped_lim", 200), ("humanoid_lim", 200),
                                          ("quadruped_terrain", 200), ("humanoid_terrain", 200),
                                          ("humanoid_damp", 200), ("quadruped_slip", 200),
                                          ("chain3_loop", 200), ("humanoid_weld", 200),
                                          ("quadruped_condim6", 200), ("humanoid_condim4", 200),
                                          ("quadruped_elliptic", 200), ("humanoid_elliptic", 200),
                                          ("cube_stack", 200), ("pincer", 200), ("humanoid_self", 200),
                                          ("pincer_cube", 400), ("quadruped_elliptic4", 200),
                                          ("humanoid_elliptic4", 200), ("quadruped_elliptic6", 200)])
def test_single_step_teacher_forced(oracle_mod, name, horizon):
    """Along the oracle's own trajectory (up to env step 1000 for the quadruped and humanoid
    workloads), hand its state (rounded to FP32) to the GPU every 25 env steps and compare one
    env step of 32 worlds: qpos, qvel and the last substep's contacts at the step tolerance
    wherever both paths made the same contacts, rows, Newton updates and active sets (checked
    from the per-substep work records of both); see StepTally for the other two cases."""
    T = teacher_forced(oracle_mod, name, horizon)
    assert T.nmatch >= 0.8 * T.n


# ------------------------------------------------------------------ contact-free rollouts
@pytest.mark.parametrize("name", ["chain3", "quadruped", "humanoid", "arm_box"])
def test_ten_step_contact_free(oracle_mod, name):
    m, q, v, u, fr, ms = _wl(name, 32)
    if name != "chain3":
        q = lifted(m, q)
    g = gpu_run(m, q, v, u, friction=fr, mass_scale=ms, nsteps=10)
    r = oracle_run(oracle_mod.Oracle(m), q, v, u, None, fr, ms, nsteps=10)
    assert rel_err(g["qpos"], r["qpos"]) <= RTOL_ROLLOUT
    assert rel_err(g["qvel"], r["qvel"]) <= RTOL_ROLLOUT


def test_chain3_500_steps(oracle_mod):
    """The chain workload at its size (64 worlds x 500 env steps, contact-free): a single step
    teacher-forced at every step of the oracle's trajectory matches at the step tolerance; every
    10-step window started from the oracle's state matches at the rollout tolerance; and the
    free-running FP32 trajectory's energy drift (semi-implicit Euler does not conserve energy)
    stays with the oracle's own drift.  Prints the divergence curve of the free runs."""
    import torch
    import paper_2601_22074_amd as rb
    m, q, v, u, fr, ms = _wl("chain3", 64)
    n, T = 64, 500
    o = oracle_mod.Oracle(m)
    M = rb.Model(m)
    B = rb.Batch(M, n)
    dev = torch.device("cuda:0")
    uz = torch.zeros(n, 0, device=dev)

    def gstep(q32, v32, k=1):
        qt = torch.tensor(q32, device=dev)
        vt = torch.tensor(v32, device=dev)
        for _ in range(k):
            B.step(uz, qt, vt)
        return qt.cpu().numpy(), vt.cpu().numpy()

    def ostep(q32, v32, k=1):
        qq = q32.astype(np.float64); vv = v32.astype(np.float64); ws = np.zeros((n, o.nv))
        for _ in range(k):
            o.step(np.zeros((n, 0)), qq, vv, ws)
        return qq, vv

    qq = q.astype(np.float64); vv = v.astype(np.float64); ws = np.zeros((n, o.nv))
    worst1 = worst10 = 0.0
    for s in range(T):
        q32, v32 = qq.astype(np.float32), vv.astype(np.float32)
        g = gstep(q32, v32)
        r = ostep(q32, v32)
        worst1 = max(worst1, rel_err(g[0], r[0]), rel_err(g[1], r[1]))
        if s % 10 == 0:
            g = gstep(q32, v32, 10)
            r = ostep(q32, v32, 10)
            worst10 = max(worst10, rel_err(g[0], r[0]), rel_err(g[1], r[1]))
        o.step(np.zeros((n, 0)), qq, vv, ws)
    assert worst1 <= RTOL_STEP, worst1
    assert worst10 <= RTOL_ROLLOUT, worst10

    def energies(qs, vs):
        return np.array([sum(o.energy(qs[w], vs[w])) for w in range(n)])

    qg, vg = q.copy(), v.copy()
    qo, vo = q.astype(np.float64), v.astype(np.float64)
    wso = np.zeros((n, o.nv))
    E0 = energies(qo, vo)
    Dg = np.zeros(n); Do = np.zeros(n); curve = {}
    qt = torch.tensor(qg, device=dev); vt = torch.tensor(vg, device=dev)
    for s in range(1, T + 1):
        B.step(uz, qt, vt)
        o.step(np.zeros((n, 0)), qo, vo, wso)
        qg, vg = qt.cpu().numpy(), vt.cpu().numpy()
        Dg = np.maximum(Dg, np.abs(energies(qg, vg) - E0))
        Do = np.maximum(Do, np.abs(energies(qo, vo) - E0))
        if s in (1, 10, 50, 100, 200, 300, 500):
            curve[s] = float(np.max(np.abs(qg - qo)))
    B.close(); M.close()
    scale = np.maximum(np.abs(E0), 1.0)
    print("chain3 x64 free-run max |qpos_gpu - qpos_oracle| by step:", curve)
    print("chain3 x64 energy drift / max(|E0|, 1): gpu median %.3e max %.3e, oracle median %.3e max %.3e"
          % (np.median(Dg / scale), np.max(Dg / scale), np.median(Do / scale), np.max(Do / scale)))
    assert curve[10] <= RTOL_ROLLOUT
    assert np.all(np.abs(Dg - Do) <= 0.02 * Do + 1e-3 * scale), np.max(np.abs(Dg - Do) / (Do + scale))


# ------------------------------------------------------------------ contact sets
@pytest.mark.parametrize("name", ["quadruped", "humanoid", "arm_box", "quadruped_terrain", "humanoid_terrain",
                                  "quadruped_slip", "quadruped_hfield", "humanoid_weld", "quadruped_condim6",
                                  "humanoid_condim4", "quadruped_elliptic", "humanoid_elliptic", "cube_stack",
                                  "pincer", "humanoid_self", "pincer_cube", "quadruped_elliptic4",
                                  "humanoid_elliptic4", "quadruped_elliptic6"])
def test_contact_sets(oracle_mod, name):
    m, q, v, u, fr, ms = _wl(name, 32)
    o = oracle_mod.Oracle(m)
    r0 = oracle_run(o, q, v, u, None, fr, ms, nsteps=40)
    q1, v1, w1 = (r0[k].astype(np.float32) for k in ("qpos", "qvel", "qacc_ws"))
    g = gpu_run(m, q1, v1, u, w1, fr, ms, contacts=True)
    r = oracle_run(o, q1, v1, u, w1, fr, ms, contacts=True)
    # contacts come from the last substep's starting state, which the two paths reach separately;
    # compare them where that state agrees to the step tolerance
    for w in range(q1.shape[0]):
        gc, gb = contact_keys(g["contacts"], w)
        rc, rb_ = contact_keys(r["contacts"], w)
        assert gc - rb_ == rc - gb, f"world {w}"


def test_box_box_contacts_random_poses(oracle_mod):
    """Cube at random orientations pressed 0.1-3 mm into the table: face, edge and vertex
    contacts (keys, depths, points, normals) against the oracle on the same FP32 state."""
    m = substeps1(by_name("arm_box"))
    n = 64
    rng = np.random.default_rng(11)
    q = np.tile(robots.qpos0(m), (n, 1))
    for w in range(n):
        qc = rng.normal(size=4)
        if w < 8:                       # a few face-down cubes turned about z only
            qc = np.array([np.cos(w / 5), 0, 0, np.sin(w / 5)])
        qc /= np.linalg.norm(qc)
        R = rot(qc)
        zext = np.abs(R[2]) @ np.full(3, 0.025)
        c = [0.5 + rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), 0.4 + zext - rng.uniform(1e-4, 3e-3)]
        q[w, -7:-4] = c
        q[w, -4:] = qc
    q = q.astype(np.float32)
    v = np.zeros((n, 13), np.float32)
    g = gpu_run(m, q, v, contacts=True)
    c = g["contacts"]
    o = oracle_mod.Oracle(m)
    kinds = set()
    for w in range(n):
        t = o.forward(q[w], v[w])
        if any(abs(d) <= MARGIN_BAND for d in t["dist"]):
            continue
        nc = t["ncon"]
        assert c["ncon"][w] == nc, f"world {w}"
        assert [tuple(x) for x in c["geom"][w, :nc]] == [tuple(x) for x in t["geom"]]
        assert list(c["feature"][w, :nc]) == list(t["feature"])
        assert np.abs(c["dist"][w, :nc] - t["dist"]).max() <= 2e-6, f"world {w}"
        assert np.abs(c["pos"][w, :nc] - t["pos"]).max() <= 2e-5, f"world {w}"
        assert np.abs(c["frame"][w, :nc].reshape(nc, 9) - t["frame"].reshape(nc, 9)).max() <= 2e-5, f"world {w}"
        kinds.add(nc)
    assert 1 in kinds and 4 in kinds


def test_frictionless_box_slides_gpu(oracle_mod):
    """A frictionless box (condim 1) on a 0.3 rad incline accelerates downhill at g sin(theta)
    on the HIP path too, with zero tangential contact force."""
    import torch
    import paper_2601_22074_amd as rb
    th, h = 0.3, 0.05
    mb = robots.ModelBuilder("incline", timestep=0.002, nsubsteps=1)
    mb.geom(0, "plane", [0, 0, 0], quat=robots.quat_axis_angle([0, 1, 0], th), contype=0, conaffinity=1)
    mb.geoms[-1]["condim"] = 1
    b = mb.body("box", 0, (0, 0, 1), 1.0, robots.box_inertia(1.0, h, h, h))
    mb.joint(b, "free")
    mb.geom(b, "box", [h, h, h], contype=1, conaffinity=0)
    mb.geoms[-1]["condim"] = 1                   # the pair takes the larger of the two
    m = mb.build()
    R = rot(robots.quat_axis_angle([0, 1, 0], th))
    q0 = np.concatenate([R[:, 2] * (h - 1e-4), robots.quat_axis_angle([0, 1, 0], th)])
    M = rb.Model(m)
    B = rb.Batch(M, 4)
    q = torch.tensor(np.tile(q0, (4, 1)), dtype=torch.float32, device="cuda")
    v = torch.zeros(4, 6, device="cuda")
    u = torch.zeros(4, 0, device="cuda")
    con = B.contacts(4)
    vs = []
    for _ in range(600):
        B.step(u, q, v, con)
        vs.append(v[0, :3].cpu().numpy().astype(np.float64))
    f = con.force[0, :int(con.ncon[0].item())].cpu().numpy()
    B.close()
    M.close()
    a = np.diff(np.array(vs) @ R[:, 0])[-100:] / 0.002
    assert np.abs(a.mean() - 9.81 * np.sin(th)) <= 1e-3 * 9.81 * np.sin(th)
    assert f.shape[0] == 4 and np.abs(f[:, 1:]).max() == 0.0
    assert abs(f[:, 0].sum() - 9.81 * np.cos(th)) <= 1e-3 * 9.81


def test_sphere_box_contacts_random_poses(oracle_mod):
    """A ball at random places around a rotated static box, within a 2 cm margin band or
    penetrating (centre outside or inside): contact keys, depths, points and normals against
    the oracle on the same FP32 state."""
    n = 64
    r = 0.05
    quat = robots.quat_axis_angle([0.3, -0.5, 0.8], 0.7)
    mb = robots.ModelBuilder("box_ball", timestep=0.005, nsubsteps=1)
    mb.geom(0, "box", [0.3, 0.2, 0.1], pos=(0.0, 0.0, 0.5), quat=quat, contype=0, conaffinity=1)
    b = mb.body("ball", 0, (0, 0, 1), 0.5, robots.sphere_inertia(0.5, r))
    mb.joint(b, "free")
    mb.geom(b, "sphere", [r], contype=1, conaffinity=0, margin=0.02)
    m = mb.build()
    rng = np.random.default_rng(5)
    R = rot(quat)
    q = np.zeros((n, 7))
    for w in range(n):
        # a point on a random face, pushed out (or in) along that face's normal
        ax = rng.integers(3)
        loc = rng.uniform(-1, 1, 3) * np.array([0.3, 0.2, 0.1])
        sg = rng.choice([-1.0, 1.0])
        loc[ax] = sg * ([0.3, 0.2, 0.1][ax] + rng.uniform(-0.06, 0.09))
        q[w, :3] = np.array([0.0, 0.0, 0.5]) + R @ loc
        q[w, 3] = 1.0
    q = q.astype(np.float32)
    v = np.zeros((n, 6), np.float32)
    g = gpu_run(m, q, v, contacts=True)
    c = g["contacts"]
    o = oracle_mod.Oracle(m)
    kinds = set()
    for w in range(n):
        t = o.forward(q[w], v[w])
        if any(abs(d - 0.02) <= MARGIN_BAND for d in t["dist"]):
            continue
        nc = t["ncon"]
        assert c["ncon"][w] == nc, f"world {w}"
        if nc == 0:
            kinds.add("none")
            continue
        assert [tuple(x) for x in c["geom"][w, :nc]] == [tuple(x) for x in t["geom"]]
        assert abs(c["dist"][w, 0] - t["dist"][0]) <= 2e-6, f"world {w}"
        assert np.abs(c["pos"][w, 0] - t["pos"][0]).max() <= 2e-6, f"world {w}"
        assert np.abs(c["frame"][w, 0].reshape(9) - t["frame"][0].reshape(9)).max() <= 2e-5, f"world {w}"
        kinds.add("inside" if t["dist"][0] < -r else ("touch" if t["dist"][0] < 0 else "band"))
    assert {"none", "band", "touch", "inside"} <= kinds


@pytest.mark.parametrize("name", ["quadruped", "humanoid", "quadruped_lim", "humanoid_lim", "humanoid_weld",
                                  "quadruped_condim6", "humanoid_condim4", "quadruped_elliptic", "humanoid_elliptic",
                                  "quadruped_elliptic4", "humanoid_elliptic4", "quadruped_elliptic6"])
def test_newton_iterations_match_oracle(oracle_mod, name):
    """The GPU ends Newton when no row changed sides since the last Hessian; the oracle ends
    it by its FP64 gradient test.  On the same states both take the same number of
    iterations, except where a row sits on its breakpoint to rounding (at most 2 %)."""
    import torch
    import paper_2601_22074_amd as rb
    m = substeps1(by_name(name))
    _, q, v, u, fr, ms = _wl(name, 64)
    o = oracle_mod.Oracle(m)
    r = oracle_run(o, q, v, u, None, fr, ms, nsteps=40)
    q1, v1, ws1 = r["qpos"].astype(np.float32), r["qvel"].astype(np.float32), r["qacc_ws"].astype(np.float32)
    dev = torch.device("cuda:0")
    M = rb.Model(m)
    B = rb.Batch(M, 64)
    B.reset(torch.arange(64, dtype=torch.int32, device=dev), torch.tensor(ws1, device=dev))
    if fr is not None:
        B.set_params(rb.PARAM_FRICTION, torch.tensor(fr, device=dev))
    if ms is not None:
        B.set_params(rb.PARAM_MASS_SCALE, torch.tensor(ms, device=dev))
    stats = torch.zeros(64, rb.rbstep.NSTATS, dtype=torch.int32, device=dev)
    B.step_taps(torch.tensor(u, device=dev), torch.tensor(q1, device=dev), torch.tensor(v1, device=dev), stats=stats)
    gi = stats[:, 2].cpu().numpy()
    B.close()
    M.close()
    args = lambda w: (q1[w], v1[w], u[w], ws1[w], None if fr is None else fr[w], None if ms is None else ms[w])
    fw = [o.forward(*args(w)) for w in range(64)]
    oi = np.array([t["niter"] for t in fw])
    keep = np.ones(64, bool)
    if m["opt"].get("cone") == "elliptic":
        # elliptic cones: the cost is not piecewise quadratic and the iteration ends in its
        # quadratic-convergence tail, where the FP64 and FP32 improvement tests fire one update
        # apart; counts are compared where the oracle's iterate is not yet converged to FP32
        # resolution
        o.set_mode("converged")
        for w in range(64):
            qc = o.forward(*args(w))["qacc"]
            keep[w] = np.abs(fw[w]["qacc"] - qc).max() > CONV_TRUNC * max(np.abs(qc).max(), 1.0)
        o.set_mode("mirror")
    if keep.any():
        assert np.mean(gi[keep] == oi[keep]) >= (0.90 if m["opt"].get("cone") == "elliptic" else 0.98), (gi, oi, keep)


# ------------------------------------------------------------------ system properties
@pytest.mark.parametrize("name", ["quadruped", "arm_box", "humanoid_lim", "humanoid_weld", "humanoid_condim4",
                                  "humanoid_elliptic4"])
def test_plain_launch_occupancy_bitwise(name):
    """The 3- and 4-wave instantiations of the plain step (plain and extended code) compute the
    same bits."""
    import torch
    import paper_2601_22074_amd as rb
    m, q, v, u, fr, ms = _wl(name, 256)
    out = []
    for waves in (3, 4):
        M = rb.Model(m)
        B = rb.Batch(M, 256)
        B.set_waves(waves)
        if fr is not None:
            B.set_params(rb.PARAM_FRICTION, torch.tensor(fr, device="cuda"))
            B.set_params(rb.PARAM_MASS_SCALE, torch.tensor(ms, device="cuda"))
        qt, vt = torch.tensor(q, device="cuda"), torch.tensor(v, device="cuda")
        ut = torch.tensor(u, device="cuda")
        for _ in range(20):
            B.step(ut, qt, vt)
        torch.cuda.synchronize()
        out.append((qt.cpu().numpy(), vt.cpu().numpy()))
        B.close()
        M.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_run_twice_bitwise(oracle_mod):
    m, q, v, u, fr, ms = _wl("humanoid", 128)
    a = gpu_run(m, q, v, u, friction=fr, mass_scale=ms, nsteps=5, contacts=True)
    b = gpu_run(m, q, v, u, friction=fr, mass_scale=ms, nsteps=5, contacts=True)
    for k in ("qpos", "qvel", "qacc_ws", "status"):
        np.testing.assert_array_equal(a[k], b[k])
    for k in a["contacts"]:
        np.testing.assert_array_equal(a["contacts"][k], b["contacts"][k])


@pytest.mark.parametrize("name", ["chain3", "quadruped", "humanoid", "arm_box", "humanoid_lim", "quadruped_terrain",
                                  "humanoid_terrain", "humanoid_damp", "quadruped_hfield", "chain3_loop",
                                  "humanoid_weld", "quadruped_condim6", "humanoid_condim4", "quadruped_elliptic",
                                  "humanoid_elliptic", "cube_stack", "pincer", "humanoid_self",
                                  "pincer_cube", "quadruped_elliptic4", "humanoid_elliptic4", "quadruped_elliptic6"])
def test_json_model_bitwise(name):
    """A model created from its JSON file (rb_model_create_json) steps exactly like the same
    model created from the description struct."""
    import os
    m, q, v, u, fr, ms = _wl(name, 64)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "workloads", "models", name + ".json")) as f:
        text = f.read()
    a = gpu_run(m, q, v, u, friction=fr, mass_scale=ms, nsteps=5, contacts=True)
    b = gpu_run(text, q, v, u, friction=fr, mass_scale=ms, nsteps=5, contacts=True)
    for k in ("qpos", "qvel", "qacc_ws", "status"):
        np.testing.assert_array_equal(a[k], b[k])
    for k in a["contacts"]:
        np.testing.assert_array_equal(a["contacts"][k], b["contacts"][k])


def test_nan_isolated_and_frozen():
    m, q, v, u, fr, ms = _wl("quadruped", 16)
    clean = gpu_run(m, q, v, u, nsteps=3)
    v2 = v.copy()
    v2[5, 7] = np.nan
    bad = gpu_run(m, q, v2, u, nsteps=3)
    assert bad["status"][5] & 1
    np.testing.assert_array_equal(bad["qpos"][5], q[5])      # frozen: never advanced
    others = [w for w in range(16) if w != 5]
    np.testing.assert_array_equal(bad["qpos"][others], clean["qpos"][others])
    np.testing.assert_array_equal(bad["qvel"][others], clean["qvel"][others])
    assert np.all(bad["status"][others] & 1 == 0)


def test_checkpoint_resume_bitwise():
    m, q, v, u, fr, ms = _wl("humanoid", 64)
    full = gpu_run(m, q, v, u, friction=fr, mass_scale=ms, nsteps=8)
    half = gpu_run(m, q, v, u, friction=fr, mass_scale=ms, nsteps=4)
    rest = gpu_run(m, half["qpos"], half["qvel"], u, half["qacc_ws"], fr, ms, nsteps=4)
    np.testing.assert_array_equal(rest["qpos"], full["qpos"])
    np.testing.assert_array_equal(rest["qvel"], full["qvel"])


def test_resting_box_forces_gpu():
    m = robots.free_body("box", size=(0.1, 0.1, 0.1), mass=1.0, pos=(0, 0, 0.1))
    q = robots.qpos0(m)[None].astype(np.float32)
    v = np.zeros((1, 6), np.float32)
    g = gpu_run(m, q, v, nsteps=400, contacts=True)
    c = g["contacts"]
    assert c["ncon"][0] == 4
    assert abs(c["force"][0, :4, 0].sum() / 9.81 - 1) < 1e-4


def test_contact_overflow_flag():
    m, q, v, u, fr, ms = _wl("humanoid", 4)
    q = q.copy()
    q[:, 2] = 0.1                      # pelvis pushed into the floor: many contacts
    g = gpu_run(m, q, v, u, friction=fr, mass_scale=ms, contacts=True, contact_capacity=4)
    assert np.all(g["status"] & 4)
    assert np.all(g["contacts"]["ncon"] == 4)


def test_capsule_box_contacts_random_poses(oracle_mod):
    """A capsule at random poses around a rotated static box, its ends within a 2 cm margin band
    or penetrating (centres outside or inside): contact keys, depths, points and normals
    against the oracle on the same FP32 state."""
    n = 64
    r, hl = 0.04, 0.15
    quat = robots.quat_axis_angle([0.3, -0.5, 0.8], 0.7)
    mb = robots.ModelBuilder("box_capsule", timestep=0.005, nsubsteps=1)
    mb.geom(0, "box", [0.3, 0.2, 0.1], pos=(0.0, 0.0, 0.5), quat=quat, contype=0, conaffinity=1)
    b = mb.body("capsule", 0, (0, 0, 1), 0.8, robots.capsule_inertia(0.8, r, 2 * hl))
    mb.joint(b, "free")
    mb.geom(b, "capsule", [r, hl], contype=1, conaffinity=0, margin=0.02)
    m = mb.build()
    rng = np.random.default_rng(15)
    R = rot(quat)
    q = np.zeros((n, 7))
    for w in range(n):
        # one end near a point of a random face, the capsule at a random orientation
        ax = rng.integers(3)
        loc = rng.uniform(-1, 1, 3) * np.array([0.3, 0.2, 0.1])
        sg = rng.choice([-1.0, 1.0])
        loc[ax] = sg * ([0.3, 0.2, 0.1][ax] + rng.uniform(-0.06, 0.09))
        end = np.array([0.0, 0.0, 0.5]) + R @ loc
        cq = rng.normal(size=4)
        cq /= np.linalg.norm(cq)
        q[w, :3] = end + hl * rot(cq)[:, 2]          # the -z end sits at `end`
        q[w, 3:] = cq
    q = q.astype(np.float32)
    v = np.zeros((n, 6), np.float32)
    g = gpu_run(m, q, v, contacts=True)
    c = g["contacts"]
    o = oracle_mod.Oracle(m)
    kinds = set()
    for w in range(n):
        t = o.forward(q[w], v[w])
        if any(abs(d - 0.02) <= MARGIN_BAND for d in t["dist"]):
            continue
        nc = t["ncon"]
        assert c["ncon"][w] == nc, f"world {w}"
        kinds.add(nc)
        if nc == 0:
            continue
        assert [tuple(x) for x in c["geom"][w, :nc]] == [tuple(x) for x in t["geom"]]
        assert list(c["feature"][w, :nc]) == list(t["feature"])
        assert np.abs(c["dist"][w, :nc] - t["dist"]).max() <= 2e-6, f"world {w}"
        assert np.abs(c["pos"][w, :nc] - t["pos"]).max() <= 2e-6, f"world {w}"
        assert np.abs(c["frame"][w, :nc].reshape(nc, 9) - t["frame"].reshape(nc, 9)).max() <= 2e-5, f"world {w}"
    assert {0, 1} <= kinds


def test_capsule_rests_on_box_gpu():
    """A capsule dropped flat onto a box comes to rest on its two ends, each carrying half its
    weight (HIP path, 3 s)."""
    import torch
    import paper_2601_22074_amd as rb
    r, hl, mass = 0.04, 0.15, 0.8
    mb = robots.ModelBuilder("box_capsule", timestep=0.002, nsubsteps=1)
    mb.geom(0, "box", [0.3, 0.2, 0.1], pos=(0.0, 0.0, 0.1), contype=0, conaffinity=1)
    b = mb.body("capsule", 0, (0, 0, 1), mass, robots.capsule_inertia(mass, r, 2 * hl))
    mb.joint(b, "free")
    mb.geom(b, "capsule", [r, hl], contype=1, conaffinity=0)
    m = mb.build()
    quat = robots.quat_axis_angle([0, 1, 0], np.pi / 2)
    M = rb.Model(m)
    B = rb.Batch(M, 4)
    q = torch.tensor(np.tile(np.concatenate([[0.0, 0.0, 0.2 + r + 0.01], quat]), (4, 1)), dtype=torch.float32,
                     device="cuda")
    v = torch.zeros(4, 6, device="cuda")
    con = B.contacts(4)
    for _ in range(1500):
        B.step(torch.zeros(4, 0, device="cuda"), q, v, con)
    f = con.force[0, :int(con.ncon[0].item())].cpu().numpy()
    vmax = float(v.abs().max().item())
    B.close()
    M.close()
    assert f.shape[0] == 2
    np.testing.assert_allclose(f[:, 0], [mass * 9.81 / 2] * 2, rtol=1e-4)
    assert vmax < 1e-4


def test_humanoid_limbs_touch_the_tiles():
    """On the tile grid the humanoid's limbs come down on the tiles: along a 200-step rollout of
    64 worlds, capsule-tile contacts appear in the contacts output (their parity with the
    oracle is the teacher-forced humanoid_terrain test's)."""
    m, q, v, u, fr, ms = _wl("humanoid_terrain", 64)
    ctab = inputs.ctrl_table(m, "humanoid_terrain", range(64), 10)
    import torch
    import paper_2601_22074_amd as rb
    dev = torch.device("cuda:0")
    M = rb.Model(m)
    B = rb.Batch(M, 64)
    B.set_params(rb.PARAM_FRICTION, torch.tensor(fr, device=dev))
    B.set_params(rb.PARAM_MASS_SCALE, torch.tensor(ms, device=dev))
    qt, vt = torch.tensor(q, device=dev), torch.tensor(v, device=dev)
    con = B.contacts(64)
    tiles = [i for i, g in enumerate(m["geoms"]) if g["body"] == 0 and g["type"] == "box"]
    caps = {i for i, g in enumerate(m["geoms"]) if g["type"] == "capsule"}
    hits = 0
    for s in range(200):
        B.step(torch.tensor(ctab[s // 20], device=dev), qt, vt, con)
        if s % 10 == 9:
            n_ = con.ncon.cpu().numpy()
            gg = con.geom.cpu().numpy()
            hits += sum(1 for w in range(64) for i in range(n_[w]) if gg[w, i, 0] in caps and gg[w, i, 1] in tiles)
    B.close()
    M.close()
    assert hits > 0
