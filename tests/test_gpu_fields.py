"""Per-world model fields on the HIP path (needs an MI355X): geom sizes, body positions and
actuator gains expanded to one value per world (rb_batch_set_params), against the oracle's
per-world fields, against models built from descriptions carrying those values, and in a
captured graph replayed after the expansion."""
import numpy as np
import pytest

from gpu_common import (StepTally, band_worlds, by_name, fp32_floor, gpu_run, gpu_step_records, oracle_step_records,
                        with_fields)
from workloads import inputs

pytestmark = pytest.mark.gpu


def _fields(name, field, n, seed=7):
    """Per-world values of a field around the model's: sizes and gains scaled by U[0.8, 1.2]
    (colliding geoms; all gains), body positions (non-root bodies) moved by up to 1 cm."""
    m = by_name(name)
    rng = np.random.default_rng(seed)
    if field == "geom_size":
        base = np.array([g["size"] for g in m["geoms"]], np.float64)
        scale = np.ones((n, len(base), 1))
        for i, g in enumerate(m["geoms"]):
            if g["type"] != "plane" and (g["contype"] or g["conaffinity"]):
                scale[:, i, 0] = rng.uniform(0.8, 1.2, n)
        return {"geom_size": (base[None] * scale).astype(np.float32)}
    if field == "body_pos":
        base = np.array([b["pos"] for b in m["bodies"]], np.float64)
        d = rng.uniform(-0.01, 0.01, (n,) + base.shape)
        d[:, :2] = 0.0
        return {"body_pos": (base[None] + d).astype(np.float32)}
    kp = np.array([a["kp"] for a in m["actuators"]], np.float64)
    kd = np.array([a["kd"] for a in m["actuators"]], np.float64)
    return {"act_kp": (kp[None] * rng.uniform(0.8, 1.2, (n, len(kp)))).astype(np.float32),
            "act_kd": (kd[None] * rng.uniform(0.8, 1.2, (n, len(kd)))).astype(np.float32)}


@pytest.mark.parametrize("name,field", [("humanoid", "geom_size"), ("arm_box", "geom_size"),
                                        ("quadruped", "gains"), ("quadruped", "body_pos"), ("humanoid", "gains")])
def test_expanded_fields_against_oracle(oracle_mod, name, field):
    """Along the oracle's own trajectory with the per-world values, every 10 env steps, one env
    step of 32 worlds against the oracle's (StepTally)."""
    m = by_name(name)
    n, horizon = 32, 80
    f = _fields(name, field, n)
    worlds = range(n)
    q, v = inputs.initial_state(m, name, worlds)
    fr, ms = inputs.world_params(m, name, worlds)
    ctab = inputs.ctrl_table(m, name, worlds, horizon // 20 + 1)
    o = oracle_mod.Oracle(m)
    qq, vv, ws = q.astype(np.float64), v.astype(np.float64), np.zeros((n, o.nv))
    f64 = lambda a: None if a is None else a.astype(np.float64)
    T = StepTally(f"{name} with per-world {field}")
    for s in range(horizon):
        uu = ctab[s // 20].astype(np.float64)
        if s % 10 == 9:
            q32, v32, w32, u32 = (x.astype(np.float32) for x in (qq, vv, ws, uu))
            g = gpu_step_records(m, q32, v32, u32, w32, fr, ms, fields=f)
            r = oracle_step_records(o, q32, v32, u32, w32, fr, ms, fields=f)
            band = band_worlds(oracle_mod, m, q32, v32, u32, w32, fr, ms, fields=f)
            for w in range(n):
                T.add(g, r, w, w, band[w], (name, field, s, w),
                      floor=lambda w=w: fp32_floor(o, m, q32, v32, u32, w32, fr, ms, w, fields=f))
        o.step(uu, qq, vv, ws, f64(fr), f64(ms), fields=f)
    T.finish()


@pytest.mark.parametrize("name,field", [("humanoid", "geom_size"), ("quadruped", "gains")])
def test_expanded_fields_equal_description_models(name, field):
    """A world whose fields were expanded steps bit for bit like the same world of a model built
    from a description carrying its values (geom sizes and gains leave every other model table,
    including the tolerance scale, unchanged)."""
    m = by_name(name)
    n = 8
    f = _fields(name, field, n, seed=3)
    q, v = inputs.initial_state(m, name, range(n))
    fr, ms = inputs.world_params(m, name, range(n))
    u = inputs.ctrl_table(m, name, range(n), 1)[0]
    g = gpu_run(m, q, v, u, friction=fr, mass_scale=ms, nsteps=40, contacts=True, fields=f)
    for w in range(n):
        sl = slice(w, w + 1)
        gw = gpu_run(with_fields(m, f, w), q[sl], v[sl], u[sl], friction=None if fr is None else fr[sl],
                     mass_scale=None if ms is None else ms[sl], nsteps=40, contacts=True)
        np.testing.assert_array_equal(g["qpos"][w], gw["qpos"][0])
        np.testing.assert_array_equal(g["qvel"][w], gw["qvel"][0])
        for k in ("ncon", "dist", "force"):
            np.testing.assert_array_equal(g["contacts"][k][w], gw["contacts"][k][0])


def test_captured_graph_picks_up_an_expansion():
    """A fused plan's captured graph, replayed after a batch expanded a field and took per-world
    values, computes what eager fused steps with those values compute (its argument blocks are
    rewritten before the replay; no new capture)."""
    import torch
    import paper_2601_22074_amd as rb
    dev = torch.device("cuda:0")
    name, n = "quadruped", 64
    m = by_name(name)
    f = _fields(name, "geom_size", n, seed=9)
    q, v = inputs.initial_state(m, name, range(n))
    u = inputs.ctrl_table(m, name, range(n), 1)[0]
    out = []
    for graph in (False, True):
        M = rb.Model(m)
        B = rb.Batch(M, n)
        qt, vt, ut = (torch.tensor(x, device=dev) for x in (q, v, u))
        P = rb.Multi([B])
        P.bind(0, ut, qt, vt)
        P.set_schedule(rb.ORDER_HEAVY_FIRST, 0)
        s = torch.cuda.Stream()
        if graph:
            with torch.cuda.stream(s):
                P.graph_capture(5, s)
        B.set_params(rb.PARAM_GEOM_SIZE, torch.tensor(f["geom_size"], device=dev))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            if graph:
                P.graph_launch(s)
                P.graph_launch(s)
            else:
                for _ in range(10):
                    P.step(s)
        torch.cuda.synchronize()
        out.append((qt.cpu().numpy(), vt.cpu().numpy()))
        P.close()
        B.close()
        M.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
