"""Parity at the benchmark sizes, in the launch configuration bench.py times (all worlds in one
launch, contacts returned), on a sample of worlds the oracle computes one by one."""
import numpy as np
import pytest

from gpu_common import RTOL_ROLLOUT, RTOL_STEP, gpu_run, oracle_run, rel_err
from workloads import inputs

pytestmark = pytest.mark.gpu


def _sample_check(o, g, qs, vs, ws, u, fr, ms, idx, tol_trunc=True):
    """Oracle on the sampled worlds from the same FP32 state; per-world tolerance as in the
    teacher-forced test (1e-4, plus a tenth of the truncation distance where the 4-iteration
    Newton has not converged)."""
    sub = lambda a: None if a is None else a[idx]
    r = oracle_run(o, qs[idx], vs[idx], u[idx], ws[idx], sub(fr), sub(ms))
    o.set_mode("converged")
    rc = oracle_run(o, qs[idx], vs[idx], u[idx], ws[idx], sub(fr), sub(ms))
    o.set_mode("mirror")
    strict = 0
    for j, w in enumerate(idx):
        trunc = max(rel_err(rc[k][j], r[k][j]) for k in ("qpos", "qvel"))
        tol = RTOL_STEP + 0.1 * trunc
        strict += trunc <= RTOL_STEP
        err = max(rel_err(g[k][w], r[k][j]) for k in ("qpos", "qvel"))
        assert err <= tol, (int(w), err, trunc)
    return strict


@pytest.mark.parametrize("name,n,start", [("humanoid", 8192, 0), ("humanoid", 8192, 20), ("quadruped", 4096, 20)])
def test_full_size_sampled_worlds(oracle_mod, name, n, start):
    W = inputs.workload(name, n, start + 1)
    m = W["model"]
    o = oracle_mod.Oracle(m)
    idx = np.arange(0, n, n // 64)
    q, v = W["qpos"].copy(), W["qvel"].copy()
    ws = np.zeros((n, o.nv), np.float32)
    if start:
        # the sampled worlds' states after `start` env steps come from the oracle (FP64, then
        # rounded to FP32); the other worlds keep their initial states, so the launch is the
        # full-size one and every world is in a valid state
        sub = lambda a: None if a is None else a[idx]
        qq = q[idx].astype(np.float64)
        vv = v[idx].astype(np.float64)
        wd = np.zeros((len(idx), o.nv))
        st = np.zeros(len(idx), np.uint32)
        for s in range(start):
            u = W["ctrl"][s // inputs.CTRL_PERIOD][idx].astype(np.float64)
            o.step(u, qq, vv, wd, None if W["friction"] is None else W["friction"][idx].astype(np.float64),
                   None if W["mass_scale"] is None else W["mass_scale"][idx].astype(np.float64), st)
        q[idx], v[idx], ws[idx] = qq.astype(np.float32), vv.astype(np.float32), wd.astype(np.float32)
    u = W["ctrl"][start // inputs.CTRL_PERIOD]
    g = gpu_run(m, q, v, u, ws, W["friction"], W["mass_scale"], contacts=True)
    assert np.all(g["status"] & 1 == 0)
    strict = _sample_check(o, g, q, v, ws, u, W["friction"], W["mass_scale"], idx)
    assert strict >= len(idx) // 2


def test_chain_rollout_500_steps(oracle_mod):
    """The 3-link chain workload (64 worlds, 500 steps, dt 2 ms): along the GPU's own 500-step
    rollout, every 50 steps the oracle takes the GPU's state and both advance 10 steps."""
    W = inputs.workload("chain3", 64, 500)
    m = W["model"]
    o = oracle_mod.Oracle(m)
    q, v = W["qpos"].copy(), W["qvel"].copy()
    for start in range(0, 500, 50):
        g10 = gpu_run(m, q, v, nsteps=10)
        r10 = oracle_run(o, q, v, nsteps=10)
        assert rel_err(g10["qpos"], r10["qpos"]) <= RTOL_ROLLOUT
        assert rel_err(g10["qvel"], r10["qvel"]) <= RTOL_ROLLOUT
        g50 = gpu_run(m, q, v, nsteps=50)
        q, v = g50["qpos"], g50["qvel"]
    assert np.all(np.isfinite(q))
