"""Parity at the benchmark sizes, in the launch configuration bench.py times (all worlds in one
launch, contacts returned), on a sample of worlds the oracle computes one by one."""
import numpy as np
import pytest

from gpu_common import StepTally, band_worlds, fp32_floor, gpu_step_records, oracle_step_records
from workloads import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,n,start", [("humanoid", 8192, 0), ("humanoid", 8192, 20), ("quadruped", 4096, 20),
                                          ("humanoid_elliptic4", 8192, 20)])
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
    fr, ms = W["friction"], W["mass_scale"]
    g = gpu_step_records(m, q, v, u, ws, fr, ms)
    assert np.all(g["status"] & 1 == 0)
    sub = lambda a: None if a is None else a[idx]
    r = oracle_step_records(o, q[idx], v[idx], u[idx], ws[idx], sub(fr), sub(ms))
    band = band_worlds(oracle_mod, m, q[idx], v[idx], u[idx], ws[idx], sub(fr), sub(ms))
    ell = m["opt"].get("cone") == "elliptic"   # elliptic cones: the smooth-cost rules of the tally
    T = StepTally(f"{name} x{n} from step {start}", smooth=ell,
                  force_scale=max(1.0, m["opt"].get("impratio", 1.0)) if ell else 1.0)
    for j, w in enumerate(idx):
        T.add(g, r, w, j, band[j], (name, n, start, int(w)),
              floor=lambda j=j: fp32_floor(o, m, q[idx], v[idx], u[idx], ws[idx], sub(fr), sub(ms), j))
    T.finish()
