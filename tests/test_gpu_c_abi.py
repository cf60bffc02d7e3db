"""The C ABI from a C program (tests/c_abi_step.c, no Python in its process): 64 quadruped and
32 humanoid worlds advanced 20 env steps end bitwise where the Python binding's steps of the
same inputs put them (per-world parameters at the batch's defaults on both sides), with clean
status words."""
import os
import subprocess

import numpy as np
import pytest

from c_abi_build import build_c_caller
from workloads import inputs

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("name,n", [("quadruped", 64), ("humanoid", 32)])
def test_c_caller_matches_binding(tmp_path, name, n):
    import torch
    import paper_2601_22074_amd as rb
    exe = build_c_caller(str(tmp_path / "c_abi_step"))
    W = inputs.workload(name, n, 1)
    m = W["model"]
    # (both callers leave the per-world parameters at the batch's defaults)
    q0 = np.ascontiguousarray(W["qpos"], np.float32)
    v0 = np.ascontiguousarray(W["qvel"], np.float32)
    u0 = np.ascontiguousarray(W["ctrl"][0], np.float32)
    for nm, a in (("q", q0), ("v", v0), ("u", u0)):
        a.tofile(str(tmp_path / f"{nm}.f32"))
    model_json = os.path.join(ROOT, "workloads", "models", name + ".json")
    steps = 20
    r = subprocess.run([exe, model_json, str(n), str(steps), str(tmp_path / "q.f32"), str(tmp_path / "v.f32"),
                        str(tmp_path / "u.f32"), str(tmp_path / "out.bin")], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    out = np.fromfile(str(tmp_path / "out.bin"), dtype=np.uint8)
    nq, nv = q0.shape[1], v0.shape[1]
    qc = out[:4 * n * nq].view(np.float32).reshape(n, nq)
    vc = out[4 * n * nq:4 * n * (nq + nv)].view(np.float32).reshape(n, nv)
    sc = out[4 * n * (nq + nv):].view(np.uint32)
    dev = torch.device("cuda:0")
    M = rb.Model(m)
    B = rb.Batch(M, n)
    q = torch.tensor(q0, device=dev)
    v = torch.tensor(v0, device=dev)
    u = torch.tensor(u0, device=dev)
    st = torch.zeros(n, dtype=torch.int32, device=dev)
    for _ in range(steps):
        B.step(u, q, v, None, st)
    torch.cuda.synchronize()
    assert np.array_equal(qc, q.cpu().numpy()) and np.array_equal(vc, v.cpu().numpy())
    assert np.array_equal(sc.astype(np.int64), st.cpu().numpy().astype(np.int64))
    assert not np.any(sc & 1)
