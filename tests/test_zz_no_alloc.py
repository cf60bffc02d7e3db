"""The allocation-free step (rb_step_noalloc) against rb_step on freshly reset batches (needs an
MI355X).  Calls through the C ABI."""
import numpy as np
import pytest

from gpu_common import by_name
from workloads import inputs

pytestmark = pytest.mark.gpu

CON_KEYS = ("ncon", "geom", "feature", "dist", "pos", "frame", "force")


def _plain(m, q, v, u, fr, ms):
    import torch
    import paper_2601_22074_amd as rb
    dev = torch.device("cuda:0")
    M = rb.Model(m)
    n = q.shape[0]
    B = rb.Batch(M, n)
    if fr is not None:
        B.set_params(rb.PARAM_FRICTION, torch.tensor(fr, device=dev))
    if ms is not None:
        B.set_params(rb.PARAM_MASS_SCALE, torch.tensor(ms, device=dev))
    qt, vt = torch.tensor(q, device=dev), torch.tensor(v, device=dev)
    st = torch.zeros(n, dtype=torch.int32, device=dev)
    con = B.contacts(n)
    B.step(torch.tensor(u, device=dev) if M.nu else None, qt, vt, con, st)
    torch.cuda.synchronize()
    out = dict(qpos=qt.cpu().numpy(), qvel=vt.cpu().numpy(), status=st.cpu().numpy(),
               **{k: getattr(con, k).cpu().numpy() for k in CON_KEYS})
    B.close()
    M.close()
    return out


@pytest.mark.parametrize("name", ["humanoid", "arm_box"])
def test_noalloc_step_matches_rb_step(name):
    """Two calls in a row on one model (the second with fewer worlds, so the fixed array holds
    the first call's larger state when it starts): each equals rb_step on a batch just created
    with the same inputs, bit for bit (the two share their kernels)."""
    import torch
    import paper_2601_22074_amd as rb
    dev = torch.device("cuda:0")
    m = by_name(name)
    M = rb.Model(m)
    try:
        for n, first, steps_in in ((512, 0, 30), (37, 100, 10)):
            worlds = range(first, first + n)
            q, v = inputs.initial_state(m, name, worlds)
            u = inputs.ctrl_table(m, name, worlds, 1)[0]
            fr, ms = inputs.world_params(m, name, worlds)
            # states in contact: advanced by plain steps first
            if steps_in:
                g = _plain(m, q, v, u, fr, ms)
                for _ in range(steps_in - 1):
                    g = _plain(m, g["qpos"], g["qvel"], u, fr, ms)
                q, v = g["qpos"], g["qvel"]
            ref = _plain(m, q, v, u, fr, ms)
            qt, vt = torch.tensor(q, device=dev), torch.tensor(v, device=dev)
            st = torch.zeros(n, dtype=torch.int32, device=dev)
            con = rb.Contacts(n, M.contact_capacity)
            M.step_noalloc(torch.tensor(u, device=dev) if M.nu else None, qt, vt,
                           None if fr is None else torch.tensor(fr, device=dev),
                           None if ms is None else torch.tensor(ms, device=dev), con, st)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(qt.cpu().numpy(), ref["qpos"])
            np.testing.assert_array_equal(vt.cpu().numpy(), ref["qvel"])
            np.testing.assert_array_equal(st.cpu().numpy(), ref["status"])
            for k in CON_KEYS:
                np.testing.assert_array_equal(getattr(con, k).cpu().numpy(), ref[k])
            assert int(ref["ncon"].sum()) > 0
    finally:
        M.close()


def test_noalloc_rejects_sizes_beyond_the_array():
    import torch
    import paper_2601_22074_amd as rb
    m = by_name("humanoid")
    M = rb.Model(m)
    per = M.nv + 2 + M.nbody
    n = rb.rbstep.NOALLOC_MAX_FLOATS // per + 1
    q = torch.zeros(n, M.nq, device="cuda")
    v = torch.zeros(n, M.nv, device="cuda")
    u = torch.zeros(n, M.nu, device="cuda")
    with pytest.raises(rb.RbError, match="RB_NOALLOC_MAX_FLOATS"):
        M.step_noalloc(u, q, v)
    M.close()
