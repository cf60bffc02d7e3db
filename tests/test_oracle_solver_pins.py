"""Independent pins of the oracle's impedance curve, of its bias forces for floating trees under
gravity, of its exact line search, and of its work counters (CPU)."""
import copy

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from helpers import q_plus
from workloads import inputs, robots

DEFAULT_SOLIMP = (0.9, 0.95, 0.001, 0.5, 2.0)


# ---------------------------------------------------------------- impedance
def _sphere_model(solimp):
    m = robots.free_body("sphere", size=(0.05,), friction=0.5)
    m["opt"]["solimp"] = list(solimp)
    return m


def _imp_of(o, depth):
    """The oracle's impedance at penetration depth `depth`, read back from a single contact's
    rows: D = imp / ((1 - imp) A-hat), so imp = D A / (1 + D A)."""
    q = np.array([0, 0, 0.05 - depth, 1, 0, 0, 0.0])
    t = o.forward(q, np.zeros(6))
    assert t["ncon"] == 1
    assert abs(-t["dist"][0] - depth) <= 1e-15 + 1e-12 * depth
    x = t["D"] * t["Ahat"]
    imp = x / (1 + x)
    np.testing.assert_allclose(imp, imp[0], rtol=1e-12)   # the contact's four rows share it
    return float(imp[0])


@pytest.mark.parametrize("solimp", [DEFAULT_SOLIMP, (0.5, 0.99, 0.01, 0.3, 3.0)])
def test_impedance_curve_properties(oracle_mod, solimp):
    """Properties the impedance sigmoid's definition fixes (solimp = dmin, dmax, width,
    midpoint, power), checked without re-implementing it: imp -> dmin as the depth -> 0,
    imp = dmax from the width on, imp = dmin + mid (dmax - dmin) at the midpoint, a power law
    of the given order near 0, monotone, and continuous with a continuous slope p (dmax - dmin)
    / width where its two branches meet."""
    dmin, dmax, width, mid, p = solimp
    o = oracle_mod.Oracle(_sphere_model(solimp))
    span = dmax - dmin
    assert abs(_imp_of(o, 1e-9 * width) - dmin) <= 1e-12
    for r in (width, 1.5 * width, 3 * width):
        assert abs(_imp_of(o, r) - dmax) <= 1e-12
    assert abs(_imp_of(o, mid * width) - (dmin + mid * span)) <= 1e-12
    # power law near zero: (imp(2x) - dmin) / (imp(x) - dmin) = 2^p
    x = 0.05 * mid * width
    ratio = (_imp_of(o, 2 * x) - dmin) / (_imp_of(o, x) - dmin)
    assert abs(ratio - 2 ** p) <= 1e-8 * 2 ** p
    grid = np.linspace(0.01, 0.99, 45) * width
    vals = np.array([_imp_of(o, r) for r in grid])
    assert np.all(np.diff(vals) > 0)
    # slope on both sides of the midpoint
    h = 1e-4 * width
    c = mid * width
    left = (_imp_of(o, c) - _imp_of(o, c - h)) / h
    right = (_imp_of(o, c + h) - _imp_of(o, c)) / h
    slope = p * span / width
    assert abs(left / slope - 1) < 2e-3 and abs(right / slope - 1) < 2e-3


def test_impedance_clamped(oracle_mod):
    """The impedance is kept inside [1e-4, 0.9999] whatever solimp asks for."""
    o = oracle_mod.Oracle(_sphere_model((0.0, 1.0, 0.001, 0.5, 2.0)))
    assert abs(_imp_of(o, 1e-12) - 1e-4) <= 1e-15
    assert abs(_imp_of(o, 0.002) - 0.9999) <= 1e-15


# ---------------------------------------------------------------- bias forces of floating trees
def hamel_bias(o, model, q, v, eps=1e-5):
    """c(q, v) from the Boltzmann-Hamel equations in the joint velocities, which are
    quasi-velocities for a free joint (world linear velocity, body-frame angular velocity):
        c_i = sum_jk (X_k M_ij) v_j v_k - 1/2 sum_jk (X_i M_jk) v_j v_k + (w x p_w)_i + X_i V,
    where X_k is the derivative along the configuration flow of unit velocity k (taken by
    central differences through q_plus), p = M v, and the last-but-one term (rotational dofs of
    the free joint only) comes from the brackets of the body-frame rotation fields,
    [X_i, X_j] = eps_ijk X_k; for a single body with its centre of mass at the joint it reduces
    to Euler's w x I w.  Uses only M and the potential V of the oracle, never its bias."""
    n = o.nv
    XM = np.zeros((n, n, n))
    XV = np.zeros(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = eps
        qp, qm = q_plus(model, q, e), q_plus(model, q, -e)
        XM[k] = (o.forward(qp, np.zeros(n))["M"] - o.forward(qm, np.zeros(n))["M"]) / (2 * eps)
        XV[k] = (o.energy(qp, np.zeros(n))[1] - o.energy(qm, np.zeros(n))[1]) / (2 * eps)
    M = o.forward(q, np.zeros(n))["M"]
    pm = M @ v
    c = np.einsum("kij,j,k->i", XM, v, v) - 0.5 * np.einsum("ijk,j,k->i", XM, v, v) + XV
    da = 0
    for j in model["joints"]:
        if j["type"] == "free":
            c[da + 3:da + 6] += np.cross(v[da + 3:da + 6], pm[da + 3:da + 6])
            da += 6
        else:
            da += 1
    return c


def _random_config(model, o, rng):
    q = robots.qpos0(model).astype(float)
    qa = 0
    for j in model["joints"]:
        if j["type"] == "free":
            q[qa:qa + 3] = rng.normal(0, 0.3, 3) + [0, 0, 1.0]
            qv = rng.normal(size=4)
            q[qa + 3:qa + 7] = qv / np.linalg.norm(qv)
            qa += 7
        else:
            q[qa] = rng.uniform(-1, 1)
            qa += 1
    return q


@pytest.mark.parametrize("which", ["free_offset", "quadruped", "humanoid"])
def test_bias_floating_tree_matches_hamel(oracle_mod, which):
    """Bias forces of floating-base trees under gravity against the Boltzmann-Hamel equations
    (the free joint moved through q_plus): a single body with an offset centre of mass and
    rotated principal axes, the floating quadruped and the floating humanoid."""
    model = {"free_offset": robots.free_offset, "quadruped": robots.quadruped, "humanoid": robots.humanoid}[which]()
    model = copy.deepcopy(model)
    model["per_world"] = {"friction": False, "mass_scale": False}
    o = oracle_mod.Oracle(model)
    rng = np.random.default_rng(17)
    for _ in range(2):
        q = _random_config(model, o, rng)
        v = rng.normal(0, 1.0, o.nv)
        c = o.forward(q, v)["bias"]
        ch = hamel_bias(o, model, q, v)
        np.testing.assert_allclose(c, ch, rtol=1e-6, atol=1e-6 * np.abs(ch).max())
        # v = 0: gravity alone
        c0 = o.forward(q, np.zeros(o.nv))["bias"]
        np.testing.assert_allclose(c0, hamel_bias(o, model, q, np.zeros(o.nv)), rtol=1e-6,
                                   atol=1e-7 * np.abs(c0).max())


# ---------------------------------------------------------------- exact line search
def _ground_state(oracle_mod, name, steps, w):
    m = copy.deepcopy(robots.by_name(name))
    m["opt"]["nsubsteps"] = 1
    q, v = inputs.initial_state(m, name, [w])
    u = inputs.ctrl_table(m, name, [w], 1)[0]
    fr, ms = inputs.world_params(m, name, [w])
    o = oracle_mod.Oracle(m)
    qq, vv = q.astype(np.float64), v.astype(np.float64)
    ws = np.zeros((1, o.nv))
    frd = None if fr is None else fr.astype(np.float64)
    msd = None if ms is None else ms.astype(np.float64)
    for _ in range(steps):
        o.step(u.astype(np.float64), qq, vv, ws, frd, msd)
    return o, m, qq[0], vv[0], u[0].astype(np.float64), ws[0], None if fr is None else float(fr[0]), \
        None if ms is None else ms[0].astype(np.float64)


def _phis(t, a, p, alphas):
    M, a0, J, aref, D = t["M"], t["a0"], t["J"], t["aref"], t["D"]
    A = a[None, :] + np.asarray(alphas, float)[:, None] * p[None, :]
    dA = A - a0[None, :]
    quad = 0.5 * np.einsum("ni,ij,nj->n", dA, M, dA)
    jar = A @ J.T - aref[None, :]
    return quad + 0.5 * np.sum(D[None, :] * np.minimum(jar, 0.0) ** 2, axis=1)


@pytest.mark.parametrize("name,steps,w", [("humanoid", 150, 3), ("quadruped", 120, 5), ("humanoid", 200, 11)])
def test_line_search_is_exact(oracle_mod, name, steps, w):
    """alpha* of the oracle's breakpoint sweep against a dense one-dimensional minimisation of
    phi(alpha) = f(a + alpha p), on states in contact with many rows, along directions that
    cross several breakpoints (rows switching on or off)."""
    o, m, q, v, u, ws, fr, ms = _ground_state(oracle_mod, name, steps, w)
    t = o.forward(q, v, u, ws, fr, ms)
    nr = len(t["aref"])
    assert nr >= 8, nr
    rng = np.random.default_rng(w)
    tested = 0
    for trial in range(12):
        a = t["a0"] + rng.normal(0, 1.0, o.nv) * np.abs(t["qacc"] - t["a0"]).max()
        p = (t["qacc"] - a) * rng.uniform(0.5, 3.0) + rng.normal(0, 0.3, o.nv) * np.abs(t["qacc"] - a).max()
        # the oracle's own cost agrees with the definition written from the taps
        f_or, alpha = o.line_search(q, v, a, p, u, ws, fr, ms)
        np.testing.assert_allclose(f_or, _phis(t, a, p, [0.0])[0], rtol=1e-10)
        hi = max(4.0 * alpha, 1.0)
        grid = np.linspace(0.0, hi, 4001)
        vals = _phis(t, a, p, grid)
        # rows crossing their threshold inside the bracket
        jar0 = t["J"] @ a - t["aref"]
        s = t["J"] @ p
        with np.errstate(divide="ignore", invalid="ignore"):
            bp = -jar0 / s
        nbp = int(np.sum((bp > 0) & (bp < hi)))
        k = int(np.argmin(vals))
        lo_b, hi_b = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
        if k == 0:
            ref = 0.0 if _phis(t, a, p, [1e-9 * hi])[0] >= vals[0] else None
        else:
            ref = None
        if ref is None:
            r = minimize_scalar(lambda x: _phis(t, a, p, [x])[0], bounds=(lo_b, hi_b), method="bounded",
                                options={"xatol": 1e-13 * hi})
            ref = r.x
        fa = _phis(t, a, p, [alpha])[0]
        assert fa <= vals.min() * (1 + 1e-12) + 1e-12, (fa, vals.min())
        assert abs(alpha - ref) <= 1e-6 * max(abs(ref), 1e-3), (alpha, ref)
        if nbp >= 3:
            tested += 1
    assert tested >= 4, tested


# ---------------------------------------------------------------- work counters
def _fingerprint(rows):
    return int(sum((int(r) + 1) * 2654435761 for r in rows) % 2 ** 32)


@pytest.mark.parametrize("name", ["humanoid", "quadruped", "humanoid_lim"])
def test_work_counters_match_taps(oracle_mod, name):
    """The per-substep work record of one substep agrees with the stage taps of the same state:
    contacts, rows and Newton updates, and the first update's active-set fingerprint equals the
    fingerprint of the rows active at the Newton start (the better of the warm start and a0)."""
    o, m, q, v, u, ws, fr, ms = _ground_state(oracle_mod, name, 100, 2)
    t = o.forward(q, v, u, ws, fr, ms)
    wk = {}
    qq, vv, ww = q[None].copy(), v[None].copy(), ws[None].copy()
    o.step(u[None], qq, vv, ww, None if fr is None else np.array([fr]), None if ms is None else ms[None], work=wk)
    sub = wk["sub"][0, 0]
    nc, nr = t["ncon"], len(t["aref"])
    assert sub[0] == nc and sub[1] == nr and sub[2] == t["niter"]
    if t["niter"] == 0:
        pytest.skip("no Newton update at this state")
    ids = []
    for c in range(nc):
        ids += [4 * c + e for e in range(4)]
    nlim = nr - 4 * nc
    if nlim:
        # limit rows: J = +-e_dof
        ids += [256 + int(np.flatnonzero(t["J"][4 * nc + i])[0]) for i in range(nlim)]
    f0 = _phis(t, t["a0"], np.zeros(o.nv), [0.0])[0]
    fw = _phis(t, ws, np.zeros(o.nv), [0.0])[0]
    a = ws if fw < f0 else t["a0"]
    jar = t["J"] @ a - t["aref"]
    assert int(sub[5]) & 0xffffffff == _fingerprint([ids[e] for e in np.flatnonzero(jar < 0)])
    jar_end = t["J"] @ t["qacc"] - t["aref"]
    assert sub[3] == int(np.sum(jar_end < 0))
    assert sub[4] >= sub[2]


def test_operation_counts(oracle_mod):
    """Operation counts: no Newton work without contacts, proportional to the substeps for a
    contact-free model, and the tree-sparse formulation never above the plain definitions."""
    m = robots.chain3()
    o = oracle_mod.Oracle(m)
    q, v = inputs.initial_state(m, "chain3", range(4))
    wk = {}
    qq, vv, ws = q.astype(np.float64), v.astype(np.float64), np.zeros((4, 3))
    o.step(np.zeros((4, 0)), qq, vv, ws, work=wk)
    ops1 = wk["ops"]
    assert np.all(ops1[:, :, 5] == 0) and np.all(ops1[:, :, :5].sum(-1) > 0)
    m2 = copy.deepcopy(m)
    m2["opt"]["nsubsteps"] = 2
    o2 = oracle_mod.Oracle(m2)
    wk2 = {}
    qq, vv, ws = q.astype(np.float64), v.astype(np.float64), np.zeros((4, 3))
    o2.step(np.zeros((4, 0)), qq, vv, ws, work=wk2)
    np.testing.assert_allclose(wk2["ops"], 2 * ops1)
    W = inputs.workload("humanoid", 8, 1)
    wk3 = {}
    o3 = oracle_mod.Oracle(W["model"])
    qq, vv = W["qpos"].astype(np.float64), W["qvel"].astype(np.float64)
    ws = np.zeros_like(vv)
    o3.step(W["ctrl"][0].astype(np.float64), qq, vv, ws, W["friction"].astype(np.float64),
            W["mass_scale"].astype(np.float64), work=wk3)
    assert np.all(wk3["ops"][:, 1] <= wk3["ops"][:, 0])
