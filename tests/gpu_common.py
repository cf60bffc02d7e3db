"""Shared helpers for the GPU parity tests: run the HIP path and the oracle on the same inputs."""
from __future__ import annotations

import math

import numpy as np

from workloads import robots

RTOL_STEP = 1e-4      # single env step, per element, |x - ref| <= tol * max(|ref|, 1)
RTOL_ROLLOUT = 1e-3   # 10 contact-free env steps
MARGIN_BAND = 1e-6    # contacts this close to the inclusion threshold may differ


def rel_err(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.max(np.abs(x - ref) / np.maximum(np.abs(ref), 1.0)) if x.size else 0.0


def vec_err(x, ref):
    """max |x - ref| / max(|ref|_inf, 1): error relative to the vector's scale."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1.0) if x.size else 0.0


def gpu_run(model, qpos, qvel, ctrl=None, qacc_ws=None, friction=None, mass_scale=None, nsteps=1,
            contacts=False, taps=False, contact_capacity=0, fields=None):
    """Run the HIP path from float32 inputs; returns a dict of numpy results."""
    import torch
    import paper_2601_22074_amd as rb
    dev = torch.device("cuda:0")
    M = rb.Model(model)
    n = qpos.shape[0]
    B = rb.Batch(M, n, contact_capacity)
    q = torch.tensor(np.asarray(qpos, np.float32), device=dev).contiguous()
    v = torch.tensor(np.asarray(qvel, np.float32), device=dev).contiguous()
    u = torch.tensor(np.asarray(ctrl if ctrl is not None else np.zeros((n, M.nu)), np.float32), device=dev).contiguous()
    if qacc_ws is not None:
        B.reset(torch.arange(n, dtype=torch.int32, device=dev),
                torch.tensor(np.asarray(qacc_ws, np.float32), device=dev).contiguous())
    if friction is not None:
        B.set_params(rb.PARAM_FRICTION, torch.tensor(np.asarray(friction, np.float32), device=dev).contiguous())
    if mass_scale is not None:
        B.set_params(rb.PARAM_MASS_SCALE, torch.tensor(np.asarray(mass_scale, np.float32), device=dev).contiguous())
    for k, a in (fields or {}).items():
        B.set_params(getattr(rb, FIELD_PARAMS[k]), torch.tensor(np.asarray(a, np.float32), device=dev).contiguous())
    st = torch.zeros(n, dtype=torch.int32, device=dev)
    con = B.contacts(n) if contacts else None
    out = {}
    for k in range(nsteps):
        if taps and k == 0:
            nv = M.nv
            Mt = torch.zeros(n, nv, nv, device=dev); bias = torch.zeros(n, nv, device=dev)
            a0 = torch.zeros(n, nv, device=dev); qacc = torch.zeros(n, nv, device=dev)
            efc = torch.zeros(n, B.ncap, 4, 3, device=dev)
            from paper_2601_22074_amd.rbstep import NSTATS
            stats = torch.zeros(n, NSTATS, dtype=torch.int32, device=dev)
            B.step_taps(u, q, v, con, st, M=Mt, bias=bias, a0=a0, qacc=qacc, efc=efc, stats=stats)
            out.update(M=Mt, bias=bias, a0=a0, qacc=qacc, efc=efc, stats=stats)
        else:
            B.step(u, q, v, con, st)
    torch.cuda.synchronize()
    ws = torch.zeros(n, M.nv, device=dev)
    B.get_state(n, ws, None)
    torch.cuda.synchronize()
    res = {k: t.cpu().numpy() for k, t in out.items()}
    res.update(qpos=q.cpu().numpy(), qvel=v.cpu().numpy(), qacc_ws=ws.cpu().numpy(), status=st.cpu().numpy(),
               ncap=B.ncap)
    if con is not None:
        res["contacts"] = {k: getattr(con, k).cpu().numpy() for k in ("ncon", "geom", "feature", "dist", "pos",
                                                                      "frame", "force")}
    B.close()
    M.close()
    return res


def oracle_run(o, qpos, qvel, ctrl=None, qacc_ws=None, friction=None, mass_scale=None, nsteps=1, contacts=False):
    n = qpos.shape[0]
    q = np.array(qpos, np.float64, order="C")
    v = np.array(qvel, np.float64, order="C")
    ws = np.zeros((n, o.nv)) if qacc_ws is None else np.array(qacc_ws, np.float64, order="C")
    u = np.zeros((n, o.nu)) if ctrl is None else np.array(ctrl, np.float64)
    fr = None if friction is None else np.asarray(friction, np.float64)
    ms = None if mass_scale is None else np.asarray(mass_scale, np.float64)
    st = np.zeros(n, np.uint32)
    cs = None
    for _ in range(nsteps):
        st, cs = o.step(u, q, v, ws, fr, ms, st, contacts=contacts)
    return dict(qpos=q, qvel=v, qacc_ws=ws, status=st, contacts=cs)


def contact_keys(c, w, dist_band=MARGIN_BAND):
    """(g1, g2, feature) of world w's contacts, split into (certain, near-margin) sets."""
    n = int(c["ncon"][w])
    certain, band = set(), set()
    for i in range(n):
        k = (int(c["geom"][w, i, 0]), int(c["geom"][w, i, 1]), int(c["feature"][w, i]))
        (band if abs(c["dist"][w, i]) <= dist_band else certain).add(k)
    return certain, band


def lifted(model, qpos, height=2.0):
    q = np.array(qpos, np.float64)
    for (t, qa, _), j in zip(_layout(model), model["joints"]):
        if t == "free":
            q[:, qa + 2] += height
    return q.astype(np.float32)


def _layout(model):
    out, qa, da = [], 0, 0
    for j in model["joints"]:
        out.append((j["type"], qa, da))
        qa, da = (qa + 7, da + 6) if j["type"] == "free" else (qa + 1, da + 1)
    return out


def substeps1(model):
    m = dict(model)
    m["opt"] = dict(model["opt"], nsubsteps=1)
    return m


def by_name(name):
    return robots.by_name(name)


def band_worlds(oracle_mod, model, qpos, qvel, ctrl, qacc_ws, friction, mass_scale, fields=None):
    """Per world: whether one env step from this FP32 state passes a contact within MARGIN_BAND
    of its inclusion threshold at the start of some substep.  Such a contact may be included by
    one path only, and a contact row that acts in one path and not in the other changes the
    step by far more than rounding.  Found with the oracle alone: its substeps are replayed one
    at a time and each starting state's contacts are listed by a copy of the model whose
    margins are widened by the band."""
    import copy
    m1 = substeps1(model)
    wide = copy.deepcopy(m1)
    for g in wide["geoms"]:
        g["margin"] = g["margin"] + MARGIN_BAND
    o1, ow = oracle_mod.Oracle(m1), oracle_mod.Oracle(wide)
    n = qpos.shape[0]
    if fields:
        # per-world fields: world w's contacts listed by a widened model carrying its values
        oww = [oracle_mod.Oracle(with_fields(wide, fields, w)) for w in range(n)]
    q = np.array(qpos, np.float64); v = np.array(qvel, np.float64)
    ws = np.zeros((n, o1.nv)) if qacc_ws is None else np.array(qacc_ws, np.float64)
    u = np.zeros((n, o1.nu)) if ctrl is None else np.asarray(ctrl, np.float64)
    gm = [g["margin"] for g in model["geoms"]]
    band = np.zeros(n, bool)
    for _ in range(model["opt"]["nsubsteps"]):
        for w in range(n):
            t = (oww[w] if fields else ow).forward(q[w], v[w], u[w] if o1.nu else None, ws[w],
                                                  None if friction is None else friction[w],
                                                  None if mass_scale is None else mass_scale[w])
            band[w] |= any(abs(d - max(gm[g1], gm[g2])) <= MARGIN_BAND for (g1, g2), d in zip(t["geom"], t["dist"]))
        o1.step(u, q, v, ws, None if friction is None else np.asarray(friction, np.float64),
                None if mass_scale is None else np.asarray(mass_scale, np.float64), fields=fields)
    return band


def with_fields(model, fields, w):
    """Copy of a model description carrying world w's values of the per-world fields."""
    import copy
    m = copy.deepcopy(model)
    for k, a in fields.items():
        a = np.asarray(a, np.float64)[w]
        if k == "geom_size":
            for g, x in zip(m["geoms"], a):
                g["size"] = [float(y) for y in x]
        elif k == "body_pos":
            for b, x in zip(m["bodies"], a):
                b["pos"] = [float(y) for y in x]
        else:
            key = "kp" if k == "act_kp" else "kd"
            for act, x in zip(m["actuators"], a):
                act[key] = float(x)
    return m


# per-substep work record columns compared between the two paths: contacts, rows, Newton
# updates, rows active at the solution, and the active-set fingerprints of the first updates
# (line-search segment counts are left out: equal breakpoints may be swept as one or two)
REC_COLS = [0, 1, 2, 3, 5, 6, 7, 8]
CON_COLS = [0, 1]


FIELD_PARAMS = {"geom_size": "PARAM_GEOM_SIZE", "body_pos": "PARAM_BODY_POS", "act_kp": "PARAM_ACT_KP",
                "act_kd": "PARAM_ACT_KD"}


def gpu_step_records(model, q32, v32, u32, w32, fr, ms, fields=None):
    """One env step of every world on the GPU from FP32 inputs: the plain launch (results and
    contacts) and the diagnostic launch (per-substep work records), which must compute the same
    bits."""
    import torch
    import paper_2601_22074_amd as rb
    from paper_2601_22074_amd.rbstep import NSTATS
    dev = torch.device("cuda:0")
    n = q32.shape[0]
    M = rb.Model(model)
    B = rb.Batch(M, n)
    res = {}
    try:
        if fr is not None:
            B.set_params(rb.PARAM_FRICTION, torch.tensor(np.asarray(fr, np.float32), device=dev))
        if ms is not None:
            B.set_params(rb.PARAM_MASS_SCALE, torch.tensor(np.asarray(ms, np.float32), device=dev))
        for k, a in (fields or {}).items():
            B.set_params(getattr(rb, FIELD_PARAMS[k]), torch.tensor(np.asarray(a, np.float32), device=dev).contiguous())
        ids = torch.arange(n, dtype=torch.int32, device=dev)
        u = u32 if M.nu else np.zeros((n, 0), np.float32)
        for diag in (False, True):
            qt, vt = torch.tensor(q32, device=dev), torch.tensor(v32, device=dev)
            ut = torch.tensor(np.asarray(u, np.float32), device=dev)
            B.reset(ids, torch.tensor(w32, device=dev))
            sta = torch.zeros(n, dtype=torch.int32, device=dev)
            if diag:
                stats = torch.zeros(n, NSTATS, dtype=torch.int32, device=dev)
                B.step_taps(ut, qt, vt, None, sta, stats=stats)
                torch.cuda.synchronize()
                res["stats"] = stats.cpu().numpy()
                np.testing.assert_array_equal(qt.cpu().numpy(), res["qpos"])
                np.testing.assert_array_equal(vt.cpu().numpy(), res["qvel"])
            else:
                con = B.contacts(n)
                B.step(ut, qt, vt, con, sta)
                torch.cuda.synchronize()
                res.update(qpos=qt.cpu().numpy(), qvel=vt.cpu().numpy(), status=sta.cpu().numpy(),
                           contacts={k: getattr(con, k).cpu().numpy() for k in
                                     ("ncon", "geom", "feature", "dist", "pos", "frame", "force")})
    finally:
        B.close()
        M.close()
    K = model["opt"]["nsubsteps"] if isinstance(model, dict) else None
    res["sub"] = res["stats"][:, 14:14 + 36].reshape(n, 4, 9)[:, :K]
    return res


def oracle_step_records(o, q32, v32, u32, w32, fr, ms, fields=None):
    """The oracle's env step (mirror mode, with contacts and per-substep work records) and the
    converged-mode step from the same FP32 inputs."""
    n = q32.shape[0]
    f64 = lambda a: None if a is None else np.asarray(a, np.float64)
    u = np.zeros((n, o.nu)) if u32 is None else np.asarray(u32, np.float64)
    rq, rv, rw = (np.array(x, np.float64) for x in (q32, v32, w32))
    work = {}
    _, con = o.step(u, rq, rv, rw, f64(fr), f64(ms), contacts=True, work=work, fields=fields)
    o.set_mode("converged")
    cq, cv, cw = (np.array(x, np.float64) for x in (q32, v32, w32))
    o.step(u, cq, cv, cw, f64(fr), f64(ms), fields=fields)
    o.set_mode("mirror")
    return dict(qpos=rq, qvel=rv, qacc_ws=rw, contacts=con, sub=work["sub"], cq=cq, cv=cv)


def classify(gsub, osub, smooth=False):
    """'match': the two paths made the same contacts, rows, Newton updates and active sets in
    every substep; 'contacts': they listed different contacts or rows in some substep; 'path':
    same contacts and rows, different Newton updates or active sets.  smooth (elliptic cones):
    contacts that differ only after a substep whose solve already differed are 'path' too (the
    solve's difference moved the next substep's state)."""
    if np.array_equal(gsub[:, REC_COLS], osub[:, REC_COLS]):
        return "match"
    if not np.array_equal(gsub[:, CON_COLS], osub[:, CON_COLS]):
        if smooth:
            k = next(i for i in range(len(gsub)) if not np.array_equal(gsub[i, REC_COLS], osub[i, REC_COLS]))
            if np.array_equal(gsub[k, CON_COLS], osub[k, CON_COLS]):
                return "path"
        return "contacts"
    return "path"


DEPTH_TOL = 3e-7      # FP32 contact-depth error of the GPU's kinematics (asserted on the stage taps)


FP32_U = 2.0 ** -24    # unit roundoff of FP32
RESIDUAL_TOL = 3e-4    # same-path samples beyond RTOL_STEP and their floor: at most this error ...
RESIDUAL_FRAC = 0.005  # ... in at most this fraction (rounded up) of the same-path samples
FLOOR_ULPS = 4         # input perturbation of the FP32 floor, in unit roundoffs
CONV_TRUNC = 1e-7      # the oracle's truncated step equals its converged step below FP32 resolution
FD_REL = 1e-9          # finite-difference step, relative to max(|x|, 1)


def _floor(f, xs, scale):
    """First-order worst case of |f(xs + d) - f(xs)| over perturbations |d_i| <= FLOOR_ULPS *
    FP32_U * max(|x_i|, 1) of every element of the arrays xs, divided elementwise by
    scale(f(xs)): the componentwise condition of f at single-precision inputs on R23's scale.
    Derivatives by forward differences of FD_REL * max(|x_i|, 1), small enough that no contact
    flips its inclusion."""
    y0 = f(*xs)
    bound = np.zeros_like(y0)
    for k, x in enumerate(xs):
        for i in range(x.size):
            h = FD_REL * max(abs(x.flat[i]), 1.0)
            xp = [a.copy() for a in xs]
            xp[k].flat[i] += h
            bound += np.abs(f(*xp) - y0) / h * (FLOOR_ULPS * FP32_U * max(abs(x.flat[i]), 1.0))
    return float(np.max(bound / scale(y0)))


def fp32_floor(o, model, q32, v32, u32, w32, fr, ms, j, fields=None):
    """The FP32 floor of world j's env step (R23 metric over qpos and qvel): how far the FP64
    step can move when its inputs (qpos, qvel, warm start) carry the rounding of a few units of
    single precision (_floor).  A single-precision step that rounds backward-stably resolves the
    step only to about this; it is large where stiff contact rows (aref moves by k imp ~ 2600 /
    s^2 per metre of depth) act on light dofs, and where the 4-update Newton iterate is
    truncated.  Computed by the oracle alone."""
    sl = slice(j, j + 1)
    f64 = lambda a: None if a is None else np.asarray(a[sl], np.float64)
    u = np.zeros((1, o.nu)) if u32 is None else np.asarray(u32[sl], np.float64)

    fj = None if not fields else {k: np.asarray(a)[sl] for k, a in fields.items()}

    def step(q, v, w):
        q, v, w = q[None].copy(), v[None].copy(), w[None].copy()
        o.step(u, q, v, w, f64(fr), f64(ms), fields=fj)
        return np.concatenate([q[0], v[0]])

    xs = [np.asarray(x[j], np.float64) for x in (q32, v32, w32)]
    return _floor(step, xs, lambda y: np.maximum(np.abs(y), 1.0))


def qacc_floor(oracle_mod, model, q, v, u, ws, fr, ms):
    """fp32_floor's counterpart for one substep's constrained acceleration at one world's state
    (vec_err metric)."""
    o = oracle_mod.Oracle(model)
    acc = lambda qq, vv, ww: o.forward(qq, vv, u, ww, fr, ms)["qacc"]
    xs = [np.asarray(x, np.float64) for x in (q, v, ws)]
    return _floor(acc, xs, lambda y: max(np.max(np.abs(y)), 1.0))


def _memo(f):
    box = []
    return lambda: box[0] if box else (box.append(f()) or box[0])


class StepTally:
    """Single-step parity of one workload over many (world, state) samples.

    Per sample (R23 metric, tolerance RTOL_STEP):
      * same work records on both paths ('match'): qpos and qvel within RTOL_STEP (or, where the
        oracle's own step moves by more than that when its inputs carry single-precision rounding,
        within that FP32 floor: fp32_floor; beyond both, at most RESIDUAL_FRAC of these samples
        within RESIDUAL_TOL, each printed), and the last substep's contacts (keys exactly;
        dist and pos within RTOL_STEP m, frame within RTOL_STEP, the qpos bar carried to the
        contact geometry; force within RTOL_STEP of the world's largest contact force plus
        RTOL_STEP of the contact's own: the accelerations' bar carried to the multipliers, and
        the stage taps' bar on A-hat carried through the rows' D);
      * different contacts or rows in some substep ('contacts'): allowed only where the oracle
        finds a contact within MARGIN_BAND of its inclusion threshold at the start of a substep
        (the contact pair-set rule); qpos and qvel are then not compared;
      * same contacts and rows, different Newton updates or active sets ('path'): the truncated
        Newton iterate depends on its path, and the bar is RTOL_STEP plus a tenth of the FP64
        distance between the 4-iteration and the converged step.
    Over the workload: 'path' samples at most 5 %, iteration counts equal in at least 98 % of
    the compared samples, 'contacts' samples at most a sixth, samples on their FP32 floor at
    most 1 %."""

    def __init__(self, name, smooth=False, force_scale=1.0):
        """smooth: the model's cost is not piecewise quadratic (elliptic cones), so its Newton
        iteration ends in a quadratic-convergence tail where the FP64 and FP32 improvement tests
        fire one update apart; a sample whose records differ while the oracle's truncated step
        already equals its converged step to FP32 resolution (CONV_TRUNC) is then compared as a
        same-path sample and left out of the iteration-count statistic.
        force_scale: the contact-force bar's factor; an elliptic contact's tangential rows have
        impratio times the normal row's D, so the same acceleration error moves their forces
        impratio times as much."""
        self.name = name
        self.smooth = smooth
        self.force_scale = force_scale
        self.nconv = 0
        self.n = self.nmatch = self.npath = self.ncon = self.nband = self.iteq = self.ncmp = self.nfloor = 0
        self.nresidual = 0
        self.worst = self.worst_path = 0.0
        self.cworst = dict(dist=0.0, pos=0.0, frame=0.0, force=0.0)

    def add(self, g, r, gw, rw, band, where, floor=None):
        """floor: callable giving the sample's FP32 floors (fp32_floor), asked only where an
        error exceeds RTOL_STEP."""
        floor = _memo(floor) if floor is not None else (lambda: 0.0)
        gs, os_ = g["sub"][gw], r["sub"][rw]
        kind = classify(gs, os_, self.smooth)
        if kind == "path" and band and not np.array_equal(gs[:, CON_COLS], os_[:, CON_COLS]):
            # (smooth mode) contact sets that differ after a solve that differed: where the world
            # also has a contact on its inclusion threshold, that contact decided the later
            # substep's set, so the sample is a threshold sample like any other
            kind = "contacts"
        self.n += 1
        err = max(rel_err(g[k][gw], r[k][rw]) for k in ("qpos", "qvel"))
        if kind == "contacts":
            assert band, (where, "contact records differ with no contact on its threshold", gs.tolist(), os_.tolist())
            self.ncon += 1
            return
        trunc = None
        if kind == "path":
            trunc = max(rel_err(r["cq"][rw], r["qpos"][rw]), rel_err(r["cv"][rw], r["qvel"][rw]))
            if self.smooth and trunc <= CONV_TRUNC:
                kind = "converged"
                self.nconv += 1
        if kind != "converged":
            self.ncmp += 1
            self.iteq += bool(np.array_equal(gs[:, 2], os_[:, 2]))
        if kind in ("match", "converged"):
            self.nmatch += 1
            if err > RTOL_STEP:
                fl = floor()
                if err > fl:
                    # beyond the input-rounding floor too: FP32 formation of M and H in a frame at
                    # the root (cancellation on light distal dofs with large accelerations); capped
                    assert err <= RESIDUAL_TOL, (where, err, fl)
                    self.nresidual += 1
                    print(f"  FP32 residual: {where} err {err:.2e} floor {fl:.2e}", flush=True)
                else:
                    self.nfloor += 1
            else:
                self.worst = max(self.worst, err)
            if not band:
                self._contacts(g["contacts"], r["contacts"], gw, rw, where)
        else:
            self.npath += 1
            if self.smooth:
                # the elliptic cost's Hessian jumps at the cones' zone boundaries, so iterates
                # that crossed them differently differ by up to the truncation itself: the GPU's
                # step must lie as close to the oracle's converged step as twice the oracle's own
                conv = max(rel_err(g["qpos"][gw], r["cq"][rw]), rel_err(g["qvel"][gw], r["cv"][rw]))
                assert conv <= RTOL_STEP + 2 * trunc, (where, conv, trunc, gs.tolist(), os_.tolist())
            else:
                assert err <= RTOL_STEP + 0.1 * trunc, (where, err, trunc, gs.tolist(), os_.tolist())
            self.worst_path = max(self.worst_path, err)

    def _contacts(self, gc, rc, gw, rw, where):
        nc = int(rc["ncon"][rw])
        assert int(gc["ncon"][gw]) == nc, where
        if nc == 0:
            return
        assert [tuple(x) for x in gc["geom"][gw, :nc]] == [tuple(x) for x in rc["geom"][rw, :nc]], where
        assert list(gc["feature"][gw, :nc]) == list(rc["feature"][rw, :nc]), where
        fg, fr_ = gc["force"][gw, :nc].astype(np.float64), rc["force"][rw, :nc]
        e = dict(dist=np.abs(gc["dist"][gw, :nc] - rc["dist"][rw, :nc]).max(),
                 pos=rel_err(gc["pos"][gw, :nc], rc["pos"][rw, :nc]),
                 frame=np.abs(gc["frame"][gw, :nc].reshape(nc, 9) - rc["frame"][rw, :nc].reshape(nc, 9)).max(),
                 # per element: RTOL_STEP of the world's largest contact force (the accelerations'
                 # bar carried to the multipliers) plus RTOL_STEP of the contact's own force (A-hat's
                 # bar on the stage taps carried through D = imp / ((1 - imp) A-hat) into each of
                 # its pyramid rows, whose forces make up all three components)
                 force=np.max(np.abs(fg - fr_) / (max(np.abs(fr_).max(), 1.0)
                                                   + np.linalg.norm(fr_, axis=1, keepdims=True))))
        for k, x in e.items():
            assert x <= RTOL_STEP * (self.force_scale if k == "force" else 1.0), (where, k, x)
            self.cworst[k] = max(self.cworst[k], float(x))

    def finish(self):
        print(f"{self.name}: {self.n} samples: {self.nmatch} same path (max err {self.worst:.2e}, "
              f"{self.nfloor} above RTOL_STEP within their FP32 floor, {self.nresidual} FP32 residuals), "
              f"{self.npath} path differences (max err {self.worst_path:.2e}), {self.nconv} converged with different "
              f"update counts, {self.ncon} contact-threshold "
              f"samples not compared; iteration counts equal in {self.iteq}/{self.ncmp}; contact outputs max "
              + ", ".join(f"{k} {v:.1e}" for k, v in self.cworst.items()), flush=True)
        # (elliptic cones: zone changes make path differences, and the improvement test's FP32
        # and FP64 decisions in the quadratic tail update-count differences, more common; their
        # caps are 10 % and 90 %)
        assert self.npath <= (0.10 if self.smooth else 0.05) * self.n, (self.npath, self.n)
        assert self.iteq >= (0.90 if self.smooth else 0.98) * self.ncmp, (self.iteq, self.ncmp)
        assert self.ncon <= self.n / 6, (self.ncon, self.n)
        assert self.nfloor <= 0.01 * self.n, (self.nfloor, self.n)
        assert self.nresidual <= math.ceil(RESIDUAL_FRAC * (self.nmatch + self.nconv)), (self.nresidual, self.nmatch)


def teacher_forced(oracle_mod, name, horizon, every=25, n=32):
    """Along the oracle's own trajectory of n worlds, hand its state (rounded to FP32) to the GPU
    every ``every`` env steps and compare one env step of every world (StepTally)."""
    from workloads import inputs
    m = by_name(name)
    worlds = list(range(n))
    q, v = inputs.initial_state(m, name, worlds)
    fr, ms = inputs.world_params(m, name, worlds)
    o = oracle_mod.Oracle(m)
    ctab = inputs.ctrl_table(m, name, worlds, horizon // 20 + 1)
    qq = q.astype(np.float64); vv = v.astype(np.float64); ws = np.zeros((n, o.nv)); st = np.zeros(n, np.uint32)
    frd = None if fr is None else fr.astype(np.float64)
    msd = None if ms is None else ms.astype(np.float64)
    ell = m["opt"].get("cone") == "elliptic"
    T = StepTally(name, smooth=ell, force_scale=max(1.0, m["opt"].get("impratio", 1.0)) if ell else 1.0)
    for s in range(horizon):
        uu = ctab[s // 20].astype(np.float64)
        if s % every == every - 1:
            q32, v32, w32, u32 = (x.astype(np.float32) for x in (qq, vv, ws, uu))
            g = gpu_step_records(m, q32, v32, u32, w32, fr, ms)
            r = oracle_step_records(o, q32, v32, u32, w32, fr, ms)
            band = band_worlds(oracle_mod, m, q32, v32, u32, w32, fr, ms)
            assert np.all(g["status"] & 1 == 0)
            for w in range(n):
                T.add(g, r, w, w, band[w], (name, s, w),
                      floor=lambda w=w: fp32_floor(o, m, q32, v32, u32, w32, fr, ms, w))
        o.step(uu, qq, vv, ws, frd, msd, st)
    T.finish()
    return T
