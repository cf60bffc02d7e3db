"""ctypes marshalling for the FP64 oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_GEOM = {"plane": 0, "sphere": 1, "capsule": 2, "box": 3, "hfield": 4}
_EQ = {"connect": 0, "weld": 1}
_JNT = {"free": 0, "hinge": 1}
_ACT = {"position": 0, "motor": 1}

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)


class _Desc(C.Structure):
    _fields_ = [("nbody", C.c_int32), ("njnt", C.c_int32), ("ngeom", C.c_int32), ("nu", C.c_int32),
                ("body_parent", _i32p),
                ("body_pos", _f64p), ("body_quat", _f64p), ("body_ipos", _f64p), ("body_iquat", _f64p),
                ("body_mass", _f64p), ("body_inertia", _f64p),
                ("jnt_type", _i32p), ("jnt_body", _i32p),
                ("jnt_pos", _f64p), ("jnt_axis", _f64p), ("jnt_armature", _f64p),
                ("geom_type", _i32p), ("geom_body", _i32p), ("geom_contype", _i32p), ("geom_conaffinity", _i32p),
                ("geom_pos", _f64p), ("geom_quat", _f64p), ("geom_size", _f64p), ("geom_friction", _f64p),
                ("geom_margin", _f64p),
                ("act_type", _i32p), ("act_joint", _i32p),
                ("act_kp", _f64p), ("act_kd", _f64p), ("act_gear", _f64p),
                ("timestep", C.c_double), ("nsubsteps", C.c_int32), ("gravity", C.c_double * 3),
                ("iterations", C.c_int32), ("tolerance", C.c_double), ("solref", C.c_double * 2),
                ("solimp", C.c_double * 5), ("friction_per_world", C.c_int32), ("mass_scale_per_world", C.c_int32),
                ("jnt_range", _f64p), ("jnt_damping", _f64p), ("geom_condim", _i32p),
                ("hfield_nrow", C.c_int32), ("hfield_ncol", C.c_int32), ("hfield_data", _f64p),
                ("neq", C.c_int32), ("eq_type", _i32p), ("eq_body", _i32p), ("eq_anchor", _f64p), ("eq_target", _f64p),
                ("geom_friction_spin", _f64p), ("geom_friction_roll", _f64p),
                ("cone", C.c_int32), ("impratio", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("nq", C.c_int32), ("nv", C.c_int32), ("nu", C.c_int32), ("nbody", C.c_int32),
                ("ngeom", C.c_int32), ("maxcon", C.c_int32), ("maxrows", C.c_int32), ("npair", C.c_int32),
                ("meaninertia", C.c_double)]


class _Contacts(C.Structure):
    _fields_ = [("ncon", _i32p), ("geom", _i32p), ("feature", _i32p), ("dist", _f64p), ("pos", _f64p),
                ("frame", _f64p), ("force", _f64p)]


_TAP_FIELDS = [("xpos", "f", "nb3"), ("xquat", "f", "nb4"), ("xmat", "f", "nb9"), ("com", "f", "nb3"),
               ("gpos", "f", "ng3"), ("gmat", "f", "ng9"),
               ("M", "f", "nvnv"), ("bias", "f", "nv"), ("tau", "f", "nv"), ("a0", "f", "nv"),
               ("ncon", "i", "1"), ("geom", "i", "mc2"), ("feature", "i", "mc"),
               ("dist", "f", "mc"), ("pos", "f", "mc3"), ("frame", "f", "mc9"), ("mu", "f", "mc"),
               ("J", "f", "mrnv"), ("aref", "f", "mr"), ("D", "f", "mr"), ("Ahat", "f", "mr"),
               ("efc_force", "f", "mr"), ("qacc", "f", "nv"), ("cforce", "f", "mc3"),
               ("niter", "i", "1"), ("cost", "f", "1"), ("nrows", "i", "1")]


class _Taps(C.Structure):
    _fields_ = [(n, _f64p if t == "f" else _i32p) for n, t, _ in _TAP_FIELDS]


_lib = None

FPITER = 4                 # active-set fingerprints per substep (rbo.h)
SUBCOLS = 5 + FPITER       # per-substep work columns
NSTAGE = 7                 # operation-count stages
STAGES = ("kinematics", "inertia and bias", "factorisation and a0", "collision", "constraint rows", "newton",
          "integration")


def build_if_missing() -> None:
    if not os.path.exists(_build.LIB):
        _build.build()


class _Fields(C.Structure):
    _fields_ = [("geom_size", _f64p), ("body_pos", _f64p), ("act_kp", _f64p), ("act_kd", _f64p)]


FIELDS = ("geom_size", "body_pos", "act_kp", "act_kd")


def lib():
    global _lib
    if _lib is None:
        build_if_missing()
        L = C.CDLL(_build.LIB)
        L.rbo_last_error.restype = C.c_char_p
        L.rbo_model_create.argtypes = [C.POINTER(_Desc), C.POINTER(C.c_void_p)]
        L.rbo_model_destroy.argtypes = [C.c_void_p]
        L.rbo_model_info.argtypes = [C.c_void_p, C.POINTER(_Info)]
        L.rbo_set_mode.argtypes = [C.c_void_p, C.c_int32]
        L.rbo_forward.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, C.POINTER(_Taps)]
        L.rbo_step.argtypes = [C.c_void_p, C.c_int32, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p,
                               C.POINTER(C.c_uint32), C.POINTER(_Contacts), C.c_int32]
        L.rbo_step_work.argtypes = [C.c_void_p, C.c_int32, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p,
                                    C.POINTER(C.c_uint32), C.POINTER(_Contacts), _i32p, _f64p, C.c_int32]
        L.rbo_step_fields.argtypes = [C.c_void_p, C.c_int32, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p,
                                      C.POINTER(_Fields), C.POINTER(C.c_uint32), C.POINTER(_Contacts), _i32p, _f64p,
                                      C.c_int32]
        L.rbo_line_search.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p,
                                      _f64p, _f64p]
        L.rbo_energy.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p, _f64p]
        L.rbo_jacobian.argtypes = [C.c_void_p, _f64p, C.c_int32, _f64p, _f64p, _f64p]
        L.rbo_integrate.argtypes = [C.c_void_p, _f64p, _f64p, _f64p, _f64p, _f64p]
        _lib = L
    return _lib


def _f(a):
    return None if a is None else a.ctypes.data_as(_f64p)


def _d(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return a if n is None else a.reshape(n)


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle: " + lib().rbo_last_error().decode())


class Oracle:
    """FP64 reference for one model description (see ``workloads.robots``)."""

    def __init__(self, model: dict):
        L = lib()
        B, Jt, G, A = model["bodies"], model["joints"], model["geoms"], model["actuators"]
        keep = []

        def i32(x):
            a = np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(-1))
            keep.append(a)
            return a.ctypes.data_as(_i32p)

        def f64(x):
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
            keep.append(a)
            return a.ctypes.data_as(_f64p)

        d = _Desc()
        d.nbody, d.njnt, d.ngeom, d.nu = len(B), len(Jt), len(G), len(A)
        d.body_parent = i32([b["parent"] for b in B])
        d.body_pos = f64([b["pos"] for b in B]); d.body_quat = f64([b["quat"] for b in B])
        d.body_ipos = f64([b["ipos"] for b in B]); d.body_iquat = f64([b["iquat"] for b in B])
        d.body_mass = f64([b["mass"] for b in B]); d.body_inertia = f64([b["inertia"] for b in B])
        d.jnt_type = i32([_JNT[j["type"]] for j in Jt] or [0]); d.jnt_body = i32([j["body"] for j in Jt] or [0])
        d.jnt_pos = f64([j["pos"] for j in Jt] or [0.0]); d.jnt_axis = f64([j["axis"] for j in Jt] or [0.0])
        d.jnt_armature = f64([j["armature"] for j in Jt] or [0.0])
        d.geom_type = i32([_GEOM[g["type"]] for g in G] or [0]); d.geom_body = i32([g["body"] for g in G] or [0])
        d.geom_contype = i32([g["contype"] for g in G] or [0])
        d.geom_conaffinity = i32([g["conaffinity"] for g in G] or [0])
        d.geom_pos = f64([g["pos"] for g in G] or [0.0]); d.geom_quat = f64([g["quat"] for g in G] or [0.0])
        d.geom_size = f64([g["size"] for g in G] or [0.0]); d.geom_friction = f64([g["friction"] for g in G] or [0.0])
        d.geom_margin = f64([g["margin"] for g in G] or [0.0])
        d.act_type = i32([_ACT[a["type"]] for a in A] or [0]); d.act_joint = i32([a["joint"] for a in A] or [0])
        d.act_kp = f64([a["kp"] for a in A] or [0.0]); d.act_kd = f64([a["kd"] for a in A] or [0.0])
        d.act_gear = f64([a["gear"] for a in A] or [0.0])
        o = model["opt"]
        d.timestep = o["timestep"]; d.nsubsteps = o["nsubsteps"]
        d.gravity = (C.c_double * 3)(*o["gravity"])
        d.iterations = o["iterations"]; d.tolerance = o["tolerance"]
        d.solref = (C.c_double * 2)(*o["solref"]); d.solimp = (C.c_double * 5)(*o["solimp"])
        d.friction_per_world = int(bool(model["per_world"].get("friction")))
        d.mass_scale_per_world = int(bool(model["per_world"].get("mass_scale")))
        d.jnt_range = f64([j.get("range", [0.0, 0.0]) for j in Jt] or [0.0, 0.0])
        d.jnt_damping = f64([j.get("damping", 0.0) for j in Jt] or [0.0])
        d.geom_condim = i32([g.get("condim", 3) for g in G] or [3])
        d.geom_friction_spin = f64([g.get("friction_spin", 0.005) for g in G] or [0.0])
        d.geom_friction_roll = f64([g.get("friction_roll", 0.0001) for g in G] or [0.0])
        d.cone = {"pyramidal": 0, "elliptic": 1}[o.get("cone", "pyramidal")]
        d.impratio = float(o.get("impratio", 1.0))
        hf = model.get("hfield")
        if hf:
            d.hfield_nrow, d.hfield_ncol = int(hf["nrow"]), int(hf["ncol"])
            d.hfield_data = f64(hf["data"])
        E = model.get("equality", [])
        if E:
            d.neq = len(E)
            d.eq_type = i32([_EQ[e["type"]] for e in E]); d.eq_body = i32([e["body"] for e in E])
            d.eq_anchor = f64([e["anchor"] for e in E])
            d.eq_target = f64([list(e["target"]) + list(e.get("quat", [1.0, 0.0, 0.0, 0.0])) for e in E])
        h = C.c_void_p()
        _check(L.rbo_model_create(C.byref(d), C.byref(h)))
        self._h = h
        self.model = model
        info = _Info()
        _check(L.rbo_model_info(h, C.byref(info)))
        self.nq, self.nv, self.nu, self.nbody = info.nq, info.nv, info.nu, info.nbody
        self.ngeom, self.maxcon, self.maxrows, self.npair = info.ngeom, info.maxcon, info.maxrows, info.npair
        self.meaninertia = info.meaninertia

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().rbo_model_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def set_mode(self, mode: str) -> None:
        _check(lib().rbo_set_mode(self._h, {"mirror": 0, "converged": 1}[mode]))

    # ------------------------------------------------------------------------------
    def forward(self, qpos, qvel, ctrl=None, qacc_ws=None, friction=None, mass_scale=None) -> dict:
        """Stage taps of one substep (no integration) for one world."""
        nv, nb, ng, mc, mr = self.nv, self.nbody, self.ngeom, self.maxcon, self.maxrows
        sizes = {"nb3": nb * 3, "nb4": nb * 4, "nb9": nb * 9, "ng3": ng * 3, "ng9": ng * 9, "nvnv": nv * nv,
                 "nv": nv, "1": 1, "mc": mc, "mc2": mc * 2, "mc3": mc * 3, "mc9": mc * 9, "mr": mr,
                 "mrnv": mr * nv}
        bufs, taps = {}, _Taps()
        for n, t, s in _TAP_FIELDS:
            a = np.zeros(max(1, sizes[s]), np.float64 if t == "f" else np.int32)
            bufs[n] = a
            setattr(taps, n, a.ctypes.data_as(_f64p if t == "f" else _i32p))
        q, v = _d(qpos, self.nq), _d(qvel, nv)
        u = _d(ctrl if ctrl is not None else np.zeros(self.nu), self.nu) if self.nu else None
        ws = _d(qacc_ws, nv) if qacc_ws is not None else None
        fr = _d([friction]) if friction is not None else None
        ms = _d(mass_scale, nb) if mass_scale is not None else None
        _check(lib().rbo_forward(self._h, _f(q), _f(v), _f(u), _f(ws), _f(fr), _f(ms), C.byref(taps)))
        nc = int(bufs["ncon"][0])
        nr = int(bufs["nrows"][0])
        out = dict(xpos=bufs["xpos"].reshape(nb, 3), xquat=bufs["xquat"].reshape(nb, 4),
                   xmat=bufs["xmat"].reshape(nb, 3, 3), com=bufs["com"].reshape(nb, 3),
                   gpos=bufs["gpos"][:ng * 3].reshape(ng, 3), gmat=bufs["gmat"][:ng * 9].reshape(ng, 3, 3),
                   M=bufs["M"][:nv * nv].reshape(nv, nv), bias=bufs["bias"][:nv], tau=bufs["tau"][:nv],
                   a0=bufs["a0"][:nv], ncon=nc, geom=bufs["geom"][:2 * nc].reshape(nc, 2),
                   feature=bufs["feature"][:nc], dist=bufs["dist"][:nc], pos=bufs["pos"][:3 * nc].reshape(nc, 3),
                   frame=bufs["frame"][:9 * nc].reshape(nc, 3, 3), mu=bufs["mu"][:nc],
                   J=bufs["J"][:nr * nv].reshape(nr, nv), aref=bufs["aref"][:nr], D=bufs["D"][:nr],
                   Ahat=bufs["Ahat"][:nr], efc_force=bufs["efc_force"][:nr], qacc=bufs["qacc"][:nv],
                   cforce=bufs["cforce"][:3 * nc].reshape(nc, 3), niter=int(bufs["niter"][0]),
                   cost=float(bufs["cost"][0]))
        return out

    def step(self, ctrl, qpos, qvel, qacc_ws, friction=None, mass_scale=None, status=None, contacts=False,
             nthreads=0, work=None, fields=None):
        """One env step (K substeps) for n worlds, in place on float64 arrays; returns (status, contacts).

        fields: an optional dict of per-world model fields (``geom_size`` [n, ngeom, 3], ``body_pos``
        [n, nbody, 3], ``act_kp`` / ``act_kd`` [n, nu]); world w steps as the model with its values.
        work: an optional dict that receives ``sub`` [n, K, SUBCOLS] int32 (per substep: contacts,
        rows, Newton updates, active rows at the solution, line-search segments, active-set
        fingerprints of the first FPITER updates) and ``ops`` [n, 2, NSTAGE] float64 (operation
        counts per stage: the oracle's plain definitions, the tree-sparse formulation)."""
        n = qpos.shape[0]
        for a in (qpos, qvel, qacc_ws):
            assert a.dtype == np.float64 and a.flags.c_contiguous
        u = _d(ctrl, (n, self.nu)) if self.nu else None
        fr = _d(friction, n) if friction is not None else None
        ms = _d(mass_scale, (n, self.nbody)) if mass_scale is not None else None
        st = np.zeros(n, np.uint32) if status is None else status
        cs = None
        out = None
        keep = []
        if contacts:
            mc = max(1, self.maxcon)
            out = dict(ncon=np.zeros(n, np.int32), geom=np.zeros((n, mc, 2), np.int32),
                       feature=np.zeros((n, mc), np.int32), dist=np.zeros((n, mc)), pos=np.zeros((n, mc, 3)),
                       frame=np.zeros((n, mc, 3, 3)), force=np.zeros((n, mc, 3)))
            cs = _Contacts()
            for k, v in out.items():
                setattr(cs, k, v.ctypes.data_as(_i32p if v.dtype == np.int32 else _f64p))
        fs = None
        if fields:
            shapes = dict(geom_size=(n, self.ngeom, 3), body_pos=(n, self.nbody, 3), act_kp=(n, self.nu),
                          act_kd=(n, self.nu))
            fs = _Fields()
            for k, a in fields.items():
                if k not in FIELDS:
                    raise KeyError(k)
                arr = _d(a, shapes[k])
                keep.append(arr)
                setattr(fs, k, _f(arr))
        if work is None and fs is None:
            _check(lib().rbo_step(self._h, n, _f(u), _f(qpos), _f(qvel), _f(qacc_ws), _f(fr), _f(ms),
                                  st.ctypes.data_as(C.POINTER(C.c_uint32)), C.byref(cs) if cs is not None else None,
                                  int(nthreads)))
        elif work is None:
            _check(lib().rbo_step_fields(self._h, n, _f(u), _f(qpos), _f(qvel), _f(qacc_ws), _f(fr), _f(ms),
                                         C.byref(fs), st.ctypes.data_as(C.POINTER(C.c_uint32)),
                                         C.byref(cs) if cs is not None else None, None, None, int(nthreads)))
        else:
            K = self.model["opt"]["nsubsteps"]
            sub = np.zeros((n, K, SUBCOLS), np.int32)
            ops = np.zeros((n, 2, NSTAGE), np.float64)
            _check(lib().rbo_step_fields(self._h, n, _f(u), _f(qpos), _f(qvel), _f(qacc_ws), _f(fr), _f(ms),
                                         C.byref(fs) if fs is not None else None,
                                         st.ctypes.data_as(C.POINTER(C.c_uint32)),
                                         C.byref(cs) if cs is not None else None, sub.ctypes.data_as(_i32p),
                                         ops.ctypes.data_as(_f64p), int(nthreads)))
            work["sub"] = sub
            work["ops"] = ops
        return st, out

    def line_search(self, qpos, qvel, a, p, ctrl=None, qacc_ws=None, friction=None, mass_scale=None):
        """(f(a), alpha*) for the rows of one substep's state: the constraint cost at a and the
        exact line search's step along p."""
        nv = self.nv
        u = _d(ctrl if ctrl is not None else np.zeros(self.nu), self.nu) if self.nu else None
        ws = _d(qacc_ws, nv) if qacc_ws is not None else None
        fr = _d([friction]) if friction is not None else None
        ms = _d(mass_scale, self.nbody) if mass_scale is not None else None
        c, al = C.c_double(), C.c_double()
        _check(lib().rbo_line_search(self._h, _f(_d(qpos, self.nq)), _f(_d(qvel, nv)), _f(u), _f(ws), _f(fr),
                                     _f(ms), _f(_d(a, nv)), _f(_d(p, nv)), C.byref(c), C.byref(al)))
        return c.value, al.value

    def energy(self, qpos, qvel, mass_scale=None):
        T, V = C.c_double(), C.c_double()
        ms = _d(mass_scale, self.nbody) if mass_scale is not None else None
        _check(lib().rbo_energy(self._h, _f(_d(qpos, self.nq)), _f(_d(qvel, self.nv)), _f(ms), C.byref(T),
                                C.byref(V)))
        return T.value, V.value

    def jacobian(self, qpos, body, point):
        jp = np.zeros((3, self.nv)); jr = np.zeros((3, self.nv))
        _check(lib().rbo_jacobian(self._h, _f(_d(qpos, self.nq)), int(body), _f(_d(point, 3)), _f(jp), _f(jr)))
        return jp, jr

    def integrate(self, qpos, qvel, qacc):
        qo = np.zeros(self.nq); vo = np.zeros(self.nv)
        _check(lib().rbo_integrate(self._h, _f(_d(qpos, self.nq)), _f(_d(qvel, self.nv)), _f(_d(qacc, self.nv)),
                                   _f(qo), _f(vo)))
        return qo, vo

    def rollout(self, qpos, qvel, ctrl=None, nsteps=1, qacc_ws=None, friction=None, mass_scale=None, nthreads=0):
        """Run ``nsteps`` env steps from float arrays [n, ...]; returns (qpos, qvel, qacc_ws, status) float64."""
        q = np.array(qpos, np.float64, order="C", ndmin=2)
        v = np.array(qvel, np.float64, order="C", ndmin=2)
        n = q.shape[0]
        ws = np.zeros((n, self.nv)) if qacc_ws is None else np.array(qacc_ws, np.float64, order="C", ndmin=2)
        st = np.zeros(n, np.uint32)
        u = np.zeros((n, self.nu)) if ctrl is None else ctrl
        for _ in range(nsteps):
            self.step(u, q, v, ws, friction, mass_scale, st, nthreads=nthreads)
        return q, v, ws, st
