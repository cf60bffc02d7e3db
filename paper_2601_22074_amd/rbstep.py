"""ctypes binding of librbstep (include/rbstep.h) over torch device tensors.

Argument marshalling only: every step of the physics runs in the HIP library.  torch
supplies device memory and streams; tensors are passed by pointer.  The library must be
built (``python -m paper_2601_22074_amd.build``); importing the binding without it, or
using it without a GPU, raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbstep.so")

RB_OK, RB_EINVAL, RB_ENOMEM, RB_EHIP, RB_EBUDGET, RB_ESTATE = 0, -1, -2, -3, -4, -5
STATUS_NONFINITE, STATUS_ITERCAP, STATUS_CONOVERFLOW = 1, 2, 4
PARAM_FRICTION, PARAM_MASS_SCALE, PARAM_GEOM_SIZE, PARAM_BODY_POS, PARAM_ACT_KP, PARAM_ACT_KD = 0, 1, 2, 3, 4, 5
NSTAGE = 10             # timed stages in the stats tap
STATS_SUB = 4           # substeps with a per-substep record in the stats tap
STATS_FP = 4            # Newton updates with an active-set fingerprint per substep
SUBSTAT = 5 + STATS_FP  # per substep: contacts, rows, updates, active rows, segments, fingerprints
NSTATS = 4 + NSTAGE + STATS_SUB * SUBSTAT
STAGES = ["kinematics", "inertia+bias+M", "factor M + a0", "collision", "constraint rows", "newton start",
          "gradient+hessian", "hessian factor+solve", "line search+update", "integrate"]

_GEOM = {"plane": 0, "sphere": 1, "capsule": 2, "box": 3, "hfield": 4}
_EQTYPE = {"connect": 0, "weld": 1}
_JNT = {"free": 0, "hinge": 1}
_ACT = {"position": 0, "motor": 1}

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)

EXPORTED = ["rb_last_error", "rb_model_create", "rb_model_create_json", "rb_model_destroy", "rb_model_info_get", "rb_batch_create",
            "rb_batch_destroy", "rb_batch_contact_capacity", "rb_batch_set_params", "rb_batch_set_params_at", "rb_batch_set_waves",
            "rb_world_reset",
            "rb_get_state", "rb_step", "rb_step_taps", "rb_step_noalloc", "rb_multi_create", "rb_multi_destroy", "rb_multi_bind",
            "rb_multi_set_schedule", "rb_multi_set_items", "rb_multi_set_occupancy", "rb_multi_set_group", "rb_multi_step", "rb_multi_graph_capture", "rb_multi_graph_launch"]
ORDER_BATCH, ORDER_HEAVY_FIRST, ORDER_INTERLEAVE = 0, 1, 2
NOALLOC_MAX_FLOATS = 4 << 20   # RB_NOALLOC_MAX_FLOATS


class RbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rbstep error {code}: {msg}")
        self.code = code


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
                ("neq", C.c_int32), ("eq_type", _i32p), ("eq_body", _i32p), ("eq_anchor", _f64p),
                ("eq_target", _f64p), ("geom_friction_spin", _f64p), ("geom_friction_roll", _f64p),
                ("cone", C.c_int32), ("impratio", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("nq", C.c_int32), ("nv", C.c_int32), ("nu", C.c_int32), ("nbody", C.c_int32),
                ("ngeom", C.c_int32), ("npair", C.c_int32), ("maxcon", C.c_int32), ("max_depth", C.c_int32),
                ("lds_bytes", C.c_int32), ("bytes_per_world", C.c_int32), ("meaninertia", C.c_double)]


class _Contacts(C.Structure):
    _fields_ = [("ncon", C.c_void_p), ("geom", C.c_void_p), ("feature", C.c_void_p), ("dist", C.c_void_p),
                ("pos", C.c_void_p), ("frame", C.c_void_p), ("force", C.c_void_p)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"librbstep.so not built at {LIB_PATH}; run python -m paper_2601_22074_amd.build")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.rb_last_error.restype = C.c_char_p
        L.rb_model_create.argtypes = [C.POINTER(_Desc), C.POINTER(vp)]
        L.rb_model_create_json.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.rb_model_destroy.argtypes = [vp]
        L.rb_model_info_get.argtypes = [vp, C.POINTER(_Info)]
        L.rb_batch_create.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(vp)]
        L.rb_batch_destroy.argtypes = [vp]
        L.rb_batch_contact_capacity.argtypes = [vp]
        L.rb_batch_contact_capacity.restype = C.c_int32
        L.rb_batch_set_params.argtypes = [vp, C.c_int32, C.c_int32, vp, vp]
        L.rb_batch_set_params_at.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp, vp]
        L.rb_batch_set_waves.argtypes = [vp, C.c_int32]
        L.rb_world_reset.argtypes = [vp, vp, C.c_int32, vp, vp]
        L.rb_get_state.argtypes = [vp, C.c_int32, vp, vp, vp]
        L.rb_step.argtypes = [vp, C.c_int32, vp, vp, vp, C.POINTER(_Contacts), vp, vp]
        L.rb_step_taps.argtypes = [vp, C.c_int32, vp, vp, vp, C.POINTER(_Contacts), vp, vp, vp, vp, vp, vp, vp, vp]
        L.rb_step_noalloc.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, C.POINTER(_Contacts), vp, vp]
        L.rb_multi_create.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(vp)]
        L.rb_multi_destroy.argtypes = [vp]
        L.rb_multi_bind.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp, C.POINTER(_Contacts), vp]
        L.rb_multi_set_schedule.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_float)]
        L.rb_multi_set_items.argtypes = [vp, C.POINTER(C.c_int32), C.c_int32, C.c_int32, vp]
        L.rb_multi_set_occupancy.argtypes = [vp, C.c_int32]
        L.rb_multi_set_group.argtypes = [vp, C.c_int32]
        L.rb_multi_step.argtypes = [vp, vp]
        L.rb_multi_graph_capture.argtypes = [vp, C.c_int32, vp]
        L.rb_multi_graph_launch.argtypes = [vp, vp]
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != RB_OK:
        raise RbError(rc, lib().rb_last_error().decode())


def _ptr(t, dtype=None, shape=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (or None), after shape/dtype checks."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def marshal_desc(model: dict):
    """rb_model_desc for a model dict (see workloads.robots); returns (desc, keepalive)."""
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
    eqs = model.get("equality") or []
    if eqs:
        # target: the world point, then the orientation quaternion (identity for a connect)
        d.neq = len(eqs)
        d.eq_type = i32([_EQTYPE[e["type"]] for e in eqs])
        d.eq_body = i32([e["body"] for e in eqs])
        d.eq_anchor = f64([e["anchor"] for e in eqs])
        d.eq_target = f64([[*e["target"], *(e["quat"] if e["type"] == "weld" else (1.0, 0.0, 0.0, 0.0))] for e in eqs])
    return d, keep


class Model:
    """A compiled model resident on the current GPU (rb_model_create)."""

    def __init__(self, model: dict | str):
        """model: a description dict, or JSON text of the same fields (rb_model_create_json)."""
        L = lib()
        h = C.c_void_p()
        if isinstance(model, str):
            _check(L.rb_model_create_json(model.encode(), C.byref(h)))
            import json
            model = json.loads(model)
        else:
            d, keep = marshal_desc(model)
            _check(L.rb_model_create(C.byref(d), C.byref(h)))
        self._h = h
        self.desc = model
        info = _Info()
        _check(L.rb_model_info_get(h, C.byref(info)))
        self.nq, self.nv, self.nu, self.nbody, self.ngeom = info.nq, info.nv, info.nu, info.nbody, info.ngeom
        self.npair, self.maxcon, self.max_depth, self.lds_bytes = info.npair, info.maxcon, info.max_depth, info.lds_bytes
        self.meaninertia = info.meaninertia
        self.bytes_per_world = info.bytes_per_world

    @property
    def contact_capacity(self) -> int:
        """Contact slots per world of a batch created with the default capacity."""
        return max(1, min(self.maxcon, 64))

    def step_noalloc(self, ctrl, qpos, qvel, friction=None, mass_scale=None, contacts=None, status=None,
                     stream=None) -> None:
        """rb_step_noalloc: one env step of worlds [0, n) without any device allocation, as a
        freshly reset batch would step them (the warm start does not carry between calls)."""
        import torch
        n = qpos.shape[0]
        pc = _ptr(ctrl, torch.float32, (n, self.nu), "ctrl") if self.nu else None
        cs = C.byref(contacts._struct(n, self.contact_capacity)) if contacts is not None else None
        _check(lib().rb_step_noalloc(self._h, int(n), pc, _ptr(qpos, torch.float32, (n, self.nq), "qpos"),
                                     _ptr(qvel, torch.float32, (n, self.nv), "qvel"),
                                     _ptr(friction, torch.float32, (n,), "friction"),
                                     _ptr(mass_scale, torch.float32, (n, self.nbody), "mass_scale"), cs,
                                     _ptr(status, torch.int32, (n,), "status"), _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().rb_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Contacts:
    """Device tensors receiving the last substep's contacts, ``cap`` slots per world."""

    def __init__(self, n: int, cap: int, device="cuda"):
        import torch
        self.ncon = torch.zeros(n, dtype=torch.int32, device=device)
        self.geom = torch.zeros(n, cap, 2, dtype=torch.int32, device=device)
        self.feature = torch.zeros(n, cap, dtype=torch.int32, device=device)
        self.dist = torch.zeros(n, cap, dtype=torch.float32, device=device)
        self.pos = torch.zeros(n, cap, 3, dtype=torch.float32, device=device)
        self.frame = torch.zeros(n, cap, 3, 3, dtype=torch.float32, device=device)
        self.force = torch.zeros(n, cap, 3, dtype=torch.float32, device=device)
        self.n, self.cap = n, cap

    def _struct(self, n, cap):
        if n > self.n:
            raise ValueError("contact buffers hold fewer worlds than stepped")
        if cap != self.cap:
            raise ValueError(f"contact buffers have {self.cap} slots per world, the batch needs {cap}")
        s = _Contacts()
        for k in ("ncon", "geom", "feature", "dist", "pos", "frame", "force"):
            setattr(s, k, getattr(self, k).data_ptr())
        return s


class Batch:
    """World slots of one model (rb_batch_create): resident warm start, status, parameters."""

    def __init__(self, model: Model, capacity: int, contact_capacity: int = 0):
        L = lib()
        h = C.c_void_p()
        _check(L.rb_batch_create(model._h, int(capacity), int(contact_capacity), C.byref(h)))
        self._h = h
        self.model = model
        self.capacity = int(capacity)
        self.ncap = int(L.rb_batch_contact_capacity(h))

    def close(self):
        if getattr(self, "_h", None):
            lib().rb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def contacts(self, n: int | None = None, device="cuda") -> Contacts:
        return Contacts(self.capacity if n is None else n, self.ncap, device)

    def set_params(self, field: int, vals, stream=None) -> None:
        import torch
        n = vals.shape[0]
        _check(lib().rb_batch_set_params(self._h, int(field), int(n),
                                         _ptr(vals, torch.float32, self._param_shape(field, n), "vals"), _stream(stream)))

    def set_params_at(self, field: int, first: int, vals, stream=None) -> None:
        """Per-world parameters of slots [first, first + n), n = vals.shape[0]."""
        import torch
        n = vals.shape[0]
        _check(lib().rb_batch_set_params_at(self._h, int(field), int(first), int(n),
                                            _ptr(vals, torch.float32, self._param_shape(field, n), "vals"),
                                            _stream(stream)))

    def _param_shape(self, field: int, n: int):
        M = self.model
        return {PARAM_FRICTION: (n,), PARAM_MASS_SCALE: (n, M.nbody), PARAM_GEOM_SIZE: (n, M.ngeom, 3),
                PARAM_BODY_POS: (n, M.nbody, 3), PARAM_ACT_KP: (n, M.nu), PARAM_ACT_KD: (n, M.nu)}.get(field, (n,))

    def set_waves(self, waves: int) -> None:
        """Resident waves per SIMD of plain launches: 3, 4, or 0 (automatic)."""
        _check(lib().rb_batch_set_waves(self._h, int(waves)))

    def reset(self, ids, qacc_ws=None, stream=None) -> None:
        import torch
        n = ids.shape[0]
        _check(lib().rb_world_reset(self._h, _ptr(ids, torch.int32, (n,), "ids"), int(n),
                                    _ptr(qacc_ws, torch.float32, (n, self.model.nv), "qacc_ws"), _stream(stream)))

    def get_state(self, n: int, qacc_ws=None, status=None, stream=None) -> None:
        import torch
        _check(lib().rb_get_state(self._h, int(n), _ptr(qacc_ws, torch.float32, (n, self.model.nv), "qacc_ws"),
                                  _ptr(status, torch.int32, (n,), "status"), _stream(stream)))

    def _common(self, ctrl, qpos, qvel, status):
        import torch
        n = qpos.shape[0]
        m = self.model
        pc = _ptr(ctrl, torch.float32, (n, m.nu), "ctrl") if m.nu else None
        return n, pc, _ptr(qpos, torch.float32, (n, m.nq), "qpos"), _ptr(qvel, torch.float32, (n, m.nv), "qvel"), \
            _ptr(status, torch.int32, (n,), "status")

    def step(self, ctrl, qpos, qvel, contacts: Contacts | None = None, status=None, stream=None) -> None:
        """One env step (K substeps) of worlds [0, n), n = qpos.shape[0]; qpos/qvel in place."""
        n, pc, pq, pv, ps = self._common(ctrl, qpos, qvel, status)
        cs = C.byref(contacts._struct(n, self.ncap)) if contacts is not None else None
        _check(lib().rb_step(self._h, int(n), pc, pq, pv, cs, ps, _stream(stream)))

    def step_taps(self, ctrl, qpos, qvel, contacts=None, status=None, M=None, bias=None, a0=None, qacc=None,
                  efc=None, stats=None, stream=None) -> None:
        import torch
        n, pc, pq, pv, ps = self._common(ctrl, qpos, qvel, status)
        nv = self.model.nv
        cs = C.byref(contacts._struct(n, self.ncap)) if contacts is not None else None
        _check(lib().rb_step_taps(self._h, int(n), pc, pq, pv, cs, ps,
                                  _ptr(M, torch.float32, (n, nv, nv), "M"), _ptr(bias, torch.float32, (n, nv), "bias"),
                                  _ptr(a0, torch.float32, (n, nv), "a0"), _ptr(qacc, torch.float32, (n, nv), "qacc"),
                                  _ptr(efc, torch.float32, (n, self.ncap, 4, 3), "efc"),
                                  _ptr(stats, torch.int32, (n, NSTATS), "stats"), _stream(stream)))


class Multi:
    """One fused launch over several batches (rb_multi_*): the batching form."""

    def __init__(self, batches):
        L = lib()
        arr = (C.c_void_p * len(batches))(*[b._h for b in batches])
        h = C.c_void_p()
        _check(L.rb_multi_create(arr, len(batches), C.byref(h)))
        self._h = h
        self.batches = list(batches)
        self.bound = [None] * len(batches)

    def close(self):
        if getattr(self, "_h", None):
            lib().rb_multi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bind(self, i, ctrl, qpos, qvel, contacts: Contacts | None = None, status=None) -> None:
        """Step inputs of batch i (kept alive by the plan until rebound)."""
        n, pc, pq, pv, ps = self.batches[i]._common(ctrl, qpos, qvel, status)
        cs = C.byref(contacts._struct(n, self.batches[i].ncap)) if contacts is not None else None
        _check(lib().rb_multi_bind(self._h, int(i), int(n), pc, pq, pv, cs, ps))
        self.bound[i] = (ctrl, qpos, qvel, contacts, status)

    def set_schedule(self, order: int = ORDER_HEAVY_FIRST, grid: int = 0, cost=None) -> None:
        c = None
        if cost is not None:
            c = (C.c_float * len(self.batches))(*[float(x) for x in cost])
        _check(lib().rb_multi_set_schedule(self._h, int(order), int(grid), c))

    def set_items(self, items, grid: int = 0, stream=None) -> None:
        """Explicit work list (host int32 array of batch << 24 | world), uploaded on the stream."""
        a = np.ascontiguousarray(np.asarray(items, dtype=np.int32).reshape(-1))
        _check(lib().rb_multi_set_items(self._h, a.ctypes.data_as(C.POINTER(C.c_int32)), int(a.size), int(grid),
                                        _stream(stream)))

    def set_occupancy(self, waves_per_simd: int) -> None:
        """Cap resident waves per SIMD of the fused launch (0 = no cap)."""
        _check(lib().rb_multi_set_occupancy(self._h, int(waves_per_simd)))

    def set_group(self, worlds_per_workgroup: int) -> None:
        """Worlds (one wave each) per workgroup of the fused launch: 1, 2 or 4."""
        _check(lib().rb_multi_set_group(self._h, int(worlds_per_workgroup)))

    def step(self, stream=None) -> None:
        _check(lib().rb_multi_step(self._h, _stream(stream)))

    def graph_capture(self, nsteps: int, stream) -> None:
        _check(lib().rb_multi_graph_capture(self._h, int(nsteps), _stream(stream)))

    def graph_launch(self, stream=None) -> None:
        _check(lib().rb_multi_graph_launch(self._h, _stream(stream)))
