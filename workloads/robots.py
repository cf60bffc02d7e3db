"""Synthetic robot descriptions.

The paper's robots (a humanoid, a quadruped and an arm lifting a cube; section
"Tasks", robot-morphology figure) come from a model zoo that is not available
here, so these are stand-ins with the degree-of-freedom and geom structure the
benchmark workloads state: a 3-link planar hinge chain, a 12-joint quadruped on a
free base, a 29-joint humanoid on a free base with 40 colliding geoms, and a
7-joint arm with a free cube on a table.

A model description is a plain dict:

``bodies``     list of {name, parent, pos[3], quat[4], ipos[3], iquat[4], mass, inertia[3]};
               body 0 is the world, ``parent[b] < b``.
``joints``     list of {type: "free"|"hinge", body, pos[3], axis[3], armature};
               at most one joint per body.
``geoms``      list of {type: "plane"|"sphere"|"capsule"|"box", body, pos[3], quat[4],
               size[3], friction, contype, conaffinity, margin}.  Sizes: sphere (r),
               capsule (r, half-length of the cylinder part along local z), box
               (half-sizes), plane (ignored; its normal is local +z).
``actuators``  list of {type: "position"|"motor", joint, kp, kd, gear}.
``opt``        {timestep, nsubsteps, gravity[3], iterations, tolerance, solref[2], solimp[5]}.
``per_world``  {friction: bool, mass_scale: bool} -- which fields vary per world.

Quaternions are (w, x, y, z).  Masses and inertias are those of uniform solids of
the stated shape (the formulas below are the only arithmetic in this module).
"""
from __future__ import annotations

import copy
import math

import numpy as np

GEOM_TYPES = ("plane", "sphere", "capsule", "box")
JOINT_TYPES = ("free", "hinge")
ACT_TYPES = ("position", "motor")

DEFAULT_OPT = {
    "timestep": 0.005,
    "nsubsteps": 4,
    "gravity": [0.0, 0.0, -9.81],
    "iterations": 4,
    "tolerance": 1e-8,
    "solref": [0.02, 1.0],
    "solimp": [0.9, 0.95, 0.001, 0.5, 2.0],
}


# --------------------------------------------------------------------------------------
# solid-shape inertias (principal moments about the centre of mass)
# --------------------------------------------------------------------------------------
def capsule_inertia(mass: float, radius: float, length: float) -> list[float]:
    """Uniform solid capsule: cylinder of ``length`` along z plus two hemispherical caps."""
    r, L = radius, length
    v_cyl = math.pi * r * r * L
    v_sph = 4.0 / 3.0 * math.pi * r ** 3
    rho = mass / (v_cyl + v_sph)
    mc, ms = rho * v_cyl, rho * v_sph
    izz = mc * r * r / 2.0 + ms * 2.0 * r * r / 5.0
    ixx = mc * (r * r / 4.0 + L * L / 12.0) + ms * (2.0 * r * r / 5.0 + L * L / 4.0 + 3.0 * L * r / 8.0)
    return [ixx, ixx, izz]


def box_inertia(mass: float, hx: float, hy: float, hz: float) -> list[float]:
    return [mass / 3.0 * (hy * hy + hz * hz), mass / 3.0 * (hx * hx + hz * hz), mass / 3.0 * (hx * hx + hy * hy)]


def sphere_inertia(mass: float, radius: float) -> list[float]:
    i = 0.4 * mass * radius * radius
    return [i, i, i]


def quat_axis_angle(axis, angle) -> list[float]:
    a = np.asarray(axis, dtype=float)
    a = a / np.linalg.norm(a)
    s = math.sin(angle / 2.0)
    return [math.cos(angle / 2.0), s * a[0], s * a[1], s * a[2]]


def quat_z_to(direction) -> list[float]:
    """Unit quaternion rotating local +z onto ``direction``."""
    d = np.asarray(direction, dtype=float)
    d = d / np.linalg.norm(d)
    z = np.array([0.0, 0.0, 1.0])
    c = float(np.dot(z, d))
    if c > 1.0 - 1e-12:
        return [1.0, 0.0, 0.0, 0.0]
    if c < -1.0 + 1e-12:
        return [0.0, 1.0, 0.0, 0.0]
    ax = np.cross(z, d)
    return quat_axis_angle(ax, math.acos(c))


# --------------------------------------------------------------------------------------
# builder
# --------------------------------------------------------------------------------------
class ModelBuilder:
    def __init__(self, name: str, **opt):
        self.name = name
        self.opt = copy.deepcopy(DEFAULT_OPT)
        self.opt.update(opt)
        self.bodies = [dict(name="world", parent=-1, pos=[0, 0, 0], quat=[1, 0, 0, 0], ipos=[0, 0, 0],
                            iquat=[1, 0, 0, 0], mass=0.0, inertia=[0, 0, 0])]
        self.joints: list[dict] = []
        self.geoms: list[dict] = []
        self.actuators: list[dict] = []
        self.per_world = {"friction": False, "mass_scale": False}
        self.hfield_grid = None
        self.equalities: list[dict] = []

    def body(self, name, parent, pos, mass, inertia, ipos=(0, 0, 0), iquat=(1, 0, 0, 0), quat=(1, 0, 0, 0)) -> int:
        pid = parent if isinstance(parent, int) else self.body_id(parent)
        self.bodies.append(dict(name=name, parent=pid, pos=list(map(float, pos)), quat=list(map(float, quat)),
                                ipos=list(map(float, ipos)), iquat=list(map(float, iquat)), mass=float(mass),
                                inertia=list(map(float, inertia))))
        return len(self.bodies) - 1

    def body_id(self, name) -> int:
        for i, b in enumerate(self.bodies):
            if b["name"] == name:
                return i
        raise KeyError(name)

    def capsule_body(self, name, parent, pos, a, b, radius, mass, quat=(1, 0, 0, 0)) -> int:
        """Body whose inertia is that of a uniform capsule from point ``a`` to ``b`` (body frame)."""
        a, b = np.asarray(a, float), np.asarray(b, float)
        length = float(np.linalg.norm(b - a))
        return self.body(name, parent, pos, mass, capsule_inertia(mass, radius, length),
                         ipos=(a + b) / 2.0, iquat=quat_z_to(b - a) if length > 0 else (1, 0, 0, 0), quat=quat)

    def joint(self, body, type_, axis=(0, 0, 1), pos=(0, 0, 0), armature=0.0, range_=None, damping=0.0) -> int:
        """range_: (lower, upper) angle limits of a hinge, or None for an unlimited joint;
        damping: passive torque -damping * velocity on a hinge (integrated implicitly)."""
        bid = body if isinstance(body, int) else self.body_id(body)
        j = dict(type=type_, body=bid, pos=list(map(float, pos)), axis=list(map(float, axis)),
                 armature=float(armature))
        if range_ is not None:
            j["range"] = [float(range_[0]), float(range_[1])]
        if damping:
            j["damping"] = float(damping)
        self.joints.append(j)
        return len(self.joints) - 1

    def geom(self, body, type_, size, pos=(0, 0, 0), quat=(1, 0, 0, 0), friction=1.0, contype=1, conaffinity=1,
             margin=0.0) -> int:
        bid = body if isinstance(body, int) else self.body_id(body)
        s = list(map(float, size)) + [0.0] * (3 - len(size))
        self.geoms.append(dict(type=type_, body=bid, pos=list(map(float, pos)), quat=list(map(float, quat)), size=s,
                               friction=float(friction), contype=int(contype), conaffinity=int(conaffinity),
                               margin=float(margin)))
        return len(self.geoms) - 1

    def capsule(self, body, a, b, radius, **kw) -> int:
        a, b = np.asarray(a, float), np.asarray(b, float)
        half = float(np.linalg.norm(b - a)) / 2.0
        return self.geom(body, "capsule", [radius, half], pos=(a + b) / 2.0, quat=quat_z_to(b - a), **kw)

    def hfield(self, heights) -> None:
        """The model's height grid [nrow, ncol] (rows along y, columns along x) used by its
        "hfield" geoms, whose size[0], size[1] are the grid's half extents."""
        h = np.asarray(heights, float)
        self.hfield_grid = dict(nrow=int(h.shape[0]), ncol=int(h.shape[1]), data=[float(x) for x in h.ravel()])

    def equality(self, type_, body, anchor, target, quat=None) -> int:
        """An equality constraint of a moving body with the world: "connect" holds the body point
        ``anchor`` (body frame) at the world point ``target``; "weld" also holds the body's
        orientation at the unit quaternion ``quat``."""
        bid = body if isinstance(body, int) else self.body_id(body)
        e = dict(type=type_, body=bid, anchor=list(map(float, anchor)), target=list(map(float, target)))
        if type_ == "weld":
            e["quat"] = list(map(float, quat if quat is not None else (1, 0, 0, 0)))
        self.equalities.append(e)
        return len(self.equalities) - 1

    def actuator(self, joint, type_="position", kp=0.0, kd=0.0, gear=1.0) -> int:
        self.actuators.append(dict(type=type_, joint=int(joint), kp=float(kp), kd=float(kd), gear=float(gear)))
        return len(self.actuators) - 1

    def build(self) -> dict:
        m = dict(name=self.name, opt=copy.deepcopy(self.opt), bodies=copy.deepcopy(self.bodies),
                 joints=copy.deepcopy(self.joints), geoms=copy.deepcopy(self.geoms),
                 actuators=copy.deepcopy(self.actuators), per_world=dict(self.per_world))
        if self.hfield_grid is not None:
            m["hfield"] = copy.deepcopy(self.hfield_grid)
        if self.equalities:
            m["equality"] = copy.deepcopy(self.equalities)
        return m


# --------------------------------------------------------------------------------------
# model dimensions derived from a description (pure bookkeeping)
# --------------------------------------------------------------------------------------
def dims(model: dict) -> dict:
    nq = sum(7 if j["type"] == "free" else 1 for j in model["joints"])
    nv = sum(6 if j["type"] == "free" else 1 for j in model["joints"])
    return dict(nbody=len(model["bodies"]), njnt=len(model["joints"]), ngeom=len(model["geoms"]), nq=nq, nv=nv,
                nu=len(model["actuators"]))


def qpos0(model: dict) -> np.ndarray:
    """Reference configuration: free joints at their body's position with unit quaternion, hinges at 0."""
    out = []
    for j in model["joints"]:
        if j["type"] == "free":
            b = model["bodies"][j["body"]]
            out += list(b["pos"]) + list(b["quat"])
        else:
            out.append(0.0)
    return np.array(out, dtype=np.float64)


# --------------------------------------------------------------------------------------
# the benchmark robots
# --------------------------------------------------------------------------------------
CAPSULE_GEOM = dict(contype=1, conaffinity=0)      # collides with the ground only
GROUND_GEOM = dict(contype=0, conaffinity=1)
GHOST_GEOM = dict(contype=0, conaffinity=0)        # never collides


def chain(nlinks: int = 3, name: str | None = None, timestep: float = 0.002, gravity=(0, 0, -9.81)) -> dict:
    """Planar hinge chain hanging from a fixed base at the origin.

    Each link is a 0.5 m capsule of radius 0.05 and mass 1 kg running from its
    joint to (0, 0, -0.5) in its own frame; hinge axes are +y; q = 0 hangs along -z.
    No geom collides (contact-free), no actuators.
    """
    mb = ModelBuilder(name or f"chain{nlinks}", timestep=timestep, nsubsteps=1, gravity=list(gravity))
    parent = 0
    for i in range(nlinks):
        pos = (0, 0, 0) if i == 0 else (0, 0, -0.5)
        b = mb.capsule_body(f"link{i + 1}", parent, pos, (0, 0, 0), (0, 0, -0.5), 0.05, 1.0)
        mb.joint(b, "hinge", axis=(0, 1, 0))
        mb.capsule(b, (0, 0, 0), (0, 0, -0.5), 0.05, **GHOST_GEOM)
        parent = b
    return mb.build()


def chain3() -> dict:
    return chain(3, "chain3")


def quadruped() -> dict:
    """Free-floating box torso with four 3-hinge legs ending in sphere feet."""
    mb = ModelBuilder("quadruped", timestep=0.005, nsubsteps=4)
    mb.geom(0, "plane", [0, 0, 0], friction=1.0, **GROUND_GEOM)
    torso = mb.body("torso", 0, (0, 0, 0.45), 6.0, box_inertia(6.0, 0.20, 0.08, 0.05))
    mb.joint(torso, "free")
    mb.geom(torso, "box", [0.20, 0.08, 0.05], friction=1.0, **CAPSULE_GEOM)
    for leg, (sx, sy) in (("FL", (1, 1)), ("FR", (1, -1)), ("RL", (-1, 1)), ("RR", (-1, -1))):
        hip = mb.capsule_body(f"{leg}_hip", torso, (0.18 * sx, 0.07 * sy, 0), (0, 0, 0), (0, 0.05 * sy, 0), 0.03, 0.6)
        jh = mb.joint(hip, "hinge", axis=(1, 0, 0), armature=0.01)
        mb.capsule(hip, (0, 0, 0), (0, 0.05 * sy, 0), 0.03, **GHOST_GEOM)
        thigh = mb.capsule_body(f"{leg}_thigh", hip, (0, 0.05 * sy, 0), (0, 0, 0), (0, 0, -0.2), 0.02, 1.0)
        jt = mb.joint(thigh, "hinge", axis=(0, 1, 0), armature=0.01)
        mb.capsule(thigh, (0, 0, 0), (0, 0, -0.2), 0.02, **GHOST_GEOM)
        calf = mb.capsule_body(f"{leg}_calf", thigh, (0, 0, -0.2), (0, 0, 0), (0, 0, -0.2), 0.015, 0.25)
        jc = mb.joint(calf, "hinge", axis=(0, 1, 0), armature=0.01)
        mb.capsule(calf, (0, 0, 0), (0, 0, -0.2), 0.015, **GHOST_GEOM)
        mb.geom(calf, "sphere", [0.02], pos=(0, 0, -0.2), friction=1.0, **CAPSULE_GEOM)
        for j in (jh, jt, jc):
            mb.actuator(j, "position", kp=20.0, kd=0.5)
    return mb.build()


def humanoid() -> dict:
    """Free pelvis, 3-hinge waist, two 6-hinge legs and two 7-hinge arms (30 bodies, 29 hinges).

    40 colliding geoms (32 capsules and 8 boxes) collide with the ground plane only.
    Per-world friction and per-body mass scale are enabled.
    """
    mb = ModelBuilder("humanoid", timestep=0.005, nsubsteps=4)
    mb.per_world = {"friction": True, "mass_scale": True}
    mb.geom(0, "plane", [0, 0, 0], friction=1.0, **GROUND_GEOM)
    cg = CAPSULE_GEOM
    pelvis_z = 0.765 + 0.001          # feet 1 mm above the plane at qpos0
    pelvis = mb.body("pelvis", 0, (0, 0, pelvis_z), 5.0, box_inertia(5.0, 0.07, 0.12, 0.06))
    mb.joint(pelvis, "free")
    mb.geom(pelvis, "box", [0.07, 0.12, 0.06], **cg)
    arm = 0.01
    hinges = []
    for side, sy in (("L", 1), ("R", -1)):
        b = mb.capsule_body(f"{side}_hip_pitch", pelvis, (0, 0.09 * sy, -0.06), (0, 0, 0), (0, 0.04 * sy, 0), 0.04, 1.2)
        hinges.append(mb.joint(b, "hinge", (0, 1, 0), armature=arm))
        mb.capsule(b, (0, 0, 0), (0, 0.04 * sy, 0), 0.04, **cg)
        b = mb.capsule_body(f"{side}_hip_roll", b, (0, 0.04 * sy, 0), (0, 0, 0), (0, 0, -0.06), 0.045, 1.0)
        hinges.append(mb.joint(b, "hinge", (1, 0, 0), armature=arm))
        mb.capsule(b, (0, 0, 0), (0, 0, -0.06), 0.045, **cg)
        b = mb.capsule_body(f"{side}_hip_yaw", b, (0, 0, -0.06), (0, 0, 0), (0, 0, -0.26), 0.055, 3.0)
        hinges.append(mb.joint(b, "hinge", (0, 0, 1), armature=arm))
        mb.capsule(b, (0, 0, 0), (0, 0, -0.13), 0.055, **cg)
        mb.capsule(b, (0, 0, -0.13), (0, 0, -0.26), 0.05, **cg)
        b = mb.capsule_body(f"{side}_knee", b, (0, 0, -0.26), (0, 0, 0), (0, 0, -0.32), 0.045, 2.0)
        hinges.append(mb.joint(b, "hinge", (0, 1, 0), armature=arm))
        mb.capsule(b, (0, 0, 0), (0, 0, -0.16), 0.045, **cg)
        mb.capsule(b, (0, 0, -0.16), (0, 0, -0.30), 0.04, **cg)
        b = mb.capsule_body(f"{side}_ankle_pitch", b, (0, 0, -0.32), (0, 0, 0), (0, 0, -0.02), 0.02, 0.2)
        hinges.append(mb.joint(b, "hinge", (0, 1, 0), armature=arm))
        mb.capsule(b, (0, 0, 0), (0, 0, -0.02), 0.02, **cg)
        b = mb.body(f"{side}_ankle_roll", b, (0, 0, -0.02), 0.6, box_inertia(0.6, 0.09, 0.04, 0.015),
                    ipos=(0.015, 0, -0.03))
        hinges.append(mb.joint(b, "hinge", (1, 0, 0), armature=arm))
        mb.geom(b, "box", [0.05, 0.04, 0.015], pos=(0.06, 0, -0.03), **cg)
        mb.geom(b, "box", [0.04, 0.04, 0.015], pos=(-0.04, 0, -0.03), **cg)
    b = mb.capsule_body("waist_yaw", pelvis, (0, 0, 0.06), (0, 0, 0), (0, 0, 0.04), 0.05, 0.5)
    hinges.append(mb.joint(b, "hinge", (0, 0, 1), armature=arm))
    mb.capsule(b, (0, 0, 0), (0, 0, 0.04), 0.05, **cg)
    b = mb.capsule_body("waist_roll", b, (0, 0, 0.04), (0, 0, 0), (0, 0, 0.03), 0.05, 0.5)
    hinges.append(mb.joint(b, "hinge", (1, 0, 0), armature=arm))
    mb.capsule(b, (0, 0, 0), (0, 0, 0.03), 0.05, **cg)
    torso = mb.body("torso", b, (0, 0, 0.03), 8.0, box_inertia(8.0, 0.08, 0.12, 0.18), ipos=(0, 0, 0.2))
    hinges.append(mb.joint(torso, "hinge", (0, 1, 0), armature=arm))
    mb.geom(torso, "box", [0.08, 0.12, 0.18], pos=(0, 0, 0.2), **cg)
    for side, sy in (("L", 1), ("R", -1)):
        b = mb.capsule_body(f"{side}_shoulder_pitch", torso, (0, 0.16 * sy, 0.3), (0, 0, 0), (0, 0.05 * sy, 0), 0.04, 0.5)
        hinges.append(mb.joint(b, "hinge", (0, 1, 0), armature=arm))
        mb.capsule(b, (0, 0, 0), (0, 0.05 * sy, 0), 0.04, **cg)
        b = mb.capsule_body(f"{side}_shoulder_roll", b, (0, 0.05 * sy, 0), (0, 0, 0), (0, 0, -0.05), 0.035, 0.5)
        hinges.append(mb.joint(b, "hinge", (1, 0, 0), armature=arm))
        mb.capsule(b, (0, 0, 0), (0, 0, -0.05), 0.035, **cg)
        b = mb.capsule_body(f"{side}_shoulder_yaw", b, (0, 0, -0.05), (0, 0, 0), (0, 0, -0.2), 0.035, 0.8)
        hinges.append(mb.joint(b, "hinge", (0, 0, 1), armature=arm))
        mb.capsule(b, (0, 0, 0), (0, 0, -0.1), 0.035, **cg)
        mb.capsule(b, (0, 0, -0.1), (0, 0, -0.2), 0.03, **cg)
        b = mb.capsule_body(f"{side}_elbow", b, (0, 0, -0.2), (0, 0, 0), (0, 0, -0.18), 0.03, 0.6)
        hinges.append(mb.joint(b, "hinge", (0, 1, 0), armature=arm))
        mb.capsule(b, (0, 0, 0), (0, 0, -0.1), 0.03, **cg)
        mb.capsule(b, (0, 0, -0.1), (0, 0, -0.18), 0.028, **cg)
        b = mb.capsule_body(f"{side}_wrist_roll", b, (0, 0, -0.18), (0, 0, 0), (0, 0, -0.03), 0.025, 0.2)
        hinges.append(mb.joint(b, "hinge", (0, 0, 1), armature=arm))
        mb.capsule(b, (0, 0, 0), (0, 0, -0.03), 0.025, **cg)
        b = mb.capsule_body(f"{side}_wrist_pitch", b, (0, 0, -0.03), (0, 0, 0), (0, 0, -0.02), 0.025, 0.2)
        hinges.append(mb.joint(b, "hinge", (0, 1, 0), armature=arm))
        mb.capsule(b, (0, 0, 0), (0, 0, -0.02), 0.025, **cg)
        b = mb.body(f"{side}_wrist_yaw", b, (0, 0, -0.02), 0.3, box_inertia(0.3, 0.02, 0.04, 0.05), ipos=(0, 0, -0.05))
        hinges.append(mb.joint(b, "hinge", (1, 0, 0), armature=arm))
        mb.geom(b, "box", [0.02, 0.04, 0.05], pos=(0, 0, -0.05), **cg)
    for j in hinges:
        mb.actuator(j, "position", kp=20.0, kd=0.5)
    return mb.build()


def arm_box() -> dict:
    """Fixed-base 7-hinge arm (non-colliding capsule links) beside a static table with a 5 cm free cube on it."""
    mb = ModelBuilder("arm_box", timestep=0.005, nsubsteps=4)
    mb.geom(0, "plane", [0, 0, 0], friction=1.0, **GROUND_GEOM)
    mb.geom(0, "box", [0.3, 0.3, 0.2], pos=(0.5, 0, 0.2), friction=1.0, contype=0, conaffinity=1)
    axes = [(0, 0, 1), (0, 1, 0), (0, 0, 1), (0, 1, 0), (0, 0, 1), (0, 1, 0), (0, 0, 1)]
    lengths = [0.15, 0.25, 0.05, 0.25, 0.05, 0.1, 0.05]
    masses = [2.0, 1.5, 1.0, 1.0, 0.5, 0.4, 0.3]
    parent, pos = 0, (0, 0, 0.0)
    for i, (ax, L, m) in enumerate(zip(axes, lengths, masses)):
        b = mb.capsule_body(f"arm{i + 1}", parent, pos, (0, 0, 0), (0, 0, L), 0.04, m)
        j = mb.joint(b, "hinge", ax, armature=0.01)
        mb.capsule(b, (0, 0, 0), (0, 0, L), 0.04, **GHOST_GEOM)
        mb.actuator(j, "position", kp=20.0, kd=0.5)
        parent, pos = b, (0, 0, L)
    cube = mb.body("cube", 0, (0.5, 0.0, 0.4 + 0.025 + 0.001), 0.1, box_inertia(0.1, 0.025, 0.025, 0.025))
    mb.joint(cube, "free")
    mb.geom(cube, "box", [0.025, 0.025, 0.025], friction=1.0, contype=1, conaffinity=0)
    return mb.build()


# --------------------------------------------------------------------------------------
# small models used by the pins and edge-case tests
# --------------------------------------------------------------------------------------
def free_body(shape="box", size=(0.1, 0.1, 0.1), mass=1.0, pos=(0, 0, 1.0), quat=(1, 0, 0, 0), ground=True,
              friction=1.0, gravity=(0, 0, -9.81), timestep=0.005, nsubsteps=1, iterations=4, tolerance=1e-8,
              ground_quat=(1, 0, 0, 0), inertia=None, name=None) -> dict:
    mb = ModelBuilder(name or f"free_{shape}", timestep=timestep, nsubsteps=nsubsteps, gravity=list(gravity),
                      iterations=iterations, tolerance=tolerance)
    if ground:
        mb.geom(0, "plane", [0, 0, 0], quat=ground_quat, friction=friction, **GROUND_GEOM)
    if inertia is None:
        if shape == "box":
            inertia = box_inertia(mass, *size)
        elif shape == "sphere":
            inertia = sphere_inertia(mass, size[0])
        else:
            inertia = capsule_inertia(mass, size[0], 2 * size[1])
    b = mb.body("body", 0, pos, mass, inertia, quat=quat)
    mb.joint(b, "free")
    mb.geom(b, shape, size, friction=friction, contype=1, conaffinity=0)
    return mb.build()


def free_box_asym(gravity=(0, 0, 0), timestep=0.005) -> dict:
    """Single free box with three distinct principal moments, no ground (momentum pins)."""
    return free_body("box", size=(0.2, 0.1, 0.05), mass=2.0, ground=False, gravity=gravity, timestep=timestep,
                     name="free_box_asym")


def free_offset(gravity=(0, 0, -9.81), timestep=0.005) -> dict:
    """Single free body whose centre of mass and principal axes are offset from its frame."""
    mb = ModelBuilder("free_offset", timestep=timestep, nsubsteps=1, gravity=list(gravity))
    b = mb.body("body", 0, (0, 0, 1.0), 1.5, [0.02, 0.03, 0.04], ipos=(0.1, -0.05, 0.2),
                iquat=quat_axis_angle((1, 2, 3), 0.7))
    mb.joint(b, "free")
    mb.geom(b, "box", [0.1, 0.1, 0.1], **GHOST_GEOM)
    return mb.build()


TERRAIN_GEOM = dict(contype=0, conaffinity=2)      # terrain tiles: touched by geoms with contype bit 2


def quadruped_terrain(tile=0.4, n=3, max_height=0.04, seed=2601) -> dict:
    """The quadruped on a random-height grid: n x n static box tiles of side ``tile`` centred
    under the robot, tops at heights U[0, max_height] from a fixed seed; the sphere feet touch
    the tiles (and the plane), the torso only the plane.  The torso starts ``max_height``
    higher."""
    m = quadruped()
    m["name"] = "quadruped_terrain"
    rng = np.random.default_rng(seed)
    heights = rng.uniform(0.0, max_height, (n, n))
    half = tile / 2
    for i in range(n):
        for j in range(n):
            cx, cy = (i - (n - 1) / 2) * tile, (j - (n - 1) / 2) * tile
            m["geoms"].append(dict(type="box", body=0, pos=[cx, cy, float(heights[i, j]) - 0.05],
                                   quat=[1.0, 0.0, 0.0, 0.0], size=[half, half, 0.05], friction=1.0,
                                   margin=0.0, **TERRAIN_GEOM))
    for g in m["geoms"]:
        if g["type"] == "sphere":
            g["contype"] = 3
    m["bodies"][1]["pos"][2] += max_height
    return m


def quadruped_hfield(nrow=41, half=2.0, amp=0.03, seed=2603) -> dict:
    """The quadruped on smooth height-field terrain instead of the plane: a 41 x 41 grid over
    4 m x 4 m, heights a sum of three sinusoids of wavelength 0.6-1.5 m and random phase from a
    fixed seed, scaled to +-``amp``, shifted to zero under the robot's start; feet and torso
    collide with it (5 height-field pairs)."""
    m = quadruped()
    m["name"] = "quadruped_hfield"
    rng = np.random.default_rng(seed)
    xs = np.linspace(-half, half, nrow)
    X, Y = np.meshgrid(xs, xs)          # rows along y, columns along x
    H = np.zeros_like(X)
    for _ in range(3):
        lam = rng.uniform(0.6, 1.5)
        th = rng.uniform(0, np.pi)
        H += np.sin(2 * np.pi * (np.cos(th) * X + np.sin(th) * Y) / lam + rng.uniform(0, 2 * np.pi))
    H *= amp / np.abs(H).max()
    H -= H[nrow // 2, nrow // 2]
    planes = [g for g in m["geoms"] if g["type"] == "plane"]
    for g in planes:
        g.update(type="hfield", size=[half, half, 0.0])
    m["hfield"] = dict(nrow=nrow, ncol=nrow, data=[float(x) for x in H.ravel()])
    return m


LIMB_BODIES = ("hip_yaw", "knee", "shoulder_yaw", "elbow")   # thighs, shins, upper arms, forearms


def humanoid_terrain(tile=0.6, n=2, max_height=0.03, seed=2602) -> dict:
    """The humanoid on a random-height grid: n x n static box tiles of side ``tile`` centred
    under the robot, tops at heights U[0, max_height] from a fixed seed; the four foot boxes
    touch the tiles (box against box) and so do the limb capsules (thighs, shins, upper arms,
    forearms: capsule against box), every other geom only the plane.  The pelvis starts
    ``max_height`` higher."""
    m = humanoid()
    m["name"] = "humanoid_terrain"
    rng = np.random.default_rng(seed)
    heights = rng.uniform(0.0, max_height, (n, n))
    half = tile / 2
    for i in range(n):
        for j in range(n):
            cx, cy = (i - (n - 1) / 2) * tile, (j - (n - 1) / 2) * tile
            m["geoms"].append(dict(type="box", body=0, pos=[cx, cy, float(heights[i, j]) - 0.05],
                                   quat=[1.0, 0.0, 0.0, 0.0], size=[half, half, 0.05], friction=1.0,
                                   margin=0.0, **TERRAIN_GEOM))
    for g in m["geoms"]:
        bname = m["bodies"][g["body"]]["name"]
        if g["type"] == "box" and bname.endswith("ankle_roll"):
            g["contype"] = 3
        if g["type"] == "capsule" and bname.endswith(LIMB_BODIES):
            g["contype"] = 3
    m["bodies"][1]["pos"][2] += max_height
    return m


def with_limits(model: dict, lower: float, upper: float, name: str | None = None) -> dict:
    """Copy of ``model`` whose hinges are limited to [lower, upper] (radians)."""
    out = copy.deepcopy(model)
    for j in out["joints"]:
        if j["type"] == "hinge":
            j["range"] = [float(lower), float(upper)]
    if name:
        out["name"] = name
    return out


def with_damping(model: dict, damping: float, name: str | None = None) -> dict:
    """Copy of ``model`` whose hinges carry joint damping ``damping`` (N m s / rad)."""
    out = copy.deepcopy(model)
    for j in out["joints"]:
        if j["type"] == "hinge":
            j["damping"] = float(damping)
    if name:
        out["name"] = name
    return out


def chain3_damp() -> dict:
    """chain3 with strong joint damping (2 N m s / rad on each hinge)."""
    return with_damping(chain3(), 2.0, "chain3_damp")


def humanoid_damp() -> dict:
    """humanoid with joint damping 0.5 N m s / rad on every hinge."""
    return with_damping(humanoid(), 0.5, "humanoid_damp")


def quadruped_slip() -> dict:
    """quadruped whose sphere feet are frictionless (condim 1) against the ground."""
    m = quadruped()
    m["name"] = "quadruped_slip"
    for g in m["geoms"]:
        if g["type"] == "sphere":
            g["condim"] = 1
    return m


def chain3_lim() -> dict:
    """chain3 with every hinge limited to +-0.6 rad."""
    return with_limits(chain3(), -0.6, 0.6, "chain3_lim")


def quadruped_lim() -> dict:
    """quadruped with every hinge limited to +-0.25 rad (the control targets often lie beyond)."""
    return with_limits(quadruped(), -0.25, 0.25, "quadruped_lim")


def humanoid_lim() -> dict:
    """humanoid with every hinge limited to +-0.15 rad (the control targets often lie beyond)."""
    return with_limits(humanoid(), -0.15, 0.15, "humanoid_lim")


LOOP_POINT = (0.5, 0.0, -1.1)   # world point holding chain3_loop's tip


def chain3_loop() -> dict:
    """chain3 whose tip (the end of link 3) is connected to the world point LOOP_POINT: a closed
    planar loop with one degree of freedom, swinging under gravity."""
    m = chain(3, "chain3_loop")
    m["equality"] = [dict(type="connect", body=3, anchor=[0.0, 0.0, -0.5], target=list(LOOP_POINT))]
    return m


def humanoid_weld() -> dict:
    """humanoid whose pelvis is welded to the world at its reference pose (a fixed-base humanoid:
    the limbs move under position control, the feet reach the ground)."""
    m = humanoid()
    m["name"] = "humanoid_weld"
    m["equality"] = [dict(type="weld", body=1, anchor=[0.0, 0.0, 0.0], target=list(m["bodies"][1]["pos"]),
                          quat=[1.0, 0.0, 0.0, 0.0])]
    return m


def quadruped_condim6() -> dict:
    """quadruped whose sphere feet have torsional and rolling friction (condim 6: mu_spin 0.02,
    mu_roll 0.002 against the ground)."""
    m = quadruped()
    m["name"] = "quadruped_condim6"
    for g in m["geoms"]:
        if g["type"] == "sphere":
            g.update(condim=6, friction_spin=0.02, friction_roll=0.002)
    return m


def humanoid_condim4() -> dict:
    """humanoid whose four foot boxes have torsional friction (condim 4, mu_spin 0.02)."""
    m = humanoid()
    m["name"] = "humanoid_condim4"
    feet = {i for i, b in enumerate(m["bodies"]) if b.get("name", "").endswith("ankle_roll")}
    for g in m["geoms"]:
        if g["type"] == "box" and g["body"] in feet:
            g.update(condim=4, friction_spin=0.02)
    return m


def with_elliptic(model: dict, impratio: float, name: str) -> dict:
    out = copy.deepcopy(model)
    out["opt"]["cone"] = "elliptic"
    out["opt"]["impratio"] = float(impratio)
    out["name"] = name
    return out


def quadruped_elliptic() -> dict:
    """quadruped with elliptic friction cones (impratio 1)."""
    return with_elliptic(quadruped(), 1.0, "quadruped_elliptic")


def humanoid_elliptic() -> dict:
    """humanoid with elliptic friction cones (impratio 1)."""
    return with_elliptic(humanoid(), 1.0, "humanoid_elliptic")


def quadruped_elliptic4() -> dict:
    """quadruped with elliptic friction cones (impratio 1) whose sphere feet have torsional
    friction (condim 4, mu_spin 0.02): four rows per foot contact in one cone."""
    m = with_elliptic(quadruped(), 1.0, "quadruped_elliptic4")
    for g in m["geoms"]:
        if g["type"] == "sphere":
            g.update(condim=4, friction_spin=0.02)
    return m


def quadruped_elliptic6() -> dict:
    """quadruped with elliptic friction cones (impratio 1) whose sphere feet have torsional and
    rolling friction (condim 6: mu_spin 0.02, mu_roll 0.002): six rows per foot contact in one
    cone."""
    m = with_elliptic(quadruped(), 1.0, "quadruped_elliptic6")
    for g in m["geoms"]:
        if g["type"] == "sphere":
            g.update(condim=6, friction_spin=0.02, friction_roll=0.002)
    return m


def humanoid_elliptic4() -> dict:
    """humanoid with elliptic friction cones (impratio 1) whose four foot boxes have torsional
    friction (condim 4, mu_spin 0.02), with up to 8 Newton updates per substep: a spin row in
    each foot corner's cone puts more contacts on their cones' surfaces, where the cost is not
    quadratic, and 4 updates leave about a tenth of the steps short of convergence."""
    m = with_elliptic(humanoid_condim4(), 1.0, "humanoid_elliptic4")
    m["opt"]["iterations"] = 8
    return m


CUBE_HALF = 0.05   # cube_stack: cube half size (m)


def cube_stack(ncube: int = 3) -> dict:
    """Free 10 cm cubes (0.3, 0.2, 0.1 kg from the bottom) stacked on a plane: box-box contacts
    between two moving bodies (each pair of cubes) and box-plane contacts."""
    mb = ModelBuilder("cube_stack", timestep=0.002, nsubsteps=4)
    mb.geom(0, "plane", [0, 0, 0], friction=1.0, contype=0, conaffinity=1)
    h = CUBE_HALF
    for k in range(ncube):
        m = 0.3 - 0.1 * k
        b = mb.body(f"cube{k}", 0, (0, 0, h + 2 * h * k), m, box_inertia(m, h, h, h))
        mb.joint(b, "free")
        mb.geom(b, "box", [h, h, h], friction=0.8, contype=1, conaffinity=1)
    return mb.build()


def pincer() -> dict:
    """A palm on a hinge about x under a fixed mount, with two box fingers (4 and 3 cm deep) on
    hinges about y at x = -+4 cm hanging 10 cm below it; position actuators close the fingers until their tips
    press on each other: box-box contacts between two moving bodies whose chains share the palm's
    dof (and a ground plane under them)."""
    mb = ModelBuilder("pincer", timestep=0.002, nsubsteps=4)
    mb.geom(0, "plane", [0, 0, 0], friction=1.0, **GROUND_GEOM)
    palm = mb.body("palm", 0, (0, 0, 0.3), 0.5, box_inertia(0.5, 0.06, 0.03, 0.01))
    jp = mb.joint(palm, "hinge", (1, 0, 0), armature=0.01)
    mb.geom(palm, "box", [0.06, 0.03, 0.01], **GHOST_GEOM)
    mb.actuator(jp, "position", kp=5.0, kd=0.2)
    # the right finger is narrower along y, so that no edge of one finger's face lies exactly on a
    # side plane of the other's (a clipping tie)
    for side, sx, hy in (("L", -1, 0.02), ("R", 1, 0.015)):
        f = mb.body(f"finger{side}", palm, (0.04 * sx, 0, 0), 0.05, box_inertia(0.05, 0.015, hy, 0.05),
                    ipos=(0, 0, -0.05))
        jf = mb.joint(f, "hinge", (0, 1, 0), armature=0.001)
        mb.geom(f, "box", [0.015, hy, 0.05], pos=(0, 0, -0.05), friction=0.8, contype=1, conaffinity=1)
        mb.actuator(jf, "position", kp=2.0, kd=0.05)
    return mb.build()


def pincer_cube() -> dict:
    """The pincer holding a free 4 cm cube (50 g) between its fingertips: the fingers squeeze it
    and friction carries its weight while the palm swings (finger-cube contacts between moving
    bodies, the analogue of the paper's cube lifting)."""
    m = pincer()
    m["name"] = "pincer_cube"
    mb_cube = {"name": "cube", "parent": 0, "pos": [0.0, 0.0, 0.3 - 0.08], "quat": [1.0, 0.0, 0.0, 0.0],
               "ipos": [0.0, 0.0, 0.0], "iquat": [1.0, 0.0, 0.0, 0.0], "mass": 0.05,
               "inertia": box_inertia(0.05, 0.02, 0.02, 0.02)}
    m["bodies"].append(mb_cube)
    cb = len(m["bodies"]) - 1
    m["joints"].append({"type": "free", "body": cb, "pos": [0.0, 0.0, 0.0], "axis": [0.0, 0.0, 1.0],
                        "armature": 0.0})
    m["geoms"].append({"type": "box", "body": cb, "pos": [0.0, 0.0, 0.0], "quat": [1.0, 0.0, 0.0, 0.0],
                       "size": [0.02, 0.02, 0.02], "friction": 1.0, "contype": 1, "conaffinity": 1, "margin": 0.0})
    return m


def humanoid_self() -> dict:
    """humanoid whose left and right leg capsules (thighs and shins) collide with each other:
    self-collision between two branches of the tree below the pelvis (16 capsule pairs), with a
    Newton budget of 8 updates for the extra rows."""
    m = humanoid()
    m["name"] = "humanoid_self"
    m["opt"]["iterations"] = 8
    names = [b.get("name", "") for b in m["bodies"]]
    for g in m["geoms"]:
        if g["type"] != "capsule":
            continue
        bn = names[g["body"]]
        if bn in ("L_hip_yaw", "L_knee"):
            g["contype"] = g["contype"] | 4
        elif bn in ("R_hip_yaw", "R_knee"):
            g["conaffinity"] = g["conaffinity"] | 4
    return m


BENCH_MODELS = {"chain3": chain3, "quadruped": quadruped, "humanoid": humanoid, "arm_box": arm_box,
                "chain3_lim": chain3_lim, "quadruped_lim": quadruped_lim, "humanoid_lim": humanoid_lim,
                "quadruped_terrain": quadruped_terrain, "humanoid_terrain": humanoid_terrain,
                "chain3_damp": chain3_damp, "humanoid_damp": humanoid_damp, "quadruped_slip": quadruped_slip,
                "quadruped_hfield": quadruped_hfield, "chain3_loop": chain3_loop, "humanoid_weld": humanoid_weld,
                "quadruped_condim6": quadruped_condim6, "humanoid_condim4": humanoid_condim4,
                "quadruped_elliptic": quadruped_elliptic, "humanoid_elliptic": humanoid_elliptic,
                "quadruped_elliptic4": quadruped_elliptic4, "humanoid_elliptic4": humanoid_elliptic4,
                "quadruped_elliptic6": quadruped_elliptic6,
                "cube_stack": cube_stack, "pincer": pincer, "humanoid_self": humanoid_self,
                "pincer_cube": pincer_cube}


def by_name(name: str) -> dict:
    return BENCH_MODELS[name]()
