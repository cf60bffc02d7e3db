"""Seeded synthetic inputs: initial states, control tables and per-world parameters.

World ``w`` of workload ``c`` draws from ``numpy.random.Generator(PCG64(SeedSequence([c, w, s])))``
with stream ``s`` = 0 for the initial state, 1 for controls, 2 for per-world
parameters, so a world's inputs never depend on how many worlds run beside it.
Values are drawn in float64 and rounded to float32; both the oracle and the HIP
path consume the same float32 values (the oracle widens them to float64).
"""
from __future__ import annotations

import math

import numpy as np

from . import robots

WORKLOAD_IDS = {"chain3": 1, "quadruped": 2, "humanoid": 3, "arm_box": 4,
                "chain3_lim": 6, "quadruped_lim": 7, "humanoid_lim": 8, "quadruped_terrain": 9,
                "humanoid_terrain": 10, "chain3_damp": 11, "humanoid_damp": 12,
                "quadruped_slip": 13, "quadruped_hfield": 14, "chain3_loop": 15, "humanoid_weld": 16,
                "quadruped_condim6": 17, "humanoid_condim4": 18, "quadruped_elliptic": 19,
                "humanoid_elliptic": 20, "cube_stack": 21, "pincer": 22,
                "humanoid_self": 23, "pincer_cube": 24, "quadruped_elliptic4": 25, "humanoid_elliptic4": 26,
                "quadruped_elliptic6": 27}
CTRL_PERIOD = 20          # env steps between control resamples
CTRL_STD = {"chain3": 0.0, "quadruped": 0.3, "humanoid": 0.2, "arm_box": 0.3,
            "chain3_lim": 0.0, "quadruped_lim": 0.3, "humanoid_lim": 0.2, "quadruped_terrain": 0.3,
            "humanoid_terrain": 0.2, "chain3_damp": 0.0, "humanoid_damp": 0.2,
            "quadruped_slip": 0.3, "quadruped_hfield": 0.3, "chain3_loop": 0.0, "humanoid_weld": 0.2,
            "quadruped_condim6": 0.3, "humanoid_condim4": 0.2, "quadruped_elliptic": 0.3,
            "humanoid_elliptic": 0.2, "cube_stack": 0.0, "pincer": 0.1,
            "humanoid_self": 0.2, "pincer_cube": 0.1, "quadruped_elliptic4": 0.3, "humanoid_elliptic4": 0.2,
            "quadruped_elliptic6": 0.3}
# mean control target per actuator where it is not 0: the pincer's fingers close past each other
CTRL_MEAN = {"pincer": [0.0, -0.4, 0.4], "pincer_cube": [0.0, -0.2, 0.2],
             # the humanoid's hips adducted (left roll -, right roll +) so that its legs meet
             "humanoid_self": [0.0, -0.25] + [0.0] * 5 + [0.25] + [0.0] * 21}


def rng(workload_id: int, world: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(workload_id), int(world), int(stream)])))


def _hinge_qadr(model: dict) -> list[int]:
    out, adr = [], 0
    for j in model["joints"]:
        if j["type"] == "hinge":
            out.append(adr)
            adr += 1
        else:
            adr += 7
    return out


def initial_state(model: dict, name: str, worlds, workload_id: int | None = None):
    """(qpos[n, nq], qvel[n, nv]) float32 for the given world ids."""
    wid = WORKLOAD_IDS.get(name, 0) if workload_id is None else workload_id
    d = robots.dims(model)
    q0 = robots.qpos0(model)
    hq = _hinge_qadr(model)
    worlds = list(worlds)
    qpos = np.zeros((len(worlds), d["nq"]), np.float64)
    qvel = np.zeros((len(worlds), d["nv"]), np.float64)
    for i, w in enumerate(worlds):
        g = rng(wid, w, 0)
        qpos[i] = q0
        if name in ("chain3", "chain3_damp"):
            qpos[i, :] = g.uniform(-math.pi, math.pi, d["nq"])
            qvel[i, :] = g.normal(0.0, 0.5, d["nv"])
        elif name == "chain3_lim":
            # inside the +-0.6 rad limits, fast enough to reach them
            qpos[i, :] = g.uniform(-0.5, 0.5, d["nq"])
            qvel[i, :] = g.normal(0.0, 2.0, d["nv"])
        elif name in ("quadruped_lim", "quadruped_terrain", "quadruped_slip", "quadruped_hfield", "quadruped_condim6",
                      "quadruped_elliptic", "quadruped_elliptic4", "quadruped_elliptic6"):
            qpos[i, hq] = g.uniform(-0.1, 0.1, len(hq))
        elif name == "pincer":
            # palm angle U[+-0.2], fingers open U[0, 0.3] / U[-0.3, 0] (tips apart), at rest
            qpos[i, :] = [g.uniform(-0.2, 0.2), g.uniform(0.0, 0.3), g.uniform(-0.3, 0.0)]
        elif name == "pincer_cube":
            # palm angle U[+-0.05], fingertips just touching the cube (U[0, 0.01] rad past contact),
            # the cube between them at rest
            qpos[i, :3] = [g.uniform(-0.05, 0.05), -0.0625 - g.uniform(0, 0.01), 0.0625 + g.uniform(0, 0.01)]
        elif name == "cube_stack":
            # each cube over the one below with a horizontal offset U[+-1.5 cm], yaw U[+-0.3],
            # a tilt U[0, 0.02] rad about a random horizontal axis, lifted 1 mm per level, at rest
            h = robots.CUBE_HALF
            for k in range(len(model["bodies"]) - 1):
                yaw, tilt, ax = g.uniform(-0.3, 0.3), g.uniform(0.0, 0.02), g.uniform(0, 2 * math.pi)
                qy = np.array([math.cos(yaw / 2), 0, 0, math.sin(yaw / 2)])
                s = math.sin(tilt / 2)
                qt = np.array([math.cos(tilt / 2), s * math.cos(ax), s * math.sin(ax), 0])
                qq = np.array([qt[0] * qy[0] - qt[3] * qy[3], qt[1] * qy[0] + qt[2] * qy[3],
                               qt[2] * qy[0] - qt[1] * qy[3], qt[0] * qy[3] + qt[3] * qy[0]])
                qpos[i, 7 * k:7 * k + 3] = [g.uniform(-0.015, 0.015), g.uniform(-0.015, 0.015),
                                            h + 2 * h * k + 0.001 * (k + 1)]
                qpos[i, 7 * k + 3:7 * k + 7] = qq / np.linalg.norm(qq)
        elif name == "chain3_loop":
            # on the loop: link 1's angle uniform around the direction of the held point, links 2
            # and 3 closing the loop (elbow bent either way, the knee's sign drawn), at rest
            P = np.array([robots.LOOP_POINT[0], robots.LOOP_POINT[2]])
            phi = math.atan2(-P[0], -P[1])
            while True:
                q1 = phi + g.uniform(-0.6, 0.6)
                p1 = 0.5 * np.array([-math.sin(q1), -math.cos(q1)])
                dd = P - p1
                r = float(np.hypot(*dd))
                if r < 0.98:
                    break
            # absolute directions of links 2 and 3: the chord's direction -+ the half-angle
            base = math.atan2(-dd[0], -dd[1])
            half = math.acos(r / 1.0)
            sgn = 1.0 if g.uniform() < 0.5 else -1.0
            a2, a3 = base + sgn * half, base - sgn * half
            qpos[i, :] = [q1, a2 - q1, a3 - a2]
        elif name in ("humanoid_lim", "humanoid_terrain", "humanoid_damp", "humanoid_weld", "humanoid_condim4",
                      "humanoid_elliptic", "humanoid_self", "humanoid_elliptic4"):
            qpos[i, hq] = g.uniform(-0.05, 0.05, len(hq))
        elif name == "quadruped":
            qpos[i, hq] = g.uniform(-0.1, 0.1, len(hq))
        elif name == "humanoid":
            qpos[i, hq] = g.uniform(-0.05, 0.05, len(hq))
        elif name == "arm_box":
            qpos[i, hq] = g.uniform(-0.1, 0.1, len(hq))
        else:
            raise KeyError(name)
    return qpos.astype(np.float32), qvel.astype(np.float32)


def ctrl_table(model: dict, name: str, worlds, nseg: int, workload_id: int | None = None) -> np.ndarray:
    """Control targets [nseg, n, nu] float32; segment k is held for env steps [k*20, (k+1)*20)."""
    wid = WORKLOAD_IDS.get(name, 0) if workload_id is None else workload_id
    nu = len(model["actuators"])
    worlds = list(worlds)
    out = np.zeros((nseg, len(worlds), nu), np.float64)
    std = CTRL_STD.get(name, 0.0)
    if nu and std > 0:
        for i, w in enumerate(worlds):
            out[:, i, :] = rng(wid, w, 1).normal(0.0, std, (nseg, nu))
    if name in CTRL_MEAN:
        out += np.asarray(CTRL_MEAN[name], np.float64)
    return out.astype(np.float32)


def world_params(model: dict, name: str, worlds, workload_id: int | None = None):
    """Per-world (friction[n], mass_scale[n, nbody]) float32, or None where the model shares the field."""
    wid = WORKLOAD_IDS.get(name, 0) if workload_id is None else workload_id
    nb = len(model["bodies"])
    worlds = list(worlds)
    fr = ms = None
    if model["per_world"].get("friction") or model["per_world"].get("mass_scale"):
        fr = np.zeros(len(worlds), np.float64)
        ms = np.ones((len(worlds), nb), np.float64)
        for i, w in enumerate(worlds):
            g = rng(wid, w, 2)
            fr[i] = g.uniform(0.3, 1.2)
            ms[i, 1:] = g.uniform(0.8, 1.2, nb - 1)
        fr = fr.astype(np.float32) if model["per_world"].get("friction") else None
        ms = ms.astype(np.float32) if model["per_world"].get("mass_scale") else None
    return fr, ms


def workload(name: str, nworlds: int, nsteps: int, first_world: int = 0):
    """Everything one benchmark workload needs: model, initial state, control table, per-world params."""
    model = robots.by_name(name)
    worlds = range(first_world, first_world + nworlds)
    qpos, qvel = initial_state(model, name, worlds)
    nseg = max(1, -(-nsteps // CTRL_PERIOD))
    ctrl = ctrl_table(model, name, worlds, nseg)
    fr, ms = world_params(model, name, worlds)
    return dict(model=model, name=name, qpos=qpos, qvel=qvel, ctrl=ctrl, friction=fr, mass_scale=ms,
                nsteps=nsteps, worlds=list(worlds))
