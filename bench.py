"""Benchmark of the batched physics step on one MI355X.

Default workload: the 29-hinge humanoid (free base, 30 bodies, 40 colliding geoms vs a
plane), 8192 worlds, dt 5 ms x 4 substeps, Newton <= 4 iterations, per-world friction and
mass scale, controls ~N(0, 0.2) resampled every 20 env steps, contacts returned every step.
Inputs are synthetic and seeded (workloads/), resident on the GPU before timing starts.

Prints one JSON line: env-steps/s over the timed steps, per-call p50/p99 latency, the
roofline of the step kernel (FP32 ALU bound: algorithmic FLOPs per launch over the measured
launch time, against the 157.3 TFLOP/s vector peak), HBM bytes and their fraction of 8 TB/s,
and the FP64 oracle timed on this host's cores on a bounded sample (a baseline only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

WORKLOAD_TEXT = {
    "humanoid": "humanoid: free base + 29 hinges, 30 bodies, 40 capsule/box geoms vs plane, dt 5 ms x 4 substeps, "
                "Newton <= 4 iters, per-world friction U[0.3,1.2] and mass scale U[0.8,1.2], ctrl N(0,0.2)/20 steps",
    "quadruped": "quadruped: free base + 12 hinges, 13 bodies, sphere feet + box torso vs plane, friction 1, "
                 "PD kp 20 kd 0.5, dt 5 ms x 4 substeps, ctrl N(0,0.3)/20 steps",
    "chain3": "3-link planar hinge chain, contact-free, dt 2 ms, K = 1",
    "arm_box": "7-hinge arm (non-colliding links) beside a static table box with a 5 cm free cube on it: "
               "box-box and box-plane contacts, dt 5 ms x 4 substeps, ctrl N(0,0.2)/20 steps",
    "mix": "mixed batch: chain3 x512 + quadruped x4096 + humanoid x2048 + arm_box x1024 (7680 worlds), "
           "each model's own dt and substeps, contacts returned",
    "humanoid_lim": "humanoid with every hinge limited to +-0.15 rad (limit rows solved with the contacts), "
                    "otherwise as humanoid",
    "quadruped_lim": "quadruped with every hinge limited to +-0.25 rad, otherwise as quadruped",
    "quadruped_terrain": "quadruped on a 3x3 random-height grid of 0.4 m box tiles (tops U[0, 4 cm]): "
                         "sphere feet vs static boxes, otherwise as quadruped",
    "humanoid_terrain": "humanoid on a 2x2 random-height grid of 0.6 m box tiles (tops U[0, 3 cm]): foot boxes vs "
                        "static boxes (16 box-box pairs), limb capsules vs static boxes (64 capsule-box pairs), "
                        "otherwise as humanoid",
    "humanoid_damp": "humanoid with joint damping 0.5 N m s/rad on every hinge (implicit in the step), "
                     "otherwise as humanoid",
    "quadruped_hfield": "quadruped on smooth height-field terrain (41x41 grid over 4 m x 4 m, +-3 cm) instead of the "
                        "plane: feet and torso vs the triangle under each candidate point, otherwise as quadruped",
    "humanoid_weld": "humanoid with its pelvis welded to the world at the reference pose (6 equality rows solved "
                     "with the contacts): limbs under position control, feet reaching the floor, otherwise as humanoid",
    "chain3_loop": "chain3 with its tip connected to a world point (3 equality rows): a closed one-degree-of-freedom "
                   "loop swinging under gravity, dt 2 ms, K = 1",
    "quadruped_condim6": "quadruped whose sphere feet have torsional and rolling friction (condim 6, mu_spin 0.02, "
                         "mu_roll 0.002: 10 pyramid rows per foot contact), otherwise as quadruped",
    "humanoid_condim4": "humanoid whose four foot boxes have torsional friction (condim 4, mu_spin 0.02: 6 pyramid "
                        "rows per foot contact), otherwise as humanoid",
    "quadruped_elliptic": "quadruped with elliptic friction cones (impratio 1): 3 frame rows per contact costed by "
                          "the soft elliptic cone, Newton line search on phi', otherwise as quadruped",
    "humanoid_elliptic": "humanoid with elliptic friction cones (impratio 1), otherwise as humanoid",
    "quadruped_elliptic4": "quadruped with elliptic friction cones (impratio 1) and torsional friction on the "
                           "sphere feet (condim 4, mu_spin 0.02): 4 rows per foot contact in one cone",
    "humanoid_elliptic4": "humanoid with elliptic friction cones (impratio 1) and torsional friction on the "
                          "foot boxes (condim 4, mu_spin 0.02)",
    "quadruped_elliptic6": "quadruped with elliptic friction cones (impratio 1) and torsional and rolling friction "
                           "on the sphere feet (condim 6, mu_spin 0.02, mu_roll 0.002): 6 rows per foot contact "
                           "in one cone",
    "cube_stack": "three free 10 cm cubes (0.3/0.2/0.1 kg) stacked on a plane with random offsets, yaws and tilts: "
                  "box-box contacts between moving bodies (dense Newton Hessian), dt 2 ms x 4 substeps",
    "pincer": "a hinged palm with two hinged box fingers closed onto each other by position actuators: box-box "
              "contacts between bodies whose chains share the palm's dof, dt 2 ms x 4 substeps",
    "pincer_cube": "the pincer holding a free 4 cm cube between its fingertips while the palm swings (finger-cube "
                   "contacts between moving bodies, friction carrying the cube), dt 2 ms x 4 substeps",
    "humanoid_self": "humanoid whose left and right thigh and shin capsules collide with each other (16 capsule "
                     "pairs, hips adducted so the legs meet; dense Newton Hessian), otherwise as humanoid",
}
MIX = [("chain3", 512), ("quadruped", 4096), ("humanoid", 2048), ("arm_box", 1024)]
DEFAULT_WORLDS = {"humanoid": 8192, "quadruped": 4096, "chain3": 64, "arm_box": 1024, "humanoid_lim": 8192,
                  "quadruped_lim": 4096, "quadruped_terrain": 4096, "humanoid_terrain": 8192,
                  "humanoid_damp": 8192, "quadruped_hfield": 4096, "humanoid_weld": 8192, "chain3_loop": 8192,
                  "quadruped_condim6": 4096, "humanoid_condim4": 8192, "quadruped_elliptic": 4096,
                  "humanoid_elliptic": 8192, "quadruped_elliptic4": 4096, "humanoid_elliptic4": 8192, "quadruped_elliptic6": 4096, "cube_stack": 8192, "pincer": 8192, "humanoid_self": 8192,
                  "pincer_cube": 8192}
WORKLOAD_TEXT["serve"] = ("serving: Poisson arrivals of rollout requests, model uniform over chain3/quadruped/humanoid/"
                          "arm_box, worlds log-uniform 16-4096, horizon uniform 50-500 env steps, device-side seeded "
                          "inputs, HBM-budget admission, continuous batching in one fused launch per tick")


# ------------------------------------------------------------------ mixed-model batching
def run_mix(args, emit=True):
    """The batching form on the mixed batch: one env step of every world per call, timed for
    (a) separate plain launches back to back on one stream, (b) the same on one stream per
    model, (c) the fused launch under the autotuned schedule and (d) that launch replayed from
    a captured hipGraph of one control period.  Every form starts from the same state; its
    final state is compared bit for bit with (a).  Returns the result (printed when emit)."""
    import torch
    import paper_2601_22074_amd as rb
    from paper_2601_22074_amd import autotune
    from workloads import inputs

    dev = torch.device("cuda:0")
    K, warm = args.steps, args.warmup
    P = inputs.CTRL_PERIOD
    K = max(P, K // P * P)
    warm = (warm + P - 1) // P * P
    Ws = [inputs.workload(name, n, warm + K) for name, n in MIX]
    models = [rb.Model(W["model"]) for W in Ws]

    def fresh():
        S = []
        for (name, n), W, model in zip(MIX, Ws, models):
            b = rb.Batch(model, n)
            if W["friction"] is not None:
                b.set_params(rb.PARAM_FRICTION, torch.tensor(W["friction"], device=dev))
            if W["mass_scale"] is not None:
                b.set_params(rb.PARAM_MASS_SCALE, torch.tensor(W["mass_scale"], device=dev))
            ctab = torch.tensor(W["ctrl"], device=dev).contiguous()
            if ctab.shape[-1] == 0:
                ctab = torch.zeros(ctab.shape[0], n, 1, device=dev)
            S.append(dict(batch=b, n=n, ctab=ctab, u=ctab[0].clone(), q=torch.tensor(W["qpos"], device=dev),
                          v=torch.tensor(W["qvel"], device=dev), con=b.contacts(n),
                          st=torch.zeros(n, dtype=torch.int32, device=dev)))
        torch.cuda.synchronize()
        return S

    def seg(S, s):
        return [x["ctab"][min(s // P, x["ctab"].shape[0] - 1)] for x in S]

    def timed(S, step_fn, period_fn=None):
        stream = torch.cuda.current_stream()
        for s in range(warm):
            if s % P == 0 and period_fn:
                period_fn(S, s)
            step_fn(S, s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for s in range(warm, warm + K):
            if s % P == 0 and period_fn:
                period_fn(S, s)
            step_fn(S, s)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K

    def finals(S):
        return [(x["q"].cpu().numpy(), x["v"].cpu().numpy(), x["st"].cpu().numpy()) for x in S]

    nworlds = sum(n for _, n in MIX)
    res, equal = {}, {}
    # (a) separate launches, one stream
    S = fresh()

    def sep(S, s):
        for x, u in zip(S, seg(S, s)):
            x["batch"].step(u, x["q"], x["v"], x["con"], x["st"])
    res["separate"] = timed(S, sep)
    ref = finals(S)

    # (b) separate launches, one stream per model (default priority), joined every step
    S = fresh()
    streams = [torch.cuda.Stream() for _ in S]
    main = torch.cuda.current_stream()

    def sep4(S, s):
        ev = torch.cuda.Event()
        ev.record(main)
        for x, u, st in zip(S, seg(S, s), streams):
            st.wait_event(ev)
            x["batch"].step(u, x["q"], x["v"], x["con"], x["st"], stream=st)
        for st in streams:
            e = torch.cuda.Event()
            e.record(st)
            main.wait_event(e)
    res["separate_streams"] = timed(S, sep4)
    equal["separate_streams"] = all(all(np.array_equal(a, b) for a, b in zip(r, f)) for r, f in zip(ref, finals(S)))

    # (c) fused launch, autotuned schedule
    S = fresh()
    plan = rb.Multi([x["batch"] for x in S])
    for i, x in enumerate(S):
        plan.bind(i, x["u"], x["q"], x["v"], x["con"], x["st"])
    choice, timings = autotune.tune(plan, [(x["u"], x["q"], x["v"]) for x in S], reps=10, resident=args.resident,
                                    advance=warm)
    for i, x in enumerate(S):
        plan.bind(i, x["u"], x["q"], x["v"], x["con"], x["st"])
    if choice[0] != "fused":
        choice = ("fused", rb.ORDER_HEAVY_FIRST, 0, 0, 1)
    plan.set_schedule(choice[1], choice[2])
    plan.set_occupancy(choice[3])
    plan.set_group(choice[4])

    def load_ctrl(S, s):
        for x, u in zip(S, seg(S, s)):
            x["u"].copy_(u)

    res["fused"] = timed(S, lambda S, s: plan.step(), load_ctrl)
    equal["fused"] = all(all(np.array_equal(a, b) for a, b in zip(r, f)) for r, f in zip(ref, finals(S)))
    plan.close()

    # (d) fused launch replayed from a hipGraph of one control period (P env steps)
    S = fresh()
    plan = rb.Multi([x["batch"] for x in S])
    for i, x in enumerate(S):
        plan.bind(i, x["u"], x["q"], x["v"], x["con"], x["st"])
    plan.set_schedule(choice[1], choice[2])
    plan.set_occupancy(choice[3])
    plan.set_group(choice[4])
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    plan.graph_capture(P, side)
    torch.cuda.synchronize()

    def graph_period(S, s):
        load_ctrl(S, s)
        plan.graph_launch(torch.cuda.current_stream())

    ms = timed(S, lambda S, s: None, graph_period)
    res["fused_graph"] = ms
    equal["fused_graph"] = all(all(np.array_equal(a, b) for a, b in zip(r, f)) for r, f in zip(ref, finals(S)))
    plan.close()

    rates = {k: nworlds / (v / 1e3) for k, v in res.items()}
    best = max(("fused", "fused_graph"), key=lambda k: rates[k])
    out = {
        "metric": "env-steps/sec, mixed batch (chain3 x512 + quadruped x4096 + humanoid x2048 + arm_box x1024)",
        "value": rates[best],
        "unit": "env-steps/s",
        "n_gpus": 1, "steps": K, "warmup": warm,
        "ms_per_step": res[best],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["mix"], "worlds": nworlds, "env_steps": K, "form": best,
                   "schedule": {"order": choice[1], "grid": choice[2], "waves_per_simd_cap": choice[3],
                                "worlds_per_workgroup": choice[4]},
                   "graph_steps": P},
        "forms_env_steps_per_s": rates,
        "forms_ms_per_step": res,
        "speedup_vs_separate": rates[best] / rates["separate"],
        "bitwise_equal_to_separate": equal,
        "autotune_timings_ms": timings,
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


# ------------------------------------------------------------------ serving
def run_serve(args):
    """The serving form: (a) the offered load (Poisson rate --rate for --seconds), stopped at
    that time with whatever is still queued counted as backlog, served by the fused server and,
    on the same trace, by the plain-launch baseline (one rb_step launch per live request per
    tick); (b) a rate the fused server's measured throughput sustains (80 % of it), run to
    completion, for steady-state latency."""
    import torch
    from paper_2601_22074_amd.serve import PlainServer, Server
    from workloads import robots
    from workloads.requests import NAMES, DeviceSource, mean_request_work, poisson_requests

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    src = DeviceSource({k: robots.by_name(k) for k in NAMES})
    # admission by the device's free memory, or by a configured budget as well
    budget = (int(args.budget_mb) << 20) if args.budget_mb > 0 else None

    for cls in (Server, PlainServer):
        srv = cls(src, budget=budget)
        # warm-up: compile and first launches outside the timed runs
        srv.run_script(poisson_requests(50.0, 0.2, seed=99, wmax=64, hmax=50))
        srv.close()

    reqs = poisson_requests(args.rate, args.seconds, seed=1)
    runs = {}
    for key, cls in (("fused", Server), ("plain", PlainServer)):
        srv = cls(src, budget=budget)
        log(f"serve ({key}): offered {len(reqs)} requests over {args.seconds} s")
        runs[key] = srv.run_timed(reqs, stop_after=args.seconds, progress=log)
        srv.close()
    a = runs["fused"]
    offered = args.rate * mean_request_work()
    lam = 0.8 * a["env_steps_per_s"] / mean_request_work()
    srv = Server(src, budget=budget)
    reqs_b = poisson_requests(lam, args.sustain_seconds, seed=2)
    log(f"serve: sustainable-rate run at {lam:.2f}/s, {len(reqs_b)} requests")
    b = srv.run_timed(reqs_b, stop_after=3 * args.sustain_seconds, progress=log)
    srv.close()
    srv = PlainServer(src, budget=budget)
    log(f"serve (plain): the same sustainable-rate trace")
    bp = srv.run_timed(reqs_b, stop_after=3 * args.sustain_seconds, progress=log)
    srv.close()
    out = {
        "metric": f"env-steps/sec served at Poisson {args.rate:g} requests/s; p50/p99 request latency",
        "value": a["env_steps_per_s"],
        "unit": "env-steps/s",
        "n_gpus": 1, "steps": a["ticks"], "warmup": 0,
        "ms_per_step": 1e3 * a["wall_s"] / max(a["ticks"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["serve"], "rate_per_s": args.rate, "seconds": args.seconds,
                   "budget_bytes": a["budget_bytes"]},
        "offered_env_steps_per_s": offered,
        "offered_load": a,
        "offered_load_plain_launches": runs["plain"],
        "sustainable_rate_per_s": lam,
        "sustainable": b,
        "sustainable_plain_launches": bp,
    }
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ work model
def tree_info(model):
    """Dof depths and per-body chain depths of a model description (bookkeeping only)."""
    bodies, joints = model["bodies"], model["joints"]
    nb = len(bodies)
    bj = {j["body"]: j for j in joints}
    last = [-1] * nb
    depth = []
    nfree = nhinge = 0
    for b in range(1, nb):
        p = bodies[b]["parent"]
        pd = last[p]
        j = bj.get(b)
        if j is None:
            last[b] = pd
            continue
        nd = 6 if j["type"] == "free" else 1
        nfree += j["type"] == "free"
        nhinge += j["type"] == "hinge"
        for k in range(nd):
            par = pd if k == 0 else len(depth) - 1
            depth.append(1 if par < 0 else depth[par] + 1)
        last[b] = len(depth) - 1
    bdepth = [0 if last[b] < 0 else depth[last[b]] for b in range(nb)]
    return dict(nb=nb, nv=len(depth), depth=depth, bdepth=bdepth, nfree=nfree, nhinge=nhinge,
                nfixed=nb - 1 - nfree - nhinge, nM=sum(depth))


def flops_per_env_step(model, stats_mean):
    """A cross-check of the roofline numerator (which comes from the oracle's operation counts):
    a per-stage hand count of the tree-sparse method's FP32 operations (multiply-add = 2) fed
    with the kernel's own work per substep.

    stats_mean: per-substep means of (contacts, active rows, Newton iterations, line-search
    segments), measured by the kernel's stats tap on a subset of the same worlds."""
    t = tree_info(model)
    nb, nv, nM = t["nb"], t["nv"], t["nM"]
    dep = np.array(t["depth"])
    nu = len(model["actuators"])
    K = model["opt"]["nsubsteps"]
    con, rows, iters, segs = stats_mean
    # pairs and colliding-body chain depth
    caps = []
    cdepth = []
    for g in model["geoms"]:
        if g["type"] == "plane" or g["contype"] == 0:
            continue
        caps.append({"sphere": 1, "capsule": 2, "box": 8}[g["type"]])
        cdepth.append(t["bdepth"][g["body"]])
    npair = len(caps)
    d_c = float(np.mean(cdepth)) if cdepth else 0.0
    ldl = float(np.sum(1.5 * (dep - 1) * dep + dep))
    solve = 4.0 * (nM - nv) + nv
    msum = 4.0 * (nM - nv) + 2 * nv
    bm = 12.0 * sum(t["bdepth"])
    smooth = (5 * nu + 190 * t["nhinge"] + 60 * t["nfree"] + 46 * t["nfixed"] + 170 * (nb - 1)
              + 42 * t["nhinge"] + 27 * t["nfree"] + 54 * t["nhinge"] + 198 * t["nfree"] + 124 * (nb - 1)
              + 48 * nv + 11 * nM + ldl + solve + nv + 4 * nv + 60 * t["nfree"])
    coll = sum(186 + 25 * c for c in caps) + con * (186 + 25 * (np.mean(caps) if caps else 0) + 28)
    rowsf = con * (42 * d_c + 3 * d_c * d_c + 100)
    newton = 0.0
    if con > 0:
        init = 2 * bm + 2 * con * 46 + msum + 6 * nv
        per_it = (con * d_c * 35 + rows * d_c * 30 + 3 * nv + 11 * nM + ldl + solve + bm + 30 * con + msum
                  + 4 * nv + 6 * nv + 20 * con)
        per_seg = 32 * con + 10
        newton = init + iters * per_it + segs * per_seg
    return K * (smooth + coll + rowsf + newton)


def hbm_bytes_per_env_step(model, con_last, contacts_on):
    t = tree_info(model)
    nq = sum(7 if j["type"] == "free" else 1 for j in model["joints"])
    nv, nb = t["nv"], t["nb"]
    nu = len(model["actuators"])
    pw = model["per_world"]
    rd = 4 * (nq + nv + nu + nv + 1) + (4 if pw.get("friction") else 0) + (4 * nb if pw.get("mass_scale") else 0)
    wr = 4 * (nq + nv + nv + 1)
    if contacts_on:
        wr += 4 + con_last * 4 * (2 + 1 + 1 + 3 + 9 + 3)
    return rd + wr


# ------------------------------------------------------------------ CPU baseline
def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


CPU_PHASE = 20        # env steps the CPU baseline's sample starts into the workload
CPU_STEPS = 10        # env steps the CPU baseline times
CPU_WORLDS = 4096     # worlds of the OpenMP run (the workload's own count if smaller)
CPU_WORLDS_1T = 256   # worlds of the single-thread run


def _oracle_inputs(W, nw, s):
    f = lambda a: None if a is None else a[:nw].astype(np.float64)
    return W["ctrl"][min(s // 20, len(W["ctrl"]) - 1)][:nw].astype(np.float64), f(W["friction"]), f(W["mass_scale"])


def cpu_baseline(W):
    """The FP64 oracle on the host cores (OpenMP over worlds) over a fixed sample of the same
    workload: min(CPU_WORLDS, worlds) worlds advanced untimed by the oracle to env step
    CPU_PHASE (the robots are down and in contact, as in the timed GPU run), then CPU_STEPS env
    steps timed; and the first CPU_WORLDS_1T of those worlds on one thread.  The sample does not
    depend on the bench's step count."""
    from oracle import Oracle
    o = Oracle(W["model"])
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        cores = min(cores, int(os.environ["OMP_NUM_THREADS"]))
    nw = min(len(W["worlds"]), CPU_WORLDS)
    q = W["qpos"][:nw].astype(np.float64)
    v = W["qvel"][:nw].astype(np.float64)
    ws = np.zeros_like(v)
    st = np.zeros(nw, np.uint32)
    for s in range(CPU_PHASE):
        u, fr, ms = _oracle_inputs(W, nw, s)
        o.step(u, q, v, ws, fr, ms, st, nthreads=cores)

    def run(n, threads):
        qq, vv, ww, ss = q[:n].copy(), v[:n].copy(), ws[:n].copy(), st[:n].copy()
        t0 = time.perf_counter()
        for s in range(CPU_PHASE, CPU_PHASE + CPU_STEPS):
            u, fr, ms = _oracle_inputs(W, n, s)
            o.step(u, qq, vv, ww, fr, ms, ss, nthreads=threads)
        return time.perf_counter() - t0

    dt = run(nw, cores)
    n1 = min(nw, CPU_WORLDS_1T)
    dt1 = run(n1, 1)
    return {"value": nw * CPU_STEPS / dt, "unit": "env-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{nw} worlds x env steps {CPU_PHASE}-{CPU_PHASE + CPU_STEPS - 1} of the same workload "
                      f"(advanced to step {CPU_PHASE} by the oracle, untimed), FP64, OpenMP over worlds, {dt:.1f} s",
            "single_thread_value": n1 * CPU_STEPS / dt1,
            "single_thread_sample": f"{n1} of those worlds, same steps, one thread, {dt1:.1f} s",
            "cpu_model": _cpu_model(), "cpu_count": os.cpu_count()}


ORACLE_STAGES = ("kinematics", "inertia+bias", "factorisation+a0", "collision", "constraint rows", "newton",
                 "integration")


def oracle_work(W, nworlds, first, nsteps):
    """Algorithmic work per env step from the oracle: its per-stage operation counts of the
    tree-sparse formulation (a multiply-add counts 2), evaluated on its own contacts, rows,
    active sets, Newton updates and line-search segments, and its per-substep work record means,
    over nworlds worlds of the workload, env steps [first, first + nsteps) of the oracle's own
    trajectory from the same initial states and controls."""
    from oracle import Oracle
    o = Oracle(W["model"])
    nw = min(nworlds, len(W["worlds"]))
    q = W["qpos"][:nw].astype(np.float64)
    v = W["qvel"][:nw].astype(np.float64)
    ws = np.zeros_like(v)
    st = np.zeros(nw, np.uint32)
    ops = np.zeros(7)
    sub = np.zeros(5)
    for s in range(first + nsteps):
        u, fr, ms = _oracle_inputs(W, nw, s)
        work = {} if s >= first else None
        o.step(u, q, v, ws, fr, ms, st, work=work)
        if work is not None:
            ops += work["ops"][:, 1, :].sum(0)
            sub += work["sub"][:, :, :5].reshape(-1, 5).sum(0)
    K = W["model"]["opt"]["nsubsteps"]
    per = ops / (nw * nsteps)
    rec = sub / (nw * nsteps * K)
    return {"flops_per_env_step": float(per.sum()),
            "stage_flops_per_env_step": {k: float(x) for k, x in zip(ORACLE_STAGES, per)},
            "per_substep": {"contacts": rec[0], "rows": rec[1], "newton_updates": rec[2], "active_rows": rec[3],
                            "line_search_segments": rec[4]},
            "sample": f"{nw} worlds x env steps {first}-{first + nsteps - 1}, the oracle's own trajectory"}


def kernel_source_hash():
    """Hash of what decides the step kernel's code: its sources and the compile flags."""
    from paper_2601_22074_amd import build as _b
    h = hashlib.sha256()
    for f in ("step_kernel.hip", "rb_internal.h"):
        with open(os.path.join(ROOT, "paper_2601_22074_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(_b.FLAGS).encode())
    return h.hexdigest()[:16]


def _is_plain_step(kernel_name):
    """The plain step kernel: rbk::step_kernel<MAXD, false, EXT> (3 waves per SIMD) or
    rbk::step_kernel_w4<MAXD, EXT> (4 waves per SIMD), not the diagnostic instantiation."""
    import re
    return re.match(r"void rbk::step_kernel(<\d+, false|_w4<)", kernel_name) is not None


def load_traffic(name, nworlds):
    """HBM bytes per launch from committed PMC counters, if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"step_kernel_{name}_x{nworlds}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


# ------------------------------------------------------------------ rocprofv3 summaries
def summarize_profiles(trace_db, fetch_db, write_db, name, nworlds, calib_mb, commands):
    """Summaries of rocprofv3 databases: per-kernel time, and HBM bytes of the step kernel from
    FETCH_SIZE / WRITE_SIZE scaled by what they read for an elementwise kernel of known size."""
    import sqlite3
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    base = f"step_kernel_{name}_x{nworlds}"
    c = sqlite3.connect(trace_db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    lines = [f"# rocprofv3 kernel trace: {name} x{nworlds}", "", "Command:", "", "```", commands["trace"], "```", "",
             "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for n, calls, tot, avg, pct in rows[:8]:
        short = n if len(n) < 70 else n[:67] + "..."
        lines.append(f"| `{short}` | {calls} | {tot:.1f} | {avg:.1f} | {pct:.2f} |")
    step = [r for r in rows if _is_plain_step(r[0])]
    if step:
        lines += ["", f"Step kernel average duration: {step[0][3]:.1f} us per launch (one env step of {nworlds} worlds)."]
    with open(os.path.join(ROOT, "profiles", base + "_trace.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    def counter(db, cname):
        cc = sqlite3.connect(db)
        q = "select kernel_name, value from counters_collection where counter_name = ?"
        step_v = [v for k, v in cc.execute(q, (cname,)) if _is_plain_step(k)]
        copy_v = [v for k, v in cc.execute(q, (cname,)) if "neg_kernel" in k or ("elementwise" in k and "neg" in k)]
        return step_v, copy_v

    fs, fc = counter(fetch_db, "FETCH_SIZE")
    ws, wc = counter(write_db, "WRITE_SIZE")
    calib_kib = calib_mb * 1024.0
    ffac = calib_kib / float(np.median(fc)) if fc else float("nan")
    wfac = calib_kib / float(np.median(wc)) if wc else float("nan")
    fetch_kib = float(np.median(fs)) if fs else float("nan")
    write_kib = float(np.median(ws)) if ws else float("nan")
    bytes_per_launch = (fetch_kib * ffac + write_kib * wfac) * 1024.0
    d = {"kernel": "plain step kernel (step_kernel_w4<16, false> for this workload)", "workload": f"{name} x{nworlds}",
         "fetch_kib_per_dispatch": fetch_kib, "write_kib_per_dispatch": write_kib,
         "calibration": {"kernel": f"elementwise neg of {calib_mb} MiB (reads and writes {calib_mb} MiB)",
                         "fetch_kib": float(np.median(fc)) if fc else None,
                         "write_kib": float(np.median(wc)) if wc else None,
                         "fetch_factor": ffac, "write_factor": wfac},
         "bytes_per_launch": bytes_per_launch, "kernel_source_hash": kernel_source_hash(),
         "commands": commands}
    with open(os.path.join(ROOT, "profiles", base + "_traffic.json"), "w") as f:
        json.dump(d, f, indent=1)
    md = [f"# HBM traffic of the step kernel: {name} x{nworlds}", "", "Commands:", "", "```", commands["fetch"],
          commands["write"], "```", "",
          f"- FETCH_SIZE per dispatch: {fetch_kib:.0f} KiB; WRITE_SIZE per dispatch: {write_kib:.0f} KiB",
          f"- calibration kernel (elementwise neg of {calib_mb} MiB): FETCH_SIZE {d['calibration']['fetch_kib']} KiB, "
          f"WRITE_SIZE {d['calibration']['write_kib']} KiB -> factors {ffac:.3f} / {wfac:.3f}",
          f"- calibrated HBM bytes per launch: {bytes_per_launch / 1e6:.2f} MB "
          f"({bytes_per_launch / nworlds:.0f} B per world per env step)",
          f"- kernel source hash: {d['kernel_source_hash']}"]
    with open(os.path.join(ROOT, "profiles", base + "_traffic.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print(json.dumps(d))


def summarize_trace(db, title, out, command, note=""):
    """Top kernels of a rocprofv3 --kernel-trace --stats database as a short markdown table."""
    import sqlite3
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    lines = [f"# rocprofv3 kernel trace: {title}", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for n, calls, tot, avg, pct in rows[:10]:
        short = n if len(n) < 70 else n[:67] + "..."
        lines.append(f"| `{short}` | {calls} | {tot:.1f} | {avg:.1f} | {pct:.2f} |")
    if note:
        lines += ["", note]
    with open(os.path.join(ROOT, "profiles", out), "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize_pmc(db, title, out, command):
    """Median per-dispatch counter values of the plain step kernel from a rocprofv3 --pmc database."""
    import sqlite3
    c = sqlite3.connect(db)
    vals = {}
    for k, cn, v in c.execute("select kernel_name, counter_name, value from counters_collection"):
        if _is_plain_step(k):
            vals.setdefault(cn, []).append(v)
    lines = [f"# rocprofv3 counters of the step kernel: {title}", "", "Command:", "", "```", command, "```", "",
             "| counter | median per dispatch |", "|---|---|"]
    for cn in sorted(vals):
        lines.append(f"| {cn} | {float(np.median(vals[cn])):.6g} |")
    lines += ["", f"kernel source hash: {kernel_source_hash()}"]
    with open(os.path.join(ROOT, "profiles", out), "w") as f:
        f.write("\n".join(lines) + "\n")
    return {cn: float(np.median(v)) for cn, v in vals.items()}


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="humanoid", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--worlds", type=int, default=None)
    ap.add_argument("--no-contacts", action="store_true", help="do not return contacts")
    ap.add_argument("--waves", type=int, default=0, choices=(0, 3, 4),
                    help="resident waves per SIMD of the plain launch (0: automatic)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-mix", action="store_true",
                    help="humanoid: skip the mixed-batch batching figures reported beside the headline")
    ap.add_argument("--stats-worlds", type=int, default=512)
    ap.add_argument("--flop-worlds", type=int, default=64,
                    help="worlds of the oracle run whose operation counts give the roofline numerator")
    ap.add_argument("--flop-steps", type=int, default=1000, help="at most this many env steps of that run")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="also run a plain device copy of this size (for counter calibration)")
    ap.add_argument("--resident", type=int, default=2048,
                    help="mix: resident-grid size the autotuner tries (persistent launch)")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: request arrival rate (1/s)")
    ap.add_argument("--seconds", type=float, default=60.0, help="serve: arrival window of the offered-load run")
    ap.add_argument("--sustain-seconds", type=float, default=20.0, help="serve: arrival window at the sustained rate")
    ap.add_argument("--budget-mb", type=int, default=0,
                    help="serve: HBM budget for admitted requests (MiB); 0: the device's free memory")
    ap.add_argument("--summarize-trace", nargs=4, metavar=("DB", "TITLE", "OUT", "COMMAND"),
                    help="write a profiles/ table of the top kernels of a trace database and exit")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("DB", "TITLE", "OUT", "COMMAND"),
                    help="write a profiles/ table of step-kernel counters from a --pmc database and exit")
    ap.add_argument("--summarize", nargs=3, metavar=("TRACE_DB", "FETCH_DB", "WRITE_DB"),
                    help="write profiles/ summaries from rocprofv3 databases and exit")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(*args.summarize_pmc)))
        return
    if args.summarize:
        wl = args.workload
        nwd = args.worlds or DEFAULT_WORLDS[wl]
        # the commands that wrote the three databases, each into the directory it was read from
        def out_dir(db):
            d = os.path.dirname(os.path.abspath(db))
            return os.path.relpath(d, os.getcwd()) if d.startswith(os.getcwd()) else d
        tdb, fdb, wdb = args.summarize
        cmds = {"trace": f"rocprofv3 --kernel-trace --stats -d {out_dir(tdb)} -o trace -- "
                         "python bench.py --steps 50 --warmup 5 --no-cpu --no-mix --stats-worlds 64",
                "fetch": f"rocprofv3 --pmc FETCH_SIZE -d {out_dir(fdb)} -o fetch -- "
                         "python bench.py --steps 10 --warmup 2 --no-cpu --no-mix --stats-worlds 16 --copy-calib-mb 256",
                "write": f"rocprofv3 --pmc WRITE_SIZE -d {out_dir(wdb)} -o write -- "
                         "python bench.py --steps 10 --warmup 2 --no-cpu --no-mix --stats-worlds 16 --copy-calib-mb 256"}
        summarize_profiles(*args.summarize, wl, nwd, args.copy_calib_mb or 256, cmds)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: worlds are independent and the step runs on a single MI355X; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "mix":
        run_mix(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    import torch
    import paper_2601_22074_amd as rb
    from workloads import inputs

    nw = args.worlds or DEFAULT_WORLDS[args.workload]
    K, warm = args.steps, args.warmup
    W = inputs.workload(args.workload, nw, warm + K)
    m = W["model"]
    dev = torch.device("cuda:0")
    model = rb.Model(m)
    batch = rb.Batch(model, nw)
    batch.set_waves(args.waves)
    q = torch.tensor(W["qpos"], device=dev)
    v = torch.tensor(W["qvel"], device=dev)
    ctab = torch.tensor(W["ctrl"], device=dev).contiguous()
    if W["friction"] is not None:
        batch.set_params(rb.PARAM_FRICTION, torch.tensor(W["friction"], device=dev))
    if W["mass_scale"] is not None:
        batch.set_params(rb.PARAM_MASS_SCALE, torch.tensor(W["mass_scale"], device=dev))
    status = torch.zeros(nw, dtype=torch.int32, device=dev)
    con = None if args.no_contacts else batch.contacts(nw)
    stream = torch.cuda.current_stream()

    if args.copy_calib_mb:
        # a plain elementwise kernel of known traffic (reads and writes calib_mb MiB each) whose
        # counter readings calibrate FETCH_SIZE / WRITE_SIZE
        a = torch.ones(args.copy_calib_mb * 2 ** 20 // 4, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()

    def ctrl_at(s):
        return ctab[min(s // inputs.CTRL_PERIOD, ctab.shape[0] - 1)]

    for s in range(warm):
        batch.step(ctrl_at(s), q, v, con, status)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for s in range(K):
        batch.step(ctrl_at(warm + s), q, v, con, status)
        ev[s + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(K)])  # ms, on the kernel's stream
    total_ms = ev[0].elapsed_time(ev[K])
    value = nw * K / (total_ms / 1e3)
    st = status.cpu().numpy()
    ncon_last = float(con.ncon.float().mean().item()) if con is not None else float("nan")

    # work statistics on a subset of the same worlds, replayed untimed from the same inputs
    ns = min(args.stats_worlds, nw)
    sub = rb.Batch(model, ns)
    qs = torch.tensor(W["qpos"][:ns], device=dev)
    vs = torch.tensor(W["qvel"][:ns], device=dev)
    if W["friction"] is not None:
        sub.set_params(rb.PARAM_FRICTION, torch.tensor(W["friction"][:ns], device=dev))
    if W["mass_scale"] is not None:
        sub.set_params(rb.PARAM_MASS_SCALE, torch.tensor(W["mass_scale"][:ns], device=dev))
    stats = torch.zeros(ns, rb.rbstep.NSTATS, dtype=torch.int32, device=dev)
    acc = np.zeros(rb.rbstep.NSTATS)
    for s in range(warm + K):
        sub.step_taps(ctab[min(s // inputs.CTRL_PERIOD, ctab.shape[0] - 1)][:ns].contiguous(), qs, vs, stats=stats)
        if s >= warm:
            acc += stats.double().sum(0).cpu().numpy()
    Ksub = m["opt"]["nsubsteps"]
    stats_mean = acc[:4] / (ns * K * Ksub)      # per substep per world
    cyc = acc[4:4 + rb.rbstep.NSTAGE]
    stage_share = {n: float(c / cyc.sum()) for n, c in zip(rb.rbstep.STAGES, cyc)} if cyc.sum() > 0 else {}
    fl_kernel = flops_per_env_step(m, stats_mean)
    # the numerator: the oracle's operation counts on its own trajectory of the same workload
    ow = oracle_work(W, args.flop_worlds, warm, min(K, args.flop_steps))
    fl = ow["flops_per_env_step"]
    hb = hbm_bytes_per_env_step(m, ncon_last if con is not None else 0, con is not None)
    launch_s = float(np.mean(per)) / 1e3
    achieved_tf = fl * nw / launch_s / 1e12
    traffic = load_traffic(args.workload, nw)

    out = {
        "metric": "env-steps/sec, 29-DoF humanoid x8192 worlds; p50/p99 rollout latency"
        if args.workload == "humanoid" else f"env-steps/sec, {args.workload} x{nw} worlds",
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": warm,
        "ms_per_step": total_ms / K,
        "p50_ms": float(np.percentile(per, 50)),
        "p99_ms": float(np.percentile(per, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "worlds": nw, "env_steps": K,
                   "substeps": Ksub, "contacts_returned": con is not None, "waves_per_simd": args.waves or "auto"},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / PEAK_FP32_TFLOPS,
                     "traffic": None if traffic is None else traffic,
                     "flops_per_env_step": fl, "flops_source": "oracle operation counts (tree-sparse formulation)",
                     "oracle_work": ow, "flops_per_env_step_kernel_stats_estimate": fl_kernel,
                     "launch_ms": launch_s * 1e3},
        "hbm": {"algorithmic_bytes_per_env_step": hb, "achieved_GBs": hb * nw / launch_s / 1e9,
                "peak_GBs": PEAK_HBM_GBS, "frac": hb * nw / launch_s / 1e9 / PEAK_HBM_GBS},
        "work_per_substep": {"contacts": stats_mean[0], "active_rows": stats_mean[1],
                             "newton_iters": stats_mean[2], "line_search_segments": stats_mean[3]},
        "stage_cycle_share": stage_share,
        "stage_cycle_share_source": "the diagnostic instantiation's shader-clock taps (compiled for 3 resident "
                                    "waves per SIMD, not the timed kernel) on the stats sample of worlds",
        "nonfinite_worlds": int(np.sum(st & 1)),
        "wall_s": wall,
        "kernel_source_hash": kernel_source_hash(),
    }
    if nw < 4 * 256:
        out["roofline"]["note"] = (f"{nw} worlds occupy {nw} of the chip's 256 compute units' wave slots once: "
                                   "the launch is latency-bound and its roofline fraction is not meaningful")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W)
    if args.workload == "humanoid" and not args.no_mix:
        # the batching form beside the headline figure, after its timed region: the mixed batch
        # at its counts, fused launch against the separate plain launches (200 env steps)
        margs = argparse.Namespace(**vars(args))
        margs.steps, margs.warmup = 200, 20
        mx = run_mix(margs, emit=False)
        out["batching"] = {"workload": mx["config"]["workload"], "worlds": mx["config"]["worlds"],
                           "env_steps": mx["steps"], "form": mx["config"]["form"],
                           "schedule": mx["config"]["schedule"],
                           "env_steps_per_s": mx["forms_env_steps_per_s"],
                           "speedup_vs_separate": mx["speedup_vs_separate"],
                           "bitwise_equal_to_separate": mx["bitwise_equal_to_separate"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
