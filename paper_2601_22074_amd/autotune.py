"""Schedule autotuner for mixed-model batching.

Given batches with bound step inputs, time each candidate schedule of one env step --
separate plain launches, or the fused launch under every dispatch order, a few grid sizes
(every world launched at once, or a persistent grid of 1x / 2x the resident capacity), the
resident waves per SIMD (automatic, 3, or capped at 2) and the worlds per workgroup (1, 2 or
4, one wave each) -- on cloned state, and keep the fastest.  The lanes per world are not a
dimension: the step runs one world on a whole 64-lane wave (its reductions, broadcasts and
pivot ballots span the wave).
Decisions are cached in a JSON file keyed by the batch signature (model shapes and world
counts), so a configuration is tuned once.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import rbstep

CACHE = os.environ.get("RBSTEP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "rbstep_tune.json"))


def signature(batches, ns) -> str:
    """Key of a tuning decision: each batch's model description, contact capacity and world
    count (two models of equal sizes but different features must not share a decision)."""
    h = hashlib.sha256()
    for b, n in zip(batches, ns):
        m = b.model
        desc = json.dumps(m.desc, sort_keys=True, default=str)
        h.update(f"{hashlib.sha256(desc.encode()).hexdigest()},{m.lds_bytes},{b.ncap},{n};".encode())
    return h.hexdigest()[:20]


def candidates(nitems: int, resident: int):
    """(kind, order, grid, waves per SIMD cap, worlds per workgroup) tuples.  The dispatch orders
    and grids are tried at every occupancy with one world per workgroup; the groups of 2 and 4
    worlds with the default grid and occupancy under each order."""
    out = [("separate", None, None, None, None)]
    for occ in (0, 3, 2):
        for order in (rbstep.ORDER_HEAVY_FIRST, rbstep.ORDER_INTERLEAVE, rbstep.ORDER_BATCH):
            out.append(("fused", order, 0, occ, 1))
            for mult in (1, 2):
                g = resident * mult
                if g < nitems:
                    out.append(("fused", order, g, occ, 1))
    for wpg in (2, 4):
        for order in (rbstep.ORDER_HEAVY_FIRST, rbstep.ORDER_INTERLEAVE, rbstep.ORDER_BATCH):
            out.append(("fused", order, 0, 0, wpg))
    return out


def _time(fn, stream, reps):
    import torch
    fn()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(multi: "rbstep.Multi", inputs, reps: int = 3, resident: int = 2048, use_cache: bool = True,
         advance: int = 0):
    """inputs: per batch (ctrl, qpos, qvel).  Every candidate is timed from the same state: the
    inputs advanced by `advance` plain env steps (on copies).  Returns the chosen (kind, order,
    grid, waves per SIMD cap, worlds per workgroup) and the timings; leaves the plan scheduled
    (or marked 'separate') and bound to `inputs`, whose state and warm starts are untouched."""
    import torch
    batches = multi.batches
    ns = [q.shape[0] for _, q, _ in inputs]
    sig = signature(batches, ns)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            with open(CACHE) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    stream = torch.cuda.current_stream()
    # tune on copies: the candidates advance the state they step
    saved_ws = []
    for b, n in zip(batches, ns):
        ws = torch.zeros(n, b.model.nv, device="cuda")
        b.get_state(n, ws)
        saved_ws.append(ws)
    clones = [(u, q.clone(), v.clone()) for u, q, v in inputs]
    for i, (u, q, v) in enumerate(clones):
        multi.bind(i, u, q, v)
    for _ in range(advance):
        for b, (u, q, v) in zip(batches, clones):
            b.step(u, q, v)
    start = [(q.clone(), v.clone()) for _, q, v in clones]
    start_ws = []
    for b, n in zip(batches, ns):
        ws = torch.zeros(n, b.model.nv, device="cuda")
        b.get_state(n, ws)
        start_ws.append(ws)

    def restart():
        # every candidate starts from the same state: the step's cost depends on the contacts
        # and Newton updates of the states it meets, which drift as the clones advance
        for b, n, ws, (q0, v0), (_, q, v) in zip(batches, ns, start_ws, start, clones):
            q.copy_(q0)
            v.copy_(v0)
            b.reset(torch.arange(n, dtype=torch.int32, device="cuda"), ws)
    timings = {}
    if use_cache and sig in cache and len(cache[sig].get("choice", ())) == 5:
        choice = tuple(cache[sig]["choice"])
    else:
        for kind, order, grid, occ, wpg in candidates(sum(ns), resident):
            restart()
            if kind == "separate":
                def fn():
                    for b, (u, q, v) in zip(batches, clones):
                        b.step(u, q, v)
            else:
                multi.set_schedule(order, grid)
                multi.set_group(1)
                multi.set_occupancy(occ)
                try:
                    multi.set_group(wpg)
                except RuntimeError:
                    continue             # the group's worlds need more LDS than a workgroup has

                def fn():
                    multi.step()
            timings[f"{kind}/{order}/{grid}/{occ}/{wpg}"] = _time(fn, stream, reps)
        best = min(timings, key=timings.get)
        choice = tuple(None if x == "None" else (x if i == 0 else int(x)) for i, x in enumerate(best.split("/")))
        cache[sig] = {"choice": list(choice), "timings_ms": timings}
        if use_cache:
            try:
                os.makedirs(os.path.dirname(CACHE), exist_ok=True)
                with open(CACHE, "w") as f:
                    json.dump(cache, f, indent=1)
            except OSError:
                pass   # an unwritable cache only means the next run tunes again
    # restore the warm starts and bind the real inputs
    for b, n, ws in zip(batches, ns, saved_ws):
        b.reset(torch.arange(n, dtype=torch.int32, device="cuda"), ws)
    for i, (u, q, v) in enumerate(inputs):
        multi.bind(i, u, q, v)
    if choice[0] == "fused":
        multi.set_schedule(choice[1], choice[2])
        multi.set_group(1)
        multi.set_occupancy(choice[3])
        multi.set_group(choice[4])
    torch.cuda.synchronize()
    return choice, timings
