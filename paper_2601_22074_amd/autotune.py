"""Schedule autotuner for mixed-model batching.

Given batches with bound step inputs, time each candidate schedule of one env step --
separate plain launches, or the fused launch under every dispatch order, a few grid sizes
(one workgroup per world, or a persistent grid of 1x / 2x the resident capacity) and the
resident waves per SIMD (automatic, 3, or capped at 2) -- on cloned state, and keep the fastest.
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
    """(kind, order, grid, waves per SIMD cap) tuples."""
    out = [("separate", None, None, None)]
    for occ in (0, 3, 2):
        for order in (rbstep.ORDER_HEAVY_FIRST, rbstep.ORDER_INTERLEAVE, rbstep.ORDER_BATCH):
            out.append(("fused", order, 0, occ))
            for mult in (1, 2):
                g = resident * mult
                if g < nitems:
                    out.append(("fused", order, g, occ))
    return out


def _time(fn, stream, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(multi: "rbstep.Multi", inputs, reps: int = 3, resident: int = 2048, use_cache: bool = True):
    """inputs: per batch (ctrl, qpos, qvel).  Returns the chosen (kind, order, grid) and the
    timings; leaves the plan scheduled (or marked 'separate') and bound to `inputs`."""
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
    timings = {}
    if use_cache and sig in cache and len(cache[sig].get("choice", ())) == 4:
        choice = tuple(cache[sig]["choice"])
    else:
        for kind, order, grid, occ in candidates(sum(ns), resident):
            if kind == "separate":
                def fn():
                    for b, (u, q, v) in zip(batches, clones):
                        b.step(u, q, v)
            else:
                multi.set_schedule(order, grid)
                multi.set_occupancy(occ)

                def fn():
                    multi.step()
            timings[f"{kind}/{order}/{grid}/{occ}"] = _time(fn, stream, reps)
        best = min(timings, key=timings.get)
        choice = tuple(None if x == "None" else (x if i == 0 else int(x)) for i, x in enumerate(best.split("/")))
        cache[sig] = {"choice": list(choice), "timings_ms": timings}
        if use_cache:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            with open(CACHE, "w") as f:
                json.dump(cache, f, indent=1)
    # restore the warm starts and bind the real inputs
    for b, n, ws in zip(batches, ns, saved_ws):
        b.reset(torch.arange(n, dtype=torch.int32, device="cuda"), ws)
    for i, (u, q, v) in enumerate(inputs):
        multi.bind(i, u, q, v)
    if choice[0] == "fused":
        multi.set_schedule(choice[1], choice[2])
        multi.set_occupancy(choice[3])
    torch.cuda.synchronize()
    return choice, timings
