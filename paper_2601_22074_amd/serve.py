"""Serving form: continuous batching of rollout requests on one GPU.

A request asks for ``horizon`` env steps of ``n`` fresh worlds of one model and gets back
their final qpos/qvel.  The server keeps one slot pool per model (a Batch whose capacity is
fixed at start, with qpos/qvel/ctrl arrays of the same capacity) and one fused launch plan
over all pools.  Every tick is one fused launch that advances each live request by one env
step; requests that arrive are admitted between ticks as soon as the HBM budget and a
contiguous slot range allow (first come, first served), and leave as soon as their horizon
is reached, so requests of all models and sizes share each launch.  Each world runs the same
code in every launch, so a request's result does not depend on what it was served beside.

``Scheduler`` is the admission core (queue, budget, slot ranges) and has no device code;
``Server`` drives the device through the C ABI.
"""
from __future__ import annotations

import bisect
import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import rbstep


# ------------------------------------------------------------------ admission core
class SlotPool:
    """First-fit allocator of contiguous slot ranges in [0, capacity), coalescing on free."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.free = [(0, self.capacity)] if capacity > 0 else []   # sorted (start, length)

    def alloc(self, n: int):
        for i, (s, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (s + n, ln - n)
                return s
        return None

    def release(self, start: int, n: int) -> None:
        i = bisect.bisect_left(self.free, (start, 0))
        if i > 0:
            ps, pl = self.free[i - 1]
            assert ps + pl <= start, "double free"
        if i < len(self.free):
            assert start + n <= self.free[i][0], "double free"
        self.free.insert(i, (start, n))
        # merge with the right, then the left neighbour
        if i + 1 < len(self.free) and start + n == self.free[i + 1][0]:
            self.free[i] = (start, n + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == start:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)

    def free_slots(self) -> int:
        return sum(ln for _, ln in self.free)


class Scheduler:
    """FIFO admission against HBM: a request is admitted when the bytes its worlds occupy
    (``bytes_per_world[name] * n``) fit in what the budget has left, in what the device reports
    free (``free_probe()``, bytes, less ``reserve``) when a probe is given, and its model's pool
    has a contiguous range of n slots.  The head of the queue blocks later requests, so large
    requests are not starved."""

    def __init__(self, capacity: dict, bytes_per_world: dict, budget: int, free_probe=None, reserve: int = 0):
        self.pools = {k: SlotPool(c) for k, c in capacity.items()}
        self.bpw = dict(bytes_per_world)
        self.budget = int(budget)
        self.free_probe = free_probe
        self.reserve = int(reserve)
        self.used = 0
        self.queue = collections.deque()
        self.peak = 0
        self.blocked_by_device = 0   # admissions deferred because the device had too little free

    def need(self, req) -> int:
        return self.bpw[req.name] * req.n

    def fits_ever(self, req) -> bool:
        return self.need(req) <= self.budget and req.n <= self.pools[req.name].capacity

    def submit(self, req) -> None:
        if not self.fits_ever(req):
            raise ValueError(f"request {req.rid} ({req.name} x{req.n}) can never fit the budget or its pool")
        self.queue.append(req)

    def admit(self):
        """Admit from the head of the queue while possible; returns [(req, start)]."""
        out = []
        while self.queue:
            r = self.queue[0]
            need = self.need(r)
            if self.used + need > self.budget:
                break
            if self.free_probe is not None and need > self.free_probe() - self.reserve:
                self.blocked_by_device += 1
                break
            s = self.pools[r.name].alloc(r.n)
            if s is None:
                break
            self.queue.popleft()
            self.used += need
            self.peak = max(self.peak, self.used)
            out.append((r, s))
        return out

    def release(self, req, start: int) -> None:
        self.pools[req.name].release(start, req.n)
        self.used -= self.need(req)


# ------------------------------------------------------------------ device side
@dataclass
class _Live:
    req: object
    pool: int
    start: int
    gen: object
    done: int = 0


@dataclass
class Result:
    rid: int
    qpos: object                  # device tensor [n, nq]
    qvel: object                  # device tensor [n, nv]
    status: object                # device tensor [n] int32
    arrival: float                # seconds after the start of the run
    event: object = None
    finish: float | None = None   # seconds after the start of the run
    extra: dict = field(default_factory=dict)


def bytes_per_world(model: "rbstep.Model", ncap: int) -> int:
    """Device bytes one world holds while served: pool state (qpos, qvel, ctrl, status out),
    the batch's per-world data (warm start, status, friction, mass scales), the result copy,
    and its share of the work list."""
    return model.bytes_per_world + 4 * (2 * model.nq + 2 * model.nv + max(model.nu, 1) + 2)


DEVICE_RESERVE = 512 << 20   # device bytes admission leaves free for everything else


def device_free_bytes() -> int:
    """Free device memory as the runtime reports it (hipMemGetInfo through torch)."""
    import torch
    return int(torch.cuda.mem_get_info()[0])


class Server:
    """Continuous-batching server over the models in ``source.models`` (name -> model dict).

    budget: HBM bytes that admitted requests may hold (default: the device's free memory at
    start, less DEVICE_RESERVE); admission also re-reads the device's free memory before each
    request (``free_probe``, default ``device_free_bytes``).  capacity: slots per model pool
    (default: what the budget could hold of that model alone, at most ``max_pool``).
    inflight: ticks the host may run ahead of the device."""

    def __init__(self, source, budget: int | None = None, capacity: dict | None = None, max_pool: int = 1 << 17,
                 inflight: int = 3, grid: int = 0, free_probe=device_free_bytes, reserve: int = DEVICE_RESERVE):
        import torch
        self.torch = torch
        self.src = source
        self.dev = source.device
        self.names = list(source.models)
        self.models = {k: rbstep.Model(m) for k, m in source.models.items()}
        bpw = {k: bytes_per_world(self.models[k], 0) for k in self.names}
        if budget is None:
            budget = max(0, (free_probe() if free_probe is not None else 1 << 30) - reserve)
        cap = capacity or {k: max(1, min(max_pool, budget // bpw[k])) for k in self.names}
        self.sched = Scheduler(cap, bpw, budget, free_probe, reserve)
        self.live: list[_Live] = []
        self.dirty = True
        self.inflight = inflight
        self.grid = grid
        self.ticks = collections.deque()
        self.pending: list[Result] = []
        self.results: dict[int, Result] = {}
        self.env_steps = 0
        self.nticks = 0
        self.launches = 0
        self.stream = torch.cuda.current_stream()
        self.t0 = None
        self.ev0 = None
        self._init_device(cap)

    def _init_device(self, cap):
        """One slot pool per model and one fused launch plan over the pools."""
        torch = self.torch
        self.pools = []
        for k in self.names:
            M, c = self.models[k], cap[k]
            b = rbstep.Batch(M, c)
            d = dict(name=k, batch=b, cap=c, q=torch.zeros(c, M.nq, device=self.dev),
                     v=torch.zeros(c, M.nv, device=self.dev), u=torch.zeros(c, max(M.nu, 1), device=self.dev),
                     st=torch.zeros(c, dtype=torch.int32, device=self.dev))
            self.pools.append(d)
        self.pool_of = {k: i for i, k in enumerate(self.names)}
        self.plan = rbstep.Multi([p["batch"] for p in self.pools])
        for i, p in enumerate(self.pools):
            M = self.models[p["name"]]
            self.plan.bind(i, p["u"] if M.nu else None, p["q"], p["v"], None, p["st"])
        # heaviest models first in the work list (rough per-world cost of one env step)
        self.cost = {k: self.models[k].nv ** 2 + 8 * self.pools[i]["batch"].ncap + 4 * self.models[k].nbody
                     for i, k in enumerate(self.names)}

    def close(self):
        self.torch.cuda.synchronize()
        self.plan.close()
        for p in self.pools:
            p["batch"].close()
        for M in self.models.values():
            M.close()

    # ---- request lifecycle
    def _admit(self, req, start: int) -> None:
        t = self.torch
        i = self.pool_of[req.name]
        p = self.pools[i]
        n = req.n
        M = self.models[req.name]
        gen = self.src.generator(req.seed)
        sl = slice(start, start + n)
        self.src.initial(req.name, n, gen, p["q"][sl], p["v"][sl])
        fr, ms = self.src.params(req.name, n, gen)
        if fr is not None:
            p["batch"].set_params_at(rbstep.PARAM_FRICTION, start, fr.contiguous())
        if ms is not None:
            p["batch"].set_params_at(rbstep.PARAM_MASS_SCALE, start, ms.contiguous())
        p["batch"].reset(t.arange(start, start + n, dtype=t.int32, device=self.dev))
        if M.nu:
            self.src.ctrl(req.name, gen, p["u"][sl])
        self.live.append(_Live(req, i, start, gen))
        self.dirty = True

    def _complete(self, L: _Live) -> None:
        p = self.pools[L.pool]
        sl = slice(L.start, L.start + L.req.n)
        r = Result(L.req.rid, p["q"][sl].clone(), p["v"][sl].clone(), p["st"][sl].clone(), L.req.arrival)
        r.event = self.torch.cuda.Event(enable_timing=True)
        r.event.record(self.stream)
        self.pending.append(r)
        self.sched.release(L.req, L.start)
        self.dirty = True

    def _items(self):
        parts = []
        for L in sorted(self.live, key=lambda L: -self.cost[L.req.name]):
            parts.append((L.pool << 24) | np.arange(L.start, L.start + L.req.n, dtype=np.int64))
        return np.concatenate(parts).astype(np.int32) if parts else np.zeros(0, np.int32)

    def _tick(self) -> None:
        if self.dirty:
            self.plan.set_items(self._items(), self.grid)
            self.dirty = False
        if len(self.ticks) >= self.inflight:
            self.ticks.popleft().synchronize()
        self.plan.step()
        self.launches += 1
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        self.ticks.append(ev)
        self.nticks += 1
        still = []
        for L in self.live:
            self.env_steps += L.req.n
            L.done += 1
            if L.done >= L.req.horizon:
                self._complete(L)
            else:
                if L.done % 20 == 0 and self.models[L.req.name].nu:
                    p = self.pools[L.pool]
                    self.src.ctrl(L.req.name, L.gen, p["u"][L.start:L.start + L.req.n])
                still.append(L)
        self.live = still

    def _poll(self, block: bool = False) -> None:
        keep = []
        for r in self.pending:
            if block:
                r.event.synchronize()
            if block or r.event.query():
                # seconds after the start of the run, on the device clock (ev0 marks the start)
                r.finish = self.ev0.elapsed_time(r.event) / 1e3
                self.results[r.rid] = r
            else:
                keep.append(r)
        self.pending = keep

    def _start(self):
        self.torch.cuda.synchronize()
        self.ev0 = self.torch.cuda.Event(enable_timing=True)
        self.ev0.record(self.stream)
        self.t0 = time.perf_counter()

    # ---- drivers
    def run_script(self, reqs) -> dict:
        """Deterministic run: request.arrival is the tick before which it is submitted.
        Returns {rid: Result} once every request has finished."""
        self._start()
        order = sorted(reqs, key=lambda r: (r.arrival, r.rid))
        k, tick = 0, 0
        while k < len(order) or self.live or self.sched.queue:
            while k < len(order) and order[k].arrival <= tick:
                self.sched.submit(order[k])
                k += 1
            for r, s in self.sched.admit():
                self._admit(r, s)
            if self.live:
                self._tick()
            tick += 1
        self._poll(block=True)
        return self.results

    def run_timed(self, reqs, stop_after: float | None = None, progress=None) -> dict:
        """Real-time run: requests are submitted when the wall clock passes their arrival
        time.  With stop_after, the run ends at that time (requests not finished by then are
        counted as backlog); otherwise it ends when every request has finished.  Returns a
        summary with latencies (finish - arrival) of the finished requests."""
        self._start()
        order = sorted(reqs, key=lambda r: r.arrival)
        k = 0
        last_report = 0.0
        while True:
            now = time.perf_counter() - self.t0
            if stop_after is not None and now >= stop_after:
                break
            while k < len(order) and order[k].arrival <= now:
                self.sched.submit(order[k])
                k += 1
            for r, s in self.sched.admit():
                self._admit(r, s)
            if self.live:
                self._tick()
            elif k < len(order):
                time.sleep(max(0.0, min(order[k].arrival - now, 1e-3)))
            elif not self.sched.queue:
                break
            self._poll()
            if progress and now - last_report >= 10.0:
                last_report = now
                progress(f"t={now:6.1f}s submitted={k} queued={len(self.sched.queue)} live={len(self.live)} "
                         f"done={len(self.results)} env_steps={self.env_steps}")
        self.torch.cuda.synchronize()
        wall = time.perf_counter() - self.t0
        self._poll(block=True)
        done = [r for r in self.results.values()]
        lat = np.array([r.finish - r.arrival for r in done]) if done else np.zeros(0)
        return {
            "submitted": k, "finished": len(done), "queued_at_end": len(self.sched.queue),
            "live_at_end": len(self.live), "wall_s": wall, "env_steps": self.env_steps,
            "env_steps_per_s": self.env_steps / wall if wall > 0 else 0.0, "ticks": self.nticks,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_latency_s": float(lat.mean()) if lat.size else None,
            "peak_budget_bytes": self.sched.peak, "budget_bytes": self.sched.budget,
            "launches": self.launches, "admissions_blocked_by_device_memory": self.sched.blocked_by_device,
        }


class PlainServer(Server):
    """The same request loop served by plain launches, the baseline of the fused server: each
    live request owns a batch of its model (batches are reused across requests of the model:
    the smallest idle one that holds the request, else a new one of the next power-of-two
    capacity) and every tick makes one plain ``rb_step`` launch per live request."""

    def _init_device(self, cap):
        self.idle = {k: [] for k in self.names}   # name -> [(capacity, state dict)]
        self.all_batches = []

    def close(self):
        self.torch.cuda.synchronize()
        for d in self.all_batches:
            d["batch"].close()
        for M in self.models.values():
            M.close()

    def _take(self, name, n):
        t = self.torch
        free = self.idle[name]
        fit = [i for i, (c, _) in enumerate(free) if c >= n]
        if fit:
            i = min(fit, key=lambda i: free[i][0])
            return free.pop(i)[1]
        M = self.models[name]
        c = 1 << max(0, (n - 1).bit_length())
        d = dict(name=name, cap=c, batch=rbstep.Batch(M, c), q=t.zeros(c, M.nq, device=self.dev),
                 v=t.zeros(c, M.nv, device=self.dev), u=t.zeros(c, max(M.nu, 1), device=self.dev),
                 st=t.zeros(c, dtype=t.int32, device=self.dev))
        self.all_batches.append(d)
        return d

    def _admit(self, req, start: int) -> None:
        t = self.torch
        n = req.n
        d = self._take(req.name, n)
        M = self.models[req.name]
        gen = self.src.generator(req.seed)
        self.src.initial(req.name, n, gen, d["q"][:n], d["v"][:n])
        fr, ms = self.src.params(req.name, n, gen)
        if fr is not None:
            d["batch"].set_params_at(rbstep.PARAM_FRICTION, 0, fr.contiguous())
        if ms is not None:
            d["batch"].set_params_at(rbstep.PARAM_MASS_SCALE, 0, ms.contiguous())
        d["batch"].reset(t.arange(n, dtype=t.int32, device=self.dev))
        if M.nu:
            self.src.ctrl(req.name, gen, d["u"][:n])
        L = _Live(req, -1, start, gen)
        L.state = d
        self.live.append(L)

    def _complete(self, L: _Live) -> None:
        d, n = L.state, L.req.n
        r = Result(L.req.rid, d["q"][:n].clone(), d["v"][:n].clone(), d["st"][:n].clone(), L.req.arrival)
        r.event = self.torch.cuda.Event(enable_timing=True)
        r.event.record(self.stream)
        self.pending.append(r)
        self.sched.release(L.req, L.start)
        # stream order keeps the batch's next user behind the copies above
        self.idle[L.req.name].append((d["cap"], d))

    def _tick(self) -> None:
        if len(self.ticks) >= self.inflight:
            self.ticks.popleft().synchronize()
        for L in self.live:
            d, n = L.state, L.req.n
            M = self.models[L.req.name]
            d["batch"].step(d["u"][:n] if M.nu else None, d["q"][:n], d["v"][:n], None, d["st"][:n])
            self.launches += 1
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        self.ticks.append(ev)
        self.nticks += 1
        still = []
        for L in self.live:
            self.env_steps += L.req.n
            L.done += 1
            if L.done >= L.req.horizon:
                self._complete(L)
            else:
                if L.done % 20 == 0 and self.models[L.req.name].nu:
                    self.src.ctrl(L.req.name, L.gen, L.state["u"][:L.req.n])
                still.append(L)
        self.live = still
