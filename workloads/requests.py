"""Seeded synthetic rollout requests for the serving form.

Arrivals form a Poisson process of the given rate; each request draws its model uniformly
from the four benchmark models, its world count log-uniformly from [16, 4096] and its
horizon uniformly from {50, ..., 500} env steps, from ``numpy`` PCG64 seeded by the run seed.

A request's own inputs (initial states, per-world parameters, control targets) are drawn on
the device from a ``torch`` Philox generator seeded by the request's seed, with the same
distributions as ``workloads.inputs``: hinge angles uniform in +-0.1 rad (quadruped, arm),
+-0.05 rad (humanoid), all angles uniform in +-pi and speeds N(0, 0.5) for the chain;
friction U[0.3, 1.2] and body mass scales U[0.8, 1.2] where the model has them per world;
control targets N(0, std) resampled every 20 env steps.  Drawing on the device keeps the
serving loop from waiting on host-side generation; a request's inputs depend only on its
seed, never on what else is being served.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import inputs, robots

NAMES = ("chain3", "quadruped", "humanoid", "arm_box")
HINGE_RANGE = {"quadruped": 0.1, "humanoid": 0.05, "arm_box": 0.1}


@dataclass
class Request:
    rid: int
    name: str
    n: int
    horizon: int
    seed: int
    arrival: float = 0.0      # seconds after the start of the run (or a tick index in scripted runs)


def poisson_requests(rate: float, duration: float, seed: int = 0, names=NAMES, wmin: int = 16, wmax: int = 4096,
                     hmin: int = 50, hmax: int = 500) -> list[Request]:
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([5, int(seed)])))
    out, t, rid = [], 0.0, 0
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            return out
        name = names[int(g.integers(len(names)))]
        n = int(math.floor(math.exp(g.uniform(math.log(wmin), math.log(wmax + 1)))))
        n = min(max(n, wmin), wmax)
        h = int(g.integers(hmin, hmax + 1))
        out.append(Request(rid, name, n, h, int(g.integers(1 << 31)), t))
        rid += 1


def mean_request_work(wmin: int = 16, wmax: int = 4096, hmin: int = 50, hmax: int = 500) -> float:
    """Expected env steps per request (worlds x horizon) of the distribution above."""
    mean_n = (wmax + 1 - wmin) / (math.log(wmax + 1) - math.log(wmin))
    return mean_n * (hmin + hmax) / 2.0


class DeviceSource:
    """Per-request device-side input generation for a set of models (name -> model dict)."""

    def __init__(self, models: dict, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.models = models
        self.q0 = {k: torch.tensor(robots.qpos0(m), dtype=torch.float32, device=self.device) for k, m in models.items()}
        self.hinge = {k: torch.tensor(inputs._hinge_qadr(m), dtype=torch.long, device=self.device)
                      for k, m in models.items()}

    def generator(self, seed: int):
        g = self.torch.Generator(device=self.device)
        g.manual_seed(int(seed))
        return g

    def initial(self, name: str, n: int, gen, q_out, v_out) -> None:
        t = self.torch
        q_out.copy_(self.q0[name].expand(n, -1))
        v_out.zero_()
        if name == "chain3":
            q_out.copy_((t.rand(q_out.shape, generator=gen, device=self.device) * 2 - 1) * math.pi)
            v_out.copy_(t.randn(v_out.shape, generator=gen, device=self.device) * 0.5)
        else:
            h = self.hinge[name]
            a = HINGE_RANGE[name]
            q_out[:, h] = (t.rand((n, h.numel()), generator=gen, device=self.device) * 2 - 1) * a

    def params(self, name: str, n: int, gen):
        """(friction[n] or None, mass_scale[n, nbody] or None) as the model requires."""
        t = self.torch
        m = self.models[name]
        fr = ms = None
        if m["per_world"].get("friction"):
            fr = 0.3 + 0.9 * t.rand(n, generator=gen, device=self.device)
        if m["per_world"].get("mass_scale"):
            nb = len(m["bodies"])
            ms = t.ones(n, nb, device=self.device)
            ms[:, 1:] = 0.8 + 0.4 * t.rand((n, nb - 1), generator=gen, device=self.device)
        return fr, ms

    def ctrl(self, name: str, gen, u_out) -> None:
        std = inputs.CTRL_STD.get(name, 0.0)
        if u_out.numel() == 0 or std == 0.0:
            u_out.zero_()
            return
        u_out.copy_(self.torch.randn(u_out.shape, generator=gen, device=self.device) * std)
