"""Seeded synthetic inputs and workload descriptions.

This module only draws parameters and starting configurations with numpy's
own generator; it holds none of the sweep's arithmetic and none of its random
stream (initial spins drawn by the method come from its Philox stream on each
side).  Both the GPU tests and the oracle tests take their inputs from here.

Workloads (the paper runs 2D Ising SW at T_c up to L = 7920, Sec. II.C, and
PCC with the extension rule, Sec. III; it names no dataset):

* parity       2D L=64 periodic at T_c, seed 1, 1000 sweeps, series recorded
* plain        2D L=8192 at T_c and 3D L=256 at T=4.5115, 200 sweeps each
* batched      512 replicas, L uniform in {64..2048}, T uniform in [2.0, 2.6]
* pcc          64 replicas of 2D L=2048, p0=0.5, dp=0.01 halved every 1000
* serving      Poisson arrivals of 2D/3D jobs admitted by memory footprint
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

TC_2D = 2.0 / math.log(1.0 + math.sqrt(2.0))   # Onsager's critical temperature, J = 1
TC_3D = 4.5115                                 # simple-cubic critical temperature used by the plain 3D case


@dataclass
class Replica:
    dim: int
    L: int
    T: float
    seed: int
    J: float = 1.0
    p_bond: float = -1.0          # < 0: P = 1 - exp(-2J/T); else explicit p (PCC start value)
    pcc: bool = False
    dp0: float = 0.01
    halve_every: int = 1000

    @property
    def nsites(self) -> int:
        return self.L ** self.dim


@dataclass
class Job:
    index: int
    arrival: float                # seconds after the start of the stream
    replica: Replica
    sweeps: int


@dataclass
class Workload:
    name: str
    replicas: List[Replica]
    sweeps: int
    extra: dict = field(default_factory=dict)

    @property
    def site_updates(self) -> int:
        return sum(r.nsites for r in self.replicas) * self.sweeps


def random_spins(dim: int, L: int, seed: int) -> np.ndarray:
    """Uniform random +-1 int8 spins (numpy generator; an explicit input)."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random(L ** dim) < 0.5, 1, -1).astype(np.int8)


def parity() -> Workload:
    return Workload("parity_2d_L64_Tc", [Replica(2, 64, TC_2D, 1)], 1000)


def plain() -> Workload:
    return Workload("plain_2d_L8192_Tc+3d_L256_T4.5115",
                    [Replica(2, 8192, TC_2D, 1), Replica(3, 256, TC_3D, 1)], 200)


def batched(n: int = 512, seed: int = 2026) -> Workload:
    rng = np.random.default_rng(seed)
    sizes = (64, 128, 256, 512, 1024, 2048)
    reps = []
    for r in range(n):
        L = int(sizes[rng.integers(0, len(sizes))])
        T = float(2.0 + 0.6 * rng.random())
        reps.append(Replica(2, L, T, 1000 + r))
    return Workload("batched_512x2d_L64-2048_T2.0-2.6", reps, 500)


def pcc(n: int = 64, L: int = 2048, sweeps: int = 10000) -> Workload:
    reps = [Replica(2, L, TC_2D, s, p_bond=0.5, pcc=True) for s in range(1, n + 1)]
    return Workload(f"pcc_{n}x2d_L{L}", reps, sweeps)


def serving(n_jobs: int = 2000, rate: float = 50.0, seed: int = 5,
            l2d=(128, 16384), l3d=(32, 512), sweeps=(100, 5000)) -> List[Job]:
    """Poisson job stream: exponential inter-arrivals of mean 1/rate seconds.

    dim is 2 or 3 with probability 1/2; L is log-uniform in the given integer
    range; T = T_c(dim) * U[0.8, 1.2]; sweeps uniform in the given range; the
    job's seed is its index + 1.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for k in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        dim = 2 if rng.random() < 0.5 else 3
        lo, hi = l2d if dim == 2 else l3d
        L = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        L = min(max(L, lo), hi)
        tc = TC_2D if dim == 2 else TC_3D
        T = float(tc * rng.uniform(0.8, 1.2))
        nsw = int(rng.integers(sweeps[0], sweeps[1] + 1))
        jobs.append(Job(k, t, Replica(dim, L, T, k + 1), nsw))
    return jobs
