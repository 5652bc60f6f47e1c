"""Seeded synthetic workloads (state points, lattice sizes, seeds, arrival
streams) shared by the benchmark and the tests.

This module holds no arithmetic of the Monte Carlo method itself: it only
draws job descriptions.  The randomness *inside* a job comes from the
job's Philox seed, drawn here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Job:
    L: int
    T: float          # K
    P: float          # MPa
    nsteps: int
    algo: str         # "met" | "sw"
    seed: int
    arrival: float = 0.0   # s, served stream only


def c1_job() -> Job:
    """Plain Metropolis, L = 64, one state point (300 K, 0.1 MPa), 1000 sweeps."""
    return Job(L=64, T=300.0, P=0.1, nsteps=1000, algo="met", seed=1)


def c2_jobs() -> list[Job]:
    """L = 1024 Metropolis 10^4 sweeps and L = 256 SW 10^3 steps, T over five
    points in 270-330 K at 0.1 MPa."""
    Ts = [270.0, 285.0, 300.0, 315.0, 330.0]
    return ([Job(1024, T, 0.1, 10_000, "met", 2 + i) for i, T in enumerate(Ts)]
            + [Job(256, T, 0.1, 1_000, "sw", 7 + i) for i, T in enumerate(Ts)])


def c3_jobs() -> list[Job]:
    """Paper-scale single jobs: Metropolis L = 4096 and SW L = 1414 at 300 K,
    P in {0.1, 25, 50} MPa, 10^3 steps each."""
    Ps = [0.1, 25.0, 50.0]
    return ([Job(4096, 300.0, P, 1000, "met", 12 + i) for i, P in enumerate(Ps)]
            + [Job(1414, 300.0, P, 1000, "sw", 15 + i) for i, P in enumerate(Ps)])


def even(x: float) -> int:
    return max(2, 2 * int(round(x / 2.0)))


def c4_jobs(nsteps: int = 1000) -> list[Job]:
    """256 replicas: L log-uniform in [64, 512] (rounded to even) from
    default_rng(4); replica k = 16 i + j at T_i = 270 + 4 i K and
    P_j = (50/15) j MPa; seed 1000 + k."""
    rng = np.random.default_rng(4)
    Ls = [even(math.exp(rng.uniform(math.log(64), math.log(512)))) for _ in range(256)]
    jobs = []
    for k in range(256):
        i, j = divmod(k, 16)
        jobs.append(Job(Ls[k], 270.0 + 4.0 * i, (50.0 / 15.0) * j, nsteps, "met", 1000 + k))
    return jobs


def c5_stream(n_jobs: int = 2000, rate: float = 200.0, seed: int = 5,
              nsteps_range=(100, 10_000), L_range=(32, 2048)) -> list[Job]:
    """Poisson arrivals (mean `rate` jobs/s): L log-uniform in L_range rounded
    to even, T ~ U(270, 330) K, P ~ U(0, 50) MPa, nsteps ~ U[nsteps_range],
    80 % Metropolis / 20 % SW, seed 5000 + job number."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for n in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        L = even(math.exp(rng.uniform(math.log(L_range[0]), math.log(L_range[1]))))
        T = float(rng.uniform(270.0, 330.0))
        P = float(rng.uniform(0.0, 50.0))
        ns = int(rng.integers(nsteps_range[0], nsteps_range[1] + 1))
        algo = "met" if rng.random() < 0.8 else "sw"
        jobs.append(Job(L, T, P, ns, algo, 5000 + n, t))
    return jobs


def c5_oracle_subset(jobs: list[Job], n_random: int = 16, seed: int = 5005) -> list[int]:
    """Indices of the served jobs whose results are checked against stored CPU
    reference runs: every job with L <= 256, plus n_random of the larger ones
    drawn uniformly (without replacement) by default_rng(seed)."""
    small = [n for n, j in enumerate(jobs) if j.L <= 256]
    rest = [n for n, j in enumerate(jobs) if j.L > 256]
    rng = np.random.default_rng(seed)
    extra = rng.choice(len(rest), size=min(n_random, len(rest)), replace=False)
    return sorted(small + [rest[int(i)] for i in extra])
