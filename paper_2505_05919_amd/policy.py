"""Choice of the MC algorithm for served jobs.

as_submitted  every job keeps the algorithm it came with.
threshold     Metropolis at T >= T_switch, Swendsen-Wang below: the paper's
              rule (Sec. II.B; 208 K for its 3-D model at its pressures).
cost          the algorithm whose independent configurations are cheaper,
              tau x time per step (Sec. III.C), from a calibration table
              measured with autocorr.measure ({T: {"met": cost, "sw": cost}},
              costs in any common unit, None for a tau beyond the measured
              window); a job takes the entry of the nearest calibrated
              temperature, and keeps its own algorithm if neither cost is
              known there.

A job's result stays a pure function of its parameters, seed and the
chosen algorithm.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

KINDS = ("as_submitted", "threshold", "cost")


@dataclass
class AlgoPolicy:
    kind: str = "as_submitted"
    T_switch: float = 208.0
    table: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.kind not in KINDS:
            raise ValueError(f"unknown policy {self.kind!r}; one of {KINDS}")
        if self.kind == "cost" and not self.table:
            raise ValueError("the cost policy needs a calibration table")

    def choose(self, job) -> str:
        if self.kind == "threshold":
            return "met" if job.T >= self.T_switch else "sw"
        if self.kind == "cost":
            T = min(self.table, key=lambda t: (abs(t - job.T), t))
            cm, cs = self.table[T].get("met"), self.table[T].get("sw")
            if cm is None and cs is None:
                return job.algo
            cm = math.inf if cm is None else cm
            cs = math.inf if cs is None else cs
            return "sw" if cs < cm else "met"
        return job.algo

    def apply(self, job):
        return dataclasses.replace(job, algo=self.choose(job))


def calibrate(cvf, torch, temperatures, L=256, P=0.1, seed=1, warm=None, n_rec=None) -> dict:
    """Cost table for the cost policy: autocorr.measure for both algorithms
    at every temperature (microseconds per independent configuration)."""
    from . import autocorr
    warm = warm or {"met": 20000, "sw": 2000}
    n_rec = n_rec or {"met": 50000, "sw": 5000}
    table = {}
    for T in temperatures:
        table[T] = {a: autocorr.measure(cvf, torch, L, T, P, seed, a, warm[a], n_rec[a])["cost_per_independent_us"]
                    for a in ("met", "sw")}
    return table
