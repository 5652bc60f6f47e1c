"""Autocorrelation of the order parameter (Sec. III.A) and the cost of an
independent configuration (Sec. III.C), from series the library records on
the device.

M(t) = max_q' N_q'(t) / n, n the number of bond indices (4N in 2-D);
C_M(dt) = (<M(t0 + dt) M(t0)> - <M>^2) / (<M^2> - <M>^2), the first mean
over the t0 with t0 + dt in the series, the others over the whole series;
tau = the lag at which C_M falls to 1/e (linear interpolation between the
two integer lags around the crossing); configurations tau steps apart count
as independent, so one costs tau times the wall time of a step.

The counts come from cvf_state_counts, one row per step, accumulated on the
device and read once; the statistics are host arithmetic on that series.
"""
import math

import numpy as np


def order_parameter(counts, n_bond: int) -> np.ndarray:
    """M(t) from a [T, 6] array of state counts."""
    c = np.asarray(counts, dtype=np.int64)
    return c.max(axis=1).astype(np.float64) / float(n_bond)


def c_m(M, max_lag: int) -> np.ndarray:
    """C_M(dt) for dt = 0..max_lag (C_M(0) = 1)."""
    x = np.asarray(M, dtype=np.float64)
    T = x.size
    if max_lag >= T:
        raise ValueError("max_lag must be below the series length")
    mean = x.mean()
    var = (x * x).mean() - mean * mean
    if not var > 0.0:
        raise ValueError("constant series: C_M is undefined")
    out = np.empty(max_lag + 1)
    for dt in range(max_lag + 1):
        out[dt] = ((x[dt:] * x[:T - dt]).mean() - mean * mean) / var
    return out


def tau_1e(C) -> float:
    """First lag at which C falls to 1/e, interpolated linearly between the
    bracketing integer lags; nan if C never gets there."""
    C = np.asarray(C, dtype=np.float64)
    target = math.exp(-1.0)
    for k in range(1, C.size):
        if C[k] <= target:
            c0, c1 = C[k - 1], C[k]
            return (k - 1) + (c0 - target) / (c0 - c1)
    return float("nan")


def record_counts(cvf, chain, step, nsteps: int):
    """Run nsteps steps of chain with step(n) (e.g. chain.metropolis) and
    return the [nsteps, 6] state counts after each step (one device read)."""
    import torch
    out = torch.zeros((nsteps, 6), dtype=torch.int64, device=chain.sigma.device)
    base = out.data_ptr()
    for i in range(nsteps):
        step(1)
        cvf.cvf_state_counts(chain.h, base + 48 * i, chain.stream)
    return out.cpu().numpy()
