"""Autocorrelation of the order parameter (Sec. III.A) and the cost of an
independent configuration (Sec. III.C), from series the library records on
the device.

M(t) = max_q' N_q'(t) / n, n the number of bond indices (4N in 2-D);
C_M(dt) = (<M(t0 + dt) M(t0)> - <M>^2) / (<M^2> - <M>^2) (Eq. (4)),
estimated from the mean-centred series d(t) = M(t) - <M> as
<d(t0 + dt) d(t0)> / <d^2>, the first mean over the t0 with t0 + dt in the
series.  For a stationary series this has the expectation of Eq. (4); the
uncentred form <M(t0 + dt) M(t0)> - <M>^2 mixes in the difference between
the means of the two lagged sub-series times <M>, which swamps the variance
when M barely moves about a large mean (an ordered lattice under cluster
shifts).  tau = the lag at which C_M falls to 1/e (linear interpolation
between the two integer lags around the crossing); configurations tau steps
apart count as independent, so one costs tau times the wall time of a step.

The counts come from cvf_state_counts, one row per step, accumulated on the
device and read once; the statistics are host arithmetic on that series.
"""
import math
import time

import numpy as np


def order_parameter(counts, n_bond: int) -> np.ndarray:
    """M(t) from a [T, 6] array of state counts."""
    c = np.asarray(counts, dtype=np.int64)
    return c.max(axis=1).astype(np.float64) / float(n_bond)


def c_m(M, max_lag: int) -> np.ndarray:
    """C_M(dt) for dt = 0..max_lag (C_M(0) = 1), from the mean-centred
    lagged products."""
    x = np.asarray(M, dtype=np.float64)
    T = x.size
    if max_lag >= T:
        raise ValueError("max_lag must be below the series length")
    d = x - x.mean()
    var = (d * d).mean()
    if not var > 0.0:
        raise ValueError("constant series: C_M is undefined")
    out = np.empty(max_lag + 1)
    for dt in range(max_lag + 1):
        out[dt] = (d[dt:] * d[:T - dt]).mean() / var
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


def measure(cvf, torch, L: int, T: float, P: float, seed: int, algo: str, warm: int, n_rec: int,
            n_time: int = 2000, max_lag: int = 2000) -> dict:
    """tau, time per step and cost of one independent configuration (Sec.
    III.C) of one algorithm ("met" or "sw") at one state point: a warm-up,
    n_rec recorded steps, C_M up to min(max_lag, n_rec / 2), then n_time
    steps timed without recording.  tau and the cost are None when C_M does
    not reach 1/e inside the window."""
    p = cvf.cvf_params_from_si(T, P, L=L, seed=seed)
    ch = cvf.Chain(p, cvf.CVF_ALGO_METROPOLIS | cvf.CVF_ALGO_SW)
    step = ch.metropolis if algo == "met" else ch.sw
    step(warm)
    counts = record_counts(cvf, ch, step, n_rec)
    C = c_m(order_parameter(counts, 4 * L * L), min(max_lag, n_rec // 2))
    tau = tau_1e(C)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step(n_time)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / n_time
    consistent = ch.obs()["consistent"] == 1
    ch.close()
    ok = not math.isnan(tau)
    return {"warmup_steps": warm, "steps_recorded": n_rec, "tau_steps": round(float(tau), 3) if ok else None,
            "C_M_1": round(float(C[1]), 4), "step_us": round(t_step * 1e6, 2),
            "cost_per_independent_us": round(float(tau) * t_step * 1e6, 2) if ok else None,
            "consistent": consistent}


def record_counts3(cvf3, chain, step, nsteps: int):
    """The cubic-lattice chain's [nsteps, 6] state counts after each of
    nsteps steps of step(n) (chain.steps or chain.sw), one device read."""
    import torch
    out = torch.zeros((nsteps, 6), dtype=torch.int64, device=chain.sigma.device)
    base = out.data_ptr()
    for i in range(nsteps):
        step(1)
        cvf3.cvf3_state_counts(chain.h, base + 48 * i, chain.stream)
    return out.cpu().numpy()


def measure3(cvf, cvf3, torch, L: int, T: float, P: float, seed: int, algo: str, warm: int, n_rec: int,
             n_time: int = 2000, max_lag: int = 2000) -> dict:
    """measure() for the cubic lattice with eta (the paper's own model, Sec.
    III.A and III.C): arm-domain Metropolis ("met") or Swendsen-Wang ("sw")
    steps, M normalised by the 6N bond indices."""
    p = cvf.cvf_params_from_si(T, P, L=L, seed=seed)
    ch = cvf3.Chain3(p, algo_mask=cvf.CVF_ALGO_METROPOLIS | cvf.CVF_ALGO_SW)
    step = ch.steps if algo == "met" else ch.sw
    step(warm)
    counts = record_counts3(cvf3, ch, step, n_rec)
    M = order_parameter(counts, 6 * L ** 3)
    C = c_m(M, min(max_lag, n_rec // 2))
    tau = tau_1e(C)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step(n_time)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / n_time
    o = ch.obs()
    ch.close()
    ok = not math.isnan(tau)
    return {"warmup_steps": warm, "steps_recorded": n_rec, "tau_steps": round(float(tau), 3) if ok else None,
            "C_M_1": round(float(C[1]), 4), "step_us": round(t_step * 1e6, 2),
            "cost_per_independent_us": round(float(tau) * t_step * 1e6, 2) if ok else None,
            "v": round(o["v"], 4), "M_mean": round(float(M.mean()), 4), "M_std": float("%.3g" % M.std()),
            "consistent": o["consistent"] == 1}
