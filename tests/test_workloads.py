"""The seeded synthetic inputs (job descriptions only): each configuration's
generator produces the sizes, state points, step counts, seeds and arrival
statistics that the input recipe states."""
import math

import numpy as np

from paper_2505_05919_amd import workloads as w


def test_single_and_scan_configurations():
    c1 = w.c1_job()
    assert (c1.L, c1.T, c1.P, c1.nsteps, c1.algo, c1.seed) == (64, 300.0, 0.1, 1000, "met", 1)
    c2 = w.c2_jobs()
    met = [j for j in c2 if j.algo == "met"]
    sw = [j for j in c2 if j.algo == "sw"]
    assert [j.T for j in met] == [270.0, 285.0, 300.0, 315.0, 330.0] == [j.T for j in sw]
    assert all(j.L == 1024 and j.nsteps == 10_000 and j.P == 0.1 for j in met)
    assert all(j.L == 256 and j.nsteps == 1_000 and j.P == 0.1 for j in sw)
    assert [j.seed for j in c2] == list(range(2, 12))
    c3 = w.c3_jobs()
    assert [(j.L, j.P, j.algo, j.seed) for j in c3] == (
        [(4096, P, "met", 12 + i) for i, P in enumerate((0.1, 25.0, 50.0))]
        + [(1414, P, "sw", 15 + i) for i, P in enumerate((0.1, 25.0, 50.0))])
    assert all(j.T == 300.0 and j.nsteps == 1000 for j in c3)


def test_batched_replicas():
    jobs = w.c4_jobs()
    assert len(jobs) == 256
    Ls = np.array([j.L for j in jobs])
    assert np.all(Ls % 2 == 0) and Ls.min() >= 64 and Ls.max() <= 512
    # log-uniform: the median sits near the geometric mean of the range
    assert 150 <= np.median(Ls) <= 215
    for k, j in enumerate(jobs):
        i, jj = divmod(k, 16)
        assert j.T == 270.0 + 4.0 * i and math.isclose(j.P, 50.0 / 15.0 * jj)
        assert j.seed == 1000 + k and j.nsteps == 1000 and j.algo == "met"
    assert w.c4_jobs() == jobs                     # seeded: the same replicas every time


def test_served_stream():
    jobs = w.c5_stream()
    assert len(jobs) == 2000
    arr = np.array([j.arrival for j in jobs])
    assert np.all(np.diff(arr) > 0)
    # Poisson at 200 jobs/s: 2000 arrivals span about 10 s
    assert 9.0 < arr[-1] < 11.0
    gaps = np.diff(np.concatenate(([0.0], arr)))
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1   # exponential gaps: coefficient of variation 1
    Ls = np.array([j.L for j in jobs])
    assert np.all(Ls % 2 == 0) and Ls.min() >= 32 and Ls.max() <= 2048
    assert 200 <= np.median(Ls) <= 310                # geometric mean of 32..2048 is 256
    assert all(270.0 <= j.T <= 330.0 and 0.0 <= j.P <= 50.0 for j in jobs)
    assert all(100 <= j.nsteps <= 10_000 for j in jobs)
    sw = sum(j.algo == "sw" for j in jobs) / len(jobs)
    assert 0.17 < sw < 0.23
    assert [j.seed for j in jobs] == [5000 + n for n in range(2000)]


def test_served_oracle_subset():
    jobs = w.c5_stream()
    sub = w.c5_oracle_subset(jobs)
    assert sub == sorted(set(sub))
    small = [n for n, j in enumerate(jobs) if j.L <= 256]
    assert set(small) <= set(sub)
    extra = [n for n in sub if jobs[n].L > 256]
    assert len(extra) == 16
    assert len(sub) == len(small) + 16 == 1008
