"""Host-side logic of the job server (no GPU): the least-remaining-work
selection of a quantum's members, the FCFS latency model of the
one-job-at-a-time baseline, the latency summary and the device footprint
used for admission."""
import numpy as np

from paper_2505_05919_amd import serve
from paper_2505_05919_amd.workloads import Job


def run_of(L, nsteps, done, seed):
    return serve.Running(Job(L, 300.0, 0.1, nsteps, "met", seed), chain=None, done=done)


def test_srpt_takes_least_remaining_work_until_the_fill():
    runs = [run_of(64, 1000, 0, 1),        # 64^2 * 1000 cells left
            run_of(32, 1000, 900, 2),      # 32^2 * 100
            run_of(128, 100, 50, 3),       # 128^2 * 50
            run_of(16, 10, 0, 4)]          # 16^2 * 10
    got = serve._srpt(runs, fill_cells=32 * 32 + 16 * 16)
    assert [r.job.seed for r in got] == [4, 2]            # stops once the fill is reached
    got = serve._srpt(runs, fill_cells=1 << 30)
    assert [r.job.seed for r in got] == [4, 2, 3, 1]      # all, in order of remaining work
    tie = [run_of(16, 10, 0, 9), run_of(16, 10, 0, 5)]
    assert [r.job.seed for r in serve._srpt(tie, 1 << 30)] == [5, 9]   # ties by seed


def test_fcfs_latencies_by_hand():
    jobs = [Job(8, 300.0, 0.1, 1, "met", k, a) for k, a in enumerate((0.0, 0.2, 5.0))]
    lat = serve.fcfs_latencies(jobs, [1.0, 0.5, 2.0])
    # completions 1.0, 1.5, 7.0
    assert np.allclose(lat, [1.0, 1.3, 2.0])


def test_summary_of_records():
    recs = [serve.Record(Job(8, 300.0, 0.1, 10, "met", k, float(k)), admitted=float(k) + 0.5,
                         completed=float(k) + 2.0, obs={}, t_ref=float(k)) for k in range(4)]
    recs.append(serve.Record(Job(8, 300.0, 0.1, 10, "sw", 9, 0.0), admitted=0.0, completed=10.0, obs={}))
    s = serve.summarize(recs)
    assert s["jobs"] == 5
    assert np.isclose(s["p50_s"], 2.0) and s["p99_s"] > 9.0
    assert np.isclose(s["makespan_s"], 10.0)
    assert np.isclose(s["met_updates_per_ns"], 4 * 4 * 64 * 10 / 10.0 / 1e9)
    assert np.isclose(s["sw_cell_steps_per_ns"], 64 * 10 / 10.0 / 1e9)


def test_footprint_is_sigma_plus_workspace():
    from paper_2505_05919_amd import cvf
    for L, algo in ((64, "met"), (130, "sw"), (1414, "sw")):
        job = Job(L, 300.0, 0.1, 10, algo, 1)
        mask = cvf.CVF_ALGO_METROPOLIS | (cvf.CVF_ALGO_SW if algo == "sw" else 0)
        p = cvf.cvf_params_from_si(300.0, 0.1, L=L, seed=1)
        assert serve.footprint(job) == 4 * L * L + cvf.cvf_workspace_bytes(p, mask)
    assert serve.footprint(Job(1414, 300.0, 0.1, 10, "sw", 1)) > serve.footprint(Job(1414, 300.0, 0.1, 10, "met", 1))
