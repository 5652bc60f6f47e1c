"""Algorithm choice for served jobs: the paper's temperature switch (Sec.
II.B), the cost-per-independent-configuration rule (Sec. III.C) with the
nearest calibrated temperature, and the default that keeps every job's own
algorithm."""
import pytest

from paper_2505_05919_amd.policy import AlgoPolicy
from paper_2505_05919_amd.workloads import Job


def job(T, algo="met"):
    return Job(L=8, T=T, P=0.1, nsteps=10, algo=algo, seed=1)


def test_threshold_is_the_papers_switch():
    pol = AlgoPolicy("threshold")
    assert pol.choose(job(208.0, "sw")) == "met"          # Metropolis at T >= 208 K
    assert pol.choose(job(207.999, "met")) == "sw"
    assert pol.apply(job(190.0)).algo == "sw" and pol.apply(job(190.0)).T == 190.0
    assert AlgoPolicy("threshold", T_switch=250.0).choose(job(240.0)) == "sw"


def test_cost_uses_the_nearest_calibrated_temperature():
    table = {270.0: {"met": None, "sw": 22.0}, 300.0: {"met": 2000.0, "sw": 19.0}, 400.0: {"met": 5.0, "sw": 9.0}}
    pol = AlgoPolicy("cost", table=table)
    assert pol.choose(job(265.0)) == "sw"                  # tau beyond the window counts as infinite
    assert pol.choose(job(310.0)) == "sw"
    assert pol.choose(job(380.0, "sw")) == "met"
    assert pol.choose(job(350.0)) == "sw"                  # equidistant: the lower temperature
    assert AlgoPolicy("cost", table={300.0: {"met": None, "sw": None}}).choose(job(300.0, "sw")) == "sw"


def test_default_and_errors():
    assert AlgoPolicy().choose(job(100.0, "met")) == "met"
    with pytest.raises(ValueError):
        AlgoPolicy("fastest")
    with pytest.raises(ValueError):
        AlgoPolicy("cost")
