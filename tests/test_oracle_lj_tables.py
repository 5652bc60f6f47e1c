"""Pins for the oracle's model constants: the Lennard-Jones lattice energy,
the reduced-unit conversion of Table I, and the acceptance / bond tables.

Each check goes through a route independent of the oracle's code: Jacobi's
two-square theorem, a direct sum over 2-D lattice vectors, the closed-form
infinite lattice sums (Epstein zeta = 4 zeta(s) beta(s)), and 40-digit
decimal arithmetic.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

getcontext().prec = 40
TWO32 = 1 << 32


def jacobi_r2(m):
    """r2(m) = 4 (d1(m) - d3(m)) (Jacobi's two-square theorem), r2(0) = 1."""
    if m == 0:
        return 1
    d1 = sum(1 for d in range(1, m + 1) if m % d == 0 and d % 4 == 1)
    d3 = sum(1 for d in range(1, m + 1) if m % d == 0 and d % 4 == 3)
    return 4 * (d1 - d3)


def test_r2_two_square_theorem(oracle_mod):
    for m in range(0, 60):
        assert oracle_mod.r2(m) == jacobi_r2(m), m


def direct_lattice_energy(v):
    """Half the LJ energy of one molecule with every other molecule of a square
    lattice of spacing sqrt(v) r0, cutoff 6 r0 (inclusive), hard core r0."""
    e = 0.0
    for i in range(-7, 8):
        for j in range(-7, 8):
            if i == 0 and j == 0:
                continue
            if v * (i * i + j * j) > 36.0:
                continue
            d = math.sqrt(v) * math.hypot(i, j)
            e += 0.5 * 4.0 * ((1.0 / d) ** 12 - (1.0 / d) ** 6)
    return e


@pytest.mark.parametrize("v", [1.0, 1.0 + 1e-9, 1.1, 1.2038, 1.25, 1.5, 1.999, 2.0, 3.7, 12.0, 35.9, 36.0, 40.0])
def test_u_lj_direct_sum(oracle_mod, v):
    assert oracle_mod.u_lj(v) == pytest.approx(direct_lattice_energy(v), rel=1e-12, abs=1e-300)


def test_u_lj_hard_core_and_beyond_cutoff(oracle_mod):
    assert math.isinf(oracle_mod.u_lj(0.999999))
    assert oracle_mod.u_lj(36.0) != 0.0          # |n| = 1 sits exactly at the cutoff
    assert oracle_mod.u_lj(36.0000001) == 0.0


def dirichlet_beta(s, terms=200000):
    k = np.arange(terms, dtype=np.float64)
    return float(np.sum((-1.0) ** k / (2 * k + 1) ** s))


@pytest.mark.parametrize("v", [1.0, 1.2, 1.5, 2.5])
def test_u_lj_vs_infinite_lattice_closed_form(oracle_mod, v):
    """sum_{n != 0} |n|^-2s over Z^2 = 4 zeta(s) beta(s); the cutoff removes an
    attractive tail of about pi / (1296 v) (integral estimate)."""
    zeta3 = 1.2020569031595942854
    beta3 = math.pi ** 3 / 32.0
    zeta6 = math.pi ** 6 / 945.0
    beta6 = dirichlet_beta(6)
    S3 = 4 * zeta3 * beta3
    S6 = 4 * zeta6 * beta6
    u_inf = 2.0 * (v ** -6 * S6 - v ** -3 * S3)
    tail = math.pi / (1296.0 * v)
    diff = oracle_mod.u_lj(v) - u_inf
    assert 0.5 * tail < diff < 1.5 * tail


def test_u_lj_minimum_near_expected(oracle_mod):
    vs = np.linspace(1.0, 1.6, 6001)
    us = np.array([oracle_mod.u_lj(float(v)) for v in vs])
    i = int(np.argmin(us))
    # the 2-D lattice minimum: d/dv [S6 v^-6 - S3 v^-3] = 0 -> v^3 = 2 S6/S3 (cutoff shifts it slightly)
    zeta3 = 1.2020569031595942854
    S3 = 4 * zeta3 * math.pi ** 3 / 32.0
    S6 = 4 * (math.pi ** 6 / 945.0) * dirichlet_beta(6)
    v_star = (2 * S6 / S3) ** (1.0 / 3.0)
    assert abs(vs[i] - v_star) < 2e-3


def test_params_from_si_table1(oracle_mod):
    p = oracle_mod.params_from_si(300.0, 0.1)
    R = 6.02214076e23 * 1.380649e-23
    assert p.beta == pytest.approx(5500.0 / (R * 300.0), rel=1e-15)
    assert p.beta == pytest.approx(2.2049931758, rel=1e-9)
    assert p.P == pytest.approx(1e5 * (2.9e-10) ** 3 * 6.02214076e23 / 5500.0, rel=1e-14)
    assert p.P == pytest.approx(2.6704362e-4, rel=1e-7)
    assert p.J == 2.0 and p.Jsigma == pytest.approx(0.32, rel=1e-15) and p.vHB == 0.6
    assert p.q == 6 and p.v_init == 1.25 and p.dv_max == pytest.approx(0.0125)


def dec_exp_floor(x: Decimal) -> int:
    """floor(exp(x) 2^32) in 40-digit arithmetic."""
    return int((x.exp() * TWO32).to_integral_value(rounding="ROUND_FLOOR"))


@pytest.mark.parametrize("T,P", [(270.0, 0.1), (300.0, 0.1), (330.0, 50.0), (300.0, 2000.0), (200.0, 25.0)])
def test_metropolis_table_vs_decimal(oracle_mod, T, P):
    p = oracle_mod.params_from_si(T, P)
    met, _ = oracle_mod.tables(p)
    beta, J, Js, Ps, vHB = (Decimal(repr(x)) for x in (p.beta, p.J, p.Jsigma, p.P, p.vHB))
    Jeff = J - Ps * vHB
    for th in (0, 1):
        for dh in (-1, 0, 1):
            for dc in range(-3, 4):
                dH = -(th * Jeff * dh) - Js * dc
                got = int(met[th, dh + 1, dc + 3])
                if dH <= 0:
                    # dH == 0 exactly only for dh == dc == 0 or theta*dh == 0 == dc
                    assert got == 0xFFFFFFFF, (th, dh, dc)
                else:
                    ref = min(dec_exp_floor(-beta * dH), 0xFFFFFFFE)
                    assert abs(got - ref) <= 1, (th, dh, dc, got, ref)
                    # detailed balance of the pair (s -> s', s' -> s): reverse move always accepted
                    assert int(met[th, 1 - dh, 3 - dc]) == 0xFFFFFFFF


def test_metropolis_table_beta_zero_always_accepts(oracle_mod):
    p = oracle_mod.params_from_si(300.0, 0.1)
    p.beta = 0.0
    met, sw = oracle_mod.tables(p)
    assert np.all(met == 0xFFFFFFFF)
    assert list(sw) == [0, 0, 0]


@pytest.mark.parametrize("T,P", [(270.0, 0.1), (330.0, 50.0), (300.0, 2000.0)])
def test_sw_thresholds_vs_decimal(oracle_mod, T, P):
    p = oracle_mod.params_from_si(T, P)
    _, sw = oracle_mod.tables(p)
    beta, J, Js, Ps, vHB = (Decimal(repr(x)) for x in (p.beta, p.J, p.Jsigma, p.P, p.vHB))
    Jeff = abs(J - Ps * vHB)

    def thr(x):
        return int(((1 - (-beta * x).exp()) * TWO32).to_integral_value(rounding="ROUND_FLOOR"))
    assert abs(int(sw[0]) - thr(Js)) <= 1
    assert int(sw[1]) == 0
    assert abs(int(sw[2]) - thr(Jeff)) <= 1
