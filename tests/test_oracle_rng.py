"""Pins for the oracle's random-number primitives.

* Philox4x32-10 (Salmon et al., SC'11) against rocRAND's independent
  implementation of the same published generator (library routine, run on
  the host through its public engine API).
* ``pick`` (exactly uniform integer from a 32-bit word) against the block
  boundaries that its definition fixes.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND helper")
    exe = str(tmp_path_factory.mktemp("kat") / "rocrand_philox_kat")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "helpers", "rocrand_philox_kat.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(rows):
        text = "".join(f"{a} {b} {c} {d} {s}\n" for a, b, c, d, s in rows)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return np.array([[int(x) for x in ln.split()] for ln in out.strip().splitlines()], dtype=np.uint64)
    return run


def test_philox_matches_rocrand(oracle_mod, rocrand_kat):
    rng = np.random.default_rng(123)
    rows = [(0, 0, 0, 0, 0),
            (0xFFFFFFFF, (1 << 30) - 1, 0xFFFFFFFF, 0xFFFFFFFF, (1 << 64) - 1),
            (1, 0, 0, 0, 1), (0, 1, 0, 0, 1), (0, 0, 1, 0, 1), (0, 0, 0, 1, 1),
            (4095, 999, 1, 2, 1), (0, 7, 0, 1, 12345678901234567)]
    for _ in range(200):
        rows.append((int(rng.integers(0, 1 << 32)), int(rng.integers(0, 1 << 30)),
                     int(rng.integers(0, 1 << 32)), int(rng.integers(0, 1 << 32)),
                     int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))))
    ref = rocrand_kat(rows)
    got = np.array([oracle_mod.philox(r[:4], r[4]) for r in rows], dtype=np.uint64)
    assert np.array_equal(got, ref)


def test_philox_zero_block_known_value(oracle_mod, rocrand_kat):
    # the all-zero counter and key is the first block rocRAND produces for seed 0
    ref = rocrand_kat([(0, 0, 0, 0, 0)])[0]
    assert list(oracle_mod.philox([0, 0, 0, 0], 0)) == list(ref)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_pick_block_boundaries(oracle_mod, k):
    d = (1 << 32) // k
    for i in range(k):
        assert oracle_mod.pick(i * d, k) == i
        assert oracle_mod.pick(i * d + d - 1, k) == i
    if k * d < (1 << 32):
        assert oracle_mod.pick(k * d, k) == -1
        assert oracle_mod.pick(0xFFFFFFFF, k) == -1
    else:
        assert oracle_mod.pick(0xFFFFFFFF, k) == k - 1


def test_pick_q6_only_top_word_is_none(oracle_mod):
    # 2^32 - 1 = 3*5*17*257*65537: for k = 5 only the top word is rejected
    assert oracle_mod.pick(0xFFFFFFFE, 5) == 4
    assert oracle_mod.pick(0xFFFFFFFF, 5) == -1
    # for k = 6, 2^32 mod 6 = 4 words are rejected
    assert [oracle_mod.pick(0xFFFFFFFF - i, 6) for i in range(5)] == [-1, -1, -1, -1, 5]
