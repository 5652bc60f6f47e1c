"""Host-side launch shapes (no GPU): the Metropolis colour launch covers every
row and column of every L with whole row pairs, within the kernel's limits,
and the Swendsen-Wang grid has one tile per 64 x 16 cells."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def shapes(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("shapes") / "launch_shapes")
    subprocess.run([hipcc, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2505_05919_amd", "csrc"),
                    os.path.join(HERE, "helpers", "launch_shapes.cpp"), "-o", exe], check=True)
    Ls = list(range(2, 4100, 2)) + [4094, 4096, 5000, 8192, 16384, 32764, 32766]
    out = subprocess.run([exe], input="\n".join(map(str, Ls)), capture_output=True, text=True, check=True).stdout
    rows = {}
    for line in out.split("\n"):
        if line.strip():
            L, quad, r, rb, tiles = map(int, line.split())
            rows[L] = (quad, r, rb, tiles)
    return rows


def test_metropolis_shapes_cover_the_lattice(shapes):
    for L, (quad, rows, row_blocks, _) in shapes.items():
        assert rows % 2 == 0 and 2 <= rows <= 32, L          # whole row pairs, within the kernel's limit
        assert 4 * rows * row_blocks >= L > 4 * rows * (row_blocks - 1), L   # four wavefronts per workgroup
        if L % 4 == 0:
            assert quad == 1, L
        else:
            assert quad == (2 if L >= 1024 else 0), L        # ragged quads from L = 1024, else column pairs


def test_metropolis_shape_at_the_benchmark_size(shapes):
    quad, rows, row_blocks, _ = shapes[4096]
    # 16 rows per wavefront, 16 x 64 = 1024 workgroups of four wavefronts: 4096 wavefronts
    assert (quad, rows, row_blocks) == (1, 16, 64)


def test_sw_tiles(shapes):
    for L, (_, _, _, tiles) in shapes.items():
        assert tiles == -(-L // 64) * -(-L // 16), L
    assert shapes[1414][3] == 2047
