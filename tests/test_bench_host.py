"""Host logic of bench.py (no GPU): the algorithmic byte counts behind the
roofline figures, the launch filter, and the one-GPU guard.

The extended-cell counts are the sizes worked out independently for the
benchmark configurations (2D 32x32 with 4x4 boxes and overlap 1; 2D 512x512
with 16x16 boxes and overlap 2, its 256x256 coarse level with overlap 1;
3D 128x128x64 with 8x8x4 boxes; 3D 96x96x48 with 6x6x3 boxes): a box q of
P along n cells holds n//P + (q < n%P) cells, extended by the overlap on
each side and clipped at the boundary."""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("dims,boxes,delta,expect", [
    ((32, 32, 1), (4, 4, 1), 1, 1444),
    ((512, 512, 1), (16, 16, 1), 2, 327184),
    ((256, 256, 1), (16, 16, 1), 1, 81796),
    ((128, 128, 64), (8, 8, 4), 1, 1411480),
    ((96, 96, 48), (6, 6, 3), 1, 584272),
])
def test_extended_cells(dims, boxes, delta, expect):
    assert bench.ext_cells(*dims, *boxes, delta) == expect


def test_extended_cells_brute_force():
    # every box's extended range counted cell by cell on a small uneven grid
    nx, ny, px, py, d = 13, 7, 4, 3, 2

    def ranges(n, P):
        base, rem = divmod(n, P)
        lo = 0
        for q in range(P):
            hi = lo + base + (1 if q < rem else 0)
            yield max(0, lo - d), min(n, hi + d)
            lo = hi
    total = 0
    for (x0, x1) in ranges(nx, px):
        for (y0, y1) in ranges(ny, py):
            total += sum(1 for _ in range(x0, x1) for _ in range(y0, y1))
    assert bench.ext_cells(nx, ny, 1, px, py, 1, d) == total


def test_roofline_bytes_2d_512():
    import synthetic as S
    case = S.case_2d_512()
    s = S.with_solver(case, precision="fp64").solver
    nbytes, next_ = bench.apply_bytes(case.problems, s, "fp64")
    # 4 off-diagonal factors, 1/u_ii and the gathered residual per extended
    # cell, the written correction per owned cell
    assert next_ == 327184
    assert nbytes == 327184 * (4 * 8 + 8 + 8) + 262144 * 8 == 17801984


def test_launch_split_drops_masked_launches():
    d = np.array([1.2, 1.0, 12.0, 12.5, 11.8, 13.1, 2.0])
    kept = bench.launch_split(d)
    assert sorted(kept.tolist()) == [11.8, 12.0, 12.5, 13.1]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
