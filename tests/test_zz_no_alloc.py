"""The allocation-free residual (nks_residual_noalloc) through the C ABI
against nks_residual on the same inputs: two calls in a row on one GPU, the
second on a smaller grid, and the size limit of its fixed scratch."""
import ctypes as C
import sys

import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nks():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2007_13966_amd as P
    P.lib()
    return P


def _inputs(g, seed):
    rng = np.random.default_rng(seed)
    base = g.initial_pressure().cpu().numpy()
    p = base + 3e4 * rng.standard_normal(g.N)
    pn = base + 1e4 * rng.standard_normal(g.N)
    pnm1 = base + 1e4 * rng.standard_normal(g.N)
    return g.from_numpy(p), g.from_numpy(pn), g.from_numpy(pnm1)


def _abi_noalloc(nks, g, p, pn, pnm1, dt, order, F):
    vp = lambda t: C.c_void_p(t.data_ptr())
    return nks.lib().nks_residual_noalloc(g.h, vp(p), vp(pn), vp(pnm1), C.c_double(dt), C.c_int(order), vp(F))


@pytest.mark.parametrize("order", [1, 2])
def test_noalloc_residual_matches_residual_twice(nks, order):
    import torch
    # first call: two reservoirs (one 3D with gravity would need a separate
    # grid: every reservoir of a grid shares the fluid and gravity), then a
    # smaller grid on the same GPU, so the second call reuses the scratch
    big = S.small_case(nx=150, ny=130, seed=3)
    other = S.small_case(nx=61, ny=47, seed=4)
    small = S.small_case(nx=23, ny=17, seed=5, bc=((2, 1, 2.2e7), (3, 2, -1e-6)))
    for k, recs in enumerate([big.problems + other.problems, small.problems]):
        g = nks.Grid(recs)
        say("noalloc residual", k, "cells", g.N, "order", order)
        p, pn, pnm1 = _inputs(g, 10 + k)
        F_ref = g.residual(p, pn, pnm1, big.dt, order).cpu().numpy()
        F = g.zeros()
        F.fill_(np.nan)
        torch.cuda.synchronize()
        rc = _abi_noalloc(nks, g, p, pn, pnm1, big.dt, order, F)
        assert rc == 0, nks.lib().nks_last_error()
        g.stream.synchronize()
        Fn = F.cpu().numpy()
        assert np.array_equal(Fn, F_ref), np.max(np.abs(Fn - F_ref))
        # the grid's own path still gives the same answer afterwards
        F2 = g.residual(p, pn, pnm1, big.dt, order).cpu().numpy()
        assert np.array_equal(F2, F_ref)


def test_noalloc_residual_rejects_grids_beyond_its_scratch(nks):
    import torch
    n = 1700   # 2,890,000 cells > NKS_NOALLOC_MAX_CELLS = 2,621,440
    case = S.small_case(nx=n, ny=n, seed=6, rate=0.0)
    g = nks.Grid(case.problems)
    p = g.initial_pressure()
    F = g.zeros()
    torch.cuda.synchronize()
    rc = _abi_noalloc(nks, g, p, p, p, case.dt, 1, F)
    assert rc == -1
    assert b"exceed" in nks.lib().nks_last_error()
