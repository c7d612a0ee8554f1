"""Degenerate and boundary inputs through the libnks C ABI against the oracle:
a single-cell reservoir, one-cell-wide strips, more boxes than cells,
overlap wider than a box, coarsening down to a single coarse cell, a batch
holding a 1x1 reservoir, and the error paths (non-physical state, bad
descriptors)."""
import sys

import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu
TOL = dict(eps_r=1e-8, eps_a=1e-6)


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


def _single_cell(rate=1e-3):
    k = np.full(1, 100 * S.MD)
    return S.Problem(1, 1, 1, 10.0, 10.0, 10.0, k, k.copy(), k.copy(), np.full(1, 0.2),
                     np.array([0], np.int32), np.array([rate]))


def _compare(nks, orc, recs, settings, dt=S.DAY):
    g = nks.Grid(recs)
    p0 = g.initial_pressure()
    p = p0.clone()
    st = g.newton_step(p, p0, p0, dt, 1, settings)
    parts = g.split(p)
    for k, rec in enumerate(recs):
        prob = orc.Problem(rec)
        q0 = prob.initial_pressure()
        q, sto = orc.newton_step(prob, settings, q0, q0, q0, dt, 1)
        assert sto["status"] == 0
        dq, dg = q - q0, parts[k] - q0
        scale = max(np.linalg.norm(dq), 1e-30)
        err = np.linalg.norm(dg - dq) / scale
        say(f"  reservoir {k} ({rec.nx}x{rec.ny}x{rec.nz}): dp error {err:.2e} (|dp| {scale:.3e})")
        assert err <= 1e-6 or np.linalg.norm(dg - dq) <= 1e-9
    return st


def test_single_cell_reservoir(nks, orc):
    rec = _single_cell()
    st = _compare(nks, orc, [rec], S.SolverSettings(px=1, py=1, **TOL))
    assert st["status"] == 0


@pytest.mark.parametrize("name,cfg", [
    ("strip 1x37", dict(nx=1, ny=37, px=1, py=4)),
    ("strip 41x1", dict(nx=41, ny=1, px=5, py=1)),
    ("more boxes than cells", dict(nx=5, ny=6, px=8, py=8)),
    ("overlap wider than a box", dict(nx=8, ny=8, px=4, py=4, overlap=(3,))),
    ("coarsening to one cell", dict(nx=4, ny=4, px=2, py=2, levels=3, overlap=(1, 1, 1))),
    ("3D column 1x1x5", dict(nx=1, ny=1, nz=5, px=1, py=1, pz=2, gravity=True)),
    ("3D slab 9x7x2 boxes 2x2x3", dict(nx=9, ny=7, nz=2, px=2, py=2, pz=3)),
])
def test_degenerate_grids(nks, orc, name, cfg):
    say(name)
    case = S.small_case(**TOL, **cfg)
    _compare(nks, orc, case.problems, case.solver, case.dt)


def test_batch_with_single_cell_reservoir(nks, orc):
    recs = [S.small_case(nx=12, ny=9, seed=3).problems[0], _single_cell(2e-3),
            S.small_case(nx=7, ny=15, seed=4).problems[0]]
    settings = S.SolverSettings(px=1, py=1, tile=(4, 4, 0), levels=2, overlap=(1, 1), **TOL)
    _compare(nks, orc, recs, settings)


def test_nonphysical_state_is_an_error(nks):
    rec = S.small_case(nx=6, ny=5).problems[0]
    g = nks.Grid([rec])
    p0 = g.initial_pressure()
    bad = p0.clone()
    bad[3] = -1.0e5
    with pytest.raises(nks.NksError) as e:
        g.newton_step(bad.clone(), bad, bad, S.DAY, 1, S.SolverSettings(px=2, py=2))
    assert "NONPHYSICAL" in str(e.value)


def test_bad_descriptors_are_errors(nks):
    rec = S.small_case(nx=6, ny=5).problems[0]
    g = nks.Grid([rec])
    p0 = g.initial_pressure()
    J = g.jacobian(p0, p0, None, S.DAY, 1)
    for bad in (dict(levels=0), dict(variant="left_ras", interp_order=4), dict(coarse_restart=0),
                dict(tile=(-1, 0, 0))):
        kw = dict(px=2, py=2)
        kw.update(bad)
        with pytest.raises((nks.NksError, KeyError, ValueError)):
            nks.Ras(J, S.SolverSettings(**kw))
    with pytest.raises(nks.NksError):
        g.newton_step(p0.clone(), p0, p0, -1.0, 1, S.SolverSettings(px=2, py=2))


def test_handles_destroyed_in_any_order(nks):
    # a matrix and a preconditioner keep their grid's memory: destroying the
    # grid handle first (as a garbage collector may when the three sit in a
    # reference cycle) leaves them usable, and the last one frees the grid
    import ctypes as C
    case = S.small_case(nx=24, ny=20, px=2, py=2, levels=2, overlap=(1, 1))
    g = nks.Grid(case.problems)
    p = g.initial_pressure()
    J = g.jacobian(p, p, None, case.dt, 1)
    M = nks.Ras(J, case.solver)
    r = g.from_numpy(np.cos(np.arange(g.N)))
    z_ref = M.apply(r).cpu().numpy()
    lib = nks.lib()
    assert lib.nks_destroy_grid(g.h) == 0
    g.h = None
    z = M.apply(r).cpu().numpy()
    assert np.array_equal(z, z_ref)
    assert lib.nks_destroy_matrix(J.h) == 0
    J.h = None
    z = M.apply(r).cpu().numpy()
    assert np.array_equal(z, z_ref)
    assert lib.nks_destroy_ras(M.h) == 0
    M.h = None
