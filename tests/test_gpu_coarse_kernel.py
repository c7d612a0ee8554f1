"""The coarsest level's GMRES in its two forms: the persistent launch (one
workgroup per reservoir iterating until its own convergence test stops it)
and the chunked launches (one kernel per step, a host test after each
captured chunk).  Both run the same iteration (Remark 2: GMRES with the
one-level preconditioner to coarse_rtol), so their corrections agree up to
the order of the FP64 sums, and the persistent one matches the oracle's
multilevel apply with a fixed number of coarse iterations, restarts
included.  Uneven reservoirs in one batch, every coarse stencil shape (the
5-point rediscretised operator, the 3x3-interpolated 5x5 box, the 21-point
one of second-order interpolation) and every precision."""
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


SIZES = [(37, 29, 1), (64, 50, 2), (20, 20, 3), (9, 33, 4), (96, 80, 5)]


def _batch(nks, orc, sizes=SIZES):
    recs = [S.small_case(nx=n, ny=m, seed=s, rate=2e-3).problems[0] for n, m, s in sizes]
    g = nks.Grid(recs)
    ps, pns, rs = [], [], []
    for k, rec in enumerate(recs):
        op = orc.Problem(rec)
        rng = np.random.default_rng(40 + k)
        base = op.initial_pressure()
        ps.append(base + 3e4 * rng.standard_normal(op.N))
        pns.append(base + 1e4 * rng.standard_normal(op.N))
        rs.append(np.cos(np.arange(op.N) * (k + 1) * 0.37))
    p = g.from_numpy(np.concatenate(ps))
    pn = g.from_numpy(np.concatenate(pns))
    return recs, g, ps, pns, rs, p, pn


def _apply(nks, g, J, settings, rs):
    M = nks.Ras(J, settings)
    return M.apply(g.from_numpy(np.concatenate(rs))).cpu().numpy()


SHAPES = [dict(interp_order=2), dict(interp_order=1), dict(coarse_op="rediscretised")]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 2e-5), ("bf16", 2e-3)])
@pytest.mark.parametrize("shape", SHAPES, ids=["order2", "order1", "rediscretised"])
@pytest.mark.parametrize("ratio", [2, 4])
def test_persistent_equals_chunked(nks, orc, precision, tol, shape, ratio):
    # the default stop (rtol 0.2, 30 iterations) on every reservoir: the same
    # correction from both forms
    recs, g, ps, pns, rs, p, pn = _batch(nks, orc)
    if shape.get("coarse_op") == "rediscretised":
        # the upscaled coarse problem needs sizes that are multiples of r
        sizes = [(48, 32, 1), (64, 56, 2), (24, 24, 3), (8, 40, 4), (96, 80, 5)]
        recs, g, ps, pns, rs, p, pn = _batch(nks, orc, sizes)
    J = g.jacobian(p, pn, pn, S.DAY, 1)
    base = dict(px=1, py=1, tile=(16, 16, 0), levels=2, overlap=(2, 1), ratio=ratio, precision=precision, **shape)
    zc = _apply(nks, g, J, S.SolverSettings(coarse_kernel="chunked", **base), rs)
    zp = _apply(nks, g, J, S.SolverSettings(coarse_kernel="persistent", **base), rs)
    for k in range(len(recs)):
        a, b = zp[g.offsets[k]:g.offsets[k + 1]], zc[g.offsets[k]:g.offsets[k + 1]]
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        say(precision, shape, "ratio", ratio, "reservoir", k, "persistent vs chunked", f"{err:.2e}")
        assert err <= tol, (k, err)


@pytest.mark.parametrize("restart,maxit", [(30, 6), (3, 7)])
def test_persistent_oracle_parity(nks, orc, restart, maxit):
    # a fixed number of coarse iterations (rtol 0), with restarts every
    # `restart` iterations: each reservoir against its own oracle
    recs, g, ps, pns, rs, p, pn = _batch(nks, orc)
    J = g.jacobian(p, pn, pn, S.DAY, 1)
    kw = dict(px=1, py=1, tile=(12, 12, 0), levels=2, overlap=(2, 1), coarse_rtol=0.0, coarse_maxit=maxit,
              coarse_restart=restart)
    zg = _apply(nks, g, J, S.SolverSettings(coarse_kernel="persistent", **kw), rs)
    for k, rec in enumerate(recs):
        op = orc.Problem(rec)
        Jo = op.jacobian(ps[k], pns[k], pns[k], S.DAY, 1)
        zo = orc.Multilevel(rec, Jo, S.SolverSettings(**kw)).apply(rs[k])
        part = zg[g.offsets[k]:g.offsets[k + 1]]
        err = np.max(np.abs(part - zo)) / np.max(np.abs(zo))
        say("restart", restart, "maxit", maxit, "reservoir", k, f"{err:.2e}")
        assert err <= 1e-9, (k, err)


def test_persistent_three_levels(nks, orc):
    # the persistent kernel on the coarsest of three levels
    case = S.small_case(nx=96, ny=80, px=4, py=4, levels=3, overlap=(2, 1, 1), coarse_rtol=0.0, coarse_maxit=5,
                        coarse_kernel="persistent")
    rec = case.problems[0]
    op = orc.Problem(rec)
    rng = np.random.default_rng(5)
    p = op.initial_pressure() + 3e4 * rng.standard_normal(op.N)
    Jo = op.jacobian(p, p, p, case.dt, 1)
    r = np.sin(0.21 * np.arange(op.N))
    zo = orc.Multilevel(rec, Jo, case.solver).apply(r)
    g = nks.Grid([rec])
    pg = g.from_numpy(p)
    J = g.jacobian(pg, pg, pg, case.dt, 1)
    zg = nks.Ras(J, case.solver).apply(g.from_numpy(r)).cpu().numpy()
    assert np.max(np.abs(zg - zo)) <= 1e-9 * np.max(np.abs(zo))


def test_persistent_refused_where_not_allowed(nks, orc):
    # AS keeps the chunked form; asking for the persistent one is an error
    recs, g, ps, pns, rs, p, pn = _batch(nks, orc)
    J = g.jacobian(p, pn, pn, S.DAY, 1)
    kw = dict(px=1, py=1, tile=(16, 16, 0), levels=2, overlap=(1, 1), variant="as")
    with pytest.raises(nks.NksError):
        nks.Ras(J, S.SolverSettings(coarse_kernel="persistent", **kw))
    # auto falls back to the chunked form
    za = _apply(nks, g, J, S.SolverSettings(**kw), rs)
    zc = _apply(nks, g, J, S.SolverSettings(coarse_kernel="chunked", **kw), rs)
    assert np.array_equal(za, zc)


def test_persistent_newton_batch(nks, orc):
    # two implicit steps of a batch with either form: the same iteration
    # counts, pressures within the FP64 parity bar
    recs, g, ps, pns, rs, p, pn = _batch(nks, orc)
    out = {}
    for kind in ("chunked", "persistent"):
        s = S.SolverSettings(px=1, py=1, tile=(16, 16, 0), levels=2, overlap=(2, 1), ratio=4, precision="fp32",
                             coarse_kernel=kind, eps_r=1e-8)
        gg = nks.Grid(recs)
        hist, stats = gg.simulate(2, 5 * S.DAY, s)
        out[kind] = (hist[-1].cpu().numpy(), [(x["newton_its"], x["linear_its"]) for x in stats])
        say(kind, out[kind][1])
    assert out["chunked"][1] == out["persistent"][1]
    a, b = out["persistent"][0], out["chunked"][0]
    p0 = g.initial_pressure().cpu().numpy()
    assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(b - p0)
