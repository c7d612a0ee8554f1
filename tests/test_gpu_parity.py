"""GPU parity: every step of the hot path through the libnks C ABI against the
FP64 CPU oracle on the same seeded inputs (sizes that span several
subdomains, ragged partitions and clipped boundary boxes)."""
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


def _state(orc_prob, seed, amp=3e4):
    rng = np.random.default_rng(seed)
    base = orc_prob.initial_pressure()
    p = base + amp * rng.standard_normal(orc_prob.N)
    pn = base + amp / 3 * rng.standard_normal(orc_prob.N)
    pnm1 = base + amp / 3 * rng.standard_normal(orc_prob.N)
    return p, pn, pnm1


CASES = [
    dict(nx=37, ny=23, nz=1, seed=1),
    dict(nx=9, ny=7, nz=5, seed=2, gravity=True, kv_ratio=0.1),
    dict(nx=16, ny=16, nz=1, seed=3, sigma=2.0),
]


@pytest.mark.parametrize("cfg", CASES)
@pytest.mark.parametrize("order", [1, 2])
def test_residual_and_jacobian_parity(nks, orc, cfg, order):
    say("residual/jacobian", cfg, order)
    case = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, pnm1 = _state(op, cfg["seed"])
    Fo = op.residual(p, pn, pnm1, case.dt, order)
    Jo = op.jacobian(p, pn, pnm1, case.dt, order)
    g = nks.Grid([rec])
    dp, dpn, dpnm1 = g.from_numpy(p), g.from_numpy(pn), g.from_numpy(pnm1)
    Fg = g.residual(dp, dpn, dpnm1, case.dt, order).cpu().numpy()
    assert np.max(np.abs(Fg - Fo)) <= 1e-12 * np.max(np.abs(Fo))
    F2 = g.zeros()
    J = g.jacobian(dp, dpn, dpnm1, case.dt, order, F=F2)
    assert np.array_equal(F2.cpu().numpy(), Fg)
    rp, ci, v = J.export_csr()
    assert np.array_equal(rp, Jo.rp) and np.array_equal(ci, Jo.ci)
    rowmax = np.repeat(np.maximum.reduceat(np.abs(Jo.v), Jo.rp[:-1]), np.diff(Jo.rp))
    assert np.all(np.abs(v - Jo.v) <= 1e-12 * rowmax)
    # J x and J^T x against the oracle's CSR
    x = np.random.default_rng(9).standard_normal(op.N)
    y = J.apply(g.from_numpy(x)).cpu().numpy()
    assert np.allclose(y, Jo.matvec(x), rtol=1e-12, atol=1e-12 * np.abs(y).max())
    yt = J.apply_transpose(g.from_numpy(x)).cpu().numpy()
    assert np.allclose(yt, Jo.scipy().T @ x, rtol=1e-12, atol=1e-12 * np.abs(yt).max())


def test_hydrostatic_parity(nks, orc):
    case = S.small_case(nx=6, ny=5, nz=9, gravity=True)
    rec = case.problems[0]
    po = orc.Problem(rec).hydrostatic(2e7)
    g = nks.Grid([rec])
    pg = g.hydrostatic(2e7).cpu().numpy()
    assert np.max(np.abs(pg - po)) <= 1e-13 * po.max()


def _gpu_jac(nks, g, p, pn, dt):
    return g.jacobian(g.from_numpy(p), g.from_numpy(pn), None, dt, 1)


ONE_LEVEL = [
    dict(nx=37, ny=29, nz=1, px=4, py=3, overlap=(1,)),
    dict(nx=40, ny=40, nz=1, px=3, py=5, overlap=(2,)),
    dict(nx=11, ny=9, nz=8, px=2, py=2, pz=3, overlap=(1,), gravity=True),
    dict(nx=8, ny=8, nz=1, px=8, py=8, overlap=(0,)),     # one cell per box
    dict(nx=20, ny=7, nz=1, px=1, py=1, overlap=(1,)),    # one subdomain
    # 3D boxes of more than 64 (y, z) rows: swept in slabs of z planes,
    # one wavefront each (9x9x9 extended boxes: two slabs; 8x7x31: four)
    dict(nx=16, ny=16, nz=16, px=2, py=2, pz=2, overlap=(1,), gravity=True),
    dict(nx=14, ny=12, nz=60, px=2, py=2, pz=2, overlap=(1,)),
    dict(nx=4, ny=4, nz=4, px=4, py=4, pz=4, overlap=(0,)),   # one cell per 3D box
    dict(nx=3, ny=12, nz=14, px=3, py=1, pz=1, overlap=(0,)),  # rows of one cell, three slabs
]


@pytest.mark.parametrize("cfg", ONE_LEVEL)
@pytest.mark.parametrize("variant", ["left_ras", "as", "right_ras"])
def test_one_level_apply_parity(nks, orc, cfg, variant):
    say("one-level", cfg, variant)
    case = S.small_case(variant=variant, **cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 5)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    mo = orc.Multilevel(rec, Jo, case.solver)
    g = nks.Grid([rec])
    J = _gpu_jac(nks, g, p, pn, case.dt)
    M = nks.Ras(J, case.solver)
    r = np.random.default_rng(7).standard_normal(op.N)
    zo = mo.apply(r)
    zg = M.apply(g.from_numpy(r)).cpu().numpy()
    assert np.max(np.abs(zg - zo)) <= 1e-11 * np.max(np.abs(zo))
    # left-RAS writes every owned cell exactly once: bitwise repeatable
    zg2 = M.apply(g.from_numpy(r)).cpu().numpy()
    assert np.array_equal(zg, zg2)


ILUK = [
    dict(nx=37, ny=29, nz=1, px=4, py=3, overlap=(1,), fill=1),
    dict(nx=24, ny=20, nz=1, px=2, py=2, overlap=(2,), fill=2, variant="as"),
    dict(nx=11, ny=9, nz=8, px=2, py=2, pz=3, overlap=(1,), gravity=True, fill=1),
    dict(nx=40, ny=36, nz=1, px=4, py=4, levels=2, overlap=(1, 1), fill=1, coarse_rtol=0.0, coarse_maxit=4),
]


@pytest.mark.parametrize("variant", ["left_ras", "as"])
def test_full_fill_is_the_exact_lu_subsolve(nks, orc, variant):
    # exact (LU) subdomain solves (Section 4.2 compares ILU(k) with LU): with
    # boxes at most 4 cells wide, ILU(4) keeps every entry of each box's LU
    # band, so the library's ILU(4) apply equals the oracle's dense-LU apply
    cfg = dict(nx=10, ny=8, px=5, py=2, overlap=(1,), seed=3, variant=variant)
    say("ILU(4) as LU", cfg)
    case = S.small_case(fill=4, **cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 23)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    r = np.random.default_rng(8).standard_normal(op.N)
    zo = orc.Multilevel(rec, Jo, S.with_solver(case, subsolve="lu", fill=0).solver).apply(r)
    g = nks.Grid([rec])
    M = nks.Ras(_gpu_jac(nks, g, p, pn, case.dt), case.solver)
    zg = M.apply(g.from_numpy(r)).cpu().numpy()
    assert np.max(np.abs(zg - zo)) <= 1e-10 * np.max(np.abs(zo))


@pytest.mark.parametrize("cfg", ILUK)
def test_iluk_apply_parity(nks, orc, cfg):
    # ILU(k) subdomain solves: the oracle factors each box on its own
    # level-of-fill pattern; the library uses the stencil's pattern on an
    # unbounded grid restricted to the box
    say("ILU(k)", cfg)
    case = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 4)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    zo = orc.Multilevel(rec, Jo, case.solver).apply(np.sin(np.arange(op.N)))
    g = nks.Grid([rec])
    M = nks.Ras(_gpu_jac(nks, g, p, pn, case.dt), case.solver)
    zg = M.apply(g.from_numpy(np.sin(np.arange(op.N)))).cpu().numpy()
    assert np.max(np.abs(zg - zo)) <= 1e-10 * np.max(np.abs(zo))
    # the fill changes the preconditioner: ILU(0) gives a different result
    z0 = orc.Multilevel(rec, Jo, S.small_case(**dict(cfg, fill=0)).solver).apply(np.sin(np.arange(op.N)))
    assert np.max(np.abs(z0 - zo)) > 1e-6 * np.max(np.abs(zo))


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-5), ("bf16", 5e-2)])
@pytest.mark.parametrize("cfg", [dict(nx=12, ny=10, nz=8, px=2, py=2, pz=2, overlap=(1,), gravity=True),
                                 dict(nx=16, ny=16, nz=16, px=2, py=2, pz=2, overlap=(1,), gravity=True)])
def test_mixed_precision_apply_error(nks, orc, prec, tol, cfg):
    case = S.small_case(precision=prec, **cfg)
    case64 = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 6)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    zo = orc.Multilevel(rec, Jo, case64.solver).apply(np.ones(op.N))
    g = nks.Grid([rec])
    M = nks.Ras(_gpu_jac(nks, g, p, pn, case.dt), case.solver)
    zg = M.apply(g.from_numpy(np.ones(op.N))).cpu().numpy()
    err = np.max(np.abs(zg - zo)) / np.max(np.abs(zo))
    say(prec, "relative error of the one-level apply vs FP64 oracle", err)
    assert err <= tol


@pytest.mark.parametrize("prec,tol,cfg", [
    # 17^3 extended boxes: 17 (y) rows per z plane, three planes per slab, six
    # slabs (an eight-wavefront workgroup); the BF16 runs (16 B per cell) fit
    # in LDS, the FP32 ones one run at a time
    ("bf16", 5e-2, dict(nx=32, ny=32, nz=32, px=2, py=2, pz=2, overlap=(1,), gravity=True)),
    ("fp32", 2e-5, dict(nx=32, ny=32, nz=32, px=2, py=2, pz=2, overlap=(1,), gravity=True)),
    # 11 x 11 x 31 extended boxes: five planes per slab, seven slabs; FP32 and
    # BF16 hold both runs, FP64 takes the hyperplane kernel
    ("fp32", 2e-5, dict(nx=20, ny=20, nz=60, px=2, py=2, pz=2, overlap=(1,))),
    ("bf16", 5e-2, dict(nx=20, ny=20, nz=60, px=2, py=2, pz=2, overlap=(1,))),
    ("fp64", 1e-11, dict(nx=20, ny=20, nz=60, px=2, py=2, pz=2, overlap=(1,))),
])
def test_rows3d_many_slabs_apply_parity(nks, orc, prec, tol, cfg):
    case = S.small_case(precision=prec, **cfg)
    case64 = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 12)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    r = np.cos(0.37 * np.arange(op.N))
    zo = orc.Multilevel(rec, Jo, case64.solver).apply(r)
    g = nks.Grid([rec])
    M = nks.Ras(_gpu_jac(nks, g, p, pn, case.dt), case.solver)
    zg = M.apply(g.from_numpy(r)).cpu().numpy()
    form = M.level_sweep(0)
    err = np.max(np.abs(zg - zo)) / np.max(np.abs(zo))
    say(prec, cfg["nx"], cfg["nz"], "form", form, "relative error vs FP64 oracle", err)
    assert err <= tol
    if prec != "fp64":
        assert form[0] == "rows3d"
    zg2 = M.apply(g.from_numpy(r)).cpu().numpy()
    assert np.array_equal(zg, zg2)


GALERKIN = [
    dict(nx=40, ny=36, nz=1, levels=3, interp_order=2),
    dict(nx=41, ny=27, nz=1, levels=2, interp_order=1),
    dict(nx=32, ny=24, nz=1, levels=2, interp_order=3),
    dict(nx=16, ny=12, nz=10, levels=3, interp_order=2, gravity=True),
    # odd sizes under third order: the short last coarse cell at its centroid
    dict(nx=41, ny=27, nz=1, levels=3, interp_order=3),
    # coarse-to-fine ratios 4, 8 and 16 (Section 4.2), sizes they do not divide
    dict(nx=64, ny=50, nz=1, levels=2, interp_order=2, ratio=4),
    dict(nx=70, ny=45, nz=1, levels=2, interp_order=3, ratio=8),
    dict(nx=100, ny=64, nz=1, levels=2, interp_order=1, ratio=16),
    dict(nx=20, ny=18, nz=13, levels=2, interp_order=2, ratio=4, gravity=True),
]


@pytest.mark.parametrize("cfg", GALERKIN)
def test_galerkin_and_transfer_parity(nks, orc, cfg):
    say("galerkin", cfg)
    case = S.small_case(px=2, py=2, pz=1, overlap=(1, 1, 1), **cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 8)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    mo = orc.Multilevel(rec, Jo, case.solver)
    g = nks.Grid([rec])
    M = nks.Ras(_gpu_jac(nks, g, p, pn, case.dt), case.solver)
    for lev in range(1, cfg["levels"]):
        Ao = mo.level_matrix(lev).dense()
        rp, ci, v = M.level_export(lev)
        Ag = orc.CSR(rp, ci, v).dense()
        assert Ag.shape == Ao.shape
        assert np.max(np.abs(Ag - Ao)) <= 1e-12 * np.max(np.abs(Ao)), lev
    n0 = op.N
    P = mo.level_prolong(0).dense()
    r = np.random.default_rng(3).standard_normal(n0)
    rc = M.restrict(0, g.from_numpy(r)).cpu().numpy()
    assert np.allclose(rc, P.T @ r, rtol=1e-13, atol=1e-13 * np.abs(rc).max())
    ec = np.random.default_rng(4).standard_normal(P.shape[1])
    z0 = np.random.default_rng(5).standard_normal(n0)
    zf = g.from_numpy(z0)
    import torch
    M.prolong_add(0, torch.as_tensor(ec, device=zf.device), zf)
    assert np.allclose(zf.cpu().numpy(), z0 + P @ ec, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("cycle", ["vcycle", "left_kaskade", "right_kaskade", "additive",
                                   "coarse_only"])
def test_multilevel_apply_parity(nks, orc, cycle):
    # a fixed number of coarse GMRES iterations (rtol 0) so both sides take
    # the same steps
    cfg = dict(nx=48, ny=40, nz=1, px=4, py=4, levels=2, overlap=(2, 1), cycle=cycle,
               coarse_rtol=0.0, coarse_maxit=6)
    say("multilevel", cycle)
    case = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 9)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    zo = orc.Multilevel(rec, Jo, case.solver).apply(np.sin(np.arange(op.N)))
    g = nks.Grid([rec])
    M = nks.Ras(_gpu_jac(nks, g, p, pn, case.dt), case.solver)
    zg = M.apply(g.from_numpy(np.sin(np.arange(op.N)))).cpu().numpy()
    assert np.max(np.abs(zg - zo)) <= 1e-9 * np.max(np.abs(zo))


@pytest.mark.parametrize("cycle,mu,nu,levels", [("vcycle", 1, 2, 2), ("left_kaskade", 1, 1, 2),
                                               ("vcycle", 1, 1, 3)])
def test_multilevel_transpose_apply_parity(nks, orc, cycle, mu, nu, levels):
    # M^{-T} of the multilevel preconditioner: the transposed composition
    # (smoothing counts swapped, Kaskade sides exchanged) with a fixed number
    # of coarse GMRES iterations on A_0^T, against the oracle's transposed cycle
    cfg = dict(nx=48, ny=40, nz=1, px=4, py=4, levels=levels, overlap=(2,) + (1,) * (levels - 1),
               cycle=cycle, mu=mu, nu=nu, coarse_rtol=0.0, coarse_maxit=6)
    say("multilevel transpose", cycle, mu, nu, levels)
    case = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 19)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    r = np.cos(0.7 * np.arange(op.N))
    zo = orc.Multilevel(rec, Jo, case.solver).apply_transpose(r)
    g = nks.Grid([rec])
    M = nks.Ras(_gpu_jac(nks, g, p, pn, case.dt), case.solver)
    zg = M.apply_transpose(g.from_numpy(r)).cpu().numpy()
    assert np.max(np.abs(zg - zo)) <= 1e-9 * np.max(np.abs(zo))


@pytest.mark.parametrize("ratio,order", [(4, 2), (8, 2), (16, 3)])
def test_multilevel_ratio_apply_parity(nks, orc, ratio, order):
    # two-level V-cycle with coarse-to-fine ratio r, fixed coarse iterations
    cfg = dict(nx=96, ny=80, nz=1, px=4, py=4, levels=2, overlap=(2, 1), ratio=ratio,
               interp_order=order, coarse_rtol=0.0, coarse_maxit=5)
    say("multilevel ratio", ratio, "order", order)
    case = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 21)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    r = np.sin(0.37 * np.arange(op.N))
    zo = orc.Multilevel(rec, Jo, case.solver).apply(r)
    g = nks.Grid([rec])
    M = nks.Ras(_gpu_jac(nks, g, p, pn, case.dt), case.solver)
    zg = M.apply(g.from_numpy(r)).cpu().numpy()
    assert np.max(np.abs(zg - zo)) <= 1e-9 * np.max(np.abs(zo))


def test_multilevel_many_coarse_boxes_parity(nks, orc):
    # 17 x 17 = 289 boxes on each level, more than the 256 CUs of the device:
    # the box kernels run in several rounds of workgroups
    cfg = dict(nx=120, ny=120, nz=1, px=17, py=17, levels=2, overlap=(1, 1),
               coarse_rtol=0.0, coarse_maxit=6)
    say("multilevel, 289 coarse boxes")
    case = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 12)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    r = np.sin(0.3 * np.arange(op.N))
    zo = orc.Multilevel(rec, Jo, case.solver).apply(r)
    g = nks.Grid([rec])
    M = nks.Ras(_gpu_jac(nks, g, p, pn, case.dt), case.solver)
    zg = M.apply(g.from_numpy(r)).cpu().numpy()
    assert np.max(np.abs(zg - zo)) <= 1e-9 * np.max(np.abs(zo))


@pytest.mark.parametrize("cfg", [
    dict(nx=16, ny=16, nz=8, px=2, py=2, pz=2, levels=3, overlap=(1, 1, 1)),
    # fine boxes of 17^3 extended cells (hyperplane kernel), coarse boxes of
    # 9^3 (the row sweep in two slabs of z planes)
    dict(nx=32, ny=32, nz=32, px=2, py=2, pz=2, levels=2, overlap=(1, 1)),
])
def test_multilevel_3d_apply_parity(nks, orc, cfg):
    cfg = dict(cfg, gravity=True, coarse_rtol=0.0, coarse_maxit=4, kv_ratio=0.1)
    case = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 10)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    r = np.cos(np.arange(op.N))
    zo = orc.Multilevel(rec, Jo, case.solver).apply(r)
    g = nks.Grid([rec])
    M = nks.Ras(_gpu_jac(nks, g, p, pn, case.dt), case.solver)
    zg = M.apply(g.from_numpy(r)).cpu().numpy()
    assert np.max(np.abs(zg - zo)) <= 1e-9 * np.max(np.abs(zo))


@pytest.mark.parametrize("levels,flex", [(1, False), (2, True)])
def test_gmres_parity(nks, orc, levels, flex):
    case = S.small_case(nx=40, ny=32, px=4, py=4, levels=levels, overlap=(1, 1))
    rec = case.problems[0]
    op = orc.Problem(rec)
    p, pn, _ = _state(op, 11)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    b = np.random.default_rng(12).standard_normal(op.N)
    mo = orc.Multilevel(rec, Jo, case.solver)
    xo, its_o, _, _ = orc.gmres(Jo, b, M=mo, rtol=1e-10, atol=0.0, flexible=flex)
    g = nks.Grid([rec])
    J = _gpu_jac(nks, g, p, pn, case.dt)
    M = nks.Ras(J, case.solver)
    xg, st = nks.gmres_solve(J, M, g.from_numpy(b), rtol=1e-10, atol=0.0, flexible=flex)
    xg = xg.cpu().numpy()
    say("gmres its gpu", st["iterations"], "oracle", its_o)
    xd = np.linalg.solve(Jo.dense(), b)
    assert np.linalg.norm(xg - xd) <= 1e-8 * np.linalg.norm(xd)
    assert np.linalg.norm(xo - xd) <= 1e-8 * np.linalg.norm(xd)
    assert abs(st["iterations"] - its_o) <= 2


def _run_steps(nks, orc, case, nsteps, gpu=True):
    recs = case.problems
    if gpu:
        g = nks.Grid(recs)
        p = g.initial_pressure()
        hist = [p.clone()]
        stats = []
        for n in range(nsteps):
            order = 1 if n == 0 else 2
            pn = hist[-1]
            pnm1 = hist[-2] if len(hist) > 1 else hist[-1]
            p = pn.clone()
            st = g.newton_step(p, pn, pnm1, case.dt, order, case.solver)
            hist.append(p.clone())
            stats.append(st)
        return [h.cpu().numpy() for h in hist], stats, g
    out = orc.simulate(case, nsteps=nsteps)
    return out


# Parity runs converge Newton to eps_r = 1e-8 with an absolute floor of 1e-6:
# in FP64 the residual of these workloads cannot drop below ~3e-7 (rounding
# of the ~5e4 accumulation and flux terms), which the oracle shows too.
PARITY = dict(eps_r=1e-8, eps_a=1e-6)


def test_newton_2d_32_end_to_end(nks, orc):
    case = S.with_solver(S.case_2d_32(), **PARITY)
    say("newton 2d 32x32")
    hist_g, st_g, g = _run_steps(nks, orc, case, 2)
    (hist_o, st_o), = _run_steps(nks, orc, case, 2, gpu=False)
    op = orc.Problem(case.problems[0])
    for n in range(1, 3):
        dpg = hist_g[n] - hist_g[0]
        dpo = hist_o[n] - hist_o[0]
        err = np.linalg.norm(dpg - dpo) / np.linalg.norm(dpo)
        order = 1 if n == 1 else 2
        Fo = op.residual(hist_g[n], hist_g[n - 1], hist_g[n - 2] if n > 1 else hist_g[n - 1],
                         case.dt, order)
        F0 = op.residual(hist_g[n - 1], hist_g[n - 1], hist_g[n - 2] if n > 1 else hist_g[n - 1],
                         case.dt, order)
        rel = np.linalg.norm(Fo) / np.linalg.norm(F0)
        say("step", n, "dp err", err, "rel res", rel, "gpu", st_g[n - 1], "oracle", st_o[n - 1])
        assert err <= 1e-6
        assert rel <= 1e-8 or np.linalg.norm(Fo) <= PARITY["eps_a"]
        assert abs(st_g[n - 1]["newton_its"] - st_o[n - 1]["newton_its"]) <= 1


def test_newton_two_level_small(nks, orc):
    case = S.small_case(nx=48, ny=40, px=4, py=4, levels=2, overlap=(2, 1), rate=3e-3,
                        nsteps=2, dt=5 * S.DAY, **PARITY)
    hist_g, st_g, g = _run_steps(nks, orc, case, 2)
    (hist_o, st_o), = _run_steps(nks, orc, case, 2, gpu=False)
    for n in range(1, 3):
        dpg, dpo = hist_g[n] - hist_g[0], hist_o[n] - hist_o[0]
        err = np.linalg.norm(dpg - dpo) / np.linalg.norm(dpo)
        say("two-level step", n, err, st_g[n - 1]["linear_its"], st_o[n - 1]["linear_its"])
        assert err <= 1e-6


def test_batched_equals_unbatched(nks, orc):
    recs = [S.small_case(nx=n, ny=m, seed=s, rate=2e-3).problems[0]
            for n, m, s in [(24, 20, 1), (17, 31, 2), (32, 32, 3)]]
    settings = S.SolverSettings(px=3, py=3, levels=2, overlap=(1, 1), **PARITY)
    case = S.Case("batch", recs, S.DAY, 2, settings)
    hist_b, st_b, gb = _run_steps(nks, orc, case, 2)
    for k, rec in enumerate(recs):
        single = S.Case("one", [rec], S.DAY, 2, settings)
        hist_s, st_s, gs = _run_steps(nks, orc, single, 2)
        for n in range(3):
            part = hist_b[n][gb.offsets[k]:gb.offsets[k + 1]]
            assert np.array_equal(part, hist_s[n]), (k, n)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 2e-5)])
def test_batched_uneven_tile_apply_parity(nks, orc, precision, tol):
    # uneven reservoirs in one batch, boxes set by a tile edge, two-level V-cycle
    # with a fixed number of coarse iterations; each reservoir against its own oracle
    recs = [S.small_case(nx=n, ny=m, seed=s, rate=2e-3).problems[0]
            for n, m, s in [(37, 29, 1), (64, 50, 2), (20, 20, 3), (9, 33, 4)]]
    settings = S.SolverSettings(px=1, py=1, tile=(12, 12, 0), levels=2, overlap=(2, 1),
                                coarse_rtol=0.0, coarse_maxit=5, precision=precision)
    settings64 = S.SolverSettings(px=1, py=1, tile=(12, 12, 0), levels=2, overlap=(2, 1),
                                  coarse_rtol=0.0, coarse_maxit=5)
    g = nks.Grid(recs)
    ps, pns, Js, rs = [], [], [], []
    for k, rec in enumerate(recs):
        op = orc.Problem(rec)
        p, pn, _ = _state(op, 20 + k)
        ps.append(p)
        pns.append(pn)
        rs.append(np.cos(np.arange(op.N) * (k + 1)))
    p = g.from_numpy(np.concatenate(ps))
    pn = g.from_numpy(np.concatenate(pns))
    J = g.jacobian(p, pn, pn, S.DAY, 1)
    M = nks.Ras(J, settings)
    zg = M.apply(g.from_numpy(np.concatenate(rs))).cpu().numpy()
    for k, rec in enumerate(recs):
        op = orc.Problem(rec)
        Jo = op.jacobian(ps[k], pns[k], pns[k], S.DAY, 1)
        zo = orc.Multilevel(rec, Jo, settings64).apply(rs[k])
        part = zg[g.offsets[k]:g.offsets[k + 1]]
        err = np.max(np.abs(part - zo)) / np.max(np.abs(zo))
        say("reservoir", k, precision, "relative error", err)
        assert err <= tol, (k, err)


def test_determinism(nks, orc):
    case = S.small_case(nx=40, ny=40, px=4, py=4, levels=2, overlap=(1, 1), nsteps=1)
    h1, _, _ = _run_steps(nks, orc, case, 1)
    h2, _, _ = _run_steps(nks, orc, case, 1)
    assert np.array_equal(h1[-1], h2[-1])


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 2e-5), ("bf16", 5e-2)])
def test_many_small_boxes_apply_parity(nks, orc, precision, tol):
    # 32 x 32 = 1024 boxes per level, more than four per CU: the sweeps run
    # one wavefront per box, staging a box's lower factors for the forward
    # sweep and then its upper factors in their place; one level (5-point)
    # and two levels (21-point coarse operator, fixed coarse iterations)
    for levels in (1, 2):
        cfg = dict(nx=128, ny=128, nz=1, px=32, py=32, levels=levels, overlap=(1, 1), coarse_rtol=0.0,
                   coarse_maxit=4, seed=31)
        case = S.small_case(**cfg)
        case64 = case
        case = S.with_solver(case, precision=precision)
        say("many small boxes", precision, "levels", levels)
        rec = case.problems[0]
        op = orc.Problem(rec)
        p, pn, _ = _state(op, 31)
        Jo = op.jacobian(p, pn, pn, case.dt, 1)
        r = np.sin(0.29 * np.arange(op.N))
        zo = orc.Multilevel(rec, Jo, case64.solver).apply(r)
        g = nks.Grid([rec])
        M = nks.Ras(_gpu_jac(nks, g, p, pn, case.dt), case.solver)
        zg = M.apply(g.from_numpy(r)).cpu().numpy()
        err = np.max(np.abs(zg - zo)) / np.max(np.abs(zo))
        say("  relative error", err)
        assert err <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 2e-5), ("bf16", 5e-2)])
@pytest.mark.parametrize("variant", ["left_ras", "as", "right_ras"])
def test_packed_sweep_apply_parity(nks, orc, precision, variant, tol):
    # Small boxes (4 x 4 owned cells, ragged where the side is not a
    # multiple of 4, clipped at the reservoir edges) in three reservoirs of
    # different shapes on one grid: the level sweeps pack several boxes into
    # one wavefront, a group never spanning two reservoirs.  Each
    # reservoir's apply is checked against the oracle; the kernel form used
    # is reported and the packed form must be among them.
    recs, cases = [], []
    for k, (nx, ny) in enumerate([(131, 97), (61, 75), (40, 40)]):
        c = S.small_case(nx=nx, ny=ny, nz=1, tile=(4, 4, 0), levels=2, overlap=(1, 1), coarse_rtol=0.0,
                         coarse_maxit=3, seed=41 + k, variant=variant)
        cases.append(c)
        recs.append(c.problems[0])
    s = S.with_solver(cases[0], precision=precision).solver
    say("packed sweep", precision, variant)
    g = nks.Grid(recs)
    states = []
    for rec, c in zip(recs, cases):
        op = orc.Problem(rec)
        states.append((op,) + _state(op, 7)[:2])
    p = np.concatenate([st[1] for st in states])
    pn = np.concatenate([st[2] for st in states])
    M = nks.Ras(_gpu_jac(nks, g, p, pn, cases[0].dt), s)
    r = np.concatenate([np.sin(0.29 * np.arange(st[0].N) + k) for k, st in enumerate(states)])
    zg = M.apply(g.from_numpy(r)).cpu().numpy()
    forms = [M.level_sweep(l) for l in range(2)]
    say("  forms", forms)
    assert "packed" in [f for f, _ in forms]
    off = 0
    for k, (rec, c, st) in enumerate(zip(recs, cases, states)):
        op = st[0]
        Jo = op.jacobian(st[1], st[2], st[2], c.dt, 1)
        zo = orc.Multilevel(rec, Jo, c.solver).apply(r[off:off + op.N])
        err = np.max(np.abs(zg[off:off + op.N] - zo)) / np.max(np.abs(zo))
        say("  reservoir", k, "relative error", err)
        assert err <= tol
        off += op.N
