"""GPU parity of the outer-face boundary conditions (Section 2: p = p^D on
Dirichlet faces, v.n = q^N on Neumann faces) against the oracle: residual,
Jacobian, dF/dlnK and a strongly nonlinear Dirichlet flood through Newton."""
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


BC_CASES = [
    # 2D: Dirichlet inflow and outflow on the x faces, Neumann on both y faces
    dict(nx=37, ny=23, nz=1, seed=1, bc=((0, 1, 22e6), (1, 1, 19e6), (2, 2, -2e-6), (3, 2, 1e-6))),
    # 3D with gravity: Dirichlet top, Neumann bottom, Dirichlet -y, the rest closed
    dict(nx=9, ny=7, nz=5, seed=2, gravity=True, kv_ratio=0.1,
         bc=((4, 1, 20e6), (5, 2, 3e-7), (2, 1, 20.3e6))),
    # every face Dirichlet, no wells
    dict(nx=12, ny=10, nz=4, seed=3, rate=0.0,
         bc=tuple((f, 1, 20e6 + 1e5 * f) for f in range(6))),
]


@pytest.mark.parametrize("cfg", BC_CASES)
def test_boundary_residual_jacobian_dlogk_parity(nks, orc, cfg):
    say("boundary residual/jacobian", cfg)
    case = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    rng = np.random.default_rng(cfg["seed"])
    base = op.initial_pressure()
    p = base + 3e4 * rng.standard_normal(op.N)
    pn = base + 1e4 * rng.standard_normal(op.N)
    Fo = op.residual(p, pn, pn, case.dt, 1)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    g = nks.Grid([rec])
    dp, dpn = g.from_numpy(p), g.from_numpy(pn)
    Fg = g.residual(dp, dpn, dpn, case.dt, 1).cpu().numpy()
    assert np.max(np.abs(Fg - Fo)) <= 1e-12 * np.max(np.abs(Fo))
    # the boundary terms are present: closing the faces changes F
    closed = orc.Problem(S.small_case(**dict(cfg, bc=())).problems[0]).residual(p, pn, pn, case.dt, 1)
    assert np.max(np.abs(closed - Fo)) > 1e-6 * np.max(np.abs(Fo))
    J = g.jacobian(dp, dpn, None, case.dt, 1)
    rp, ci, v = J.export_csr()
    assert np.array_equal(rp, Jo.rp) and np.array_equal(ci, Jo.ci)
    rowmax = np.repeat(np.maximum.reduceat(np.abs(Jo.v), Jo.rp[:-1]), np.diff(Jo.rp))
    assert np.all(np.abs(v - Jo.v) <= 1e-12 * rowmax)
    lam = rng.standard_normal(op.N)
    want = op.residual_dlogk_t(p, lam)
    got = g.residual_dlogk_t(dp, g.from_numpy(lam)).cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


def test_acentric_from_boiling_point_parity(nks, orc):
    # omega from Tb (Section 2's correlation) on both sides, at 20 MPa where Z
    # is sensitive to it; a different omega changes the residual
    from dataclasses import replace
    case = S.small_case(nx=20, ny=17, seed=6, bc=((0, 1, 21e6),))
    rec = case.problems[0]
    rec.fluid = replace(rec.fluid, Tc=190.58, pc=4.604e6, Tb=111.67, omega=0.5)
    op = orc.Problem(rec)
    rng = np.random.default_rng(6)
    p = 20e6 + 3e4 * rng.standard_normal(op.N)
    pn = 20e6 + 1e4 * rng.standard_normal(op.N)
    Fo = op.residual(p, pn, pn, case.dt, 1)
    g = nks.Grid([rec])
    Fg = g.residual(g.from_numpy(p), g.from_numpy(pn), g.from_numpy(pn), case.dt, 1).cpu().numpy()
    assert np.max(np.abs(Fg - Fo)) <= 1e-12 * np.max(np.abs(Fo))
    rec.fluid = replace(rec.fluid, Tb=None)
    Fw = orc.Problem(rec).residual(p, pn, pn, case.dt, 1)
    assert np.max(np.abs(Fw - Fo)) > 1e-8 * np.max(np.abs(Fo))


def test_bad_boundary_rejected(nks):
    rec = S.small_case(nx=6, ny=5, bc=((0, 1, -5.0),)).problems[0]
    with pytest.raises(Exception, match="p\\^D"):
        nks.Grid([rec])


PARITY = dict(eps_r=1e-8, eps_a=1e-6)


@pytest.mark.parametrize("levels", [1, 2])
def test_dirichlet_flood_newton_parity(nks, orc, levels):
    # strongly nonlinear: a tenfold pressure rise enters through the -y face
    case = S.case_2d_flood(32, 28, 2, 2)
    case = S.with_solver(case, levels=levels, overlap=(1,) * levels, **PARITY)
    say("flood newton", levels)
    g = nks.Grid(case.problems)
    p = g.initial_pressure()
    hist_g, st_g = [p.cpu().numpy()], []
    for n in range(3):
        order = 1 if n == 0 else 2
        pn = g.from_numpy(hist_g[-1])
        pnm1 = g.from_numpy(hist_g[-2] if n > 0 else hist_g[-1])
        p = pn.clone()
        st_g.append(g.newton_step(p, pn, pnm1, case.dt, order, case.solver))
        hist_g.append(p.cpu().numpy())
    (hist_o, st_o), = orc.simulate(case, nsteps=3)
    for n in range(1, 4):
        err = np.linalg.norm((hist_g[n] - hist_g[0]) - (hist_o[n] - hist_o[0])) / np.linalg.norm(hist_o[n] - hist_o[0])
        say("step", n, "err", err, "newton", st_g[n - 1]["newton_its"], st_o[n - 1]["newton_its"])
        assert err <= 1e-6
        assert abs(st_g[n - 1]["newton_its"] - st_o[n - 1]["newton_its"]) <= 1
    assert st_o[0]["newton_its"] >= 3          # the regime is nonlinear


@pytest.mark.parametrize("lag,levels,flood", [(3, 1, True), (100, 2, False)])
def test_lagged_factorisation_newton_parity(nks, orc, lag, levels, flood):
    # subdomain factors refreshed every lag Newton iterations on both sides
    if flood:
        case = S.case_2d_flood(32, 28, 2, 2)
    else:
        case = S.small_case(nx=32, ny=28, px=2, py=2, rate=5e-2, dt=20 * S.DAY)
    case = S.with_solver(case, lag=lag, levels=levels, overlap=(1,) * levels, **PARITY)
    say("lagged newton", lag, levels)
    g = nks.Grid(case.problems)
    hist_g, st_g = [g.initial_pressure().cpu().numpy()], []
    for n in range(2):
        order = 1 if n == 0 else 2
        pn = g.from_numpy(hist_g[-1])
        pnm1 = g.from_numpy(hist_g[-2] if n > 0 else hist_g[-1])
        p = pn.clone()
        st_g.append(g.newton_step(p, pn, pnm1, case.dt, order, case.solver))
        hist_g.append(p.cpu().numpy())
    (hist_o, st_o), = orc.simulate(case, nsteps=2)
    for n in range(1, 3):
        err = np.linalg.norm((hist_g[n] - hist_g[0]) - (hist_o[n] - hist_o[0])) / np.linalg.norm(hist_o[n] - hist_o[0])
        say("step", n, "err", err, "its", st_g[n - 1]["newton_its"], st_o[n - 1]["newton_its"],
            st_g[n - 1]["linear_its"], st_o[n - 1]["linear_its"])
        assert err <= 1e-6
        assert abs(st_g[n - 1]["newton_its"] - st_o[n - 1]["newton_its"]) <= 1
