"""Pins of the oracle's rediscretised coarse operators (the alternative to
the Galerkin product for the coarse matrices of Section 3.2): the upscaled
coarse problem (mean permeability and porosity, r times the cell size), its
Jacobian at the coarsened state, and what fixes them independently of the
code: closed forms of the coarse transmissibility and pore volume, the
relation to the first-order Galerkin product on a homogeneous medium at a
uniform state, and Newton reaching the same solution as with Galerkin
levels (the preconditioner does not move the fixed point)."""
import numpy as np
import pytest

import synthetic as S


def _jac(orc, p_amp=0.0, **kw):
    case = S.small_case(**kw)
    rec = case.problems[0]
    prob = orc.Problem(rec)
    p0 = prob.initial_pressure()
    p = p0 + p_amp * np.random.default_rng(4).standard_normal(prob.N)
    return case, rec, prob, p, prob.jacobian(p, p0, p0, case.dt, 1)


@pytest.mark.parametrize("ratio,dims", [(2, (8, 6, 1)), (4, (8, 12, 1)), (2, (4, 6, 8))])
def test_homogeneous_rediscretisation_closed_form(orc, ratio, dims):
    # homogeneous K, uniform p, no gravity or wells: the fine Jacobian is
    # c I + T lambda L_h.  Piecewise-constant (first-order) Galerkin sums the
    # r^(d-1) fine faces across a coarse face, while the rediscretised coarse
    # face carries K (r h)^(d-1)/(r h) = r^(d-2) T: its couplings are the
    # Galerkin ones divided by r; both keep the summed accumulation c r^d
    case, rec, prob, p, J = _jac(orc, nx=dims[0], ny=dims[1], nz=dims[2], sigma=0.0, rate=0.0, px=1, py=1,
                                 levels=2, overlap=(1, 1), ratio=ratio, interp_order=1)
    rec.phi[:] = 0.2
    prob = orc.Problem(rec)
    J = prob.jacobian(p, p, p, case.dt, 1)
    g = orc.Multilevel(rec, J, case.solver).level_matrix(1).dense()
    rs = S.with_solver(case, coarse_op="rediscretised").solver
    r = orc.Multilevel(rec, J, rs, state=(p, case.dt, 1)).level_matrix(1).dense()
    off = ~np.eye(g.shape[0], dtype=bool)
    assert np.allclose(r[off], g[off] / ratio, rtol=1e-12, atol=1e-12 * np.abs(g).max())
    # accumulation: the row sums (fluxes cancel) are the summed pore volumes' terms
    assert np.allclose(r.sum(1), g.sum(1), rtol=1e-12)
    assert abs(g.sum(1)[0] - ratio ** (3 if dims[2] > 1 else 2) * J.dense().sum(1)[0]) < 1e-9 * abs(g.sum(1)[0])


def test_coarse_problem_upscaling(orc):
    case, rec, prob, p, J = _jac(orc, nx=8, ny=4, sigma=1.5, seed=9, px=1, py=1, levels=2, overlap=(1, 1))
    rs = S.with_solver(case, coarse_op="rediscretised").solver
    mg = orc.Multilevel(rec, J, rs, state=(p, case.dt, 1))
    A = mg.level_matrix(1).dense()
    # coarse cell (0,0) and its +x neighbour (1,0): mean permeabilities of the
    # 2x2 children, cells 20 m wide (2D thickness stays 10 m)
    kx = rec.kx.reshape(4, 8)
    k0, k1 = kx[0:2, 0:2].mean(), kx[0:2, 2:4].mean()
    T = (20.0 * 10.0) / (20.0 / (2 * k0) + 20.0 / (2 * k1))
    pc = p.reshape(4, 8)[0:2, 0:4].reshape(2, 2, 2).mean(axis=(0, 2))
    fl = rec.fluid
    # coupling of coarse cell 0 to cell 1 = -T lambda_up(p_c) (no gravity)
    import oracle
    a, b, _ = oracle.pr_params(fl)
    lam = [pi / oracle.pr_z_ab(a, b, fl.T, fl.R, pi)[0] / fl.mu for pi in pc]
    up = 0 if pc[0] >= pc[1] else 1
    dm1 = oracle.pr_z_ab(a, b, fl.T, fl.R, pc[1])
    m1p = 1.0 / dm1[0] - pc[1] * dm1[1] / dm1[0] ** 2
    expect = -T * lam[up] + (T * m1p / fl.mu * (pc[0] - pc[1]) if up == 1 else 0.0)
    assert abs(A[0, 1] - expect) <= 1e-10 * abs(expect), (A[0, 1], expect)


def test_sizes_the_ratio_does_not_divide_are_refused(orc):
    case, rec, prob, p, J = _jac(orc, nx=9, ny=8, px=1, py=1, levels=2, overlap=(1, 1))
    rs = S.with_solver(case, coarse_op="rediscretised").solver
    with pytest.raises(ValueError):
        orc.Multilevel(rec, J, rs, state=(p, case.dt, 1))


@pytest.mark.parametrize("levels", [2, 3])
def test_newton_reaches_the_galerkin_solution(orc, levels):
    case = S.small_case(nx=32, ny=24, px=4, py=3, levels=levels, overlap=(1,) * levels, rate=3e-3, seed=5,
                        eps_r=1e-10, eps_a=1e-12, dt=5 * S.DAY)
    rec = case.problems[0]
    prob = orc.Problem(rec)
    p0 = prob.initial_pressure()
    pg, sg = orc.newton_step(prob, case.solver, p0, p0, p0, case.dt, 1)
    pr, sr = orc.newton_step(prob, S.with_solver(case, coarse_op="rediscretised").solver, p0, p0, p0,
                             case.dt, 1)
    assert sg["status"] == 0 and sr["status"] == 0, (sg, sr)
    assert np.linalg.norm((pr - p0) - (pg - p0)) <= 1e-6 * np.linalg.norm(pg - p0)
    # a working preconditioner: far fewer iterations than the unpreconditioned solve would need
    assert sr["linear_its"] < 60 * max(1, sr["newton_its"])
