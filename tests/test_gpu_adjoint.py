"""GPU parity of the differentiation form through the libnks C ABI:
(dF/dln K)^T lambda, J^T as a matrix, the transposed Schwarz apply, GMRES on
J^T, the discrete BDF1/BDF2 adjoint against the oracle's, the gradient at the
96x96x48 channelised workload against central differences of the GPU forward
solve on 20 seeded cells, and the torch.autograd.Function."""
import sys
from dataclasses import replace

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


CASES = [dict(nx=23, ny=17, nz=1, seed=1), dict(nx=9, ny=8, nz=6, seed=2, gravity=True, kv_ratio=0.1)]


@pytest.mark.parametrize("cfg", CASES)
def test_dlogk_transpose_parity(nks, orc, cfg):
    case = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    rng = np.random.default_rng(3)
    p = op.initial_pressure() + 3e4 * rng.standard_normal(op.N)
    lam = rng.standard_normal(op.N)
    want = op.residual_dlogk_t(p, lam)
    g = nks.Grid([rec])
    got = g.residual_dlogk_t(g.from_numpy(p), g.from_numpy(lam)).cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("cfg", CASES)
def test_matrix_transpose_parity(nks, orc, cfg):
    case = S.small_case(**cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p = op.initial_pressure() + 3e4 * np.random.default_rng(4).standard_normal(op.N)
    pn = op.initial_pressure()
    Jo = op.jacobian(p, pn, pn, case.dt, 1).scipy()
    g = nks.Grid([rec])
    J = g.jacobian(g.from_numpy(p), g.from_numpy(pn), None, case.dt, 1)
    rp, ci, v = J.transpose().export_csr()
    import scipy.sparse as sp
    JT = sp.csr_matrix((v, ci, rp), shape=Jo.shape)
    assert abs(JT - Jo.T).max() <= 1e-12 * abs(Jo).max()


@pytest.mark.parametrize("variant", ["left_ras", "as", "right_ras"])
@pytest.mark.parametrize("cfg", [dict(nx=37, ny=29, nz=1, px=4, py=3, overlap=(2,)),
                                 dict(nx=12, ny=10, nz=8, px=2, py=2, pz=2, overlap=(1,),
                                      gravity=True)])
def test_ras_apply_transpose_parity(nks, orc, cfg, variant):
    case = S.small_case(variant=variant, **cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    p = op.initial_pressure() + 3e4 * np.random.default_rng(5).standard_normal(op.N)
    pn = op.initial_pressure()
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    r = np.random.default_rng(6).standard_normal(op.N)
    want = orc.Multilevel(rec, Jo, case.solver).apply_transpose(r)
    g = nks.Grid([rec])
    J = g.jacobian(g.from_numpy(p), g.from_numpy(pn), None, case.dt, 1)
    M = nks.Ras(J, case.solver)
    got = M.apply_transpose(g.from_numpy(r)).cpu().numpy()
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    say("transpose apply", variant, cfg["nz"], "relative error", err)
    assert err <= 1e-11


@pytest.mark.parametrize("levels", [1, 2])
def test_gmres_transpose_with_preconditioner(nks, orc, levels):
    case = S.small_case(nx=40, ny=32, px=4, py=4, levels=levels, overlap=(1, 1))
    rec = case.problems[0]
    op = orc.Problem(rec)
    p = op.initial_pressure() + 3e4 * np.random.default_rng(7).standard_normal(op.N)
    pn = op.initial_pressure()
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    b = np.random.default_rng(8).standard_normal(op.N)
    g = nks.Grid([rec])
    J = g.jacobian(g.from_numpy(p), g.from_numpy(pn), None, case.dt, 1)
    M = nks.Ras(J, case.solver)
    x, st = nks.gmres_solve(J, M, g.from_numpy(b), rtol=1e-11, atol=0.0, flexible=levels > 1,
                            transpose=True)
    xd = np.linalg.solve(Jo.dense().T, b)
    say("transpose gmres levels", levels, "its", st["iterations"])
    assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-8 * np.linalg.norm(xd)


def _objective(rec):
    """Mean pressure over the producer cell's column."""
    prod = int(np.argmin(rec.well_rates))
    pc = int(rec.well_cells[prod])
    nxy = rec.nx * rec.ny
    col = [pc % nxy + z * nxy for z in range(rec.nz)]
    w = np.zeros(rec.N)
    w[col] = 1.0 / len(col)
    return w


@pytest.mark.parametrize("cfg,levels", [(dict(nx=20, ny=18, nz=1, px=3, py=3), 1),
                                        (dict(nx=12, ny=10, nz=6, px=2, py=2, pz=2, gravity=True,
                                              kv_ratio=0.1), 2)])
def test_adjoint_parity_against_oracle(nks, orc, cfg, levels):
    # same forward states on both sides (the oracle's), so the comparison is
    # of the adjoint alone: lambda_n per step and the gradient
    case = S.small_case(levels=levels, overlap=(1, 1), rate=2e-3, sigma=1.0, seed=9, dt=2 * S.DAY,
                        eps_r=1e-12, eps_a=0.0, **cfg)
    rec = case.problems[0]
    hist, stats = orc.simulate(case, nsteps=3)[0]
    op = orc.Problem(rec)
    w = _objective(rec)
    dG = [None, None, None, w]
    grad_o, lams_o = orc.adjoint(op, case.dt, hist, dG)
    g = nks.Grid([rec])
    ph = [g.from_numpy(h) for h in hist]
    grad_g, st = g.adjoint(ph, case.dt, [None, None, None, g.from_numpy(w)], case.solver, rtol=1e-12,
                           want_lambda=True)
    say("adjoint its per step", st["linear_its"])
    for n in (1, 2, 3):
        lg = st["lambda"][n].cpu().numpy()
        assert np.max(np.abs(lg - lams_o[n])) <= 1e-8 * np.max(np.abs(lams_o[n])), n
    gg = grad_g.cpu().numpy()
    assert np.max(np.abs(gg - grad_o)) <= 1e-8 * np.max(np.abs(grad_o))


def test_adjoint_gradient_fd_3d_96(nks):
    # the channelised 96x96x48 workload: gradient of the producer-column mean
    # pressure after 3 steps with respect to ln K, against central differences
    # of the GPU forward solve at 20 cells drawn uniformly (seed 55), chosen
    # without looking at the adjoint.  G is ~2e7 Pa, so a central difference
    # with step h resolves a gradient only to about the forward solves'
    # convergence noise over 2h; each cell is judged as |grad - fd| <=
    # 2e-3 |fd| + 1e-6 max|grad|, so a cell whose true gradient is above that
    # floor and where the adjoint returned ~0 fails.  The difference is taken
    # state by state before the weights
    base = S.case_3d_96_adjoint()
    case = S.with_solver(base, eps_r=1e-12, eps_a=0.0, eta_r=1e-10, eta_a=0.0)
    rec = case.problems[0]
    w = _objective(rec)
    g = nks.Grid([rec])
    hist, stats = g.simulate(case.nsteps, case.dt, case.solver)
    say("forward newton", [s["newton_its"] for s in stats], "gmres", [s["linear_its"] for s in stats])
    dG = [None] * case.nsteps + [g.from_numpy(w)]
    grad, st = g.adjoint(hist, case.dt, dG, case.solver, rtol=1e-10)
    grad = grad.cpu().numpy()
    scale = np.max(np.abs(grad))
    say("adjoint its", st["linear_its"], "seconds", round(st["seconds"], 3), "max |grad|", scale,
        "quantiles", np.quantile(np.abs(grad), [0.5, 0.9, 0.99, 0.999]))
    cells = np.random.default_rng(55).choice(rec.N, size=20, replace=False)
    h = 1e-2

    def final_state(c, hh):
        f = np.exp(hh)
        kx, ky, kz = rec.kx.copy(), rec.ky.copy(), rec.kz.copy()
        kx[c] *= f
        ky[c] *= f
        kz[c] *= f
        gp = nks.Grid([replace(rec, kx=kx, ky=ky, kz=kz)])
        hp, _ = gp.simulate(case.nsteps, case.dt, case.solver)
        return hp[-1].cpu().numpy()

    worst, resolved = 0.0, 0
    floor = 1e-6 * scale
    for c in cells:
        fd = float(w @ (final_state(c, h) - final_state(c, -h))) / (2 * h)
        err = abs(grad[c] - fd) / max(abs(fd), 1e-300)
        if abs(fd) > 100 * floor:
            resolved += 1
            worst = max(worst, err)
        say(f"  cell {c}: adjoint {grad[c]:.6e} fd {fd:.6e} rel {err:.1e}")
        assert abs(grad[c] - fd) <= 2e-3 * abs(fd) + floor, (c, grad[c], fd)
    say(f"worst relative difference {worst:.2e} over {resolved} of {len(cells)} cells whose gradient is "
        f"resolved (|fd| > 100 x the absolute floor {floor:.2e})")


def test_autograd_function_matches_adjoint(nks):
    import torch
    from paper_2007_13966_amd.adjoint import WellPressureObjective
    case = S.small_case(nx=16, ny=12, nz=4, px=2, py=2, pz=2, levels=2, overlap=(1, 1), gravity=True,
                        kv_ratio=0.1, rate=2e-3, seed=12, eps_r=1e-12, eps_a=0.0)
    rec = case.problems[0]
    w = _objective(rec)
    obj = WellPressureObjective(rec, case.solver, 2, case.dt, w)
    theta = torch.tensor(np.log(rec.kx), dtype=torch.float64, device="cuda:0", requires_grad=True)
    G = obj(theta)
    (2.5 * G).backward()
    # the same gradient straight from the library
    g = nks.Grid([rec])
    hist, _ = g.simulate(2, case.dt, case.solver)
    grad, _ = g.adjoint(hist, case.dt, [None, None, g.from_numpy(2.5 * w)], case.solver)
    assert abs(G.item() - float(w @ hist[-1].cpu().numpy())) <= 1e-9 * abs(G.item())
    assert torch.allclose(theta.grad, grad, rtol=1e-9, atol=1e-12 * grad.abs().max().item())
