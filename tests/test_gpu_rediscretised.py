"""GPU parity of rediscretised coarse operators (the upscaled coarse
problem's Jacobian at the coarsened state, the alternative to the Galerkin
product for the coarse matrices of Section 3.2) through the libnks C ABI
against the FP64 oracle: coarse matrices element by element, the two- and
three-level V-cycle apply with a fixed number of coarse iterations, and
implicit steps through Newton."""
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


CASES = [
    dict(nx=48, ny=40, nz=1, px=4, py=4, levels=2, overlap=(2, 1)),
    dict(nx=64, ny=48, nz=1, px=4, py=3, levels=2, overlap=(1, 1), ratio=4),
    dict(nx=48, ny=32, nz=1, px=3, py=2, levels=3, overlap=(1, 1, 1), sigma=2.0),
    dict(nx=16, ny=12, nz=8, px=2, py=2, pz=2, levels=2, overlap=(1, 1), gravity=True, kv_ratio=0.1),
]


def _setup(nks, orc, cfg, seed):
    case = S.small_case(coarse_op="rediscretised", seed=seed, **cfg)
    rec = case.problems[0]
    op = orc.Problem(rec)
    rng = np.random.default_rng(seed)
    base = op.initial_pressure()
    p = base + 3e4 * rng.standard_normal(op.N)
    pn = base + 1e4 * rng.standard_normal(op.N)
    Jo = op.jacobian(p, pn, pn, case.dt, 1)
    mo = orc.Multilevel(rec, Jo, case.solver, state=(p, case.dt, 1))
    g = nks.Grid([rec])
    J = g.jacobian(g.from_numpy(p), g.from_numpy(pn), None, case.dt, 1)
    M = nks.Ras(J, case.solver)
    return case, rec, op, mo, g, M


@pytest.mark.parametrize("cfg", CASES)
def test_rediscretised_coarse_matrices_parity(nks, orc, cfg):
    say("rediscretised coarse matrices", cfg)
    case, rec, op, mo, g, M = _setup(nks, orc, cfg, 31)
    for lev in range(1, cfg["levels"]):
        Ao = mo.level_matrix(lev)
        rp, ci, v = M.level_export(lev)
        assert np.array_equal(rp, Ao.rp) and np.array_equal(ci, Ao.ci), lev
        rowmax = np.repeat(np.maximum.reduceat(np.abs(Ao.v), Ao.rp[:-1]), np.diff(Ao.rp))
        assert np.all(np.abs(v - Ao.v) <= 1e-12 * rowmax), lev


@pytest.mark.parametrize("cfg", CASES)
def test_rediscretised_vcycle_apply_parity(nks, orc, cfg):
    cfg = dict(cfg, coarse_rtol=0.0, coarse_maxit=5)
    say("rediscretised V-cycle", cfg)
    case, rec, op, mo, g, M = _setup(nks, orc, cfg, 32)
    r = np.sin(0.41 * np.arange(op.N))
    zo = mo.apply(r)
    zg = M.apply(g.from_numpy(r)).cpu().numpy()
    assert np.max(np.abs(zg - zo)) <= 1e-9 * np.max(np.abs(zo))


def test_rediscretised_newton_steps_parity(nks, orc):
    case = S.small_case(nx=64, ny=48, px=4, py=4, levels=2, overlap=(2, 1), rate=3e-3, seed=5,
                        coarse_op="rediscretised", eps_r=1e-8, eps_a=1e-6, dt=5 * S.DAY)
    rec = case.problems[0]
    g = nks.Grid([rec])
    hist_g, st_g = g.simulate(2, case.dt, case.solver)
    hist_g = [h.cpu().numpy() for h in hist_g]
    (hist_o, st_o), = orc.simulate(case, nsteps=2)
    op = orc.Problem(rec)
    for n in (1, 2):
        dpg, dpo = hist_g[n] - hist_g[0], hist_o[n] - hist_o[0]
        err = np.linalg.norm(dpg - dpo) / np.linalg.norm(dpo)
        order = 1 if n == 1 else 2
        pm1 = hist_g[n - 2] if n > 1 else hist_g[n - 1]
        F = op.residual(hist_g[n], hist_g[n - 1], pm1, case.dt, order)
        F0 = op.residual(hist_g[n - 1], hist_g[n - 1], pm1, case.dt, order)
        # the oracle's own step: both sides may stop at the FP64 rounding floor
        pom1 = hist_o[n - 2] if n > 1 else hist_o[n - 1]
        Fo = op.residual(hist_o[n], hist_o[n - 1], pom1, case.dt, order)
        say(f"step {n}: gpu newton {st_g[n - 1]['newton_its']} gmres {st_g[n - 1]['linear_its']}, oracle "
            f"gmres {st_o[n - 1]['linear_its']}, dp error {err:.2e}")
        assert err <= 1e-6
        assert np.linalg.norm(F) <= max(1e-8 * np.linalg.norm(F0), 2.0 * np.linalg.norm(Fo), case.solver.eps_a)
        assert abs(st_g[n - 1]["linear_its"] - st_o[n - 1]["linear_its"]) <= 2 * st_g[n - 1]["newton_its"]


def test_rediscretised_refuses_sizes_the_ratio_does_not_divide(nks):
    case = S.small_case(nx=9, ny=8, px=1, py=1, levels=2, overlap=(1, 1), coarse_op="rediscretised")
    g = nks.Grid(case.problems)
    p = g.initial_pressure()
    J = g.jacobian(p, p, None, case.dt, 1)
    with pytest.raises(Exception) as e:
        nks.Ras(J, case.solver)
    assert "multiple" in str(e.value)
