"""GPU parity of the chain-rule accumulation (the BDF1 and BDF2 equations of
Section 2 as printed; the conservative form is the default reading) through
the libnks C ABI against the FP64 oracle: residual and Jacobian element by
element, and implicit steps through Newton."""
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


def _chain(case):
    return replace(case, problems=[replace(r, accum="chain_rule") for r in case.problems])


@pytest.mark.parametrize("cfg", [dict(nx=37, ny=23, nz=1, seed=1), dict(nx=9, ny=7, nz=5, seed=2, gravity=True,
                                                                          kv_ratio=0.1)])
@pytest.mark.parametrize("order", [1, 2])
def test_chain_rule_residual_and_jacobian_parity(nks, orc, cfg, order):
    say("chain-rule residual/jacobian", cfg, order)
    case = _chain(S.small_case(**cfg))
    rec = case.problems[0]
    op = orc.Problem(rec)
    rng = np.random.default_rng(cfg["seed"])
    base = op.initial_pressure()
    p = base + 3e4 * rng.standard_normal(op.N)
    pn = base + 1e4 * rng.standard_normal(op.N)
    pnm1 = base + 1e4 * rng.standard_normal(op.N)
    Fo = op.residual(p, pn, pnm1, case.dt, order)
    Jo = op.jacobian(p, pn, pnm1, case.dt, order)
    g = nks.Grid([rec])
    dp, dpn, dpnm1 = g.from_numpy(p), g.from_numpy(pn), g.from_numpy(pnm1)
    Fg = g.residual(dp, dpn, dpnm1, case.dt, order).cpu().numpy()
    assert np.max(np.abs(Fg - Fo)) <= 1e-12 * np.max(np.abs(Fo))
    J = g.jacobian(dp, dpn, dpnm1, case.dt, order)
    rp, ci, v = J.export_csr()
    assert np.array_equal(rp, Jo.rp) and np.array_equal(ci, Jo.ci)
    rowmax = np.repeat(np.maximum.reduceat(np.abs(Jo.v), Jo.rp[:-1]), np.diff(Jo.rp))
    assert np.all(np.abs(v - Jo.v) <= 1e-12 * rowmax)
    # the conservative grid on the same state gives a different residual
    gc = nks.Grid([replace(rec, accum="conservative")])
    Fc = gc.residual(gc.from_numpy(p), gc.from_numpy(pn), gc.from_numpy(pnm1), case.dt, order).cpu().numpy()
    assert np.max(np.abs(Fc - Fg)) > 1e-9 * np.max(np.abs(Fg))


def test_chain_rule_newton_steps_parity(nks, orc):
    # a BDF1 then a BDF2 step of the two-level solver on the printed form
    case = _chain(S.small_case(nx=48, ny=40, px=4, py=4, levels=2, overlap=(2, 1), rate=3e-3, seed=3,
                               eps_r=1e-8, eps_a=1e-6, dt=5 * S.DAY))
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
        say(f"step {n}: gpu newton {st_g[n - 1]['newton_its']}, dp error {err:.2e}, "
            f"relative residual {np.linalg.norm(F) / np.linalg.norm(F0):.2e}")
        assert err <= 1e-6
        assert np.linalg.norm(F) <= max(1e-8 * np.linalg.norm(F0), case.solver.eps_a)


def test_adjoint_refuses_the_chain_rule_form(nks):
    case = _chain(S.small_case(nx=8, ny=8))
    g = nks.Grid(case.problems)
    p = g.initial_pressure()
    with pytest.raises(Exception) as e:
        g.adjoint([p, p.clone()], case.dt, [None, g.zeros()], case.solver)
    assert "conservative" in str(e.value)
