"""Oracle pins for lagged preconditioner refactorisation across Newton
iterations.  The Newton solution does not depend on the preconditioner, only
the Krylov iterations do: a lagged run must reach the same state within the
Newton tolerance, take the same first linear solve (the preconditioner is
built at iteration 0 either way), and lag 1 must be the plain method."""
import numpy as np
import pytest

import oracle as orc
import synthetic as S

PARITY = dict(eps_r=1e-10, eps_a=1e-8)


def run(lag, levels=1, case=None):
    case = case or S.case_2d_flood(24, 24, 2, 2)
    case = S.with_solver(case, lag=lag, levels=levels, overlap=(1,) * levels, **PARITY)
    (hist, st), = orc.simulate(case, nsteps=2)
    return hist, st


def same_state(h1, s1, hl, sl):
    for n in (1, 2):
        d = h1[n] - h1[0]
        assert np.linalg.norm((hl[n] - hl[0]) - d) <= 1e-6 * np.linalg.norm(d)
    for a, b in zip(s1, sl):
        assert a["lits"][0] == b["lits"][0]


@pytest.mark.parametrize("lag", [2, 3, 100])
def test_lagged_newton_reaches_the_same_state(lag):
    # one level on the flood: several Newton iterations per step, and a
    # Jacobian that changes tenfold near the inflow face
    h1, s1 = run(1)
    hl, sl = run(lag)
    same_state(h1, s1, hl, sl)
    assert s1[0]["newton_its"] >= 3
    # stale factors cost linear iterations, never the answer
    assert sum(x["linear_its"] for x in sl) >= sum(x["linear_its"] for x in s1)


@pytest.mark.parametrize("lag", [2, 100])
def test_lagged_two_level_mild_regime(lag):
    # two levels where the Jacobian moves little between Newton iterations
    # (a five-spot at 20 MPa); the coarse operators stay current
    case = S.small_case(nx=32, ny=28, px=2, py=2, rate=5e-2, dt=20 * S.DAY)
    h1, s1 = run(1, 2, case)
    hl, sl = run(lag, 2, case)
    assert max(x["newton_its"] for x in s1) >= 2
    same_state(h1, s1, hl, sl)


def test_lag_one_and_zero_are_the_plain_method():
    h1, s1 = run(1)
    h0, s0 = run(0)
    for a, b in zip(h1, h0):
        assert np.array_equal(a, b)
    assert [x["lits"] for x in s1] == [x["lits"] for x in s0]
