"""Pins of the oracle's chain-rule accumulation, the BDF1 and BDF2 equations of
Section 2 as printed: the coefficient (phi p/Z)(1/p - Z'/Z) = phi m'(p) at the
new level times the difference quotient of p.  Its Jacobian needs m''(p),
from Z'' of the cubic.  Pinned by: second differences of independently
computed companion-matrix roots, the identity with the conservative form at
p = p^n (residual and Jacobian), the second-order size of the difference
between the two forms in the step, central differences of the residual, and
Newton on it."""
from dataclasses import replace

import numpy as np
import pytest

import synthetic as S
from test_oracle_pr import roots_largest_real


def _z_roots(fl, a, b, p):
    RT = fl.R * fl.T
    return roots_largest_real(a * p / RT ** 2, b * p / RT)


@pytest.mark.parametrize("T", [250.0, 350.0])
@pytest.mark.parametrize("p", [101325.0, 1e6, 1e7, 2e7, 5e7])
def test_second_derivatives_by_second_differences(orc, T, p):
    fl = S.Fluid(T=T)
    a, b, _ = orc.pr_params(fl)
    Z, dZ, d2Z, d2m = orc.pr_z2_ab(a, b, fl.T, fl.R, p)
    # at low pressure Z is nearly quadratic in p and its second difference is
    # tiny next to the roots' rounding: a wider step there
    h = (2e-2 if p < 1e6 else 2e-3) * p
    z = [_z_roots(fl, a, b, p + k * h) for k in (-2, -1, 0, 1, 2)]
    # fourth-order central second difference
    fd = (-z[0] + 16 * z[1] - 30 * z[2] + 16 * z[3] - z[4]) / (12 * h * h)
    assert abs(d2Z - fd) <= 1e-5 * abs(fd) + 1e-26, (T, p, d2Z, fd)
    m = [(p + k * h) / zz for k, zz in zip((-2, -1, 0, 1, 2), z)]
    fdm = (-m[0] + 16 * m[1] - 30 * m[2] + 16 * m[3] - m[4]) / (12 * h * h)
    assert abs(d2m - fdm) <= 1e-5 * abs(fdm) + 1e-20, (T, p, d2m, fdm)
    assert abs(dZ - (z[3] - z[1]) / (2 * h)) <= 1e-5 * abs(dZ)


def _pair(orc, chain, **kw):
    case = S.small_case(**kw)
    rec = case.problems[0]
    if chain:
        rec = replace(rec, accum="chain_rule")
    return orc.Problem(rec), case


def _state(prob, seed, amp=3e4):
    rng = np.random.default_rng(seed)
    base = prob.initial_pressure()
    return (base + amp * rng.standard_normal(prob.N), base + amp / 3 * rng.standard_normal(prob.N),
            base + amp / 3 * rng.standard_normal(prob.N))


@pytest.mark.parametrize("order", [1, 2])
def test_equal_to_conservative_at_the_old_level(orc, order):
    # at p = p^n (and p^{n-1} = p^n for BDF2) both accumulations vanish and
    # their linearisations agree: m''(p) multiplies a zero difference
    kw = dict(nx=6, ny=5, nz=3, gravity=True, seed=4)
    cons, case = _pair(orc, False, **kw)
    chain, _ = _pair(orc, True, **kw)
    p, _, _ = _state(cons, 1)
    Fc = cons.residual(p, p, p, case.dt, order)
    Fr = chain.residual(p, p, p, case.dt, order)
    assert np.allclose(Fr, Fc, rtol=0, atol=1e-12 * np.abs(Fc).max())
    Jc = cons.jacobian(p, p, p, case.dt, order).dense()
    Jr = chain.jacobian(p, p, p, case.dt, order).dense()
    assert np.allclose(Jr, Jc, rtol=1e-13, atol=1e-13 * np.abs(Jc).max())


def test_differs_from_conservative_at_second_order(orc):
    # F_chain - F_cons = V phi/dt [m'(p)(p - p^n) - (m(p) - m(p^n))], which is
    # m''/2 (p - p^n)^2 to leading order: halving the step quarters it
    kw = dict(nx=5, ny=4, seed=7, rate=0.0)
    cons, case = _pair(orc, False, **kw)
    chain, _ = _pair(orc, True, **kw)
    pn = cons.initial_pressure()
    d = np.random.default_rng(3).standard_normal(cons.N)
    diffs = []
    for amp in (4e5, 2e5, 1e5):
        p = pn + amp * d
        diffs.append(np.linalg.norm(chain.residual(p, pn, pn, case.dt, 1) - cons.residual(p, pn, pn, case.dt, 1)))
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 3.8 < r1 < 4.2 and 3.8 < r2 < 4.2, (r1, r2)


@pytest.mark.parametrize("dims,grav,order", [((5, 4, 1), False, 1), ((4, 3, 3), True, 2)])
def test_chain_rule_jacobian_matches_central_differences(orc, dims, grav, order):
    prob, case = _pair(orc, True, nx=dims[0], ny=dims[1], nz=dims[2], gravity=grav, seed=5)
    p, pn, pnm1 = _state(prob, 2)
    J = prob.jacobian(p, pn, pnm1, 86400.0, order).dense()
    for j in range(prob.N):
        h = 1e-6 * p[j]
        e = np.zeros(prob.N)
        e[j] = h
        fd = (prob.residual(p + e, pn, pnm1, 86400.0, order) -
              prob.residual(p - e, pn, pnm1, 86400.0, order)) / (2 * h)
        assert np.allclose(J[:, j], fd, rtol=1e-5, atol=1e-6 * np.max(np.abs(J))), j


def test_newton_on_the_chain_rule_form(orc):
    # Newton converges on the printed form, to a state within the O(dt^2)
    # distance of the conservative one; unlike the conservative form it does
    # not conserve mass exactly, but the imbalance is small and second order
    case = S.small_case(nx=10, ny=8, seed=6, rate=5e-3, eps_r=1e-12, eps_a=1e-14,
                        eta_r=1e-12, eta_a=1e-16)
    rec = case.problems[0]
    cons = orc.Problem(rec)
    chain = orc.Problem(replace(rec, accum="chain_rule"))
    p0 = cons.initial_pressure()
    pc, sc = orc.newton_step(cons, case.solver, p0, p0, p0, case.dt, 1)
    pr, sr = orc.newton_step(chain, case.solver, p0, p0, p0, case.dt, 1)
    assert sc["status"] == 0 and sr["status"] == 0
    assert np.linalg.norm(chain.residual(pr, p0, p0, case.dt, 1)) <= \
        1e-10 * np.linalg.norm(chain.residual(p0, p0, p0, case.dt, 1))
    dc, dr = pc - p0, pr - p0
    rel = np.linalg.norm(dr - dc) / np.linalg.norm(dc)
    assert 0 < rel < 1e-2, rel
    fl = rec.fluid
    V = rec.dx * rec.dy * rec.dz
    q = np.sum(rec.well_rates) * fl.R * fl.T / fl.W * case.dt
    mr = pr / np.array([_z_roots(fl, *orc.pr_params(fl)[:2], x) for x in pr])
    m0 = p0 / np.array([_z_roots(fl, *orc.pr_params(fl)[:2], x) for x in p0])
    gained = np.sum(V * rec.phi * (mr - m0))
    assert abs(gained - q) > 1e-12 * abs(q)       # not exactly conservative
    assert abs(gained - q) < 1e-2 * np.sum(V * rec.phi * np.abs(mr - m0))
