"""Oracle pins for the boundary conditions of Section 2 (p = p^D on the
Dirichlet part of the boundary, v.n = q^N on the Neumann part).

Each pin is a value fixed by the mathematics, not by the residual's code:
- Dirichlet faces, small pressure differences: the steady state of a column is
  the series-resistance solution of linear flow, with half-cell resistances
  Delta/(2K) at the two boundary faces (the one-sided face transmissibility);
- a Neumann inflow face against a Dirichlet face: the steady drop of each face
  is q mu Delta-resistance (Darcy's law with the prescribed velocity), and the
  sign of q^N follows the outward normal;
- gravity with a Dirichlet top or bottom face: the steady state is hydrostatic,
  half a cell of it between the face and the first cell centre;
- the analytic Jacobian with every face type agrees with finite differences.
"""
import numpy as np
import pytest
import scipy.optimize
import scipy.sparse.linalg as spla

import oracle as orc
from synthetic.configs import ATM, MD, Problem


def column(n, axis, k, bc_type, bc_value, gravity=False):
    dims = [1, 1, 1]
    dims[axis] = n
    nx, ny, nz = dims
    k = np.asarray(k, float)
    return Problem(nx, ny, nz, 10.0, 10.0, 10.0, k.copy(), k.copy(), k.copy(), np.full(n, 0.2),
                   np.zeros(0, np.int32), np.zeros(0), gravity=gravity, p_init=ATM,
                   bc_type=tuple(bc_type), bc_value=tuple(bc_value))


def steady(op, p, its=20):
    """Steady state by Newton: a time step so long that accumulation vanishes."""
    dt = 1e22
    p = np.array(p, float)
    for _ in range(its):
        F = op.residual(p, p, dt=dt)
        dp = spla.spsolve(op.jacobian(p, p, dt=dt).scipy().tocsc(), -F)
        p += dp
        if np.max(np.abs(dp)) <= 1e-13 * np.max(np.abs(p)):
            break
    return p


def faces_of(axis):
    return 2 * axis, 2 * axis + 1


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_dirichlet_series_resistance(axis):
    n = 9
    rng = np.random.default_rng(3 + axis)
    k = np.exp(rng.normal(0.0, 1.0, n)) * 100 * MD
    dp = 1e-3                                   # linear regime: dp/p ~ 1e-8
    lo, hi = faces_of(axis)
    bt, bv = [0] * 6, [0.0] * 6
    bt[lo], bv[lo] = 1, ATM + dp
    bt[hi], bv[hi] = 1, ATM
    op = orc.Problem(column(n, axis, k, bt, bv))
    p = steady(op, np.full(n, ATM))
    h = 10.0
    r = [h / (2 * k[0])] + [h / (2 * k[i]) + h / (2 * k[i + 1]) for i in range(n - 1)] + [h / (2 * k[-1])]
    R = sum(r)
    expect = np.array([ATM + dp - dp * sum(r[:i + 1]) / R for i in range(n)])
    assert np.max(np.abs(p - expect)) <= 1e-4 * dp


@pytest.mark.parametrize("axis", [0, 1])
def test_neumann_inflow_against_dirichlet(axis):
    n = 8
    rng = np.random.default_rng(11 + axis)
    k = np.exp(rng.normal(0.0, 0.7, n)) * 100 * MD
    f = 11.067e-3 * 1e-3          # viscosity of the default fluid, Pa s
    q = -1e-10                    # outward normal velocity at the inlet: inflow
    lo, hi = faces_of(axis)
    bt, bv = [0] * 6, [0.0] * 6
    bt[lo], bv[lo] = 2, q
    bt[hi], bv[hi] = 1, ATM
    op = orc.Problem(column(n, axis, k, bt, bv))
    p = steady(op, np.full(n, ATM))
    h = 10.0
    r = [h / (2 * k[i]) + h / (2 * k[i + 1]) for i in range(n - 1)] + [h / (2 * k[-1])]
    # the same mass flux |q| A m crosses every face: each drop is |q| mu r
    expect = np.array([ATM + (-q) * f * sum(r[i:]) for i in range(n)])
    drop = expect[0] - ATM
    assert drop > 1e-4
    assert np.all(np.diff(p) < 0)               # inflow: pressure falls towards the outlet
    assert np.max(np.abs(p - expect)) <= 1e-4 * drop
    # an outward velocity of the same size reverses the profile
    bv[lo] = -q
    op2 = orc.Problem(column(n, axis, k, bt, bv))
    p2 = steady(op2, np.full(n, ATM))
    assert np.max(np.abs((p2 - ATM) + (expect - ATM))) <= 1e-4 * drop


@pytest.mark.parametrize("face", [4, 5])
def test_gravity_dirichlet_face_is_hydrostatic(face):
    n = 6
    k = np.full(n, 50 * MD)
    pd = 5e6
    bt, bv = [0] * 6, [0.0] * 6
    bt[face], bv[face] = 1, pd
    rec = column(n, 2, k, bt, bv, gravity=True)
    op = orc.Problem(rec)
    p = steady(op, np.full(n, pd))
    f = rec.fluid
    crho_g = f.W / (f.R * f.T) * rec.g

    def m(x):
        return op.pr(np.array([x]))[2][0]

    half = 0.5 * rec.dz
    if face == 4:
        # top face at depth 0, first cell centre half a cell below
        top = scipy.optimize.brentq(lambda x: x - pd - 0.5 * (m(x) + m(pd)) * crho_g * half, pd, pd * 1.1,
                                    xtol=1e-12, rtol=1e-15)
    else:
        # bottom face half a cell below the last cell centre
        bot = scipy.optimize.brentq(lambda x: pd - x - 0.5 * (m(x) + m(pd)) * crho_g * half, pd * 0.9, pd,
                                    xtol=1e-12, rtol=1e-15)
        top = scipy.optimize.brentq(lambda x: op.hydrostatic(x)[-1] - bot, pd * 0.9, pd, xtol=1e-12, rtol=1e-15)
    expect = op.hydrostatic(top)
    assert np.max(np.abs(p - expect)) <= 1e-9 * pd


def test_jacobian_matches_finite_differences_with_boundaries():
    nx, ny, nz = 5, 4, 3
    rng = np.random.default_rng(5)
    N = nx * ny * nz
    k = np.exp(rng.normal(0.0, 1.0, N)) * 100 * MD
    rec = Problem(nx, ny, nz, 10.0, 10.0, 10.0, k.copy(), 0.7 * k, 0.2 * k, rng.uniform(0.1, 0.3, N),
                  np.zeros(0, np.int32), np.zeros(0), gravity=True, p_init=ATM,
                  bc_type=(1, 2, 1, 0, 1, 2), bc_value=(10 * ATM, -2e-6, 3 * ATM, 0.0, ATM, 1e-6))
    op = orc.Problem(rec)
    p = rng.uniform(2 * ATM, 8 * ATM, N)
    pn = p * 0.97
    J = op.jacobian(p, pn, dt=3600.0).dense()
    for i in rng.choice(N, 12, replace=False):
        e = np.zeros(N)
        h = 1e-3 * p[i]
        e[i] = h
        fd = (op.residual(p + e, pn, dt=3600.0) - op.residual(p - e, pn, dt=3600.0)) / (2 * h)
        assert np.max(np.abs(fd - J[:, i])) <= 1e-6 * np.max(np.abs(J[:, i]))


def test_dlogk_matches_finite_differences_with_boundaries():
    nx, ny, nz = 4, 3, 2
    rng = np.random.default_rng(9)
    N = nx * ny * nz
    k = np.exp(rng.normal(0.0, 1.0, N)) * 100 * MD
    p = rng.uniform(2 * ATM, 8 * ATM, N)
    lam = rng.normal(size=N)
    bt, bv = (1, 1, 2, 1, 1, 0), (9 * ATM, 2 * ATM, -1e-6, 4 * ATM, ATM, 0.0)

    def F(theta):
        kk = k * np.exp(theta)
        rec = Problem(nx, ny, nz, 10.0, 10.0, 10.0, kk.copy(), kk.copy(), kk.copy(), np.full(N, 0.2),
                      np.zeros(0, np.int32), np.zeros(0), gravity=True, p_init=ATM, bc_type=bt, bc_value=bv)
        return orc.Problem(rec).residual(p, p, dt=1e30)

    rec = Problem(nx, ny, nz, 10.0, 10.0, 10.0, k.copy(), k.copy(), k.copy(), np.full(N, 0.2),
                  np.zeros(0, np.int32), np.zeros(0), gravity=True, p_init=ATM, bc_type=bt, bc_value=bv)
    g = orc.Problem(rec).residual_dlogk_t(p, lam)
    for c in rng.choice(N, 8, replace=False):
        e = np.zeros(N)
        e[c] = 1e-6
        fd = lam @ (F(e) - F(-e)) / 2e-6
        assert abs(fd - g[c]) <= 1e-6 * max(abs(g[c]), 1e-30) + 1e-12 * np.max(np.abs(g))


def test_bad_boundary_rejected():
    rec = column(3, 0, np.full(3, MD), (1, 0, 0, 0, 0, 0), (-1.0, 0, 0, 0, 0, 0))
    with pytest.raises(ValueError):
        orc.Problem(rec)
    rec = column(3, 0, np.full(3, MD), (3, 0, 0, 0, 0, 0), (1.0, 0, 0, 0, 0, 0))
    with pytest.raises(ValueError):
        orc.Problem(rec)
