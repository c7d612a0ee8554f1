"""Pins of the oracle's finite-volume residual and Jacobian (Section 2,
the pressure form of the governing equation, BDF1/BDF2, Remark 1) against invariants that
hold whatever the implementation: zero residual at rest, hydrostatic
equilibrium, discrete conservation, mirror symmetry, finite differences,
and BDF temporal orders."""
import numpy as np
import pytest

import synthetic as S


def _prob(orc, **kw):
    case = S.small_case(**kw)
    return orc.Problem(case.problems[0]), case


def _no_wells(case):
    rec = case.problems[0]
    rec.well_cells = rec.well_cells[:0]
    rec.well_rates = rec.well_rates[:0]
    return case


def _m_by_roots(fl, p):
    from test_oracle_pr import roots_largest_real
    import oracle
    a, b, _ = oracle.pr_params(fl)
    RT = fl.R * fl.T
    return np.array([pi / roots_largest_real(a * pi / RT ** 2, b * pi / RT) for pi in p])


def test_transmissibility_closed_forms(orc):
    case = S.small_case(nx=3, ny=2, nz=2, sigma=0.0)
    rec = case.problems[0]
    rec.kx[:] = 2e-13
    rec.kx[1] = 6e-13          # cells 0 and 1 in series: harmonic mean 3e-13
    rec.ky[:] = 1e-13
    rec.kz[:] = 5e-14
    tx, ty, tz = orc.Problem(rec).transmissibility()
    # A_f / d times K for equal neighbours; 2 K1 K2 / (K1 + K2) A_f / d across a jump
    assert np.isclose(tx[0], 2 * 2e-13 * 6e-13 / 8e-13 * 100.0 / 10.0, rtol=1e-15)
    assert np.isclose(tx[3], 2e-13 * 10.0, rtol=1e-15)
    assert tx[2] == 0.0 and tx[5] == 0.0           # last column has no +x face
    assert np.allclose(ty[:3], 1e-13 * 10.0, rtol=1e-15) and np.all(ty[3:6] == 0.0)
    assert np.allclose(tz[:6], 5e-14 * 10.0, rtol=1e-15) and np.all(tz[6:] == 0.0)


@pytest.mark.parametrize("dims", [(6, 5, 1), (4, 3, 3)])
def test_zero_residual_at_rest(orc, dims):
    case = _no_wells(S.small_case(nx=dims[0], ny=dims[1], nz=dims[2]))
    prob = orc.Problem(case.problems[0])
    p = np.full(prob.N, 2e7)
    F = prob.residual(p, p, p, 86400.0, 1)
    assert np.max(np.abs(F)) == 0.0
    # BDF2's (3m - 4m + m)/2 cancels only up to rounding of the accumulation size
    F = prob.residual(p, p, p, 86400.0, 2)
    acc = 1000.0 * 0.3 / 86400.0 * 2e7 / 0.9
    assert np.max(np.abs(F)) < 4e-16 * acc


def test_hydrostatic_equilibrium(orc):
    case = _no_wells(S.small_case(nx=3, ny=3, nz=6, gravity=True))
    prob = orc.Problem(case.problems[0])
    p = prob.hydrostatic(2e7)
    # pressure rises with depth by about rho g dz (rho ~ 120 kg/m^3 at 20 MPa)
    nxy = 9
    dp = p[nxy:2 * nxy] - p[:nxy]
    assert np.all(dp > 0) and np.allclose(dp, 120 * 9.80665 * 10.0, rtol=0.1)
    F = prob.residual(p, p, p, 86400.0, 1)
    # each vertical flux is T lambda dPhi with dPhi = 0; compare with the size
    # of a single 1 Pa flux
    tx, ty, tz = prob.transmissibility()
    _, _, m, _ = prob.pr(p)
    scale = np.max(tz) * np.max(m) / case.problems[0].fluid.mu
    assert np.max(np.abs(F)) < 1e-6 * scale


def test_discrete_conservation(orc):
    # interior fluxes cancel pairwise: sum_i F_i = sum_i (V phi/dt) Acc_i - sum_w Q RT/W,
    # with Acc built here from independent companion roots
    case = S.small_case(nx=5, ny=4, nz=3, gravity=True, seed=3)
    rec = case.problems[0]
    prob = orc.Problem(rec)
    rng = np.random.default_rng(0)
    p = 2e7 + 1e5 * rng.standard_normal(prob.N)
    pn = 2e7 + 1e5 * rng.standard_normal(prob.N)
    pnm1 = 2e7 + 1e5 * rng.standard_normal(prob.N)
    dt = 3600.0
    fl = rec.fluid
    V = rec.dx * rec.dy * rec.dz
    m, mn, mnm1 = (_m_by_roots(fl, x) for x in (p, pn, pnm1))
    q = np.sum(rec.well_rates) * fl.R * fl.T / fl.W
    F1 = prob.residual(p, pn, pnm1, dt, 1)
    acc1 = np.sum(V * rec.phi / dt * (m - mn))
    assert abs(F1.sum() - (acc1 - q)) < 1e-9 * np.sum(np.abs(F1))
    F2 = prob.residual(p, pn, pnm1, dt, 2)
    acc2 = np.sum(V * rec.phi / dt * (3 * m - 4 * mn + mnm1) / 2)
    assert abs(F2.sum() - (acc2 - q)) < 1e-9 * np.sum(np.abs(F2))


def test_flux_direction_and_upwinding(orc):
    # two cells, no wells: flow runs from high to low pressure, so F of the
    # high cell (outflow) is positive; its size uses the upstream p/Z
    case = _no_wells(S.small_case(nx=2, ny=1, sigma=0.0))
    rec = case.problems[0]
    prob = orc.Problem(rec)
    p = np.array([2.1e7, 2.0e7])
    F = prob.residual(p, p, p, 1e30, 1)        # dt -> infinity removes accumulation
    tx, _, _ = prob.transmissibility()
    m_up = _m_by_roots(rec.fluid, p[:1])[0]
    assert F[0] > 0 and np.isclose(F[0], -F[1], rtol=1e-14)
    assert np.isclose(F[0], tx[0] * m_up / rec.fluid.mu * 1e6, rtol=1e-12)
    F_rev = prob.residual(p[::-1].copy(), p, p, 1e30, 1)
    assert np.isclose(F_rev[1], F[0], rtol=1e-14)


def test_mirror_symmetry(orc):
    # flipping the grid along x flips the residual: catches index and
    # face-assignment mistakes
    case = S.small_case(nx=5, ny=4, nz=2, gravity=True, seed=4)
    rec = case.problems[0]
    prob = orc.Problem(rec)
    rng = np.random.default_rng(1)
    p = 2e7 + 2e5 * rng.standard_normal(prob.N)
    pn = p + 1e4 * rng.standard_normal(prob.N)
    F = prob.residual(p, pn, pn, 86400.0, 1)

    def flip(a):
        return a.reshape(rec.nz, rec.ny, rec.nx)[:, :, ::-1].ravel().copy()

    cells = rec.well_cells
    x = cells % rec.nx
    rest = cells - x
    case2 = S.small_case(nx=5, ny=4, nz=2, gravity=True, seed=4)
    r2 = case2.problems[0]
    r2.kx, r2.ky, r2.kz, r2.phi = flip(rec.kx), flip(rec.ky), flip(rec.kz), flip(rec.phi)
    r2.well_cells = (rest + (rec.nx - 1 - x)).astype(np.int32)
    F2 = orc.Problem(r2).residual(flip(p), flip(pn), flip(pn), 86400.0, 1)
    assert np.allclose(flip(F), F2, rtol=1e-12, atol=1e-9 * np.max(np.abs(F)))


@pytest.mark.parametrize("dims,grav,order", [((5, 4, 1), False, 1), ((4, 3, 3), True, 2),
                                             ((3, 3, 4), True, 1)])
def test_jacobian_matches_central_differences(orc, dims, grav, order):
    case = S.small_case(nx=dims[0], ny=dims[1], nz=dims[2], gravity=grav, seed=5)
    prob = orc.Problem(case.problems[0])
    rng = np.random.default_rng(2)
    base = prob.initial_pressure()
    p = base + 3e4 * rng.standard_normal(prob.N)
    pn = base + 1e4 * rng.standard_normal(prob.N)
    pnm1 = base + 1e4 * rng.standard_normal(prob.N)
    J = prob.jacobian(p, pn, pnm1, 86400.0, order).dense()
    for j in range(prob.N):
        h = 1e-6 * p[j]
        e = np.zeros(prob.N)
        e[j] = h
        fd = (prob.residual(p + e, pn, pnm1, 86400.0, order) -
              prob.residual(p - e, pn, pnm1, 86400.0, order)) / (2 * h)
        assert np.allclose(J[:, j], fd, rtol=1e-5, atol=1e-6 * np.max(np.abs(J))), j


def test_mass_balance_per_step(orc):
    # a converged step conserves mass: sum V phi (m^{n+1} - m^n) = dt sum Q RT/W
    case = S.small_case(nx=8, ny=8, seed=6, rate=5e-3, eps_r=1e-12, eps_a=1e-14,
                        eta_r=1e-12, eta_a=1e-16)
    rec = case.problems[0]
    res = orc.simulate(case, nsteps=2)[0]
    hist = res[0]
    fl = rec.fluid
    V = rec.dx * rec.dy * rec.dz
    q = np.sum(rec.well_rates) * fl.R * fl.T / fl.W
    m = [_m_by_roots(fl, h) for h in hist]
    lhs1 = np.sum(V * rec.phi * (m[1] - m[0]))
    assert abs(lhs1 - case.dt * q) < 1e-8 * np.sum(V * rec.phi * np.abs(m[1] - m[0]))
    lhs2 = np.sum(V * rec.phi * (3 * m[2] - 4 * m[1] + m[0]) / 2)
    assert abs(lhs2 - case.dt * q) < 1e-8 * np.sum(V * rec.phi * np.abs(m[2] - m[1]))
    # injector pressure rose, producer pressure fell
    assert hist[-1][0] > hist[0][0] and hist[-1][-1] < hist[0][-1]


@pytest.mark.slow
def test_bdf_temporal_orders(orc):
    # BDF1 converges at first order in dt, BDF2 at second order (after its BDF1
    # start step); exact linear solves (one subdomain, dense LU) and tight Newton
    def run(nsteps, bdf2):
        case = S.small_case(nx=12, ny=1, seed=7, rate=2e-2, px=1, py=1, subsolve="lu",
                            kmean_md=0.05,
                            eps_r=1e-10, eps_a=1e-6, eta_r=1e-13, eta_a=1e-18,
                            dt=4 * S.DAY / nsteps, nsteps=nsteps)
        prob = orc.Problem(case.problems[0])
        p = prob.initial_pressure()
        hist = [p]
        for n in range(nsteps):
            order = 2 if (bdf2 and n > 0) else 1
            pnm1 = hist[-2] if len(hist) > 1 else hist[-1]
            p, st = orc.newton_step(prob, case.solver, hist[-1], hist[-1], pnm1, case.dt, order)
            assert st["status"] == 0
            hist.append(p)
        return hist[-1] - hist[0]
    ref = run(512, True)
    e1 = [np.linalg.norm(run(n, False) - ref) for n in (8, 16, 32)]
    e2 = [np.linalg.norm(run(n, True) - ref) for n in (8, 16, 32)]
    r1 = np.log2(e1[1] / e1[2])
    r2 = np.log2(e2[1] / e2[2])
    assert 0.8 < r1 < 1.2, e1
    assert 1.7 < r2 < 2.3, e2
