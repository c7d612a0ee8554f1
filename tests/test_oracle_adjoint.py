"""Pins of the oracle's differentiation pieces against central differences of
the oracle's own residual and forward solves: (dF/dln K)^T lam, and the
discrete BDF1/BDF2 adjoint gradient of a pressure objective."""
from dataclasses import replace

import numpy as np
import pytest

import synthetic as S


def _perturb(rec, c, h):
    f = np.exp(h)
    kx, ky, kz = rec.kx.copy(), rec.ky.copy(), rec.kz.copy()
    kx[c] *= f
    ky[c] *= f
    kz[c] *= f
    return replace(rec, kx=kx, ky=ky, kz=kz)


@pytest.mark.parametrize("dims,grav", [((6, 5, 1), False), ((4, 4, 3), True)])
def test_dlogk_transpose_matches_residual_differences(orc, dims, grav):
    case = S.small_case(nx=dims[0], ny=dims[1], nz=dims[2], gravity=grav, kv_ratio=0.1, seed=4,
                        sigma=1.0)
    rec = case.problems[0]
    prob = orc.Problem(rec)
    rng = np.random.default_rng(5)
    p = prob.initial_pressure() + 2e4 * rng.standard_normal(prob.N)
    pn = prob.initial_pressure()
    lam = rng.standard_normal(prob.N)
    got = prob.residual_dlogk_t(p, lam)
    h = 1e-5
    for c in range(prob.N):
        Fp = orc.Problem(_perturb(rec, c, h)).residual(p, pn, pn, case.dt, 1)
        Fm = orc.Problem(_perturb(rec, c, -h)).residual(p, pn, pn, case.dt, 1)
        fd = lam @ (Fp - Fm) / (2 * h)
        assert abs(got[c] - fd) <= 1e-6 * np.max(np.abs(got)) + 1e-6 * abs(fd), c


def _objective_case(dims, grav):
    case = S.small_case(nx=dims[0], ny=dims[1], nz=dims[2], gravity=grav, kv_ratio=0.1, seed=7,
                        sigma=1.0, rate=2e-3, px=1, py=1, pz=1, subsolve="lu", eps_r=1e-14,
                        eps_a=0.0, eta_r=1e-14, eta_a=0.0, dt=2 * S.DAY)
    rec = case.problems[0]
    # objective: mean pressure of the producer cell's column at the last step,
    # plus a smaller weight on the injector cell at the first step
    prod = int(np.argmin(rec.well_rates))
    inj = int(np.argmax(rec.well_rates))
    pc, ic = int(rec.well_cells[prod]), int(rec.well_cells[inj])
    nxy = rec.nx * rec.ny
    col = [pc % nxy + z * nxy for z in range(rec.nz)]
    return case, rec, col, ic


def _G(orc, case, rec, col, ic, nsteps):
    out = orc.simulate(replace(case, problems=[rec]), nsteps=nsteps)[0]
    hist, stats = out
    assert all(st["status"] == 0 for st in stats)
    return np.mean(hist[-1][col]) + 0.3 * hist[1][ic], hist


@pytest.mark.parametrize("dims,grav,nsteps", [((6, 5, 1), False, 3), ((4, 4, 3), True, 3),
                                              ((7, 3, 1), False, 1)])
def test_adjoint_gradient_matches_central_differences(orc, dims, grav, nsteps):
    case, rec, col, ic = _objective_case(dims, grav)
    G0, hist = _G(orc, case, rec, col, ic, nsteps)
    prob = orc.Problem(rec)
    dG = [None] * (nsteps + 1)
    dG[nsteps] = np.zeros(prob.N)
    dG[nsteps][col] += 1.0 / len(col)
    if dG[1] is None:
        dG[1] = np.zeros(prob.N)
    dG[1][ic] += 0.3
    grad, _ = orc.adjoint(prob, case.dt, hist, dG)
    rng = np.random.default_rng(11)
    cells = rng.choice(prob.N, size=min(8, prob.N), replace=False)
    h = 1e-4
    for c in cells:
        Gp, _ = _G(orc, case, _perturb(rec, c, h), col, ic, nsteps)
        Gm, _ = _G(orc, case, _perturb(rec, c, -h), col, ic, nsteps)
        fd = (Gp - Gm) / (2 * h)
        assert abs(grad[c] - fd) <= 1e-5 * np.max(np.abs(grad)) + 1e-4 * abs(fd), (c, grad[c], fd)
