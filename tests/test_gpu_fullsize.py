"""GPU parity at the benchmark workloads' full sizes, in the launch
configuration the benchmark times: one implicit step on the GPU through the
libnks C ABI against the FP64 CPU oracle, reservoir by reservoir (a sample of
the batch where the whole batch would take the oracle minutes).

The bar: the pressure change of the step agrees to 1e-6 relative, and the
GPU's pressure is at least as converged, judged by the oracle's own residual:
||F(p_gpu)|| <= max(1e-8 ||F(p_n)||, 2 ||F(p_oracle)||).  The second term
applies where binary64 cannot resolve 1e-8 of the initial residual: both sides
then stop at the rounding floor u || |J| |p| ||."""
import sys

import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu
PARITY = dict(eps_r=1e-8, eps_a=1e-6)


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


def _gpu_first_step(nks, case):
    g = nks.Grid(case.problems)
    p0 = g.initial_pressure()
    p = p0.clone()
    st = g.newton_step(p, p0, p0, case.dt, 1, case.solver)
    return g.split(p0), g.split(p), st


def _check(orc, case, k, p0g, pg):
    rec = case.problems[k]
    prob = orc.Problem(rec)
    q0 = prob.initial_pressure()
    assert np.max(np.abs(p0g - q0)) <= 1e-9 * np.max(np.abs(q0)), "initial state"
    q, st = orc.newton_step(prob, case.solver, q0, q0, q0, case.dt, 1)
    assert st["status"] == 0, st
    dq, dg = q - q0, pg - q0
    err = np.linalg.norm(dg - dq) / np.linalg.norm(dq)
    f0 = np.linalg.norm(prob.residual(q0, q0, q0, case.dt, 1))
    fg = np.linalg.norm(prob.residual(pg, q0, q0, case.dt, 1))
    fo = np.linalg.norm(prob.residual(q, q0, q0, case.dt, 1))
    say(f"  reservoir {k} ({rec.nx}x{rec.ny}x{rec.nz}): dp error {err:.2e}, ||F|| gpu {fg:.3e} "
        f"oracle {fo:.3e} initial {f0:.3e}")
    assert err <= 1e-6
    assert fg <= max(1e-8 * f0, 2.0 * fo, case.solver.eps_a)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_2d_512_first_step(nks, orc, precision):
    case = S.with_solver(S.case_2d_512(), precision=precision, **PARITY)
    say("2d 512x512", precision)
    p0, p, st = _gpu_first_step(nks, case)
    say("  gpu", st["newton_its"], "newton,", st["linear_its"], "gmres")
    _check(orc, case, 0, p0[0], p[0])


def test_flood_512_first_step(nks, orc):
    # Dirichlet faces at 1 and 10 atm around gas at 1 atm: several Newton
    # iterations in the first step
    case = S.with_solver(S.case_2d_flood_512(), **PARITY)
    say("2d 512x512 flood")
    p0, p, st = _gpu_first_step(nks, case)
    say("  gpu", st["newton_its"], "newton,", st["linear_its"], "gmres")
    assert st["newton_its"] >= 2
    _check(orc, case, 0, p0[0], p[0])


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_3d_128_first_step(nks, orc, precision):
    # FP32 factors (the workload's form) and BF16 off-diagonal factors with
    # FP32 accumulation: the Newton fixed point is the FP64 residual's, so the
    # bar is the FP64 one
    case = S.with_solver(S.case_3d_128(), precision=precision, **PARITY)
    say("3d 128x128x64", case.solver.precision)
    p0, p, st = _gpu_first_step(nks, case)
    say("  gpu", st["newton_its"], "newton,", st["linear_its"], "gmres")
    _check(orc, case, 0, p0[0], p[0])


def _gpu_two_steps(nks, case):
    g = nks.Grid(case.problems)
    hist, stats = g.simulate(2, case.dt, case.solver)
    return [g.split(h) for h in hist], stats


def _check_second_step(orc, case, k, hg):
    """The BDF2 step: the change p^2 - p^0 against the oracle's own two
    steps, and the oracle's BDF2 residual at the GPU's p^2 (with the GPU's
    p^1 and p^0 as history) against the same bar as the first step."""
    rec = case.problems[k]
    prob = orc.Problem(rec)
    q0 = prob.initial_pressure()
    q1, st1 = orc.newton_step(prob, case.solver, q0, q0, q0, case.dt, 1)
    q2, st2 = orc.newton_step(prob, case.solver, q1, q1, q0, case.dt, 2)
    assert st1["status"] == 0 and st2["status"] == 0
    p0, p1, p2 = hg[0][k], hg[1][k], hg[2][k]
    dq, dg = q2 - q0, p2 - q0
    err = np.linalg.norm(dg - dq) / np.linalg.norm(dq)
    f0 = np.linalg.norm(prob.residual(p1, p1, p0, case.dt, 2))
    fg = np.linalg.norm(prob.residual(p2, p1, p0, case.dt, 2))
    fo = np.linalg.norm(prob.residual(q2, q1, q0, case.dt, 2))
    say(f"  reservoir {k}: BDF2 step dp error {err:.2e}, ||F|| gpu {fg:.3e} oracle {fo:.3e} "
        f"initial {f0:.3e}")
    assert err <= 1e-6
    assert fg <= max(1e-8 * f0, 2.0 * fo, case.solver.eps_a)


@pytest.mark.parametrize("name", ["2d512", "3d128"])
def test_fullsize_second_step_bdf2(nks, orc, name):
    case = {"2d512": S.case_2d_512, "3d128": S.case_3d_128}[name]()
    case = S.with_solver(case, **PARITY)
    say("BDF2 second step", name, case.solver.precision)
    hg, stats = _gpu_two_steps(nks, case)
    say("  gpu", [x["newton_its"] for x in stats], "newton,", [x["linear_its"] for x in stats], "gmres")
    _check_second_step(orc, case, 0, hg)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp64"])
def test_batch64_first_step(nks, orc, precision):
    case = S.with_solver(S.case_batch64(), precision=precision, **PARITY)
    say("batch", len(case.problems), "reservoirs,", case.solver.precision)
    p0, p, st = _gpu_first_step(nks, case)
    say("  gpu", st["newton_its"], "newton,", st["linear_its"], "gmres")
    sizes = [r.N for r in case.problems]
    sample = sorted({0, 18, int(np.argmax(sizes)), int(np.argmin(sizes)), len(sizes) - 1})
    for k in sample:
        _check(orc, case, k, p0[k], p[k])


def test_3d_96_first_step(nks, orc):
    case = S.with_solver(S.case_3d_96_adjoint(), **PARITY)
    say("3d 96x96x48")
    p0, p, st = _gpu_first_step(nks, case)
    say("  gpu", st["newton_its"], "newton,", st["linear_its"], "gmres")
    _check(orc, case, 0, p0[0], p[0])
