"""GPU parity on the stand-ins for the paper's H-zone (2D, isotropic and
anisotropic) and layered 3D floods, at sizes the oracle runs in seconds:
several strongly nonlinear implicit steps through the libnks C ABI against
the FP64 oracle (pressure change per step and the oracle's residual at the
GPU's state)."""
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


@pytest.mark.parametrize("name", ["hzone_iso", "hzone_aniso", "layered"])
def test_standin_steps_parity(nks, orc, name):
    if name == "layered":
        case = S.case_3d_layered_flood(16, px=2, py=2, pz=2, nsteps=2)
    else:
        case = S.case_2d_hzone(48, anisotropic=name == "hzone_aniso", px=4, py=4, nsteps=3)
    case = S.with_solver(case, **PARITY)
    rec = case.problems[0]
    g = nks.Grid([rec])
    hist_g, st_g = g.simulate(case.nsteps, case.dt, case.solver)
    hist_g = [h.cpu().numpy() for h in hist_g]
    (hist_o, st_o), = orc.simulate(case, nsteps=case.nsteps)
    op = orc.Problem(rec)
    assert np.max(np.abs(hist_g[0] - hist_o[0])) <= 1e-12 * np.max(hist_o[0])
    for n in range(1, case.nsteps + 1):
        dpg, dpo = hist_g[n] - hist_g[0], hist_o[n] - hist_o[0]
        err = np.linalg.norm(dpg - dpo) / np.linalg.norm(dpo)
        order = 1 if n == 1 else 2
        pm1 = hist_g[n - 2] if n > 1 else hist_g[n - 1]
        F = op.residual(hist_g[n], hist_g[n - 1], pm1, case.dt, order)
        F0 = op.residual(hist_g[n - 1], hist_g[n - 1], pm1, case.dt, order)
        pom1 = hist_o[n - 2] if n > 1 else hist_o[n - 1]
        Fo = op.residual(hist_o[n], hist_o[n - 1], pom1, case.dt, order)
        say(f"{name} step {n}: newton gpu {st_g[n - 1]['newton_its']} oracle {st_o[n - 1]['newton_its']}, "
            f"dp error {err:.2e}")
        assert err <= 1e-6
        assert np.linalg.norm(F) <= max(1e-8 * np.linalg.norm(F0), 2.0 * np.linalg.norm(Fo), case.solver.eps_a)
        assert abs(st_g[n - 1]["newton_its"] - st_o[n - 1]["newton_its"]) <= 1
