"""Batch form: the tile/overlap autotuner through the libnks C ABI, and a
Newton step of an uneven batch with the tuned preconditioner against the
oracle, reservoir by reservoir."""
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


def test_autotune_then_newton_parity(nks, orc):
    recs = [S.small_case(nx=n, ny=m, seed=s, rate=2e-3, sigma=1.0).problems[0]
            for n, m, s in [(48, 40, 1), (33, 61, 2), (24, 24, 3)]]
    settings = S.SolverSettings(px=1, py=1, tile=(16, 16, 0), levels=2, overlap=(1, 1),
                                precision="fp32", eps_r=1e-8, eps_a=1e-6)
    case = S.Case("batch", recs, S.DAY, 1, settings)
    g = nks.Grid(recs)
    p0 = g.initial_pressure()
    tuned, table = g.autotune(p0, p0, p0, case.dt, 1, settings, tiles=(8, 12, 24), overlaps=(1, 2),
                              ratios=(2, 4))
    for e in table:
        say(e)
    ok = [e for e in table if e["ok"]]
    assert len(ok) == len(table) == 12
    assert [(e["tile"], e["overlap"], e["ratio"]) for e in table] == \
        [(t, o, r) for t in (8, 12, 24) for o in (1, 2) for r in (2, 4)]
    best = min(ok, key=lambda e: e["setup_ms"] + e["solve_ms"])
    assert tuned.tile[:2] == (best["tile"], best["tile"]) and tuned.overlap == (best["overlap"],) * 2
    assert tuned.ratio == best["ratio"]
    p = p0.clone()
    st = g.newton_step(p, p0, p0, case.dt, 1, tuned)
    assert st["status"] == 0
    parts = g.split(p)
    for k, rec in enumerate(recs):
        prob = orc.Problem(rec)
        q0 = prob.initial_pressure()
        q, sto = orc.newton_step(prob, tuned, q0, q0, q0, case.dt, 1)
        err = np.linalg.norm((parts[k] - q0) - (q - q0)) / np.linalg.norm(q - q0)
        say("reservoir", k, "dp error", err)
        assert err <= 1e-6
