"""FGMRES iterations captured in HIP graphs.  When the preconditioner runs
without a host round trip (one level, or the persistent coarse solve), the
Newton step replays its outer iterations from captured graphs, two per
graph, across Newton iterations and steps.  Every replay is checked against
the same steps run from plain launches (the profiler's graphs-off mode):
the kernels are deterministic, so the pressures agree bit for bit, and the
captured run waits on the device fewer times."""
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


SIZES = [(37, 29, 1), (64, 50, 2), (20, 20, 3), (9, 33, 4), (96, 80, 5)]


def _run(nks, recs, settings, nsteps, eager):
    lib = nks.lib()
    g = nks.Grid(recs)
    if eager:
        nks.check(lib.nks_profile_enable(2))
    try:
        hist, stats = g.simulate(nsteps, 5 * S.DAY, settings)
    finally:
        if eager:
            nks.check(lib.nks_profile_enable(0))
    return np.stack([h.cpu().numpy() for h in hist]), stats


@pytest.mark.parametrize("kind", ["one_level", "persistent_two_level"])
def test_captured_fgmres_matches_plain_launches(nks, kind):
    recs = [S.small_case(nx=n, ny=m, seed=s, rate=2e-3).problems[0] for n, m, s in SIZES]
    if kind == "one_level":
        s = S.SolverSettings(px=1, py=1, tile=(16, 16, 0), levels=1, overlap=(1,), precision="fp32", eps_r=1e-8)
    else:
        s = S.SolverSettings(px=1, py=1, tile=(16, 16, 0), levels=2, overlap=(2, 1), ratio=4, precision="fp32",
                             coarse_kernel="persistent", eps_r=1e-8)
    hg, sg = _run(nks, recs, s, 3, eager=False)
    he, se = _run(nks, recs, s, 3, eager=True)
    for a, b in zip(sg, se):
        say(kind, "graphs:", a["newton_its"], a["linear_its"], "waits", a["host_waits"], "chunk", a["graph_chunk"],
            "| plain:", b["newton_its"], b["linear_its"], "waits", b["host_waits"], "chunk", b["graph_chunk"])
        assert a["graph_chunk"] == 2 and b["graph_chunk"] == 0
        assert (a["newton_its"], a["linear_its"]) == (b["newton_its"], b["linear_its"])
        assert a["host_waits"] < b["host_waits"]
    assert np.array_equal(hg, he)


def test_chunked_coarse_is_not_captured(nks):
    # the chunked coarse solve tests convergence on the host: the outer
    # iterations stay plain launches
    recs = [S.small_case(nx=n, ny=m, seed=s, rate=2e-3).problems[0] for n, m, s in SIZES[:3]]
    s = S.SolverSettings(px=1, py=1, tile=(16, 16, 0), levels=2, overlap=(2, 1), coarse_kernel="chunked")
    g = nks.Grid(recs)
    _, stats = g.simulate(1, 5 * S.DAY, s)
    assert stats[0]["graph_chunk"] == 0
