"""Pins of the oracle's ILU(k) subdomain solver (Section 3.1's subdomain
solves with k levels of fill), by facts independent of its symbolic
algorithm:
- the pattern: an entry (i, j) has level of fill m, the least number of
  interior vertices on a path i -> ... -> j in the graph of A whose interior
  vertices are all smaller than min(i, j) (the fill-path characterisation of
  levels of fill); ILU(k) keeps the entries of level <= k.  Checked by a
  breadth-first search per entry on small boxes;
- the factors reproduce A on the pattern ((LU)_ij = a_ij wherever the
  pattern holds (i, j)), the defining property of an incomplete LU on a
  given pattern;
- with enough fill the pattern is full below the profile and ILU(k) is the
  exact LU: one subdomain without overlap then solves A z = r exactly."""
from collections import deque

import numpy as np
import pytest

import synthetic as S


def _one_box(orc, fill, dims, gravity=False):
    case = S.small_case(nx=dims[0], ny=dims[1], nz=dims[2], px=1, py=1, pz=1, overlap=(0,),
                        gravity=gravity, fill=fill)
    prob = orc.Problem(case.problems[0])
    rng = np.random.default_rng(5)
    p0 = prob.initial_pressure()
    p = p0 + 5e4 * rng.standard_normal(prob.N)
    J = prob.jacobian(p, p0, p0, 86400.0, 1)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    return J, mg


def _fill_levels(A):
    """level of fill of every (i, j) by the fill-path characterisation"""
    n = A.shape[0]
    nbr = [np.nonzero(A[i])[0] for i in range(n)]
    lev = np.full((n, n), np.iinfo(np.int32).max, dtype=np.int64)
    for i in range(n):
        for j in range(n):
            if A[i, j] != 0 or i == j:
                lev[i, j] = 0
                continue
            lim = min(i, j)
            # BFS from i through vertices below lim; distance = interior count
            dist = {i: 0}
            q = deque([i])
            best = None
            while q and best is None:
                u = q.popleft()
                for w in nbr[u]:
                    if w == j and u != i:
                        best = dist[u]
                        break
                    if w < lim and w not in dist:
                        dist[w] = dist[u] + 1
                        q.append(w)
            if best is not None:
                lev[i, j] = best
    return lev


@pytest.mark.parametrize("fill,dims", [(1, (6, 5, 1)), (2, (6, 5, 1)), (1, (4, 3, 3))])
def test_iluk_pattern_is_the_fill_path_level_set(orc, fill, dims):
    J, mg = _one_box(orc, fill, dims, gravity=dims[2] > 1)
    F = mg.subdomain(0, 0)["factors"]
    got = np.zeros((J.n, J.n), bool)
    for i in range(J.n):
        got[i, F.ci[F.rp[i]:F.rp[i + 1]]] = True
    want = _fill_levels(J.dense()) <= fill
    assert np.array_equal(got, want)
    assert got.sum() > (J.dense() != 0).sum()   # some fill was kept


@pytest.mark.parametrize("fill", [1, 2])
def test_iluk_factors_reproduce_a_on_the_pattern(orc, fill):
    J, mg = _one_box(orc, fill, (7, 6, 1))
    F = mg.subdomain(0, 0)["factors"]
    D = np.zeros((J.n, J.n))
    mask = np.zeros((J.n, J.n), bool)
    for i in range(J.n):
        cols = F.ci[F.rp[i]:F.rp[i + 1]]
        D[i, cols] = F.v[F.rp[i]:F.rp[i + 1]]
        mask[i, cols] = True
    L = np.tril(D, -1) + np.eye(J.n)
    U = np.triu(D)
    A = J.dense()
    assert np.allclose((L @ U)[mask], A[mask], rtol=1e-11, atol=1e-11 * np.abs(A).max())


def test_iluk_with_full_fill_is_the_exact_solve(orc):
    # 5 x 4 cells: the lexicographic profile has width 5, so 5 levels fill it
    J, mg = _one_box(orc, 6, (5, 4, 1))
    r = np.random.default_rng(2).standard_normal(J.n)
    z = mg.apply(r)
    assert np.allclose(z, np.linalg.solve(J.dense(), r), rtol=1e-10, atol=0)
