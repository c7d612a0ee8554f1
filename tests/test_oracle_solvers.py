"""Pins of the oracle's solver components (Section 3) against facts fixed by
the mathematics: the defining property of ILU(0), exact LU on tridiagonal
matrices, dense Schwarz operators built here from the restriction matrices'
definitions, closed-form interpolation weights, the V-cycle error-propagation
identity, dense direct solves, and Newton's quadratic convergence."""
import numpy as np
import pytest

import synthetic as S


def _jac(orc, **kw):
    case = S.small_case(**kw)
    prob = orc.Problem(case.problems[0])
    rng = np.random.default_rng(11)
    p0 = prob.initial_pressure()
    p = p0 + 5e4 * rng.standard_normal(prob.N)
    J = prob.jacobian(p, p0, p0, 86400.0, 1)
    return case, prob, J


# --------------------------------------------------------------- ILU(0)
@pytest.mark.parametrize("dims", [(7, 6, 1), (4, 5, 3)])
def test_ilu0_defining_property(orc, dims):
    # ILU(0) factors reproduce A exactly on A's sparsity pattern: (LU)_ij = a_ij
    _, _, J = _jac(orc, nx=dims[0], ny=dims[1], nz=dims[2], gravity=dims[2] > 1)
    F = orc.ilu0(J)
    D = F.dense()
    L = np.tril(D, -1) + np.eye(J.n)
    U = np.triu(D)
    A = J.dense()
    mask = A != 0
    assert np.allclose((L @ U)[mask], A[mask], rtol=1e-12, atol=1e-12 * np.abs(A).max())
    # and the solve applies (LU)^{-1}
    r = np.random.default_rng(0).standard_normal(J.n)
    assert np.allclose(orc.ilu0_solve(F, r), np.linalg.solve(L @ U, r), rtol=1e-9)


def test_ilu0_general_pattern_property(orc):
    # the same property on a wide Galerkin stencil with fill inside its pattern
    case, prob, J = _jac(orc, nx=12, ny=10, px=1, py=1, levels=2)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    Ac = mg.level_matrix(1)
    F = orc.ilu0(Ac)
    D = F.dense()
    L = np.tril(D, -1) + np.eye(Ac.n)
    U = np.triu(D)
    A = Ac.dense()
    mask = A != 0
    assert np.allclose((L @ U)[mask], A[mask], rtol=1e-11, atol=1e-11 * np.abs(A).max())


def test_ilu0_is_exact_on_tridiagonal(orc):
    _, _, J = _jac(orc, nx=15, ny=1)
    F = orc.ilu0(J)
    r = np.random.default_rng(1).standard_normal(J.n)
    assert np.allclose(orc.ilu0_solve(F, r), np.linalg.solve(J.dense(), r), rtol=1e-12)


def test_ilu0_five_point_closed_form(orc):
    # on a 5-point stencil ILU(0) only modifies the diagonal:
    # d_i = a_ii - sum_{k<i} a_ik a_ki / d_k, L = A_lower D^{-1}, U = D + A_upper
    _, _, J = _jac(orc, nx=6, ny=5)
    A = J.dense()
    n = J.n
    d = np.zeros(n)
    for i in range(n):
        d[i] = A[i, i] - sum(A[i, k] * A[k, i] / d[k] for k in range(i) if A[i, k] != 0)
    F = orc.ilu0(J).dense()
    assert np.allclose(np.diag(F), d, rtol=1e-13)
    off_up = np.triu(F, 1)
    assert np.array_equal(off_up, np.triu(A, 1))
    lo = np.tril(F, -1)
    assert np.allclose(lo, np.tril(A, -1) / d[None, :], rtol=1e-13)


# --------------------------------------------------------------- one-level Schwarz
def _boxes(n, P):
    base, rem = divmod(n, P)
    out, lo = [], 0
    for q in range(P):
        hi = lo + base + (1 if q < rem else 0)
        out.append((lo, hi))
        lo = hi
    return out


def dense_schwarz(A, dims, P, delta, variant):
    """sum_i Ra_i^T A_i^{-1} Rb_i with exact subdomain inverses, from the
    definitions of R_i^delta and R_i^0 (Section 3.1)."""
    nx, ny, nz = dims
    n = A.shape[0]
    M = np.zeros((n, n))
    bx, by, bz = _boxes(nx, P[0]), _boxes(ny, P[1]), _boxes(nz, P[2])
    for (zl, zh) in bz:
        for (yl, yh) in by:
            for (xl, xh) in bx:
                ext, own = [], []
                for z in range(max(zl - delta, 0), min(zh + delta, nz)):
                    for y in range(max(yl - delta, 0), min(yh + delta, ny)):
                        for x in range(max(xl - delta, 0), min(xh + delta, nx)):
                            ext.append(x + nx * (y + ny * z))
                            own.append(xl <= x < xh and yl <= y < yh and zl <= z < zh)
                ext = np.array(ext)
                own = np.array(own)
                Rd = np.zeros((len(ext), n))
                Rd[np.arange(len(ext)), ext] = 1.0
                R0 = Rd * own[:, None]
                Ai = Rd @ A @ Rd.T
                Ainv = np.linalg.inv(Ai)
                if variant == "left_ras":
                    M += R0.T @ Ainv @ Rd
                elif variant == "as":
                    M += Rd.T @ Ainv @ Rd
                else:
                    M += Rd.T @ Ainv @ R0
    return M


def _apply_dense(fn, n):
    return np.column_stack([fn(e) for e in np.eye(n)])


@pytest.mark.parametrize("variant", ["left_ras", "as", "right_ras"])
@pytest.mark.parametrize("dims,P,delta", [((9, 7, 1), (3, 2, 1), 1), ((6, 5, 4), (2, 2, 2), 1),
                                          ((8, 8, 1), (2, 3, 1), 2)])
def test_schwarz_exact_subsolves_match_definition(orc, variant, dims, P, delta):
    case, prob, J = _jac(orc, nx=dims[0], ny=dims[1], nz=dims[2], gravity=dims[2] > 1,
                         px=P[0], py=P[1], pz=P[2], overlap=(delta,), subsolve="lu",
                         variant=variant)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    M = _apply_dense(mg.apply, J.n)
    Md = dense_schwarz(J.dense(), dims, P, delta, variant)
    assert np.allclose(M, Md, rtol=1e-10, atol=1e-10 * np.abs(Md).max())


def test_tile_option_sets_box_counts(orc):
    # a box edge t gives ceil(n/t) boxes per direction, split as for an explicit count
    dims = (11, 7, 1)
    case, prob, J = _jac(orc, nx=dims[0], ny=dims[1], tile=(4, 3, 0), overlap=(1,), subsolve="lu")
    mg = orc.Multilevel(prob.rec, J, case.solver)
    M = _apply_dense(mg.apply, J.n)
    Md = dense_schwarz(J.dense(), dims, (3, 3, 1), 1, "left_ras")
    assert np.allclose(M, Md, rtol=1e-10, atol=1e-10 * np.abs(Md).max())


@pytest.mark.parametrize("variant", ["left_ras", "as", "right_ras"])
def test_onelevel_transpose_apply_is_the_transpose(orc, variant):
    # the dense operator of apply_transpose is the transpose of apply's (ILU(0) subsolves)
    case, prob, J = _jac(orc, nx=9, ny=8, px=3, py=2, overlap=(2,), variant=variant)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    M = _apply_dense(mg.apply, J.n)
    MT = _apply_dense(mg.apply_transpose, J.n)
    assert np.allclose(MT, M.T, rtol=1e-12, atol=1e-12 * np.abs(M).max())


def test_zero_overlap_is_block_jacobi(orc):
    # delta = 0: AS, left-RAS and right-RAS all reduce to block Jacobi
    ops = []
    for variant in ("left_ras", "as", "right_ras"):
        case, prob, J = _jac(orc, nx=8, ny=6, px=2, py=3, overlap=(0,), variant=variant)
        mg = orc.Multilevel(prob.rec, J, case.solver)
        ops.append(_apply_dense(mg.apply, J.n))
    assert np.allclose(ops[0], ops[1], rtol=0, atol=0)
    assert np.allclose(ops[0], ops[2], rtol=0, atol=0)


def test_one_subdomain_is_global_ilu0(orc):
    case, prob, J = _jac(orc, nx=7, ny=6, px=1, py=1, overlap=(1,))
    mg = orc.Multilevel(prob.rec, J, case.solver)
    r = np.random.default_rng(3).standard_normal(J.n)
    assert np.allclose(mg.apply(r), orc.ilu0_solve(orc.ilu0(J), r), rtol=1e-14)


def test_left_ras_ilu_equals_owned_rows_of_local_ilu(orc):
    # with ILU(0) subdomain solves, each owned entry of z comes from its own
    # subdomain's local solve on the gathered overlapping box
    case, prob, J = _jac(orc, nx=10, ny=9, px=3, py=2, overlap=(2,))
    mg = orc.Multilevel(prob.rec, J, case.solver)
    r = np.random.default_rng(4).standard_normal(J.n)
    z = mg.apply(r)
    A = J.dense()
    zz = np.zeros(J.n)
    for s in range(6):
        sd = mg.subdomain(0, s)
        cells = sd["cells"]
        Ai = A[np.ix_(cells, cells)]
        import scipy.sparse as sp
        Acsr = sp.csr_matrix(Ai)
        Acsr.sort_indices()
        F = orc.ilu0(orc.CSR(Acsr.indptr, Acsr.indices, Acsr.data))
        zl = orc.ilu0_solve(F, r[cells])
        zz[cells[sd["owned"]]] += zl[sd["owned"]]
    assert np.allclose(z, zz, rtol=1e-13)


# --------------------------------------------------------------- interpolation
def test_interp_weights_closed_forms(orc):
    P2 = orc.interp_1d(8, 2).dense()
    # interior fine cells sit 1/4 coarse spacing from their parent centroid
    assert np.allclose(P2[2, 0:3], [0.25, 0.75, 0.0])
    assert np.allclose(P2[3, 0:3], [0.0, 0.75, 0.25])
    # boundary rows clamp to the edge cell
    assert np.allclose(P2[0, :2], [1.0, 0.0]) and np.allclose(P2[7, 2:], [0.0, 1.0])
    P3 = orc.interp_1d(12, 3).dense()
    # Keys cubic convolution (a = -1/2) at offset 1/4: (-9, 111, 29, -3)/128
    assert np.allclose(P3[5, 1:5], np.array([-9, 111, 29, -3]) / 128.0)
    assert np.allclose(P3[6, 1:5], np.array([-3, 29, 111, -9]) / 128.0)
    P1 = orc.interp_1d(9, 1).dense()
    assert np.array_equal(P1.argmax(1), np.arange(9) // 2) and np.all(P1.max(1) == 1.0)
    for P in (P1, P2, P3, orc.interp_1d(9, 2).dense()):
        assert np.allclose(P.sum(1), 1.0, rtol=0, atol=1e-15)


def test_interp_polynomial_reproduction(orc):
    nf = 32
    xf = np.arange(nf) + 0.5
    xc = 2.0 * np.arange(nf // 2) + 1.0
    P2 = orc.interp_1d(nf, 2).dense()
    P3 = orc.interp_1d(nf, 3).dense()
    inner = slice(3, nf - 3)
    assert np.allclose((P2 @ (3 * xc + 1))[1:-1], (3 * xf + 1)[1:-1])
    q = lambda x: 0.5 * x * x - 2 * x + 3
    assert np.allclose((P3 @ q(xc))[inner], q(xf)[inner])
    # odd sizes: the last coarse cell sits at its single fine cell's centre
    P = orc.interp_1d(9, 2).dense()
    assert P[8, 4] == 1.0


def _centroids(nf, r):
    # coarse cell J covers fine cells rJ .. min(rJ + r, nf) - 1
    nc = -(-nf // r)
    return np.array([(r * J + min(r * (J + 1), nf)) / 2.0 for J in range(nc)])


def test_interp_ratio_closed_forms(orc):
    # ratio 4: the fine cells of a coarse cell sit at -3/8, -1/8, 1/8, 3/8 of a
    # coarse spacing from its centroid, so the linear weights are 5/8 and 3/8,
    # 7/8 and 1/8, ...
    P = orc.interp_1d(16, 2, ratio=4).dense()
    assert P.shape == (16, 4)
    assert np.allclose(P[4, 0:3], [0.375, 0.625, 0.0])
    assert np.allclose(P[5, 0:3], [0.125, 0.875, 0.0])
    assert np.allclose(P[6, 0:3], [0.0, 0.875, 0.125])
    assert np.allclose(P[7, 0:3], [0.0, 0.625, 0.375])
    # ratio 8, first order: each coarse cell is the parent of 8 fine cells
    P1 = orc.interp_1d(20, 1, ratio=8).dense()
    assert P1.shape == (20, 3)
    assert np.array_equal(P1.argmax(1), np.arange(20) // 8) and np.all(P1.max(1) == 1.0)
    # ratio 16, third order on uniform spacing: the cubic convolution kernel at
    # the fine centres' offsets (k + 1/2 - 8)/16
    P3 = orc.interp_1d(96, 3, ratio=16).dense()
    W = lambda t: (1.5 * abs(t) ** 3 - 2.5 * t * t + 1) if abs(t) < 1 else \
        ((-0.5 * abs(t) ** 3 + 2.5 * t * t - 4 * abs(t) + 2) if abs(t) < 2 else 0.0)
    for k in range(16):
        i = 2 * 16 + k
        sx = (i + 0.5 - 8.0) / 16.0
        ref = np.array([W(sx - J) for J in range(6)])
        assert np.allclose(P3[i], ref, atol=1e-15), (k, P3[i], ref)
    for M in (P, P1, P3):
        assert np.allclose(M.sum(1), 1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("nf,r", [(9, 2), (13, 2), (21, 4), (30, 4), (37, 8), (50, 16), (64, 16)])
def test_interp_uses_actual_centroids(orc, nf, r):
    # readings for sizes r does not divide: the short last coarse cell sits at
    # its centroid, and orders 2 and 3 interpolate in the coordinate that is
    # linear between consecutive centroids.  Order 2 then reproduces linear
    # functions of x between the first and last centroids; order 3 reproduces
    # s, s^2 (s the index coordinate) wherever its four cells are in range
    c = _centroids(nf, r)
    nc = len(c)
    x = np.arange(nf) + 0.5
    P2 = orc.interp_1d(nf, 2, ratio=r).dense()
    P3 = orc.interp_1d(nf, 3, ratio=r).dense()
    assert P2.shape == (nf, nc) and P3.shape == (nf, nc)
    inside = (x >= c[0]) & (x <= c[-1])
    assert np.allclose((P2 @ c)[inside], x[inside], atol=1e-12)
    s = np.interp(x, c, np.arange(nc, dtype=float))
    J = np.arange(nc, dtype=float)
    rows = (np.floor(s) >= 1) & (np.floor(s) <= nc - 3)
    for k in (0, 1, 2):
        assert np.allclose((P3 @ J ** k)[rows], (s ** k)[rows], atol=1e-12), k
    for M in (P2, P3):
        assert np.allclose(M.sum(1), 1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("ratio,order,K", [(4, 2, 21), (8, 2, 21), (4, 1, 5), (16, 1, 5)])
def test_galerkin_with_ratio(orc, ratio, order, K):
    # P^T A P with coarse-to-fine ratio r: the same Galerkin definition, and
    # the coarse stencil keeps its reach (the supports of P's columns scale
    # with r like the coarse spacing does)
    case, prob, J = _jac(orc, nx=64, ny=48, px=2, py=2, levels=2, ratio=ratio, interp_order=order)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    info = mg.level_info(1)
    assert info["dims"][:2] == (-(-64 // ratio), -(-48 // ratio))
    P = mg.level_prolong(0).dense()
    Ac = mg.level_matrix(1).dense()
    assert np.allclose(Ac, P.T @ J.dense() @ P, rtol=1e-12, atol=1e-12 * np.abs(Ac).max())
    assert np.diff(mg.level_matrix(1).rp).max() == K


def test_vcycle_identity_with_ratio_4(orc):
    case, prob, J = _jac(orc, nx=24, ny=20, px=2, py=2, levels=2, overlap=(1, 1), ratio=4,
                         coarse_rtol=1e-14, coarse_maxit=400)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    B = _apply_dense(mg.apply, J.n)
    M = _apply_dense(lambda e: mg.apply_onelevel(0, e), J.n)
    P = mg.level_prolong(0).dense()
    assert P.shape == (J.n, 6 * 5)
    A = J.dense()
    C = P @ np.linalg.inv(P.T @ A @ P) @ P.T
    I = np.eye(A.shape[0])
    assert np.allclose(I - A @ B, (I - A @ M) @ (I - A @ C) @ (I - A @ M), atol=1e-8)


def test_galerkin_stencil_sizes(orc):
    # bilinear P^T A P on a 5-point / 7-point operator: 21 / 81 points on the
    # first coarse level, 25 / 125 on the next (interior rows)
    case, prob, J = _jac(orc, nx=32, ny=32, px=1, py=1, levels=3)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    A1, A2 = mg.level_matrix(1), mg.level_matrix(2)
    assert np.diff(A1.rp).max() == 21 and np.diff(A2.rp).max() == 25
    case, prob, J = _jac(orc, nx=24, ny=24, nz=24, px=1, py=1, pz=1, levels=3, gravity=True)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    assert np.diff(mg.level_matrix(1).rp).max() == 81
    assert np.diff(mg.level_matrix(2).rp).max() == 125


def test_galerkin_equals_dense_product(orc):
    case, prob, J = _jac(orc, nx=10, ny=9, px=2, py=2, levels=2, interp_order=3)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    P = mg.level_prolong(0).dense()
    Ac = mg.level_matrix(1).dense()
    assert np.allclose(Ac, P.T @ J.dense() @ P, rtol=1e-12, atol=1e-12 * np.abs(Ac).max())


# --------------------------------------------------------------- multilevel compositions
def _two_level_ops(orc, cycle, mu=1, nu=1, dims=(12, 10, 1), order=2):
    # coarse solve made exact: one coarse subdomain with dense LU and a tiny
    # coarse tolerance, so M_{h_0}^{-1} = A_c^{-1}
    case, prob, J = _jac(orc, nx=dims[0], ny=dims[1], nz=dims[2], px=2, py=2, levels=2,
                         overlap=(1, 1), cycle=cycle, mu=mu, nu=nu, coarse_rtol=1e-14,
                         interp_order=order)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    B = _apply_dense(mg.apply, J.n)
    M = _apply_dense(lambda e: mg.apply_onelevel(0, e), J.n)
    P = mg.level_prolong(0).dense()
    A = J.dense()
    C = P @ np.linalg.inv(P.T @ A @ P) @ P.T
    return A, B, M, C


def test_vcycle_error_propagation_identity(orc):
    # the two-level V-cycle preconditioner of Section 3.2 with mu = nu = 1:
    # I - A B = (I - A M)(I - A P A_c^{-1} P^T)(I - A M)
    A, B, M, C = _two_level_ops(orc, "vcycle")
    I = np.eye(A.shape[0])
    E = (I - A @ M) @ (I - A @ C) @ (I - A @ M)
    assert np.allclose(I - A @ B, E, atol=1e-8)


@pytest.mark.parametrize("cycle", ["left_kaskade", "right_kaskade", "additive", "coarse_only"])
def test_two_level_compositions(orc, cycle):
    A, B, M, C = _two_level_ops(orc, cycle, order=1 if cycle == "additive" else 2)
    ref = {
        "left_kaskade": C + M - M @ A @ C,      # left Kaskade
        "right_kaskade": M + C - C @ A @ M,     # right Kaskade
        "additive": C + M,                      # additive
        "coarse_only": C,                       # coarse only
    }[cycle]
    assert np.allclose(B, ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())


@pytest.mark.parametrize("cycle,mu,nu,levels,variant", [
    ("vcycle", 1, 1, 2, "left_ras"), ("vcycle", 1, 2, 2, "left_ras"), ("vcycle", 2, 1, 3, "as"),
    ("left_kaskade", 1, 1, 2, "left_ras"), ("right_kaskade", 1, 1, 2, "right_ras"),
    ("additive", 1, 1, 2, "left_ras"), ("coarse_only", 1, 1, 3, "left_ras")])
def test_multilevel_transpose_apply_is_the_transpose(orc, cycle, mu, nu, levels, variant):
    # with the coarsest solve converged to rounding the multilevel map is
    # linear, and apply_transpose must be the transpose of its dense matrix:
    # pre- and post-smoothing trade places, left and right Kaskade exchange
    case, prob, J = _jac(orc, nx=12, ny=10, px=2, py=2, levels=levels, overlap=(1,) * levels,
                         cycle=cycle, mu=mu, nu=nu, coarse_rtol=1e-14, coarse_maxit=400,
                         variant=variant)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    B = _apply_dense(mg.apply, J.n)
    BT = _apply_dense(mg.apply_transpose, J.n)
    assert np.allclose(BT, B.T, rtol=1e-8, atol=1e-8 * np.abs(B).max())
    if cycle == "vcycle" and mu != nu:
        # and it is not the cycle itself transposed term by term without the swap
        assert not np.allclose(B, B.T, rtol=1e-3, atol=1e-3 * np.abs(B).max())


# --------------------------------------------------------------- Krylov
@pytest.mark.parametrize("dims", [(4, 4, 1), (6, 6, 1), (4, 4, 3)])
def test_gmres_matches_dense_solve(orc, dims):
    case, prob, J = _jac(orc, nx=dims[0], ny=dims[1], nz=dims[2], gravity=dims[2] > 1)
    b = np.random.default_rng(5).standard_normal(J.n)
    xd = np.linalg.solve(J.dense(), b)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    for M in (None, mg):
        x, its, res, st = orc.gmres(J, b, M=M, rtol=1e-13, atol=0.0, restart=64)
        assert st == 0 and np.allclose(x, xd, rtol=1e-9, atol=1e-9 * np.abs(xd).max())
        assert its <= 2 * J.n   # finite termination up to MGS rounding


def test_gmres_one_iteration_with_exact_preconditioner(orc):
    case, prob, J = _jac(orc, nx=6, ny=5, px=1, py=1, subsolve="lu")
    mg = orc.Multilevel(prob.rec, J, case.solver)
    b = np.random.default_rng(6).standard_normal(J.n)
    x, its, res, st = orc.gmres(J, b, M=mg, rtol=1e-10, atol=0.0)
    assert its == 1 and np.allclose(x, np.linalg.solve(J.dense(), b), rtol=1e-10)


def test_gmres_minimises_residual_over_krylov_space(orc):
    case, prob, J = _jac(orc, nx=7, ny=6)
    A = J.dense()
    b = np.random.default_rng(7).standard_normal(J.n)
    for k in (1, 3, 6):
        x, its, _, _ = orc.gmres(J, b, rtol=0.0, atol=0.0, maxit=k, restart=30)
        assert its == k
        K = np.column_stack([np.linalg.matrix_power(A, j) @ b for j in range(k)])
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
        assert np.isclose(np.linalg.norm(b - A @ x), np.linalg.norm(b - A @ Q @ y), rtol=1e-7)


def test_fgmres_equals_gmres_for_fixed_preconditioner(orc):
    case, prob, J = _jac(orc, nx=9, ny=8, px=3, py=2)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    b = np.random.default_rng(8).standard_normal(J.n)
    x1, i1, _, _ = orc.gmres(J, b, M=mg, rtol=1e-8, atol=0.0)
    x2, i2, _, _ = orc.gmres(J, b, M=mg, rtol=1e-8, atol=0.0, flexible=True)
    assert i1 == i2 and np.allclose(x1, x2, rtol=1e-7, atol=1e-9 * np.abs(x1).max())


def test_gmres_restart_and_transpose(orc):
    case, prob, J = _jac(orc, nx=10, ny=10)
    b = np.random.default_rng(9).standard_normal(J.n)
    mg = orc.Multilevel(prob.rec, J, case.solver)
    # GMRES(10) needs several restart cycles here (GMRES(5) stagnates)
    x, its, res, st = orc.gmres(J, b, M=mg, restart=10, rtol=1e-10, atol=0.0)
    assert st == 0 and its > 30
    assert np.allclose(J.dense() @ x, b, atol=1e-9 * np.linalg.norm(b))
    xt, _, _, st = orc.gmres(J, b, M=mg, restart=30, rtol=1e-11, atol=0.0, transpose=True)
    assert st == 0 and np.allclose(J.dense().T @ xt, b, atol=1e-9 * np.linalg.norm(b))


# --------------------------------------------------------------- Newton
def test_newton_quadratic_convergence(orc):
    # exact Jacobian and exact linear solves: the norms fall quadratically
    # (order estimate log(f3/f2)/log(f2/f1) near 2 while above the rounding floor)
    case = S.small_case(nx=10, ny=10, rate=0.3, px=1, py=1, subsolve="lu", eps_r=1e-12,
                        eps_a=1e-6, eta_r=1e-14, eta_a=0.0, dt=20 * S.DAY, kmean_md=1.0)
    prob = orc.Problem(case.problems[0])
    p0 = prob.initial_pressure()
    p, st = orc.newton_step(prob, case.solver, p0, p0, p0, case.dt, 1)
    f = [st["fnorm0"]] + st["fnorms"]
    assert st["status"] == 0 and all(l == 1.0 for l in st["lambdas"])
    f = [x for x in f if x > 1e-4]
    assert len(f) >= 4
    order = np.log(f[-1] / f[-2]) / np.log(f[-2] / f[-3])
    assert 1.8 < order < 2.6, f


def test_newton_stops_at_rounding_floor(orc):
    # eps_r far below what binary64 residuals can reach: with neither the
    # rounding-floor test nor the relative step test the line search must
    # fail at the floor; with either one Newton stops, and the pressure agrees
    # with a solve stopped by the ordinary test at a reachable tolerance
    case = S.small_case(nx=16, ny=12, seed=8, sigma=2.0, rate=2e-3, eps_r=1e-15, eps_a=0.0,
                        eta_r=1e-12, eta_a=0.0)
    prob = orc.Problem(case.problems[0])
    p0 = prob.initial_pressure()
    run = lambda **kw: orc.newton_step(prob, S.with_solver(case, **kw).solver, p0, p0, p0, case.dt, 1)
    _, st_off = run(floor_test=False, stol=0.0)
    assert st_off["status"] != 0
    ref, st_ref = run(eps_r=1e-8, floor_test=False, stol=0.0)
    assert st_ref["status"] == 0
    for kw in (dict(floor_test=True, stol=0.0), dict(floor_test=False, stol=1e-8)):
        p, st = run(**kw)
        assert st["status"] == 0 and st["newton_its"] <= 6, kw
        assert np.max(np.abs(p - ref)) <= 1e-9 * np.max(np.abs(ref - p0)), kw
    # the floor test never fires while the residual is well above u |J| |p|
    _, st_tight = run(eps_r=1e-6, floor_test=True)
    _, st_plain = run(eps_r=1e-6, floor_test=False)
    assert st_tight["newton_its"] == st_plain["newton_its"]
