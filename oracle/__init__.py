"""Plain FP64 CPU oracle of the Newton-Krylov-Schwarz hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The GPU library never loads it.

The arithmetic lives in ``nks_oracle.c`` (built with gcc into
``liboracle.so``); this module only marshals NumPy arrays.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nks_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CYCLES = {"vcycle": 0, "left_kaskade": 1, "right_kaskade": 2, "additive": 3, "coarse_only": 4}
VARIANTS = {"left_ras": 0, "as": 1, "right_ras": 2}
SUBSOLVES = {"ilu0": 0, "lu": 1}


def build(force=False):
    """Compile the oracle with gcc (O2, no fast-math: IEEE semantics kept)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class MgDesc(C.Structure):
    _fields_ = [("px", C.c_int), ("py", C.c_int), ("pz", C.c_int), ("levels", C.c_int),
                ("overlap", C.c_int * 8), ("variant", C.c_int), ("subsolve", C.c_int),
                ("interp_order", C.c_int), ("cycle", C.c_int), ("mu", C.c_int), ("nu", C.c_int),
                ("coarse_rtol", C.c_double), ("coarse_maxit", C.c_int),
                ("coarse_restart", C.c_int), ("tx", C.c_int), ("ty", C.c_int), ("tz", C.c_int),
                ("fill", C.c_int), ("ratio", C.c_int), ("coarse_op", C.c_int)]


class NewtonDesc(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("eps_a", C.c_double), ("eta_r", C.c_double),
                ("eta_a", C.c_double), ("restart", C.c_int), ("maxit", C.c_int),
                ("flexible", C.c_int), ("alpha", C.c_double), ("max_newton", C.c_int),
                ("max_backtracks", C.c_int), ("stol", C.c_double), ("floor_test", C.c_int),
                ("lag", C.c_int)]


class NewtonStats(C.Structure):
    _fields_ = [("newton_its", C.c_int), ("linear_its", C.c_int), ("status", C.c_int),
                ("fnorm0", C.c_double), ("fnorm", C.c_double), ("fnorms", C.c_double * 64),
                ("lits", C.c_int * 64), ("lambdas", C.c_double * 64)]


_lib = None
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        L.orc_problem_new.restype = C.c_void_p
        L.orc_problem_new.argtypes = [C.c_int] * 3 + [C.c_double] * 3 + [_D] * 4 + [C.c_int, _I, _D] + \
            [C.c_double] * 7 + [C.c_int, C.c_double]
        L.orc_problem_free.argtypes = [C.c_void_p]
        L.orc_problem_set_bc.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double]
        L.orc_problem_set_bc.restype = C.c_int
        L.orc_problem_set_accum.argtypes = [C.c_void_p, C.c_int]
        L.orc_problem_set_accum.restype = C.c_int
        L.orc_mg_new_problem.restype = C.c_void_p
        L.orc_mg_new_problem.argtypes = [C.c_void_p, _D, C.c_double, C.c_int, _I, _I, _D, C.POINTER(MgDesc)]
        L.orc_pr_z2.argtypes = [C.c_double] * 5 + [_D] * 4
        L.orc_pr_z2.restype = C.c_int
        L.orc_pr_params.argtypes = [C.c_double] * 5 + [_D] * 3
        L.orc_acentric_terms.argtypes = [C.c_double, _D, _D]
        L.orc_acentric.argtypes = [C.c_double] * 3
        L.orc_acentric.restype = C.c_double
        L.orc_pr_z.argtypes = [C.c_double] * 5 + [_D, _D]
        L.orc_pr_z.restype = C.c_int
        L.orc_pr_eval.argtypes = [C.c_void_p, C.c_int, _D, _D, _D, _D, _D]
        L.orc_transmissibility.argtypes = [C.c_void_p, _D, _D, _D]
        L.orc_residual.argtypes = [C.c_void_p, _D, _D, _D, C.c_double, C.c_int, _D]
        L.orc_jacobian.argtypes = [C.c_void_p, _D, _D, _D, C.c_double, C.c_int, _I, _I, _D]
        L.orc_jacobian.restype = C.c_int
        L.orc_hydrostatic.argtypes = [C.c_void_p, C.c_double, _D]
        L.orc_residual_dlogk_t.argtypes = [C.c_void_p, _D, _D, _D]
        L.orc_mg_new.restype = C.c_void_p
        L.orc_mg_new.argtypes = [C.c_int] * 4 + [_I, _I, _D, C.POINTER(MgDesc)]
        L.orc_mg_free.argtypes = [C.c_void_p]
        L.orc_mg_apply.argtypes = [C.c_void_p, _D, _D]
        L.orc_mg_apply_transpose.argtypes = [C.c_void_p, _D, _D]
        L.orc_mg_apply_onelevel.argtypes = [C.c_void_p, C.c_int, _D, _D]
        L.orc_mg_level_info.argtypes = [C.c_void_p, C.c_int, _I]
        L.orc_mg_level_info.restype = C.c_int
        L.orc_mg_level_matrix.argtypes = [C.c_void_p, C.c_int, _I, _I, _D]
        L.orc_mg_level_prolong.argtypes = [C.c_void_p, C.c_int, _I, _I, _D]
        L.orc_mg_sub_info.argtypes = [C.c_void_p, C.c_int, C.c_int, _I]
        L.orc_mg_sub_info.restype = C.c_int
        L.orc_mg_sub_factors.argtypes = [C.c_void_p, C.c_int, C.c_int, _I, _I, _I, _I, _D]
        L.orc_csr_matvec.argtypes = [C.c_int, _I, _I, _D, _D, _D]
        L.orc_interp_1d.argtypes = [C.c_int, C.c_int, _I, _I, _D]
        L.orc_interp_1d_r.argtypes = [C.c_int, C.c_int, C.c_int, _I, _I, _D]
        L.orc_ilu0.argtypes = [C.c_int, _I, _I, _D]
        L.orc_ilu0_solve.argtypes = [C.c_int, _I, _I, _D, _D, _D]
        L.orc_gmres.argtypes = [C.c_int, _I, _I, _D, C.c_void_p, C.c_int, _D, _D, C.c_int,
                                C.c_double, C.c_double, C.c_int, C.c_int, _D, _I]
        L.orc_gmres.restype = C.c_int
        L.orc_newton_step.argtypes = [C.c_void_p, C.POINTER(MgDesc), C.POINTER(NewtonDesc), _D, _D, _D,
                                      C.c_double, C.c_int, C.POINTER(NewtonStats)]
        L.orc_newton_step.restype = C.c_int
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _i(a):
    return a.ctypes.data_as(_I)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def acentric_terms(Tr):
    f0, f1 = C.c_double(), C.c_double()
    lib().orc_acentric_terms(Tr, C.byref(f0), C.byref(f1))
    return f0.value, f1.value


def acentric(pc, Tc, Tb):
    return lib().orc_acentric(pc, Tc, Tb)


def pr_params(fluid):
    a, b, m = C.c_double(), C.c_double(), C.c_double()
    tb = getattr(fluid, "Tb", None)
    omega = lib().orc_acentric(fluid.pc, fluid.Tc, tb) if tb else fluid.omega
    lib().orc_pr_params(fluid.Tc, fluid.pc, omega, fluid.T, fluid.R,
                        C.byref(a), C.byref(b), C.byref(m))
    return a.value, b.value, m.value


def pr_z(fluid, p):
    """Largest real root Z of the PR cubic and dZ/dp at scalar pressure p."""
    a, b, _ = pr_params(fluid)
    Z, dZ = C.c_double(), C.c_double()
    bad = lib().orc_pr_z(a, b, fluid.T, fluid.R, float(p), C.byref(Z), C.byref(dZ))
    return Z.value, dZ.value, bad


ACCUM_FORMS = {"conservative": 0, "chain_rule": 1}
COARSE_OPS = {"galerkin": 0, "rediscretised": 1}


def pr_z2_ab(a, b, T, R, p):
    """Z, dZ/dp, d2Z/dp2 and d2m/dp2 (m = p/Z) at scalar pressure p."""
    Z, dZ, d2Z, d2m = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    lib().orc_pr_z2(a, b, T, R, float(p), C.byref(Z), C.byref(dZ), C.byref(d2Z), C.byref(d2m))
    return Z.value, dZ.value, d2Z.value, d2m.value


def pr_z_ab(a, b, T, R, p):
    Z, dZ = C.c_double(), C.c_double()
    bad = lib().orc_pr_z(a, b, T, R, float(p), C.byref(Z), C.byref(dZ))
    return Z.value, dZ.value, bad


class CSR:
    def __init__(self, rp, ci, v, ncols=None):
        self.rp, self.ci, self.v = _i32(rp), _i32(ci), _f64(v)
        self.n = len(self.rp) - 1
        self.m = self.n if ncols is None else ncols

    def dense(self):
        A = np.zeros((self.n, self.m))
        for i in range(self.n):
            A[i, self.ci[self.rp[i]:self.rp[i + 1]]] += self.v[self.rp[i]:self.rp[i + 1]]
        return A

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.v, self.ci, self.rp), shape=(self.n, self.m))

    def matvec(self, x):
        x = _f64(x)
        y = np.zeros(self.n)
        lib().orc_csr_matvec(self.n, _i(self.rp), _i(self.ci), _d(self.v), _d(x), _d(y))
        return y


class Problem:
    """Oracle handle for one reservoir (synthetic.configs.Problem record)."""

    def __init__(self, rec):
        self.rec = rec
        f = rec.fluid
        self._keep = [_f64(rec.kx), _f64(rec.ky), _f64(rec.kz), _f64(rec.phi),
                      _i32(rec.well_cells), _f64(rec.well_rates)]
        kx, ky, kz, phi, wc, wr = self._keep
        # omega from the normal boiling point when the record gives one (Section 2)
        tb = getattr(f, "Tb", None)
        omega = lib().orc_acentric(f.pc, f.Tc, tb) if tb else f.omega
        self.h = lib().orc_problem_new(rec.nx, rec.ny, rec.nz, rec.dx, rec.dy, rec.dz,
                                       _d(kx), _d(ky), _d(kz), _d(phi), len(wc), _i(wc), _d(wr),
                                       f.Tc, f.pc, omega, f.T, f.W, f.R, f.mu,
                                       1 if rec.gravity else 0, rec.g)
        for f, (t, v) in enumerate(zip(rec.bc_type, rec.bc_value)):
            if lib().orc_problem_set_bc(self.h, f, int(t), float(v)) != 0:
                raise ValueError(f"bad boundary condition on face {f}: type {t}, value {v}")
        form = ACCUM_FORMS[getattr(rec, "accum", "conservative")]
        if lib().orc_problem_set_accum(self.h, form) != 0:
            raise ValueError(f"bad accumulation form {rec.accum}")
        self.N = rec.N

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_problem_free(self.h)
            self.h = None

    def pr(self, p):
        p = _f64(p)
        n = p.size
        Z, dZ, m, dm = (np.zeros(n) for _ in range(4))
        lib().orc_pr_eval(self.h, n, _d(p), _d(Z), _d(dZ), _d(m), _d(dm))
        return Z, dZ, m, dm

    def transmissibility(self):
        t = [np.zeros(self.N) for _ in range(3)]
        lib().orc_transmissibility(self.h, *[_d(x) for x in t])
        return t

    def residual(self, p, pn, pnm1=None, dt=86400.0, order=1):
        p, pn = _f64(p), _f64(pn)
        pnm1 = _f64(pn if pnm1 is None else pnm1)
        F = np.zeros(self.N)
        lib().orc_residual(self.h, _d(p), _d(pn), _d(pnm1), dt, order, _d(F))
        return F

    def jacobian(self, p, pn, pnm1=None, dt=86400.0, order=1):
        p, pn = _f64(p), _f64(pn)
        pnm1 = _f64(pn if pnm1 is None else pnm1)
        rp = np.zeros(self.N + 1, np.int32)
        ci = np.zeros(7 * self.N, np.int32)
        v = np.zeros(7 * self.N)
        nnz = lib().orc_jacobian(self.h, _d(p), _d(pn), _d(pnm1), dt, order, _i(rp), _i(ci), _d(v))
        return CSR(rp, ci[:nnz], v[:nnz])

    def hydrostatic(self, p_top):
        p = np.zeros(self.N)
        lib().orc_hydrostatic(self.h, float(p_top), _d(p))
        return p

    def initial_pressure(self):
        if self.rec.gravity:
            return self.hydrostatic(self.rec.p_init)
        return np.full(self.N, float(self.rec.p_init))

    def residual_dlogk_t(self, p, lam):
        out = np.zeros(self.N)
        lib().orc_residual_dlogk_t(self.h, _d(_f64(p)), _d(_f64(lam)), _d(out))
        return out


def mg_desc(s):
    """MgDesc from a synthetic.configs.SolverSettings record."""
    d = MgDesc()
    d.px, d.py, d.pz = s.px, s.py, s.pz
    d.levels = s.levels
    ov = list(s.overlap) + [s.overlap[-1]] * 8
    for k in range(8):
        d.overlap[k] = ov[k]
    d.variant = VARIANTS[s.variant]
    d.subsolve = SUBSOLVES[s.subsolve]
    d.interp_order = s.interp_order
    d.cycle = CYCLES[s.cycle]
    d.mu, d.nu = s.mu, s.nu
    d.coarse_rtol = s.coarse_rtol
    d.coarse_maxit = s.coarse_maxit
    d.coarse_restart = s.coarse_restart
    d.tx, d.ty, d.tz = s.tile
    d.fill = s.fill
    d.ratio = getattr(s, "ratio", 2)
    d.coarse_op = COARSE_OPS[getattr(s, "coarse_op", "galerkin")]
    return d


def newton_desc(s):
    d = NewtonDesc()
    d.eps_r, d.eps_a, d.eta_r, d.eta_a = s.eps_r, s.eps_a, s.eta_r, s.eta_a
    d.restart, d.maxit = s.restart, s.maxit
    flex = s.flexible if s.flexible is not None else (s.levels > 1 or s.precision != "fp64")
    d.flexible = 1 if flex else 0
    d.alpha = s.alpha
    d.max_newton, d.max_backtracks = s.max_newton, s.max_backtracks
    d.stol = s.stol
    d.floor_test = 1 if s.floor_test else 0
    d.lag = s.lag
    return d


class Multilevel:
    """Oracle multilevel Schwarz preconditioner built from a fine CSR matrix."""

    def __init__(self, rec_or_dims, J, settings, state=None):
        """state = (p, dt, order): the state rediscretised coarse levels are
        evaluated at (needs a reservoir record, not bare dimensions)."""
        if hasattr(rec_or_dims, "nx"):
            dims = (rec_or_dims.nx, rec_or_dims.ny, rec_or_dims.nz)
        else:
            dims = tuple(rec_or_dims)
        self.J = J
        self.desc = mg_desc(settings)
        if state is not None:
            self._prob = Problem(rec_or_dims)
            p, dt, order = state
            self._p = _f64(p)
            self.h = lib().orc_mg_new_problem(self._prob.h, _d(self._p), float(dt), int(order), _i(J.rp),
                                              _i(J.ci), _d(J.v), C.byref(self.desc))
        else:
            self.h = lib().orc_mg_new(dims[0], dims[1], dims[2], J.n, _i(J.rp), _i(J.ci), _d(J.v),
                                      C.byref(self.desc))
        if not self.h:
            raise ValueError("the preconditioner could not be built (rediscretised coarse levels need the "
                             "problem and sizes the ratio divides)")
        self.L = settings.levels

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_mg_free(self.h)
            self.h = None

    def apply(self, r):
        r = _f64(r)
        z = np.zeros(self.J.n)
        lib().orc_mg_apply(self.h, _d(r), _d(z))
        return z

    def apply_transpose(self, r):
        r = _f64(r)
        z = np.zeros(self.J.n)
        lib().orc_mg_apply_transpose(self.h, _d(r), _d(z))
        return z

    def level_info(self, lev):
        info = np.zeros(8, np.int32)
        lib().orc_mg_level_info(self.h, lev, _i(info))
        return dict(n=int(info[0]), nnz=int(info[1]), dims=tuple(int(x) for x in info[2:5]),
                    nsub=int(info[5]), nc=int(info[6]), pnnz=int(info[7]))

    def apply_onelevel(self, lev, r):
        r = _f64(r)
        n = self.level_info(lev)["n"]
        z = np.zeros(n)
        lib().orc_mg_apply_onelevel(self.h, lev, _d(r), _d(z))
        return z

    def level_matrix(self, lev):
        inf = self.level_info(lev)
        rp = np.zeros(inf["n"] + 1, np.int32)
        ci = np.zeros(inf["nnz"], np.int32)
        v = np.zeros(inf["nnz"])
        lib().orc_mg_level_matrix(self.h, lev, _i(rp), _i(ci), _d(v))
        return CSR(rp, ci, v)

    def level_prolong(self, lev):
        inf = self.level_info(lev)
        rp = np.zeros(inf["n"] + 1, np.int32)
        ci = np.zeros(inf["pnnz"], np.int32)
        v = np.zeros(inf["pnnz"])
        lib().orc_mg_level_prolong(self.h, lev, _i(rp), _i(ci), _d(v))
        return CSR(rp, ci, v, ncols=inf["nc"])

    def subdomain(self, lev, s):
        info = np.zeros(14, np.int32)
        lib().orc_mg_sub_info(self.h, lev, s, _i(info))
        n, nnz = int(info[0]), int(info[1])
        cells = np.zeros(n, np.int32)
        owned = np.zeros(n, np.int32)
        rp = np.zeros(n + 1, np.int32)
        ci = np.zeros(nnz, np.int32)
        v = np.zeros(nnz)
        lib().orc_mg_sub_factors(self.h, lev, s, _i(cells), _i(owned), _i(rp), _i(ci), _d(v))
        return dict(cells=cells, owned=owned.astype(bool), factors=CSR(rp, ci, v),
                    lo=tuple(info[2:5]), hi=tuple(info[5:8]), elo=tuple(info[8:11]),
                    ehi=tuple(info[11:14]))


def gmres(J, b, M=None, x0=None, restart=30, rtol=1e-5, atol=1e-8, maxit=10000,
          flexible=False, transpose=False):
    b = _f64(b)
    x = np.zeros(J.n) if x0 is None else _f64(x0).copy()
    res = C.c_double()
    its = C.c_int()
    st = lib().orc_gmres(J.n, _i(J.rp), _i(J.ci), _d(J.v), M.h if M is not None else None,
                         1 if transpose else 0, _d(b), _d(x), restart, rtol, atol, maxit,
                         1 if flexible else 0, C.byref(res), C.byref(its))
    return x, its.value, res.value, st


def interp_1d(nf, order, ratio=2):
    rp = np.zeros(nf + 1, np.int32)
    ci = np.zeros(4 * nf, np.int32)
    w = np.zeros(4 * nf)
    lib().orc_interp_1d_r(nf, order, ratio, _i(rp), _i(ci), _d(w))
    return CSR(rp, ci[:rp[-1]], w[:rp[-1]], ncols=(nf + ratio - 1) // ratio)


def ilu0(A):
    v = A.v.copy()
    lib().orc_ilu0(A.n, _i(A.rp), _i(A.ci), _d(v))
    return CSR(A.rp, A.ci, v)


def ilu0_solve(F, r):
    r = _f64(r)
    z = np.zeros(F.n)
    lib().orc_ilu0_solve(F.n, _i(F.rp), _i(F.ci), _d(F.v), _d(r), _d(z))
    return z


def newton_step(prob, settings, p, pn, pnm1, dt, order):
    p = _f64(p).copy()
    pn = _f64(pn)
    pnm1 = _f64(pnm1)
    md, nd, st = mg_desc(settings), newton_desc(settings), NewtonStats()
    lib().orc_newton_step(prob.h, C.byref(md), C.byref(nd), _d(p), _d(pn), _d(pnm1), dt, order,
                          C.byref(st))
    k = st.newton_its
    return p, dict(newton_its=k, linear_its=st.linear_its, status=st.status,
                   fnorm0=st.fnorm0, fnorm=st.fnorm, fnorms=list(st.fnorms[:min(k, 64)]),
                   lits=list(st.lits[:min(k, 64)]), lambdas=list(st.lambdas[:min(k, 64)]))


def simulate(case, nsteps=None, p0=None):
    """Run the case's implicit steps (BDF1 first, BDF2 after) on every
    reservoir; returns per-reservoir pressure histories and per-step stats."""
    out = []
    for rec in case.problems:
        prob = Problem(rec)
        p = prob.initial_pressure() if p0 is None else _f64(p0)
        hist = [p.copy()]
        stats = []
        for n in range(nsteps or case.nsteps):
            order = 1 if n == 0 else 2
            pn = hist[-1]
            pnm1 = hist[-2] if len(hist) > 1 else hist[-1]
            p, st = newton_step(prob, case.solver, pn, pn, pnm1, case.dt, order)
            hist.append(p.copy())
            stats.append(st)
        out.append((hist, stats))
    return out


def adjoint(prob, dt, hist, dGdp, orders=None):
    """Discrete adjoint of the implicit steps hist[0] -> hist[-1] (BDF1 first,
    BDF2 after, unless orders says otherwise) for an objective G whose
    gradient in state n is dGdp[n] (None: zero; entry 0 ignored: p^0 does not
    depend on K).  Written from the definition: with the Lagrangian
    G + sum_n lam_n^T F^n(p^n, p^{n-1}, p^{n-2}),
      J_n^T lam_n = -dG/dp^n - (dF^{n+1}/dp^n)^T lam_{n+1} - (dF^{n+2}/dp^n)^T lam_{n+2},
    where the couplings are the accumulation's dependence on earlier states
    (Section 2's BDF1/BDF2: m(p^n) enters F^{n+1} with coefficient -1 (BDF1)
    or -2 (BDF2) and F^{n+2} with 1/2, each times V phi / dt), and
      dG/dln K = sum_n (dF^n/dln K)^T lam_n.
    Each J_n^T system is solved directly (sparse LU).  Returns (grad, lams)."""
    import scipy.sparse.linalg as spla
    rec = prob.rec
    n = len(hist) - 1
    orders = orders or [1] + [2] * (n - 1)
    pv = rec.dx * rec.dy * rec.dz * _f64(rec.phi)
    lams = [None] * (n + 3)
    grad = np.zeros(prob.N)
    for k in range(n, 0, -1):
        _, _, _, dm = prob.pr(hist[k])
        rhs = -(np.zeros(prob.N) if dGdp[k] is None else _f64(dGdp[k]))
        if k + 1 <= n:
            c1 = -2.0 if orders[k] == 2 else -1.0
            rhs -= pv / dt * dm * c1 * lams[k + 1]
        if k + 2 <= n and orders[k + 1] == 2:
            rhs -= pv / dt * dm * 0.5 * lams[k + 2]
        pn = hist[k - 1]
        pnm1 = hist[k - 2] if k >= 2 else hist[k - 1]
        J = prob.jacobian(hist[k], pn, pnm1, dt, orders[k - 1]).scipy()
        lams[k] = spla.spsolve(J.T.tocsc(), rhs)
        grad += prob.residual_dlogk_t(hist[k], lams[k])
    return grad, lams[:n + 1]
