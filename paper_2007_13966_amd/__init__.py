"""MI355X Newton-Krylov-Schwarz hot path (arXiv 2007.13966) behind the libnks C ABI.

Thin Python binding: every computation runs in libnks.so (HIP kernels for
gfx950); this package marshals arguments, lets PyTorch provide device memory
(its caching allocator, via the ABI's allocator callback) and streams, and
converts results.  There is no CPU fallback: without the built library the
import of :mod:`paper_2007_13966_amd._lib` raises.
"""
import ctypes as C
import sys

import numpy as np

from . import _lib as L
from ._lib import (NKS_AS, NKS_BF16, NKS_COARSE_ONLY, NKS_FP32, NKS_FP64,  # noqa: F401
                   NKS_LEFT_KASKADE, NKS_LEFT_RAS, NKS_RIGHT_KASKADE, NKS_RIGHT_RAS,
                   NKS_ADDITIVE, NKS_VCYCLE, NksError)

_handle = None

VARIANTS = {"left_ras": NKS_LEFT_RAS, "as": NKS_AS, "right_ras": NKS_RIGHT_RAS}
CYCLES = {"vcycle": NKS_VCYCLE, "left_kaskade": NKS_LEFT_KASKADE,
          "right_kaskade": NKS_RIGHT_KASKADE, "additive": NKS_ADDITIVE,
          "coarse_only": NKS_COARSE_ONLY}
PRECISIONS = {"fp64": NKS_FP64, "fp32": NKS_FP32, "bf16": NKS_BF16}


def lib():
    global _handle
    if _handle is None:
        _handle = L.load()
    return _handle


def check(code):
    return L.check(lib(), code)


def _torch():
    import torch
    return torch


def _vp(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class TorchAllocator:
    """Allocator callback pair bound to PyTorch's caching allocator on one stream."""

    def __init__(self, device, stream):
        torch = _torch()
        self.device = device
        self.stream = stream

        def _alloc(size, ctx):
            return torch.cuda.caching_allocator_alloc(max(int(size), 8), self.device.index or 0,
                                                      self.stream)

        def _free(ptr, ctx):
            # frees can arrive while the interpreter shuts down
            tc = getattr(torch, "cuda", None)
            if tc is not None and getattr(tc, "caching_allocator_delete", None) is not None:
                tc.caching_allocator_delete(ptr)

        self.alloc = L.ALLOC_FN(_alloc)
        self.free = L.FREE_FN(_free)


def ras_desc(s):
    """nks_ras_desc from a synthetic.configs.SolverSettings record."""
    d = L.nks_ras_desc()
    d.px, d.py, d.pz = s.px, s.py, s.pz
    d.levels = s.levels
    ov = list(s.overlap) + [s.overlap[-1]] * 8
    for k in range(8):
        d.overlap[k] = ov[k]
    d.variant = VARIANTS[s.variant]
    d.interp_order = s.interp_order
    d.cycle = CYCLES[s.cycle]
    d.mu, d.nu = s.mu, s.nu
    d.coarse_rtol = s.coarse_rtol
    d.coarse_maxit = s.coarse_maxit
    d.coarse_restart = s.coarse_restart
    d.precision = PRECISIONS[s.precision]
    d.tx, d.ty, d.tz = s.tile
    d.fill = getattr(s, "fill", 0)
    d.ratio = getattr(s, "ratio", 2)
    d.coarse_op = {"galerkin": 0, "rediscretised": 1}[getattr(s, "coarse_op", "galerkin")]
    d.coarse_kernel = L.COARSE_KERNELS[getattr(s, "coarse_kernel", "auto")]
    return d


def newton_desc(s):
    d = L.nks_newton_desc()
    d.eps_r, d.eps_a, d.eta_r, d.eta_a = s.eps_r, s.eps_a, s.eta_r, s.eta_a
    d.restart, d.maxit = s.restart, s.maxit
    d.flexible = -1 if s.flexible is None else int(bool(s.flexible))
    d.alpha = s.alpha
    d.max_newton, d.max_backtracks = s.max_newton, s.max_backtracks
    d.stol = s.stol
    d.floor_test = 1 if s.floor_test else 0
    d.lag = getattr(s, "lag", 1)
    return d


class _Ordered:
    """Orders a library call on the grid stream after the caller's current
    stream, and the caller's stream after the call."""

    def __init__(self, grid):
        self.grid = grid

    def __enter__(self):
        torch = _torch()
        cur = torch.cuda.current_stream(self.grid.device)
        if cur.cuda_stream != self.grid.stream.cuda_stream:
            self.grid.stream.wait_stream(cur)
        return self

    def __exit__(self, *exc):
        torch = _torch()
        cur = torch.cuda.current_stream(self.grid.device)
        if cur.cuda_stream != self.grid.stream.cuda_stream:
            cur.wait_stream(self.grid.stream)
        return False


class Grid:
    """nks_grid over one or more reservoirs (synthetic.configs.Problem records)."""

    def __init__(self, problems, device="cuda:0", stream=None, torch_allocator=True):
        torch = _torch()
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        self.device = torch.device(device)
        # the library works on its own stream (default priority): graph capture
        # is not available on the legacy default stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        keep = []
        res = (L.nks_reservoir_desc * len(problems))()
        for k, pr in enumerate(problems):
            arrs = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)
                    for a in (pr.kx, pr.ky, pr.kz, pr.phi)]
            wc = np.ascontiguousarray(pr.well_cells, dtype=np.int32)
            wr = np.ascontiguousarray(pr.well_rates, dtype=np.float64)
            keep += arrs + [wc, wr]
            r = res[k]
            r.nx, r.ny, r.nz = pr.nx, pr.ny, pr.nz
            r.dx, r.dy, r.dz = pr.dx, pr.dy, pr.dz
            r.kx, r.ky, r.kz, r.phi = (a.data_ptr() for a in arrs)
            r.nwells = len(wc)
            r.well_cell = wc.ctypes.data_as(C.POINTER(C.c_int))
            r.well_rate = wr.ctypes.data_as(C.POINTER(C.c_double))
            bt = np.ascontiguousarray(getattr(pr, "bc_type", (0,) * 6), dtype=np.int32)
            bv = np.ascontiguousarray(getattr(pr, "bc_value", (0.0,) * 6), dtype=np.float64)
            if bt.size != 6 or bv.size != 6:
                raise ValueError("bc_type and bc_value need 6 entries (-x, +x, -y, +y, -z, +z)")
            keep += [bt, bv]
            r.bc_type = bt.ctypes.data_as(C.POINTER(C.c_int))
            r.bc_value = bv.ctypes.data_as(C.POINTER(C.c_double))
        fl = problems[0].fluid
        d = L.nks_grid_desc()
        d.nres = len(problems)
        d.res = res
        d.fluid = L.nks_fluid(fl.Tc, fl.pc, fl.omega, fl.T, fl.W, fl.R, fl.mu, getattr(fl, "Tb", None) or 0.0)
        d.gravity = 1 if problems[0].gravity else 0
        d.accum = L.ACCUM_FORMS[getattr(problems[0], "accum", "conservative")]
        d.g = problems[0].g
        d.stream = self.stream.cuda_stream
        self.allocator = TorchAllocator(self.device, self.stream) if torch_allocator else None
        if self.allocator is not None:
            d.alloc = self.allocator.alloc
            d.free = self.allocator.free
        h = C.c_void_p()
        check(lib().nks_setup_grid(C.byref(d), C.byref(h)))
        self.h = h
        n, b = C.c_int(), C.c_int()
        offs = (C.c_int * (len(problems) + 1))()
        check(lib().nks_grid_info(h, C.byref(n), C.byref(b), offs))
        self.N, self.B = n.value, b.value
        self.offsets = np.array(offs[:], dtype=np.int64)
        self.stream.synchronize()
        self._ras = None

    def __del__(self):
        h = getattr(self, "h", None)
        # at interpreter exit the allocator behind the handle (torch's) may
        # already be gone: the process is ending, leave the memory to it
        if h and _handle is not None and not sys.is_finalizing():
            _handle.nks_destroy_grid(h)
            self.h = None

    # -- vectors
    def zeros(self):
        torch = _torch()
        return torch.zeros(self.N, dtype=torch.float64, device=self.device)

    def from_numpy(self, a):
        torch = _torch()
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)

    def split(self, x):
        """Per-reservoir numpy views of a device vector."""
        a = x.detach().cpu().numpy()
        return [a[self.offsets[k]:self.offsets[k + 1]] for k in range(self.B)]

    def initial_pressure(self):
        """Uniform p_init, or the hydrostatic state from p_init at the top when gravity is on."""
        pr = self.problems[0]
        if pr.gravity:
            return self.hydrostatic(pr.p_init)
        p = self.zeros()
        p.fill_(float(pr.p_init))
        return p

    # -- entry points
    def hydrostatic(self, p_top):
        p = self.zeros()
        with _Ordered(self):
            check(lib().nks_hydrostatic_init(self.h, float(p_top), _vp(p)))
        return p

    def residual(self, p, pn, pnm1=None, dt=86400.0, order=1, out=None):
        F = self.zeros() if out is None else out
        with _Ordered(self):
            check(lib().nks_residual(self.h, _vp(p), _vp(pn), _vp(pnm1 if pnm1 is not None else pn),
                                     float(dt), int(order), _vp(F)))
        return F

    def residual_noalloc(self, p, pn, pnm1=None, dt=86400.0, order=1, out=None):
        """nks_residual_noalloc: the residual with the library's fixed device
        scratch (no allocation inside the call; `out` must be given for that)."""
        F = self.zeros() if out is None else out
        with _Ordered(self):
            check(lib().nks_residual_noalloc(self.h, _vp(p), _vp(pn), _vp(pnm1 if pnm1 is not None else pn),
                                             float(dt), int(order), _vp(F)))
        return F

    def matrix(self):
        return Matrix(self)

    def jacobian(self, p, pn, pnm1=None, dt=86400.0, order=1, J=None, F=None):
        J = J if J is not None else Matrix(self)
        with _Ordered(self):
            check(lib().nks_jacobian(self.h, _vp(p), _vp(pn), _vp(pnm1 if pnm1 is not None else pn),
                                     float(dt), int(order), J.h, _vp(F)))
        return J

    def residual_dlogk_t(self, p, lam):
        out = self.zeros()
        with _Ordered(self):
            check(lib().nks_residual_dlogk_transpose_apply(self.h, _vp(p), _vp(lam), _vp(out)))
        return out

    def simulate(self, nsteps, dt, settings, p0=None):
        """nsteps implicit steps (BDF1 first, BDF2 after) from p0 (default: the
        initial state); returns the list of states p^0..p^n and the step stats."""
        p = self.initial_pressure() if p0 is None else p0.clone()
        hist, stats = [p.clone()], []
        for n in range(nsteps):
            order = 1 if n == 0 else 2
            pn = hist[-1]
            pnm1 = hist[-2] if len(hist) > 1 else hist[-1]
            q = pn.clone()
            stats.append(self.newton_step(q, pn, pnm1, dt, order, settings))
            hist.append(q)
        return hist, stats

    def adjoint(self, p_hist, dt, dGdp, settings, orders=None, rtol=1e-10, atol=0.0, restart=30,
                maxit=10000, want_lambda=False):
        """nks_adjoint: dG/dln K for an objective with per-state gradients
        dGdp[n] (None: zero) over the states p_hist = [p^0, ..., p^n]."""
        torch = _torch()
        nsteps = len(p_hist) - 1
        orders = orders or [1] + [2] * (nsteps - 1)
        ph = (C.c_void_p * (nsteps + 1))(*[x.data_ptr() for x in p_hist])
        dg = (C.c_void_p * (nsteps + 1))(*[x.data_ptr() if x is not None else None for x in dGdp])
        od = (C.c_int * nsteps)(*orders)
        lams = [self.zeros() for _ in range(nsteps + 1)] if want_lambda else None
        lo = (C.c_void_p * (nsteps + 1))(*[x.data_ptr() for x in lams]) if want_lambda else None
        grad = self.zeros()
        rd = ras_desc(settings)
        gd = L.nks_gmres_desc(restart, rtol, atol, maxit, 1, 0)
        st = L.nks_adjoint_stats()
        with _Ordered(self):
            check(lib().nks_adjoint(self.h, nsteps, ph, od, float(dt), dg, C.byref(rd), C.byref(gd),
                                    _vp(grad), lo, C.byref(st)))
        out = dict(linear_its=list(st.linear_its[:min(nsteps, 64)]), total_linear_its=st.total_linear_its,
                   seconds=st.t_total)
        if want_lambda:
            out["lambda"] = lams
        return grad, out

    def autotune(self, p, pn, pnm1, dt, order, settings, tiles=(8, 16, 32), overlaps=(1, 2), ratios=None,
                 repeats=2, rtol=None, atol=None):
        """nks_ras_autotune: returns (settings with the best tile, overlap
        (the same on every level) and coarse-to-fine ratio, list of
        per-candidate timings); ratios None: the settings' ratio only."""
        import dataclasses
        rd = ras_desc(settings)
        nd = newton_desc(settings)
        flex = nd.flexible if nd.flexible >= 0 else int(settings.levels > 1 or settings.precision != "fp64")
        gd = L.nks_gmres_desc(nd.restart, settings.eta_r if rtol is None else rtol,
                              settings.eta_a if atol is None else atol, nd.maxit, flex, 0)
        ti = (C.c_int * len(tiles))(*tiles)
        ov = (C.c_int * len(overlaps))(*overlaps)
        ratios = list(ratios) if ratios else [getattr(settings, "ratio", 2)]
        ra = (C.c_int * len(ratios))(*ratios)
        best = L.nks_ras_desc()
        tab = (L.nks_autotune_entry * (len(tiles) * len(overlaps) * len(ratios)))()
        with _Ordered(self):
            check(lib().nks_ras_autotune(self.h, _vp(p), _vp(pn), _vp(pnm1 if pnm1 is not None else pn),
                                         float(dt), int(order), C.byref(rd), ti, len(tiles), ov,
                                         len(overlaps), ra, len(ratios), C.byref(gd), int(repeats),
                                         C.byref(best), tab))
        ovl = [best.overlap[0]] * len(settings.overlap)
        tz = best.tz if best.tz > 0 else 0
        tuned = dataclasses.replace(settings, tile=(best.tx, best.ty, tz), overlap=tuple(ovl),
                                    ratio=best.ratio if best.ratio > 0 else 2)
        table = [dict(tile=e.tile, overlap=e.overlap, ratio=e.ratio, ok=bool(e.ok), iterations=e.iterations,
                      setup_ms=e.setup_ms, solve_ms=e.solve_ms) for e in tab]
        return tuned, table

    def newton_step(self, p, pn, pnm1, dt, order, settings, raise_on_fail=True):
        st = L.nks_newton_stats()
        why = (C.c_int * self.B)()
        rel = (C.c_double * self.B)()
        st.stop_reason = C.cast(why, C.POINTER(C.c_int))
        st.rel_res = C.cast(rel, C.POINTER(C.c_double))
        nd, rd = newton_desc(settings), ras_desc(settings)
        with _Ordered(self):
            code = lib().nks_newton_step(self.h, _vp(p), _vp(pn), _vp(pnm1 if pnm1 is not None else pn),
                                         float(dt), int(order), C.byref(nd), C.byref(rd), C.byref(st))
        if code != 0 and (raise_on_fail or code != -5):
            check(code)
        k = st.newton_its
        return dict(newton_its=k, linear_its=st.linear_its, status=st.status, fnorm0=st.fnorm0,
                    fnorm=st.fnorm, fnorms=list(st.fnorms[:min(k, 64)]),
                    lits=list(st.lits[:min(k, 64)]), lambdas=list(st.lambdas[:min(k, 64)]),
                    t_residual=st.t_residual, t_jacobian=st.t_jacobian, t_setup=st.t_setup,
                    t_gmres=st.t_gmres, t_linesearch=st.t_linesearch,
                    stop_reason=[L.STOP_REASONS[int(w)] for w in why], rel_res=list(rel),
                    host_waits=st.host_waits, graph_chunk=st.graph_chunk)


class Matrix:
    """nks_matrix: the stencil Jacobian of a grid."""

    def __init__(self, grid):
        self.grid = grid
        h = C.c_void_p()
        check(lib().nks_matrix_create(grid.h, C.byref(h)))
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        # at interpreter exit the allocator behind the handle (torch's) may
        # already be gone: the process is ending, leave the memory to it
        if h and _handle is not None and not sys.is_finalizing():
            _handle.nks_destroy_matrix(h)
            self.h = None

    def export_csr(self):
        nnz = C.c_int()
        check(lib().nks_matrix_nnz(self.h, C.byref(nnz)))
        rp = np.zeros(self.grid.N + 1, np.int32)
        ci = np.zeros(nnz.value, np.int32)
        v = np.zeros(nnz.value)
        check(lib().nks_matrix_export_csr(self.h, rp.ctypes.data_as(C.POINTER(C.c_int)),
                                          ci.ctypes.data_as(C.POINTER(C.c_int)),
                                          v.ctypes.data_as(C.POINTER(C.c_double))))
        return rp, ci, v

    def apply(self, x, out=None):
        y = self.grid.zeros() if out is None else out
        with _Ordered(self.grid):
            check(lib().nks_matrix_apply(self.h, _vp(x), _vp(y)))
        return y

    def apply_transpose(self, x, out=None):
        y = self.grid.zeros() if out is None else out
        with _Ordered(self.grid):
            check(lib().nks_jacobian_transpose_apply(self.h, _vp(x), _vp(y)))
        return y

    def transpose(self, out=None):
        """J^T as a matrix on the same grid (nks_matrix_transpose)."""
        JT = Matrix(self.grid) if out is None else out
        with _Ordered(self.grid):
            check(lib().nks_matrix_transpose(self.h, JT.h))
        return JT


class Ras:
    """nks_ras: multilevel restricted additive Schwarz preconditioner."""

    def __init__(self, J, settings):
        self.J = J
        self.grid = J.grid
        self.desc = ras_desc(settings)
        self.h = C.c_void_p()
        self.setup(J)

    def setup(self, J=None):
        J = J or self.J
        self.J = J
        with _Ordered(self.grid):
            check(lib().nks_ras_setup(J.h, C.byref(self.desc), C.byref(self.h)))
        return self

    def __del__(self):
        h = getattr(self, "h", None)
        # at interpreter exit the allocator behind the handle (torch's) may
        # already be gone: the process is ending, leave the memory to it
        if h and _handle is not None and not sys.is_finalizing():
            _handle.nks_destroy_ras(h)
            self.h = None

    def level_info(self, level):
        info = (C.c_int * 8)()
        check(lib().nks_ras_level_info(self.h, int(level), info))
        return dict(n=info[0], K=info[1], nsub=info[2], dims=(info[3], info[4], info[5]),
                    levels=info[6], nnz=info[7])

    SWEEP_FORMS = {0: "none", 1: "hyperplane", 2: "rows4", 3: "rows1", 4: "packed", 5: "rows3d"}

    def level_sweep(self, level):
        """Kernel form of the level's last sweep ("none" before the first)
        and its workgroups."""
        form, wgs = C.c_int(), C.c_int()
        check(lib().nks_ras_level_sweep(self.h, int(level), C.byref(form), C.byref(wgs)))
        return self.SWEEP_FORMS[form.value], wgs.value

    def _vec(self, level):
        torch = _torch()
        n = self.level_info(level)["n"]
        return torch.zeros(n, dtype=torch.float64, device=self.grid.device)

    def apply(self, r, out=None):
        z = self.grid.zeros() if out is None else out
        with _Ordered(self.grid):
            check(lib().nks_ras_apply(self.h, _vp(r), _vp(z)))
        return z

    def apply_transpose(self, r, out=None):
        z = self.grid.zeros() if out is None else out
        with _Ordered(self.grid):
            check(lib().nks_ras_apply_transpose(self.h, _vp(r), _vp(z)))
        return z

    def apply_level(self, level, r, out=None):
        z = self._vec(level) if out is None else out
        with _Ordered(self.grid):
            check(lib().nks_ras_apply_level(self.h, int(level), _vp(r), _vp(z)))
        return z

    def coarse_solve(self, b, out=None):
        """The coarsest level's GMRES solve (vectors of that level's size)."""
        x = self._vec(self.desc.levels - 1) if out is None else out
        with _Ordered(self.grid):
            check(lib().nks_ras_coarse_solve(self.h, _vp(b), _vp(x)))
        return x

    def coarse_stats(self):
        """Per reservoir: iterations and last residual estimate of the latest
        coarse solve."""
        B = len(self.grid.offsets) - 1
        its = (C.c_int * B)()
        res = (C.c_double * B)()
        with _Ordered(self.grid):
            check(lib().nks_ras_coarse_stats(self.h, its, res))
        return list(its), list(res)

    def restrict(self, level, rf):
        rc = self._vec(level + 1)
        with _Ordered(self.grid):
            check(lib().nks_ras_restrict(self.h, int(level), _vp(rf), _vp(rc)))
        return rc

    def prolong_add(self, level, ec, zf):
        with _Ordered(self.grid):
            check(lib().nks_ras_prolong_add(self.h, int(level), _vp(ec), _vp(zf)))
        return zf

    def level_export(self, level):
        inf = self.level_info(level)
        rp = np.zeros(inf["n"] + 1, np.int32)
        ci = np.zeros(inf["nnz"], np.int32)
        v = np.zeros(inf["nnz"])
        check(lib().nks_ras_level_export(self.h, int(level), rp.ctypes.data_as(C.POINTER(C.c_int)),
                                         ci.ctypes.data_as(C.POINTER(C.c_int)),
                                         v.ctypes.data_as(C.POINTER(C.c_double))))
        return rp, ci, v


def gmres_solve(J, M, b, x=None, restart=30, rtol=1e-5, atol=1e-8, maxit=10000, flexible=False,
                transpose=False):
    """Right-preconditioned (F)GMRES through nks_gmres_solve; x is the initial guess."""
    grid = J.grid
    x = grid.zeros() if x is None else x
    d = L.nks_gmres_desc(restart, rtol, atol, maxit, int(bool(flexible)), int(bool(transpose)))
    st = L.nks_gmres_stats()
    its = (C.c_int * grid.B)()
    res = (C.c_double * grid.B)()
    st.its = C.cast(its, C.POINTER(C.c_int))
    st.res = C.cast(res, C.POINTER(C.c_double))
    with _Ordered(grid):
        check(lib().nks_gmres_solve(J.h, M.h if M is not None else None, _vp(b), _vp(x),
                                    C.byref(d), C.byref(st)))
    return x, dict(iterations=st.iterations, total=st.total_iterations, residual=st.residual,
                   converged=st.converged, its=list(its), res=list(res))
