"""Benchmark: time per implicit step of the Newton-Krylov-Schwarz hot path on one GPU.

Default workload: 2D 512x512 log-normal reservoir (sigma 1, correlation
length 8 cells), five-spot wells, BDF2 steps of 5 days, two-level V-cycle
RAS with 256 subdomains (overlap 2 on both levels), FGMRES(30), FP64.
A step is one full implicit time step: residual + PR, Jacobian, subdomain
ILU(0) and Galerkin setup, preconditioned FGMRES, line search, per Newton
iteration, to relative residual 1e-6.

Prints one JSON line.  `roofline` is the fine-level one-level Schwarz apply
(the 2D sweep kernel), timed with HIP events bound to its dispatches inside
the timed region; `cpu_baseline` times the CPU oracle on the first steps of the same
workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "time/implicit step + ras_apply GB/s, mixed-prec vs FP64 at rel.res 1e-6"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {"2d32": "case_2d_32", "2d512": "case_2d_512", "3d128": "case_3d_128",
             "batch64": "case_batch64", "3d96": "case_3d_96_adjoint", "flood512": "case_2d_flood_512"}

# HBM bytes moved per active fine-level launch of the FP64 2D sweep kernel on
# the 512x512 workload, from two rocprofv3 --pmc passes (FETCH_SIZE x 2.0 and
# WRITE_SIZE x 1.0, the factors that make a 256 MiB device copy read and write
# 256 MiB).  Valid only for the kernel source it was taken on: any edit of that
# file drops it to null until the counters are taken again.
PMC_TRAFFIC = {
    "workload": "2d_512x512_twolevel_fp64",
    "source": "paper_2007_13966_amd/csrc/schwarz.hip",
    "sha1": "412546ad8237521c76a11623611ee6fb4fcfc343",
    "fetch_kib": 8854.3, "fetch_scale": 2.0,
    "write_kib": 2048.0, "write_scale": 1.0,
}


def pmc_traffic(workload):
    import hashlib
    t = PMC_TRAFFIC
    if workload != t["workload"]:
        return None
    with open(os.path.join(HERE, t["source"]), "rb") as f:
        if hashlib.sha1(f.read()).hexdigest() != t["sha1"]:
            return None
    return 1024 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ext_cells(nx, ny, nz, px, py, pz, delta):
    """Cells of all overlapping boxes (box q gets n//P + (q < n%P), extended by
    delta and clipped at the boundary)."""
    def ext1(n, P):
        P = min(P, n)
        base, rem = divmod(n, P)
        out, lo = [], 0
        for q in range(P):
            hi = lo + base + (1 if q < rem else 0)
            out.append(min(n, hi + delta) - max(0, lo - delta))
            lo = hi
        return out
    ex, ey, ez = ext1(nx, px), ext1(ny, py), ext1(nz, pz)
    return sum(a * b * c for a in ex for b in ey for c in ez)


def boxes(rec, s):
    """Boxes per direction: from the tile edge when one is set, else the counts."""
    n, t, P = (rec.nx, rec.ny, rec.nz), s.tile, (s.px, s.py, s.pz)
    return [-(-n[a] // t[a]) if t[a] > 0 else P[a] for a in range(3)]


def apply_bytes(recs, s, precision):
    """Algorithmic bytes of one fine-level one-level Schwarz apply over all
    reservoirs: per extended cell the off-diagonal factors, 1/u_ii and the
    gathered residual; per owned cell the written correction."""
    fb = {"fp64": 8, "fp32": 4, "bf16": 2}[precision]
    db = 8 if precision == "fp64" else 4
    nbytes = nexts = 0
    for rec in recs:
        K = 7 if rec.nz > 1 else 5
        ne = ext_cells(rec.nx, rec.ny, rec.nz, *boxes(rec, s), s.overlap[0])
        nbytes += ne * ((K - 1) * fb + db + 8) + rec.N * 8
        nexts += ne
    return nbytes, nexts


def launch_split(d):
    """Active launches of the roofline kernel: the Krylov loop runs ahead of
    its host-side convergence check, so a few launches per solve find every
    reservoir masked out and exit at once (under half the median)."""
    d = np.asarray(d)
    if d.size == 0:
        return d
    return d[d >= np.median(d) / 2]


def level_bytes(P, case, s, level):
    """Algorithmic bytes of one FP64 one-level apply on `level` (coarse
    levels: the same boxes on the coarsened grids, that level's overlap and
    its Galerkin stencil size from the library)."""
    g = P.Grid(case.problems)
    p0 = g.initial_pressure()
    J = g.jacobian(p0, p0, None, case.dt, 1)
    info = P.Ras(J, s).level_info(level)
    K, n = info["K"], info["n"]
    ne = 0
    for rec in case.problems:
        d = [rec.nx, rec.ny, rec.nz]
        for _ in range(level):
            d = [-(-x // 2) if (x > 1 or k < 2) else 1 for k, x in enumerate(d)]
        nb = boxes(rec, s)
        ne += ext_cells(d[0], d[1], d[2], *nb, s.overlap[min(level, len(s.overlap) - 1)])
    return ne * ((K - 1) * 8 + 8 + 8) + n * 8, K


def copy_bandwidth(torch, mib=1024, reps=5):
    """Device-to-device copy bandwidth (bytes read + written per second):
    the attainable HBM rate on this GPU, beside the published peak."""
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del x, y
    return 2 * 8 * n / sec / 1e9


ROOFLINE_RECORDS = ["ras_apply_l0", "ras_apply_l1"]
BREAKDOWN_RECORDS = ["ras_apply_l0", "ras_apply_l1", "ras_apply_l2", "spmv_l0", "spmv_l1", "gmres_arnoldi", "residual_jacobian", "ilu_factor_l0",
                     "ilu_factor_l1", "ilu_factor_l2", "rap_l1", "rap_l2"]


def run_gpu(P, case, settings, warmup, steps, profile=True, breakdown_steps=2):
    import torch
    g = P.Grid(case.problems)
    p = g.initial_pressure()
    hist = [p.clone()]

    def step(n):
        order = 1 if n == 0 else 2
        pn = hist[-1]
        pnm1 = hist[-2] if len(hist) > 1 else hist[-1]
        pnew = pn.clone()
        st = g.newton_step(pnew, pn, pnm1, case.dt, order, settings)
        hist.append(pnew)
        if len(hist) > 3:
            hist.pop(0)
        return st

    def collect(names):
        import ctypes as C
        out = {}
        for name in names:
            c = C.c_int()
            P.check(P.lib().nks_profile_durations(name.encode(), None, 0, C.byref(c)))
            if c.value:
                buf = (C.c_double * c.value)()
                P.check(P.lib().nks_profile_durations(name.encode(), buf, c.value, C.byref(c)))
                out[name] = np.array(buf[:])
        return out

    for n in range(warmup):
        step(n)
    torch.cuda.synchronize()
    p_start = hist[-1].clone()
    if profile:
        # inside the timed region only the sweeps behind the roofline figures
        # carry events; the other launches take no host bookkeeping
        P.check(P.lib().nks_profile_filter(",".join(ROOFLINE_RECORDS).encode()))
        P.check(P.lib().nks_profile_enable(1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step(warmup + k) for k in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p_end = hist[-1].cpu().numpy()
    prof, breakdown = {}, {}
    if profile:
        prof = collect(ROOFLINE_RECORDS)
        P.check(P.lib().nks_profile_enable(0))
        if breakdown_steps:
            # every record, over separate steps after the timed ones
            P.check(P.lib().nks_profile_filter(None))
            P.check(P.lib().nks_profile_enable(1))
            for k in range(breakdown_steps):
                step(warmup + steps + k)
            torch.cuda.synchronize()
            breakdown = collect(BREAKDOWN_RECORDS)
            P.check(P.lib().nks_profile_enable(0))
    return dict(seconds=t1 - t0, stats=stats, prof=prof, breakdown=breakdown,
                p_start=p_start.cpu().numpy(), p_end=p_end)


def cpu_baseline(case, nsteps):
    import oracle
    rec = case.problems[0]
    prob = oracle.Problem(rec)
    p = prob.initial_pressure()
    hist = [p]
    t0 = time.perf_counter()
    for n in range(nsteps):
        order = 1 if n == 0 else 2
        pnm1 = hist[-2] if len(hist) > 1 else hist[-1]
        p, st = oracle.newton_step(prob, case.solver, hist[-1], hist[-1], pnm1, case.dt, order)
        hist.append(p)
    return (time.perf_counter() - t0) / nsteps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=9)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="2d512", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--lag", type=int, default=1,
                    help="refactor the preconditioner every LAG Newton iterations")
    ap.add_argument("--fill", type=int, default=0, choices=[0, 1, 2],
                    help="subdomain ILU level of fill k: ILU(k) instead of ILU(0)")
    ap.add_argument("--interp-order", type=int, default=0, choices=[0, 1, 2, 3],
                    help="interpolation order between levels (0: the workload's own)")
    ap.add_argument("--autotune", action="store_true",
                    help="choose the subdomain tile edge (8, 16, 32) and fine overlap (1, 2) with "
                         "nks_ras_autotune at the initial state before timing")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB five times (the "
                         "reference kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import synthetic as S
    import paper_2007_13966_amd as P
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        x = torch.arange(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "copies": 5}))
        return
    case = getattr(S, WORKLOADS[args.workload])()
    if args.interp_order:
        case = S.with_solver(case, interp_order=args.interp_order)
    if args.fill:
        case = S.with_solver(case, fill=args.fill)
    if args.lag != 1:
        case = S.with_solver(case, lag=args.lag)
    tuning = None
    if args.autotune:
        g0 = P.Grid(case.problems)
        p0 = g0.initial_pressure()
        tuned, table = g0.autotune(p0, p0, p0, case.dt, 1, case.solver)
        del g0
        case = S.with_solver(case, tile=tuned.tile, overlap=tuned.overlap)
        tuning = dict(tile=list(tuned.tile), overlap=list(tuned.overlap), table=table)
        log(f"autotuned: tile {tuned.tile}, overlap {tuned.overlap}")
        for e in table:
            log(f"  tile {e['tile']:3d} overlap {e['overlap']}: ok {e['ok']} its {e['iterations']:3d} "
                f"setup {e['setup_ms']:.2f} ms solve {e['solve_ms']:.2f} ms")
    s64 = S.with_solver(case, precision="fp64").solver
    log(f"workload {case.name}: {sum(r.N for r in case.problems)} cells")
    nbytes, nexts = apply_bytes(case.problems, s64, "fp64")
    r64 = run_gpu(P, case, s64, args.warmup, args.steps)
    st = r64["stats"]
    sec = r64["seconds"] / args.steps
    nits = [x["newton_its"] for x in st]
    lits = [x["linear_its"] for x in st]
    log(f"fp64: {sec:.4f} s/step, newton {nits}, gmres {lits}")
    allv = r64["prof"].get("ras_apply_l0", np.zeros(0))
    act = launch_split(allv)
    cnt = int(act.size)
    avg_s = float(act.mean()) / 1e3 if cnt else 0.0
    achieved = nbytes / avg_s / 1e9 if cnt else None
    out = {
        "metric": METRIC,
        "value": sec,
        "unit": "s/implicit step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": case.name,
            "description": " ".join((case.description or "").split()),
            "cells": sum(r.N for r in case.problems),
            "reservoirs": len(case.problems),
            "levels": s64.levels,
            "interp_order": s64.interp_order,
            "ilu_fill": s64.fill,
            "lag": s64.lag,
            "subdomains": int(sum(np.prod(boxes(r, s64)) for r in case.problems)),
            "overlap": list(s64.overlap), "precision": s64.precision,
            "newton_its_per_step": float(np.mean(nits)),
            "gmres_its_per_newton": float(np.sum(lits) / max(1, np.sum(nits))),
            "rel_res": s64.eps_r,
            "rel_res_reached": [x["fnorm"] / x["fnorm0"] for x in st],
            "tile": list(s64.tile),
            "autotune": tuning,
        },
        "roofline": {
            "kernel": ("k_ras_apply<double, double, double, 3> (fine level 3D 7-point sweeps: one-level left-RAS, "
                       "ILU(0) factors)" if case.problems[0].nz > 1 else
                       "k_ras_rows<double, double, double, 0, 256> (fine level 2D sweeps: one-level left-RAS, ILU(0) factors)"),
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": pmc_traffic(case.name),
            "bytes_per_launch": nbytes,
            "ext_cells": nexts,
            "launches": cnt,
            "masked_launches": int(allv.size - cnt),
            "avg_launch_us": avg_s * 1e6,
        },
        "roofline_coarse": None,
        "roofline_spmv": None,
        "stream_copy_gbs": None,
        # launches outside captured graphs, over 2 profiled steps after the timed ones
        "kernels_ms": {k: {"count": int(v.size), "total_ms": round(float(v.sum()), 3),
                           "avg_us": round(1e3 * float(v.mean()), 2)}
                       for k, v in r64["breakdown"].items()},
    }
    if s64.levels > 1:
        # the coarsest-but-one level's sweeps run inside every coarse GMRES
        # iteration and take most of the apply time
        cb, ck = level_bytes(P, case, s64, 1)
        cl = launch_split(r64["prof"].get("ras_apply_l1", np.zeros(0)))
        ca = cb / (float(cl.mean()) / 1e3) / 1e9 if cl.size else None
        out["roofline_coarse"] = {
            "kernel": f"level-1 one-level sweeps ({ck}-point Galerkin stencil), launches outside graphs",
            "bound": "hbm", "achieved": ca, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (ca / HBM_PEAK_GBS) if ca else None, "bytes_per_launch": cb,
            "launches": int(cl.size), "avg_launch_us": float(cl.mean()) * 1e3 if cl.size else None,
        }
    sp = r64["breakdown"].get("spmv_l0", np.zeros(0))
    if sp.size and all(r.nz == 1 for r in case.problems):
        # 2D: the 5-point launches are the fine level's residuals r = b - A x
        # (the coarse operators have more points); per cell 5 coefficients,
        # x, b and r
        nb = sum(r.N for r in case.problems) * (5 * 8 + 24)
        ga = nb / (float(sp.mean()) / 1e3) / 1e9
        out["roofline_spmv"] = {
            "kernel": "k_spmv<8> (fine-level residual b - A x, 5-point, FP64), 2 profiled steps",
            "bound": "hbm", "achieved": ga, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ga / HBM_PEAK_GBS,
            "bytes_per_launch": nb, "launches": int(sp.size), "avg_launch_us": float(sp.mean()) * 1e3,
        }
    out["stream_copy_gbs"] = copy_bandwidth(torch)
    log(f"device copy: {out['stream_copy_gbs']:.0f} GB/s")
    if not args.no_mixed:
        s32 = S.with_solver(case, precision="fp32").solver
        b32, _ = apply_bytes(case.problems, s32, "fp32")
        r32 = run_gpu(P, case, s32, args.warmup, args.steps, breakdown_steps=0)
        sec32 = r32["seconds"] / args.steps
        d64 = r64["p_end"] - r64["p_start"]
        d32 = r32["p_end"] - r32["p_start"]
        err = float(np.linalg.norm(d32 - d64) / max(np.linalg.norm(d64), 1e-300))
        act32 = launch_split(r32["prof"].get("ras_apply_l0", np.zeros(0)))
        a32 = b32 / (float(act32.mean()) / 1e3) / 1e9 if act32.size else None
        out["mixed_fp32"] = {
            "s_per_step": sec32,
            "speedup_vs_fp64": sec / sec32,
            "gmres_its_per_newton": float(sum(x["linear_its"] for x in r32["stats"]) /
                                          max(1, sum(x["newton_its"] for x in r32["stats"]))),
            "dp_rel_error_vs_fp64": err,
            "ras_apply_l0_gbs": a32,
            "ras_apply_l0_frac": (a32 / HBM_PEAK_GBS) if a32 else None,
        }
        log(f"fp32 preconditioner: {sec32:.4f} s/step, dp error vs fp64 {err:.2e}")
        sb = S.with_solver(case, precision="bf16").solver
        bb, _ = apply_bytes(case.problems, sb, "bf16")
        rb = run_gpu(P, case, sb, args.warmup, args.steps, breakdown_steps=0)
        secb = rb["seconds"] / args.steps
        db = rb["p_end"] - rb["p_start"]
        errb = float(np.linalg.norm(db - d64) / max(np.linalg.norm(d64), 1e-300))
        actb = launch_split(rb["prof"].get("ras_apply_l0", np.zeros(0)))
        ab = bb / (float(actb.mean()) / 1e3) / 1e9 if actb.size else None
        out["mixed_bf16"] = {
            "s_per_step": secb,
            "speedup_vs_fp64": sec / secb,
            "gmres_its_per_newton": float(sum(x["linear_its"] for x in rb["stats"]) /
                                          max(1, sum(x["newton_its"] for x in rb["stats"]))),
            "dp_rel_error_vs_fp64": errb,
            "ras_apply_l0_gbs": ab,
            "ras_apply_l0_frac": (ab / HBM_PEAK_GBS) if ab else None,
        }
        log(f"bf16 factors: {secb:.4f} s/step, dp error vs fp64 {errb:.2e}")
    if not args.no_cpu_baseline and args.workload == "2d512":
        n = args.cpu_steps
        v = cpu_baseline(case, n)
        out["cpu_baseline"] = {"value": v, "unit": "s/implicit step", "cores": 1, "kind": "oracle",
                               "sample": f"first {n} implicit steps (BDF1 then BDF2) of the same "
                                         f"512x512 workload, single-threaded C oracle"}
        log(f"cpu oracle: {v:.3f} s/step")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
