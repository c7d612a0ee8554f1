"""Benchmark: time per implicit step of the Newton-Krylov-Schwarz hot path on one GPU.

Default workload: 64 independent 2D reservoirs (sides 64..256, seeded
log-normal permeability with sigma 0.5..2, one injector and one producer
each), BDF2 steps of 5 days, a two-level V-cycle RAS whose subdomain tile and
fine overlap are chosen by the library's autotuner, FP32 subdomain factors
and sweeps inside FP64 FGMRES(30), FP64 residual, Jacobian and PR root.  The
plain FP64 form and the BF16-factor form run on the same reservoirs beside it.
A step is one full implicit time step of every reservoir: residual + PR,
Jacobian, subdomain ILU(0) and Galerkin setup, preconditioned FGMRES, line
search, per Newton iteration, to relative residual 1e-6 (or the binary64
rounding floor of the residual, reported per step).

Prints one JSON line.  `value` is the configured precision form's mean time per
step over the timed steps, which start from the initial state after the
untimed warm-up steps.  `roofline` is the fine-level one-level Schwarz apply
(the 2D sweep kernel), timed with HIP events bound to its dispatches inside
the timed region.  `cpu_baseline` runs the C oracle on every reservoir over
the workload's own steps, one reservoir per worker process on the host's
cores; its states also give each GPU form's pressure error against the
oracle.
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
             "batch64": "case_batch64", "3d96": "case_3d_96_adjoint", "flood512": "case_2d_flood_512",
             "hzone512": "case_2d_hzone", "layered128": "case_3d_layered_flood"}

# HBM bytes per launch of a sweep kernel over a whole level (no reservoir
# masked out), from two rocprofv3 --pmc passes over `bench.py --apply-level L`
# (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, scaled by the factors that
# make a 256 MiB device copy read and write 256 MiB), keyed by workload,
# level, tile edge, that level's overlap and the coarse-to-fine ratio.  Valid
# only for the kernel source they were taken on: any edit of that file drops
# them to null until the counters are taken again.
PMC_SOURCE = "paper_2007_13966_amd/csrc/schwarz.hip"
PMC_TRAFFIC = {
    ("batch64_2d_fp32prec", 0, 32, 2, 4): dict(
        fetch_kib=40616.25, fetch_scale=2.0, write_kib=18313.64, write_scale=1.0, algorithmic=90197384.0,
        sha1="542cfbcd8dcd61c81d7ff6a10d39e39cc7686e0a", kernel="k_ras_rows<float, float, float, 0, 256>"),
    ("batch64_2d_fp32prec", 1, 32, 2, 4): dict(
        fetch_kib=14383.76, fetch_scale=2.0, write_kib=1240.42, write_scale=1.0, algorithmic=26957568.0,
        sha1="542cfbcd8dcd61c81d7ff6a10d39e39cc7686e0a", kernel="k_ras_packed<float, float, float, 2>"),
}


def pmc_traffic(workload, level, settings):
    import hashlib
    key = (workload, level, settings.tile[0], settings.overlap[min(level, len(settings.overlap) - 1)],
           settings.ratio)
    t = PMC_TRAFFIC.get(key)
    if t is None:
        return None
    with open(os.path.join(HERE, PMC_SOURCE), "rb") as f:
        if hashlib.sha1(f.read()).hexdigest() != t["sha1"]:
            return None
    hbm = 1024 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])
    return {"hbm_bytes_per_full_launch": hbm, "algorithmic_bytes_per_full_launch": t["algorithmic"],
            "ratio": hbm / t["algorithmic"], "kernel": t["kernel"]}


def full_launches(P, case, level, repeats, settings=None):
    """One-level sweeps of `level` over the whole grid (no masks), `repeats`
    times at the initial state: the swept cells, algorithmic bytes and mean
    duration (HIP events bound to each dispatch) of one launch."""
    import ctypes as C
    import torch
    s = settings or case.solver
    g = P.Grid(case.problems)
    p0 = g.initial_pressure()
    J = g.jacobian(p0, p0, None, case.dt, 1)
    M = P.Ras(J, s)
    K = M.level_info(level)["K"]
    r = torch.ones(M.level_info(level)["n"], dtype=torch.float64, device=p0.device)
    M.apply_level(level, r)
    torch.cuda.synchronize()
    P.check(P.lib().nks_profile_filter(f"ras_apply_l{level}".encode()))
    P.check(P.lib().nks_profile_enable(1))
    for _ in range(repeats):
        M.apply_level(level, r)
    torch.cuda.synchronize()
    cells = (C.c_double * 2)()
    P.check(P.lib().nks_profile_units(f"ras_apply_l{level}".encode(), cells))
    c = C.c_int()
    t = C.c_double()
    P.check(P.lib().nks_profile_query(f"ras_apply_l{level}".encode(), C.byref(c), C.byref(t)))
    P.check(P.lib().nks_profile_enable(0))
    P.check(P.lib().nks_profile_filter(None))
    form = M.level_sweep(level)
    fb = {"fp64": 8, "fp32": 4, "bf16": 2}[s.precision]
    db = 8 if s.precision == "fp64" else 4
    ext, owned = cells[0] / repeats, cells[1] / repeats
    nbytes = ext * ((K - 1) * fb + db + 8) + owned * 8
    us = 1e3 * t.value / max(1, c.value)
    return {"workload": case.name, "level": level, "precision": s.precision, "tile": s.tile[0],
            "overlap": s.overlap[min(level, len(s.overlap) - 1)], "ratio": s.ratio, "launches": repeats,
            "form": form[0], "workgroups": form[1], "ext_cells": ext, "owned_cells": owned, "stencil_points": K,
            "algorithmic_bytes": nbytes, "avg_launch_us": us,
            "achieved": nbytes / (us * 1e-6) / 1e9, "frac": nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS}


def apply_level_mode(P, S, case, level, repeats):
    """`full_launches` for counter passes: prints its record."""
    print(json.dumps(full_launches(P, case, level, repeats)))


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


def level_stencils(P, case, s):
    """Stencil points of every level's operator (the Jacobian's on the
    finest, the coarse operators' below) for the preconditioner s builds,
    and the kernel form and workgroups of each level's one-level sweep."""
    import torch
    g = P.Grid(case.problems)
    p0 = g.initial_pressure()
    J = g.jacobian(p0, p0, None, case.dt, 1)
    M = P.Ras(J, s)
    forms = []
    for l in range(s.levels):
        r = torch.ones(M.level_info(l)["n"], dtype=torch.float64, device=g.device)
        M.apply_level(l, r)
        forms.append(M.level_sweep(l))
    return [M.level_info(l)["K"] for l in range(s.levels)], forms


def sweep_roofline(run, name, K, precision):
    """Achieved bandwidth of one sweep record over its profiled launches: the
    algorithmic bytes of the cells they swept (per extended cell the K-1
    off-diagonal factors, 1/u and the gathered residual; per owned cell the
    written correction) over their summed duration."""
    d = run["breakdown"].get(name, np.zeros(0))
    ext, owned = run["units"].get(name, (0.0, 0.0))
    if d.size == 0 or ext == 0:
        return None
    fb = {"fp64": 8, "fp32": 4, "bf16": 2}[precision]
    db = 8 if precision == "fp64" else 4
    nbytes = ext * ((K - 1) * fb + db + 8) + owned * 8
    sec = float(d.sum()) / 1e3
    ach = nbytes / sec / 1e9
    act = launch_split(d)
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "stencil_points": K, "launches": int(d.size), "masked_launches": int(d.size - act.size),
            "avg_launch_us": 1e3 * float(d.mean()), "total_ms": float(d.sum()),
            "bytes_total": nbytes, "bytes_per_launch": nbytes / d.size,
            "ext_cells_swept": ext, "owned_cells_swept": owned,
            "bytes_per_ext_cell": (K - 1) * fb + db + 8, "bytes_per_owned_cell": 8}


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


SWEEP_RECORDS = ["ras_apply_l0", "ras_apply_l1", "ras_apply_l2"]
BREAKDOWN_RECORDS = SWEEP_RECORDS + ["spmv_l0", "spmv_l1", "gmres_arnoldi", "residual_jacobian", "ilu_factor_l0",
                                     "ilu_factor_l1", "ilu_factor_l2", "rap_l1", "rap_l2"]


def step_record(st):
    """Per-step summary: Newton and FGMRES counts, the worst relative
    residual reached over the reservoirs and why each reservoir stopped."""
    reasons = {}
    for w in st.get("stop_reason", []):
        reasons[w] = reasons.get(w, 0) + 1
    rr = st.get("rel_res") or [st["fnorm"] / st["fnorm0"] if st["fnorm0"] else 0.0]
    return dict(newton=st["newton_its"], gmres=st["linear_its"], rel_res_max=float(max(rr)),
                stop=reasons, host_waits=st.get("host_waits"), fgmres_graph_chunk=st.get("graph_chunk"))


def run_gpu(P, case, settings, warmup, steps, keep_states=0, profile=True, breakdown_steps=2):
    """Warm-up steps from the initial state (untimed; the first keep_states
    states kept for the oracle comparison), then `steps` timed steps from the
    initial state again (no profiling), then `breakdown_steps` profiled steps
    continuing the trajectory: every launch recorded with HIP events on its
    dispatch (the coarse iterations otherwise replayed from captured graphs
    run as plain launches there), and the cells each sweep launch swept counted
    on the device."""
    import torch
    g = P.Grid(case.problems)
    p_init = g.initial_pressure()

    def trajectory():
        hist = [p_init.clone()]

        def step(n):
            order = 1 if n == 0 else 2
            pn = hist[-1]
            pnm1 = hist[-2] if len(hist) > 1 else hist[-1]
            pnew = pn.clone()
            st = g.newton_step(pnew, pn, pnm1, case.dt, order, settings)
            hist.append(pnew)
            if len(hist) > 3:
                hist.pop(0)
            return st, pnew
        return step

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

    states = []
    step = trajectory()
    for n in range(max(warmup, keep_states)):
        _, pnew = step(n)
        if n < keep_states:
            states.append(pnew.cpu().numpy())
    torch.cuda.synchronize()
    step = trajectory()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step(k)[0] for k in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    breakdown, units = {}, {}
    if profile and breakdown_steps:
        import ctypes as C
        P.check(P.lib().nks_profile_filter(None))
        P.check(P.lib().nks_profile_enable(2))
        for k in range(breakdown_steps):
            step(steps + k)
        torch.cuda.synchronize()
        breakdown = collect(BREAKDOWN_RECORDS)
        for name in SWEEP_RECORDS:
            cells = (C.c_double * 2)()
            P.check(P.lib().nks_profile_units(name.encode(), cells))
            units[name] = (cells[0], cells[1])
        P.check(P.lib().nks_profile_enable(0))
    return dict(seconds=t1 - t0, stats=stats, breakdown=breakdown, units=units, states=states,
                p_init=p_init.cpu().numpy(), offsets=g.offsets.copy())


_ORACLE_CASE = None


def _oracle_reservoir(args):
    """One reservoir through the oracle: nsteps implicit steps from the
    initial state; returns its states and per-step CPU seconds."""
    import oracle
    b, nsteps = args
    case = _ORACLE_CASE
    prob = oracle.Problem(case.problems[b])
    p = prob.initial_pressure()
    hist, secs = [p], []
    for n in range(nsteps):
        order = 1 if n == 0 else 2
        pnm1 = hist[-2] if len(hist) > 1 else hist[-1]
        t0 = time.process_time()
        p, _ = oracle.newton_step(prob, case.solver, hist[-1], hist[-1], pnm1, case.dt, order)
        secs.append(time.process_time() - t0)
        hist.append(p)
    return b, hist, secs


def cpu_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    # the GPU machine's CPU share for one GPU
    return max(1, min(n, 16))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_run(case, nsteps, workers):
    """The oracle over every reservoir of the case (the configured solver,
    FP64), one reservoir per worker process.  Runs before the GPU is touched
    (the workers are forked from this process)."""
    import multiprocessing as mp
    global _ORACLE_CASE
    _ORACLE_CASE = case
    jobs = [(b, nsteps) for b in range(len(case.problems))]
    # largest reservoirs first, so the pool drains evenly
    jobs.sort(key=lambda j: -case.problems[j[0]].N)
    t0 = time.perf_counter()
    if workers > 1 and len(jobs) > 1:
        with mp.get_context("fork").Pool(workers) as pool:
            res = pool.map(_oracle_reservoir, jobs, chunksize=1)
    else:
        res = [_oracle_reservoir(j) for j in jobs]
    wall = time.perf_counter() - t0
    res.sort(key=lambda r: r[0])
    states = [r[1] for r in res]
    serial = sum(sum(r[2]) for r in res)
    return dict(states=states, wall=wall, serial=serial, workers=workers if len(jobs) > 1 else 1)


def oracle_errors(run, orc, nsteps):
    """Pressure change error of a GPU form against the oracle, per reservoir
    and step: ||dp_gpu - dp_orc|| / ||dp_orc|| with dp = p^n - p^0."""
    off = run["offsets"]
    worst, num, den = 0.0, 0.0, 0.0
    for n in range(min(nsteps, len(run["states"]))):
        pg = run["states"][n]
        for b, hist in enumerate(orc["states"]):
            a, z = off[b], off[b + 1]
            dg = pg[a:z] - run["p_init"][a:z]
            do = hist[n + 1] - hist[0]
            e = float(np.linalg.norm(dg - do))
            d = float(np.linalg.norm(do))
            num += e * e
            den += d * d
            if d > 0:
                worst = max(worst, e / d)
    return dict(max_rel_dp_error=worst, rel_dp_error=float(np.sqrt(num / den)) if den > 0 else None,
                steps_compared=min(nsteps, len(run["states"])))


def form_summary(case, settings, run, steps, orc, ncheck, stencils):
    sec = run["seconds"] / steps
    recs = [step_record(x) for x in run["stats"]]
    out = {
        "s_per_step": sec,
        "newton_its_per_step": float(np.mean([r["newton"] for r in recs])),
        "gmres_its_per_newton": float(sum(r["gmres"] for r in recs) / max(1, sum(r["newton"] for r in recs))),
        "rel_res_reached_max": max(r["rel_res_max"] for r in recs),
        "steps": recs,
    }
    for lvl, K in enumerate(stencils[:2]):
        rf = sweep_roofline(run, f"ras_apply_l{lvl}", K, settings.precision)
        if rf:
            out[f"ras_apply_l{lvl}_gbs"] = rf["achieved"]
            out[f"ras_apply_l{lvl}_frac"] = rf["frac"]
    if orc is not None:
        out["vs_oracle"] = oracle_errors(run, orc, ncheck)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3,
                    help="timed implicit steps, from the initial state")
    ap.add_argument("--warmup", type=int, default=3,
                    help="untimed implicit steps from the initial state before the timed ones")
    ap.add_argument("--workload", default="batch64", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps per reservoir (0: the workload's steps, at most 3)")
    ap.add_argument("--lag", type=int, default=1,
                    help="refactor the preconditioner every LAG Newton iterations")
    ap.add_argument("--fill", type=int, default=0, choices=[0, 1, 2],
                    help="subdomain ILU level of fill k: ILU(k) instead of ILU(0)")
    ap.add_argument("--interp-order", type=int, default=0, choices=[0, 1, 2, 3],
                    help="interpolation order between levels (0: the workload's own)")
    ap.add_argument("--autotune", type=int, default=0, choices=[0, 1],
                    help="choose the subdomain tile edge (8, 16, 32), overlap (1, 2) and coarse-to-fine "
                         "ratio (2, 4, 8) with nks_ras_autotune at the initial state and run with its "
                         "choice (0: the workload's settings, for the batch the tuner's choice on MI355X)")
    ap.add_argument("--tile", type=int, default=0, help="subdomain tile edge (0: the workload's)")
    ap.add_argument("--overlap", type=int, default=-1, help="overlap on every level (-1: the workload's)")
    ap.add_argument("--ratio", type=int, default=0, help="coarse-to-fine ratio (0: the workload's)")
    ap.add_argument("--coarse-op", default="", choices=["", "galerkin", "rediscretised"],
                    help="coarse operators: Galerkin products or the upscaled problem's Jacobian")
    ap.add_argument("--coarse-kernel", default="", choices=["", "auto", "chunked", "persistent"],
                    help="form of the coarsest level's GMRES (empty: the workload's)")
    ap.add_argument("--apply-level", type=int, default=-1, metavar="L",
                    help="only run the one-level sweeps of level L over the whole workload (the tuned "
                         "defaults, no masks) --repeats times, for hardware counter passes, and exit")
    ap.add_argument("--repeats", type=int, default=20)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB five times (the "
                         "reference kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import synthetic as S
    case = getattr(S, WORKLOADS[args.workload])()
    if args.interp_order:
        case = S.with_solver(case, interp_order=args.interp_order)
    if args.fill:
        case = S.with_solver(case, fill=args.fill)
    if args.lag != 1:
        case = S.with_solver(case, lag=args.lag)
    if args.tile:
        case = S.with_solver(case, tile=(args.tile, args.tile, 0 if all(r.nz == 1 for r in case.problems)
                                         else args.tile))
    if args.overlap >= 0:
        case = S.with_solver(case, overlap=(args.overlap,) * case.solver.levels)
    if args.ratio:
        case = S.with_solver(case, ratio=args.ratio)
    if args.coarse_op:
        case = S.with_solver(case, coarse_op=args.coarse_op)
    if args.coarse_kernel:
        case = S.with_solver(case, coarse_kernel=args.coarse_kernel)
    ncheck = min(case.nsteps, 3) if args.cpu_steps <= 0 else args.cpu_steps

    # the oracle first: its workers are forked before anything touches the GPU
    orc = None
    if not args.no_cpu_baseline and not args.copy_calibration and args.apply_level < 0:
        workers = cpu_cores()
        log(f"oracle: {len(case.problems)} reservoirs x {ncheck} steps on {workers} worker processes")
        orc = oracle_run(case, ncheck, workers)
        log(f"oracle: {orc['wall']:.1f} s wall, {orc['serial']:.1f} s CPU in all")

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
    if args.apply_level >= 0:
        apply_level_mode(P, S, case, args.apply_level, args.repeats)
        return
    autotune = args.autotune
    tuning = None
    if autotune:
        g0 = P.Grid(case.problems)
        p0 = g0.initial_pressure()
        ratios = (2, 4, 8) if case.solver.levels > 1 else None
        tuned, table = g0.autotune(p0, p0, p0, case.dt, 1, case.solver, ratios=ratios)
        del g0
        case = S.with_solver(case, tile=tuned.tile, overlap=tuned.overlap, ratio=tuned.ratio)
        tuning = dict(tile=list(tuned.tile), overlap=list(tuned.overlap), ratio=tuned.ratio, table=table)
        log(f"autotuned: tile {tuned.tile}, overlap {tuned.overlap}, ratio {tuned.ratio}")
        for e in table:
            log(f"  tile {e['tile']:3d} overlap {e['overlap']} ratio {e['ratio']:2d}: ok {e['ok']} "
                f"its {e['iterations']:3d} setup {e['setup_ms']:.2f} ms solve {e['solve_ms']:.2f} ms")
    head = case.solver.precision
    forms = [head] if args.no_mixed else [head] + [f for f in ("fp64", "fp32", "bf16") if f != head]
    log(f"workload {case.name}: {sum(r.N for r in case.problems)} cells, forms {forms}")
    stencils, sweep_forms = level_stencils(P, case, case.solver)
    runs, summ = {}, {}
    for f in forms:
        sf = S.with_solver(case, precision=f).solver
        runs[f] = run_gpu(P, case, sf, args.warmup, args.steps, keep_states=ncheck if orc else 0,
                          breakdown_steps=2)
        summ[f] = form_summary(case, sf, runs[f], args.steps, orc, ncheck, stencils)
        e = summ[f].get("vs_oracle", {})
        log(f"{f}: {summ[f]['s_per_step']:.4f} s/step, newton {[r['newton'] for r in summ[f]['steps']]}, "
            f"gmres {[r['gmres'] for r in summ[f]['steps']]}, rel.res reached <= "
            f"{summ[f]['rel_res_reached_max']:.2e}, dp error vs oracle {e.get('max_rel_dp_error')}")
    # the coarse GMRES in both forms at the same settings: captured chunks of
    # launches with host convergence tests, and the persistent per-reservoir
    # launch (no host round trip; the FGMRES iterations then captured too)
    coarse_forms = None
    if case.solver.levels > 1 and all(r.nz == 1 for r in case.problems) and args.apply_level < 0:
        coarse_forms = {}
        # each form at the settings the tuner picks for it on MI355X (the
        # persistent one wants small coarse boxes: ratio 8, overlap 1)
        best = {"chunked": {}, "persistent": dict(tile=(32, 32, 0), overlap=(1, 1), ratio=8)}
        for kind in ("chunked", "persistent"):
            kw = best[kind] if args.workload == "batch64" and not args.tile and not args.ratio else {}
            sk = S.with_solver(case, precision=head, coarse_kernel=kind, **kw).solver
            try:
                rk = run_gpu(P, case, sk, args.warmup, args.steps, profile=False, breakdown_steps=0)
            except P.NksError as e:
                coarse_forms[kind] = {"error": str(e)[:160]}
                continue
            recs = [step_record(x) for x in rk["stats"]]
            coarse_forms[kind] = {"s_per_step": rk["seconds"] / args.steps,
                                  "tile": list(sk.tile), "overlap": list(sk.overlap), "ratio": sk.ratio,
                                  "host_waits_per_step": [r["host_waits"] for r in recs],
                                  "fgmres_graph_chunk": [r["fgmres_graph_chunk"] for r in recs],
                                  "newton": [r["newton"] for r in recs], "gmres": [r["gmres"] for r in recs]}
            log(f"coarse {kind}: {coarse_forms[kind]['s_per_step']:.4f} s/step, host waits "
                f"{coarse_forms[kind]['host_waits_per_step']}")
    s_head = S.with_solver(case, precision=head).solver
    r_head = runs[head]
    sec = summ[head]["s_per_step"]
    tname = {"fp64": "double, double, double", "fp32": "float, float, float",
             "bf16": "uint16_t, float, float"}[head]
    # the dominant kernel of the step: the sweep record with the most time in
    # the profiled steps (the coarse level's sweeps run inside every coarse
    # GMRES iteration; the finest level's twice per V-cycle)
    sweeps = {}
    for lvl, K in enumerate(stencils):
        rf = sweep_roofline(r_head, f"ras_apply_l{lvl}", K, head)
        if rf:
            form, wgs = sweep_forms[lvl]
            kern = {"packed": "k_ras_packed", "rows4": "k_ras_rows", "rows1": "k_ras_rows",
                    "rows3d": "k_ras_rows3d", "hyperplane": "k_ras_apply"}.get(form, "?")
            rf["kernel"] = (f"{kern}<{tname}, ...> ({form}, {wgs} workgroups): level-{lvl} one-level "
                            f"left-RAS sweeps, {K}-point operator, ILU(0) factors")
            rf["form"] = form
            sweeps[lvl] = rf
    dom = max(sweeps, key=lambda l: sweeps[l]["total_ms"]) if sweeps else None
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
        "dtype": "f64" if head == "fp64" else f"f64 (outer, residual, PR) + {'f32' if head == 'fp32' else 'bf16/f32'} "
                                              f"(subdomain factors and sweeps)",
        "data": "synthetic",
        "config": {
            "workload": case.name,
            "description": " ".join((case.description or "").split()),
            "cells": sum(r.N for r in case.problems),
            "reservoirs": len(case.problems),
            "levels": s_head.levels,
            "interp_order": s_head.interp_order,
            "ilu_fill": s_head.fill,
            "lag": s_head.lag,
            "subdomains": int(sum(np.prod(boxes(r, s_head)) for r in case.problems)),
            "overlap": list(s_head.overlap), "precision": head,
            "tile": list(s_head.tile),
            "ratio": s_head.ratio,
            "autotune": tuning,
            "timed_steps": f"steps 1..{args.steps} from the initial state (BDF1 first, BDF2 after), "
                           f"after {args.warmup} untimed warm-up steps from the same state",
            "newton_its_per_step": summ[head]["newton_its_per_step"],
            "gmres_its_per_newton": summ[head]["gmres_its_per_newton"],
            "rel_res_target": s_head.eps_r,
            "rel_res_reached_max": summ[head]["rel_res_reached_max"],
            "per_step": summ[head]["steps"],
        },
        "forms": summ,
        "roofline": dict(sweeps[dom], traffic=pmc_traffic(case.name, dom, case.solver),
                         measured="the profiled steps after the timed ones: every launch of the record "
                                  "with HIP events on its dispatch, bytes from the cells the launches swept "
                                  "(counted on the device)") if dom is not None else None,
        "roofline_sweeps": {f"level_{l}": v for l, v in sweeps.items()},
        "roofline_spmv": None,
        "stream_copy_gbs": None,
        # launches outside captured graphs, over 2 profiled steps after the timed ones
        "kernels_ms": {k: {"count": int(v.size), "total_ms": round(float(v.sum()), 3),
                           "avg_us": round(1e3 * float(v.mean()), 2)}
                       for k, v in r_head["breakdown"].items()},
    }
    if "fp64" in summ and head != "fp64":
        out["mixed_vs_fp64_speedup"] = summ["fp64"]["s_per_step"] / sec
    if coarse_forms:
        out["coarse_forms"] = coarse_forms
    sp = r_head["breakdown"].get("spmv_l0", np.zeros(0))
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
    # every sweep level alone over the whole grid (no reservoir masked out):
    # the kernels against their roofline without the coarse solve's partly
    # masked launches
    out["roofline_full_launches"] = {}
    for lvl in sweeps:
        fl = full_launches(P, case, lvl, 20, s_head)
        out["roofline_full_launches"][f"level_{lvl}"] = fl
        log(f"level {lvl} full launch ({fl['form']}): {fl['avg_launch_us']:.1f} us, "
            f"{fl['achieved']:.0f} GB/s ({100 * fl['frac']:.1f}%)")
    out["stream_copy_gbs"] = copy_bandwidth(torch)
    log(f"device copy: {out['stream_copy_gbs']:.0f} GB/s")
    if orc is not None:
        out["cpu_baseline"] = {
            "value": orc["wall"] / ncheck, "unit": "s/implicit step",
            "cores": orc["workers"], "kind": "oracle",
            "sample": f"all {len(case.problems)} reservoirs over steps 1..{ncheck} of the workload "
                      f"(BDF1 then BDF2), the single-threaded C oracle (FP64, the same solver settings) "
                      f"on one reservoir per worker process; wall time per step",
            "cpu_model": cpu_model(),
            "single_core_s_per_step": orc["serial"] / ncheck,
        }
        log(f"cpu oracle: {orc['wall'] / ncheck:.3f} s/step on {orc['workers']} cores, "
            f"{orc['serial'] / ncheck:.3f} s/step on one")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
