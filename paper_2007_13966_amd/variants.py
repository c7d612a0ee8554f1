"""Variant matrix of the Schwarz preconditioner on one workload (the trends of
the paper's Section 4.2 tables: AS, left- and right-RAS with overlaps 0..3,
V-cycle, Kaskade, additive and coarse-only compositions, interpolation orders
1..3, coarse-to-fine ratios 2..16, ILU(k) subdomain solves, Galerkin against
rediscretised coarse operators), measured on one GPU through the library.

    python -m paper_2007_13966_amd.variants [--workload 2d512] [--steps 3] [--json out.json]

Each variant runs the workload's first `steps` implicit steps twice from the
initial state (the first pass warms up) and reports, from the second pass,
the mean Newton iterations per step (N.It), FGMRES iterations per Newton
iteration (L.It) and seconds per step.  A variant whose linear solve hits the
iteration cap is reported as not converged, as the paper reports its
coarse-only composition.
"""
import argparse
import json
import sys
import time


def _variants():
    out = [("one-level left-RAS, overlap 1", dict(levels=1, overlap=(1,)))]
    for var in ("as", "left_ras", "right_ras"):
        for d in (0, 1, 2, 3):
            out.append((f"{var}, overlap {d}", dict(variant=var, overlap=(d, 1))))
    for cyc in ("vcycle", "left_kaskade", "right_kaskade", "additive", "coarse_only"):
        out.append((f"{cyc}, order 2", dict(cycle=cyc)))
    for order in (1, 2, 3):
        for ratio in (2, 4, 8, 16):
            out.append((f"order {order}, ratio {ratio}", dict(interp_order=order, ratio=ratio)))
    for fill in (0, 1, 2):
        out.append((f"ILU({fill})", dict(fill=fill)))
    out.append(("rediscretised coarse operator", dict(coarse_op="rediscretised")))
    out.append(("rediscretised coarse operator, order 1", dict(coarse_op="rediscretised", interp_order=1)))
    return out


def run(workload="2d512", steps=3, maxit=600, names=None):
    import torch
    import synthetic as S
    import paper_2007_13966_amd as P
    base = getattr(S, {"2d512": "case_2d_512", "flood512": "case_2d_flood_512",
                       "batch64": "case_batch64"}[workload])()
    rows = []
    for name, kw in _variants():
        if names and not any(n in name for n in names):
            continue
        case = S.with_solver(base, maxit=maxit, **kw)
        g = P.Grid(case.problems)
        rec = dict(variant=name)
        try:
            for rep in range(2):
                p0 = g.initial_pressure()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                hist, stats = g.simulate(steps, case.dt, case.solver, p0=p0)
                torch.cuda.synchronize()
                sec = (time.perf_counter() - t0) / steps
            nits = sum(s["newton_its"] for s in stats)
            lits = sum(s["linear_its"] for s in stats)
            rec.update(newton_per_step=nits / steps, gmres_per_newton=lits / max(1, nits), s_per_step=sec,
                       converged=True)
        except Exception as e:   # the iteration cap (NKS_ENOTCONVERGED) or a rejected option
            rec.update(converged=False, error=str(e)[:120])
        rows.append(rec)
        print(json.dumps(rec), flush=True)
        del g
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="2d512", choices=["2d512", "flood512", "batch64"])
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--maxit", type=int, default=600, help="FGMRES iteration cap per linear solve")
    ap.add_argument("--only", nargs="*", help="run the variants whose name contains one of these")
    ap.add_argument("--json", help="write the rows to this file")
    a = ap.parse_args()
    rows = run(a.workload, a.steps, a.maxit, a.only)
    print("| variant | N.It | L.It | s/step |")
    print("|---|---:|---:|---:|")
    for r in rows:
        if r["converged"]:
            print(f"| {r['variant']} | {r['newton_per_step']:.2f} | {r['gmres_per_newton']:.1f} | "
                  f"{r['s_per_step']:.4f} |")
        else:
            print(f"| {r['variant']} | - | not converged | - |")
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)
    sys.stdout.flush()


if __name__ == "__main__":
    main()
