"""Ablations of the method's knobs on the synthetic workloads.

The paper reports, per inner iteration cap j_max of the preconditioner solve
(Alg. 1 inside Alg. 4), the function evaluations, nonlinear, inner and
scalar-potential iterations and the time spent in each (Tables 1, 3 and 4),
and discusses the choice of beta* (Sec. 2.1). This module runs the same
measurements through the library: one demagnetization curve per setting, same
stopping rule, and prints one row per setting (evals, nli, li, mi, seconds,
and the time of the preconditioner and of the magnetostatics as the library
counts them, and the largest end-of-field torque). Besides j_max and beta*,
the (t1)-(t3) stopping rule of Sec. 3.1 can replace the torque tolerance, and
the other forms of eq. (precond) the paper's preconditioner.
Orchestration only: every step is a library call.

    python -m paper_1801_03690_amd.ablation --workload hard_cube --fields 41 \
        --jmax 0,1,2,4,10,20,100 --beta 0,1,2,3 --tau-f 1e-8,1e-10
"""
from __future__ import annotations

import argparse
import json
import time

from . import binding as B
from . import inputs

BETA_NAMES = {B.MM_BETA_ZA: "ZA", B.MM_BETA_FR: "FR", B.MM_BETA_PRP: "PRP", B.MM_BETA_HS: "HS"}
FORM_NAMES = {B.MM_PFORM_PAPER: "without the last term", B.MM_PFORM_FULL: "all terms",
              B.MM_PFORM_LOCAL: "projected local part"}


WORKLOADS = {"soft_cube": inputs.soft_cube, "hard_cube": inputs.hard_cube, "film": inputs.film,
             "polycrystal": inputs.polycrystal}
# scalar-potential CG preconditioner per workload when not given: multigrid
# except on the 2-layer film, whose Jacobi CG converges in a few iterations
AUTO_PREC = {"soft_cube": "amg", "hard_cube": "amg", "film": "jacobi", "polycrystal": "amg"}


def workload(name):
    return WORKLOADS[name]()


def run_curve(ctx, w, fields, **kw):
    """One curve from the workload's start state; returns the totals."""
    import numpy as np
    ctx.reset_warm_start()
    m = np.array(w.m0, copy=True)
    t0 = time.perf_counter()
    r = ctx.curve(m, fields, **kw)
    dt = time.perf_counter() - t0
    st = r["stats"]
    tot = {k: int(sum(s[k] for s in st)) for k in ("evals", "nli", "li", "mi", "restarts", "fallbacks")}
    tot.update(seconds=round(dt, 4), t_lin=round(sum(s["t_lin"] for s in st), 4),
               torque_max=float(max(s["torque_max"] for s in st)),
               t_mag=round(sum(s["t_mag"] for s in st), 4), rc=int(r["rc"]),
               max_status=int(max(s["status"] for s in st)), E_last=float(r["E"][-1]))
    return tot


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="hard_cube")
    ap.add_argument("--fields", type=int, default=0, help="first fields of the schedule (0: all)")
    ap.add_argument("--jmax", default="0,1,2,4,10,20,100", help="comma-separated j_max values (beta*ZA)")
    ap.add_argument("--beta", default="0,1,2,3", help="beta* kinds at the workload's j_max (0 ZA, 1 FR, 2 PRP, 3 HS)")
    ap.add_argument("--prec-form", default="", help="comma-separated forms of eq. (precond) at the workload's "
                    "j_max (0 the paper's, 1 all terms, 2 the projected local part)")
    ap.add_argument("--tau-f", default="", help="comma-separated tau_F of the (t1)-(t3) stopping rule "
                    "(Sec. 3.1) at the workload's j_max and beta*ZA")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--poisson-prec", choices=["auto", "jacobi", "amg"], default="auto")
    ap.add_argument("--max-nli", type=int, default=20000)
    ap.add_argument("--out", default=None, help="JSON report")
    args = ap.parse_args(argv)
    w = workload(args.workload)
    if args.poisson_prec == "auto":
        args.poisson_prec = AUTO_PREC[args.workload]
    fields = w.fields if args.fields <= 0 else w.fields[: args.fields]
    ctx = B.Context(0).upload(w.mesh)
    base = dict(precision=B.MM_FP64 if args.precision == "fp64" else B.MM_FP32_BULK,
                poisson_prec=B.MM_PREC_AMG if args.poisson_prec == "amg" else B.MM_PREC_JACOBI,
                max_nli=args.max_nli)
    ctx.set_opts(jmax=w.jmax, **base)
    # the first curve pays for the one-time set-up (graphs, hierarchy)
    run_curve(ctx, w, fields[:1], opts=B.default_opts(jmax=w.jmax, **base))
    rows = []
    print(f"# {w.name}: {len(fields)} fields, {args.precision}, {args.poisson_prec} scalar-potential CG", flush=True)
    print("| setting | evals | nli | li | mi | s | preconditioner s | magnetostatics s | max torque | status |",
          flush=True)
    print("|---|---|---|---|---|---|---|---|---|---|", flush=True)

    def report(label, tot):
        rows.append(dict(setting=label, **tot))
        print(f"| {label} | {tot['evals']} | {tot['nli']} | {tot['li']} | {tot['mi']} | {tot['seconds']:.2f} | "
              f"{tot['t_lin']:.2f} | {tot['t_mag']:.2f} | {tot['torque_max']:.1e} | {tot['max_status']} |", flush=True)

    settings = [(f"jmax={j}, beta*ZA", dict(jmax=j)) for j in [int(x) for x in args.jmax.split(",") if x != ""]]
    settings += [(f"jmax={w.jmax}, beta*{BETA_NAMES[b]}", dict(jmax=w.jmax, beta=b))
                 for b in [int(x) for x in args.beta.split(",") if x != ""]]
    settings += [(f"jmax={w.jmax}, P {FORM_NAMES[int(f)]}", dict(jmax=w.jmax, prec_form=int(f)))
                 for f in args.prec_form.split(",") if f != ""]
    settings += [(f"jmax={w.jmax}, (t1)-(t3) tau_F={t}", dict(jmax=w.jmax, stop_mode=B.MM_STOP_PAPER, tau_F=float(t)))
                 for t in args.tau_f.split(",") if t != ""]
    for label, kw in settings:
        print(f"# {label} ...", flush=True)
        report(label, run_curve(ctx, w, fields, opts=B.default_opts(**kw, **base)))
    ctx.close()
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(dict(workload=w.name, fields=len(fields), precision=args.precision,
                           poisson_prec=args.poisson_prec, rows=rows), fh, indent=1)
    return rows


if __name__ == "__main__":
    main()
