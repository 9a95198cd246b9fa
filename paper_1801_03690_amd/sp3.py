"""Single-domain limit of a soft cube with uniaxial anisotropy (Sec. 3.3).

The paper relaxes cubes of edge 8.4-8.6 exchange lengths twice, from the
saturated state (ending in the twisted flower state) and from a two-domain
state with a sharp wall (ending in the vortex state), stopping on (t1)-(t3)
with tau_F = 1e-12. The size at which the two relaxed energies are equal is
the single-domain limit; the paper finds 8.52 l_ex. Table 3 times the vortex
relaxation at 8.5 l_ex for several j_max.

This module runs the same relaxations through the library (FP64, multigrid
scalar-potential CG) on `inputs.sp3_cube` meshes, interpolates the crossing
size linearly between the sizes where the energy difference changes sign, and
sweeps j_max for the vortex relaxation. The air box is 7x the cube by
default: its zero potential understates stray-field energy, more for the
flower's dipole field than for the vortex, and a 3x box moves the crossing by
about 4%. Energies are densities in units of
Kd = mu0 Ms^2 / 2, with the anisotropy counted from the easy axis
(e = (E + K1 V) / (Kd V)). Orchestration only: every step is a library call.

    python -m paper_1801_03690_amd.sp3 --sizes 8.0,8.3,8.5,8.7,9.0 --jmax-sweep 0,2,4,8,12,20
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import binding as B
from . import inputs


def relax(ctx, w, jmax, tau_F=1e-12, max_nli=20000):
    """Relax w.m0 at zero field with the (t1)-(t3) rule; energy density in Kd."""
    t0 = time.perf_counter()
    m, E, st, rc = ctx.minimize(w.m0, [0.0, 0.0, 0.0], jmax=jmax, stop_mode=B.MM_STOP_PAPER, tau_F=tau_F,
                                precision=B.MM_FP64, poisson_prec=B.MM_PREC_AMG, max_nli=max_nli)
    dt = time.perf_counter() - t0
    vol = w.meta["volume_nm3"]
    # reduced energies are in mu0 Ms^2 nm^3 = 2 Kd nm^3; K1 V = 0.1 Kd V
    e = 2.0 * E / vol
    e_an = e[1] + 0.1
    mavg = np.asarray(m).reshape(-1, 3).mean(axis=0)
    return dict(e=float(e[4] + 0.1), e_ex=float(e[0]), e_an=float(e_an), e_d=float(e[3]),
                m_avg=[float(x) for x in mavg], evals=int(st["evals"]), nli=int(st["nli"]), li=int(st["li"]),
                mi=int(st["mi"]), seconds=round(dt, 3), status=int(st["status"]), rc=int(rc),
                torque_max=float(st["torque_max"]))


def uniform_demag(ctx, w):
    """Demagnetizing energy density (Kd) of the uniform state m = +z. For a
    cube it is exactly 1/3 (demagnetizing factor 1/3), so its shortfall is the
    error of the truncated air box."""
    m = np.zeros_like(w.m0)
    m[:, 2] = 1.0
    r = ctx.energy_grad(m, [0.0, 0.0, 0.0])
    return float(2.0 * r["E"][3] / w.meta["volume_nm3"])


def crossing(sizes, d):
    """Sizes at which the piecewise-linear interpolant of d changes sign."""
    out = []
    for i in range(len(sizes) - 1):
        if d[i] == 0.0:
            out.append(sizes[i])
        elif d[i] * d[i + 1] < 0.0:
            out.append(sizes[i] + (sizes[i + 1] - sizes[i]) * d[i] / (d[i] - d[i + 1]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--sizes", default="8.0,8.3,8.5,8.7,9.0", help="cube edges in exchange lengths")
    ap.add_argument("--n", type=int, default=24, help="cells per cube edge")
    ap.add_argument("--pad", type=int, default=None, help="air cells per side (default 3n: a 7x box)")
    ap.add_argument("--jmax", type=int, default=12)
    ap.add_argument("--jmax-sweep", default="", help="j_max values for the vortex relaxation at --sweep-size")
    ap.add_argument("--sweep-size", type=float, default=8.5)
    ap.add_argument("--tau-f", type=float, default=1e-12)
    ap.add_argument("--out", default=None, help="JSON report")
    args = ap.parse_args(argv)
    sizes = [float(x) for x in args.sizes.split(",") if x != ""]
    ctx = B.Context(0)
    rows, report = [], dict(n=args.n, jmax=args.jmax, tau_F=args.tau_f, lex_nm=inputs.lex_soft())
    print(f"# soft cube, K1 = 0.1 Kd along z, {args.n}^3 cells, l_ex = {inputs.lex_soft():.3f} nm, "
          f"jmax {args.jmax}, (t1)-(t3) tau_F {args.tau_f:g}", flush=True)
    pad = 3 * args.n if args.pad is None else args.pad
    report["pad"] = pad
    print(f"# air box {(args.n + 2 * pad) / args.n:g}x the cube", flush=True)
    print("| L / l_ex | h / l_ex | e_d uniform | e flower | <m> flower | e vortex | <m> vortex | e_f - e_v | "
          "nli f / v | s f / v |", flush=True)
    print("|---|---|---|---|---|---|---|---|---|---|", flush=True)
    for lam in sizes:
        wf = inputs.sp3_cube(lam, args.n, "flower", pad=pad)
        wv = inputs.sp3_cube(lam, args.n, "vortex", pad=pad)
        ctx.upload(wf.mesh)
        ed = uniform_demag(ctx, wf)
        rf = relax(ctx, wf, args.jmax, args.tau_f)
        rv = relax(ctx, wv, args.jmax, args.tau_f)
        d = rf["e"] - rv["e"]
        rows.append(dict(size_lex=lam, h_lex=wf.meta["h_nm"] / wf.meta["lex_nm"], e_d_uniform=ed, flower=rf,
                         vortex=rv, diff=d))
        fm = ", ".join(f"{x:.3f}" for x in rf["m_avg"])
        vm = ", ".join(f"{x:.3f}" for x in rv["m_avg"])
        print(f"| {lam:g} | {rows[-1]['h_lex']:.3f} | {ed:.4f} | {rf['e']:.5f} | ({fm}) | {rv['e']:.5f} | ({vm}) | {d:+.2e} | "
              f"{rf['nli']} / {rv['nli']} | {rf['seconds']:.1f} / {rv['seconds']:.1f} |", flush=True)
    report["sizes"] = rows
    if len(rows) > 1:
        report["crossing_lex"] = crossing([r["size_lex"] for r in rows], [r["diff"] for r in rows])
        print(f"# equal energies at L / l_ex = {report['crossing_lex']}", flush=True)
    sweep = [int(x) for x in args.jmax_sweep.split(",") if x != ""]
    if sweep:
        wv = inputs.sp3_cube(args.sweep_size, args.n, "vortex", pad=pad)
        ctx.upload(wv.mesh)
        report["jmax_sweep"] = []
        print(f"# vortex relaxation at {args.sweep_size:g} l_ex", flush=True)
        print("| j_max | evals | nli | li | mi | s | e |", flush=True)
        print("|---|---|---|---|---|---|---|", flush=True)
        for j in sweep:
            r = relax(ctx, wv, j, args.tau_f)
            report["jmax_sweep"].append(dict(jmax=j, **r))
            print(f"| {j} | {r['evals']} | {r['nli']} | {r['li']} | {r['mi']} | {r['seconds']:.2f} | {r['e']:.6f} |",
                  flush=True)
    ctx.close()
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(report, fh, indent=1)
    return report


if __name__ == "__main__":
    main()
