#!/usr/bin/env python3
"""Benchmark: demagnetization-curve time-to-solution on one MI355X.

Default workload: the soft thin film, 1000 x 1000 x 10 nm on 200 x 200 x 2
cells of 5 nm x 6 tets (121,203 magnet nodes) in a 3x air box for the scalar
potential (1.79M free potential nodes), Ms = 8e5 A/m, A = 13 pJ/m, K1 = 0,
field along x from +50 mT to -50 mT in 1 mT steps (101 values), j_max 10,
line-search rotation cap 0.5 rad, every minimization run to
max |m x h_eff| < 1e-6 (reduced units). Two forms reach the same torque
tolerance:

  * learned + FP32 (the value): the network's warm start at every field after
    the first (with --learn-mode start+scale also its Jacobi scaling),
    FP32-stored operators with FP64 reductions;
  * plain FP64: the method without the network, every operator in FP64.

One step is one stretch of the curve: the field list is split into `--steps`
consecutive chunks, each continuing from the previous chunk's minimum (the
learned proposal included), so the K timed steps together are exactly one
whole curve and `value` is its time-to-solution. With more steps than fields
each step is one field and the curve restarts from its initial state after
the last field; `value` is then the timed seconds per curve walked. The
`--warmup` untimed steps are the first chunks of the same curve, run before
the timed curve starts again from the initial state. Inputs (operators,
start state, network) are resident in HBM; assembly, the block-shape tuning
and the network's training are not timed, as in the paper (Sec. 3.1).

Printed (one JSON line): the time per curve, the plain FP64 form's time for
the same curve, the roofline of the dominant kernel (the scalar-potential CG
iteration, timed with HIP events on the library's stream around its graph
replays inside the timed region), the per-launch bandwidth of the field
kernels (C m + B^T u epilogue, B m, P v) from HIP events in the same region,
the CPU FP64 oracle timed on a bounded sample of the same workload, and the
20^3 hard cube's curve (FP32 bulk, multigrid CG) as an extra figure.

Other workloads (--workload): hard_cube, polycrystal (bound it with
--fields, or time it in pieces with --state), batch64.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
METRIC = "demag-curve time-to-solution (s) & SpMV HBM GB/s, plain vs learned+FP32, equal tol"
PROF = os.path.join(ROOT, "profiles")
SRC = os.path.join(ROOT, "paper_1801_03690_amd", "csrc")
# counter-measured traffic per CG iteration: (file, kernel source it was measured on)
TRAFFIC = {
    ("hard_cube", "jacobi"): (os.path.join(PROF, "pcg_hard_cube_20_traffic.txt"), os.path.join(SRC, "poisson.hip")),
    ("hard_cube", "amg"): (os.path.join(PROF, "amg_hard_cube_20_traffic.txt"), os.path.join(SRC, "amg.hip")),
    ("film", "jacobi"): (os.path.join(PROF, "pcg_film_traffic.txt"), os.path.join(SRC, "poisson.hip")),
    ("polycrystal", "amg"): (os.path.join(PROF, "amg_polycrystal_traffic.txt"), os.path.join(SRC, "amg.hip")),
}
# preconditioner of the scalar-potential CG per workload when --poisson-prec auto:
# multigrid where it is faster (measured), Jacobi on the thin film (a few dozen
# Jacobi iterations per solve)
AUTO_PREC = {"hard_cube": "amg", "polycrystal": "amg", "film": "jacobi", "batch64": "amg"}
NET = os.path.join(ROOT, "paper_1801_03690_amd", "data", "gnn_films_600_1400.npz")


def measured_traffic(workload, precision, pprec):
    """Counter-measured bytes per CG iteration, if taken on the current kernel source."""
    import hashlib
    if (workload, pprec) not in TRAFFIC:
        return None
    path, src = TRAFFIC[(workload, pprec)]
    try:
        kv = dict(line.split(None, 1) for line in open(path) if line.strip() and not line.startswith("#"))
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if kv.get("source_sha256_prefix", "").strip() != h or kv.get("precision", "").strip() != precision:
        return None
    return float(kv["traffic_bytes_per_iteration"])


def cg_kernel_label(pprec, fp32):
    t = "<float>" if fp32 else "<double>"
    if pprec == "jacobi":
        return "scalar-potential CG iteration: k_pcg_iter" + t
    return ("one scalar-potential CG iteration with its multigrid cycle" + t + ": k_amg_iter, k_amg_spmv "
            "(restriction, fused coarse-level operators), k_amg_dense, k_amg_prolong, k_amg_post0, k_amg_w")


def roofline(prof, label, traffic):
    it = prof["iterations"]
    avg = prof["seconds"] / max(it, 1)
    ach = prof["bytes_per_iteration"] / avg / 1e9 if it else None
    return {"bound": "hbm", "kernel": label, "achieved": None if ach is None else round(ach, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None if ach is None else round(ach / HBM_PEAK_GBS, 4),
            "traffic": traffic, "avg_iteration_us": round(1e6 * avg, 3), "iterations": it,
            "bytes_per_iteration": prof["bytes_per_iteration"]}


def kernel_fracs(kt):
    """Per-launch bandwidth of the field kernels from mm_profile_kernels."""
    out = {}
    for name, v in kt.items():
        if v["launches"] == 0:
            continue
        ach = v["bytes"] / v["seconds"] / 1e9
        out[name] = {"launches": v["launches"], "avg_us": round(1e6 * v["seconds"] / v["launches"], 2),
                     "bytes_per_launch": round(v["bytes"] / v["launches"]), "achieved_GBs": round(ach, 1),
                     "frac": round(ach / HBM_PEAK_GBS, 4)}
    return out


def tune(ctx, binding, args):
    """Block shape of the scalar-potential kernels, fixed for the run."""
    if args.tune_cache:
        return ctx.tune(binding.MM_TUNE_CACHE, args.tune_cache)
    return ctx.tune(binding.MM_TUNE_MEASURE)


def host_info():
    """CPU model, logical CPUs and memory of the machine the oracle runs on."""
    model, mem = "unknown", None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "mem_total_GiB": mem}


def chunks_of(nf, steps):
    """Field indices of each step: `steps` consecutive chunks of the curve, or
    one field per step (wrapping to a new curve) when steps > nf."""
    import numpy as np
    if steps <= nf:
        return [c.tolist() for c in np.array_split(np.arange(nf), steps)]
    return [[k % nf] for k in range(steps)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed steps: the film's curve in this many chunks (other workloads: whole curves)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["film", "hard_cube", "batch64", "polycrystal"], default="film",
                    help="film: the 1000 x 1000 x 10 nm soft film, learned + FP32 against plain FP64 (default); "
                         "hard_cube: one 20^3 grain; batch64: 64 uneven grains in shared launches; "
                         "polycrystal: the 200 nm, 96^3-cell, 27-grain magnet (use --fields to bound it)")
    ap.add_argument("--fields", type=int, default=0, help="truncate the schedule (0 = all)")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--jmax", type=int, default=None,
                    help="inner iteration cap of the preconditioner solve (default: the workload's)")
    ap.add_argument("--net", default=NET, help="trained network of the learned form (film)")
    ap.add_argument("--learn-mode", choices=["start", "start+scale"], default="start",
                    help="learned form: the warm start alone, or with the learned Jacobi scaling")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 comparison curve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-fields", type=int, default=3, help="field steps of the oracle sample")
    ap.add_argument("--cpu-nli", type=int, default=3, help="nonlinear iterations per field of the oracle sample")
    ap.add_argument("--no-hard-cube", action="store_true", help="skip the hard cube's extra figure (film)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default block shape (no autotuning)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON cache of tuned block shapes (reused when it holds this workload)")
    ap.add_argument("--poisson-prec", choices=["auto", "jacobi", "amg"], default="auto",
                    help="preconditioner of the scalar-potential CG (amg: smoothed-aggregation multigrid; "
                         "auto: the faster one for the workload)")
    ap.add_argument("--no-jacobi", action="store_true",
                    help="skip the Jacobi-preconditioned comparison curve of a multigrid headline")
    ap.add_argument("--state", default=None,
                    help="hard_cube/polycrystal: run the curve in pieces, resuming from this .npz when it exists "
                         "and saving the state to it after every --progress-every fields (a curve longer than one "
                         "run is timed over several)")
    ap.add_argument("--theta-max", type=float, default=None,
                    help="hard_cube/polycrystal: the line search's rotation cap (default: the library's, 0.2 rad)")
    ap.add_argument("--theta-adapt", type=int, choices=[0, 1], default=None,
                    help="hard_cube/polycrystal: 1 = the rotation cap follows the accepted steps (mm_opts.theta_adapt)")
    ap.add_argument("--theta-hi", type=float, default=None,
                    help="hard_cube/polycrystal: upper bound of the adapted rotation cap (rad)")
    ap.add_argument("--max-nli", type=int, default=None,
                    help="hard_cube/polycrystal: nonlinear iterations per field before a field ends unconverged")
    ap.add_argument("--time-limit", type=float, default=0.0,
                    help="with --state: stop after the piece that passes this many seconds of curve time")
    ap.add_argument("--progress-every", type=int, default=0,
                    help="hard_cube/polycrystal: run the curve in chunks of this many fields and report each")
    ap.add_argument("--calibrate", action="store_true",
                    help="only run a plain copy kernel of known size (for scaling HBM counters)")
    args = ap.parse_args()

    if args.poisson_prec == "auto":
        args.poisson_prec = AUTO_PREC[args.workload]
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: libmmncg has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate:
        # elementwise copy kernel: reads and writes exactly `nbytes` per launch
        nbytes = 256 << 20
        a = torch.rand(nbytes // 4, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "torch.mul(a, 1.0, out=b)", "bytes_read_per_launch": nbytes,
                          "bytes_written_per_launch": nbytes, "launches": 5}), flush=True)
        return
    if args.workload == "film":
        return bench_film(args)
    if args.workload == "batch64":
        return bench_batch(args)
    out = bench_curve(args)
    print(json.dumps(out), flush=True)


def log(msg):
    print("# " + msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# the film: learned + FP32 against plain FP64 (the default)
# ---------------------------------------------------------------------------

def bench_film(args):
    import numpy as np
    import torch

    from paper_1801_03690_amd import binding, inputs, learn

    w = inputs.film()
    fields = w.fields if args.fields <= 0 else w.fields[: args.fields]
    nf = len(fields)
    jmax = w.jmax if args.jmax is None else args.jmax
    pprec = binding.MM_PREC_AMG if args.poisson_prec == "amg" else binding.MM_PREC_JACOBI
    ctx = binding.Context(0)
    t0 = time.time()
    ctx.upload(w.mesh)
    info = ctx.info()
    log(f"setup {time.time() - t0:.1f}s n_mag={info['n_mag']} n_pot={info['n_pot']} nnz_K={info['nnz_K']}")
    graph = binding.Graph(ctx)
    net = learn.load_net(args.net, ctx)
    o_l = binding.default_opts(jmax=jmax, precision=binding.MM_FP32_BULK, poisson_prec=pprec, theta_max=w.theta_max)
    o_p = binding.default_opts(jmax=jmax, precision=binding.MM_FP64, poisson_prec=pprec, theta_max=w.theta_max)
    m0 = torch.tensor(w.m0, dtype=torch.float64, device="cuda")
    m = torch.empty_like(m0)
    shapes = {}

    def set_form(o, name):
        ctx.set_opts(o)
        if not args.no_tune:
            nw, spw = tune(ctx, binding, args)
            shapes[name] = (nw, spw.tolist())

    def run_steps(idx_lists, o, mode):
        """Steps over chunks of the field list; returns per-field results."""
        parts, times = [], []
        last = None
        for idx in idx_lists:
            if idx[0] == 0 or last is None or idx[0] != last + 1:
                m.copy_(m0)
                ctx.reset_warm_start()
                hp = None
            else:
                hp = fields[idx[0] - 1]
            ta = time.perf_counter()
            r = ctx.curve_learned(net, graph, mode, m, fields[idx[0]: idx[-1] + 1], opts=o, h_prev_T=hp)
            times.append(time.perf_counter() - ta)
            parts.append((idx, r))
            last = idx[-1]
        return parts, times

    # --- learned + FP32 (the value)
    lmode = binding.MM_LEARN_START | (binding.MM_LEARN_SCALE if args.learn_mode == "start+scale" else 0)
    set_form(o_l, "learned_fp32")
    steps = chunks_of(nf, args.steps)
    if args.warmup:
        run_steps(chunks_of(nf, max(args.steps, args.warmup))[: args.warmup], o_l, lmode)
        log(f"warmup: {args.warmup} steps")
    torch.cuda.synchronize()
    ctx.profile(-1)
    ctx.profile(1)
    ctx.profile_kernels(-1)
    ctx.profile_kernels(1)
    t0 = time.perf_counter()
    parts, times = run_steps(steps, o_l, lmode)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile(0)
    kt = ctx.profile_kernels(0)
    for i, dt in enumerate(times):
        log(f"step {i} fields {steps[i][0]}..{steps[i][-1]}: {dt:.3f}s")
    fields_walked = sum(len(p[0]) for p in parts)
    sec_curve = (t1 - t0) * nf / fields_walked
    first = {}
    for idx, r in parts:  # per-field results of the first walk of the curve
        for j, k in enumerate(idx):
            if k not in first:
                first[k] = (r["stats"][j], r["E"][j], r["m_avg"][j], r["accepted"][j])
    st_l = [first[k][0] for k in range(nf)]
    E_l = np.array([first[k][1] for k in range(nf)])
    mav_l = np.array([first[k][2] for k in range(nf)])
    learned = dict(seconds=round(sec_curve, 4), **count(st_l), starts_taken=int(sum(first[k][3] for k in range(nf))),
                   worst_status=max(s["status"] for s in st_l))

    out = {
        "metric": METRIC, "value": round(sec_curve, 4), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * (t1 - t0) / args.steps, 2), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 operators/f64 reductions (learned component bf16 MFMA)",
        "data": "synthetic (seeded Kuhn mesh, tilted +x start)",
        "config": {"workload": f"soft film 1000x1000x10 nm, 200x200x2 cells x6 tets + 3x air box, {nf} fields "
                               f"+50..{1e3 * fields[-1][0]:.0f} mT along x, jmax {jmax}, rotation cap "
                               f"{w.theta_max} rad, tol 1e-6; learned warm "
                               f"start{' + Jacobi scaling' if args.learn_mode == 'start+scale' else ''}, FP32 bulk; "
                               f"the curve in {min(args.steps, nf)} chunks",
                   "network": os.path.basename(args.net),
                   "poisson_preconditioner": args.poisson_prec, "n_mag": info["n_mag"], "n_pot": info["n_pot"],
                   "nnz_K": info["nnz_K"], "nnz_C_blocks": info["nnz_C_blocks"], "pcg_shapes": shapes},
        "learned_fp32": learned,
        "roofline": roofline(prof, cg_kernel_label(args.poisson_prec, True) + " (learned_fp32 form)",
                             measured_traffic("film", "fp32", args.poisson_prec)),
        "field_kernels": kernel_fracs(kt),
    }

    # --- plain FP64, the whole curve in one call
    if not args.no_plain:
        set_form(o_p, "plain_fp64")
        m.copy_(m0)
        ctx.reset_warm_start()
        ctx.curve(m, fields[:1], opts=o_p)  # warm-up of this form's kernels and graphs
        m.copy_(m0)
        ctx.reset_warm_start()
        torch.cuda.synchronize()
        ctx.profile_kernels(-1)
        ctx.profile_kernels(1)
        ta = time.perf_counter()
        rp = ctx.curve(m, fields, opts=o_p)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ktp = ctx.profile_kernels(0)
        log(f"plain fp64 curve {tb - ta:.2f}s")
        d = np.abs(mav_l - rp["m_avg"]).max(axis=1)
        out["plain_fp64"] = dict(seconds=round(tb - ta, 4), **count(rp["stats"]),
                                 worst_status=max(s["status"] for s in rp["stats"]),
                                 field_kernels=kernel_fracs(ktp))
        out["speedup_learned_fp32_vs_plain_fp64"] = round((tb - ta) / sec_curve, 3)
        out["learned_fp32"]["basin_changes_vs_plain"] = int((d > 1e-2).sum())
        out["learned_fp32"]["max_rel_dE_vs_plain"] = float(np.max(np.abs(E_l - rp["E"]) / np.abs(rp["E"])))
        out["learned_fp32"]["max_dmavg_vs_plain"] = float(d.max())
    net.close()
    graph.close()
    ctx.close()

    if not args.no_hard_cube:
        a2 = argparse.Namespace(**vars(args))
        a2.workload, a2.poisson_prec, a2.fields, a2.jmax, a2.steps, a2.warmup = "hard_cube", "amg", 0, None, 1, 1
        a2.no_cpu, a2.no_jacobi, a2.progress_every, a2.precision = True, True, 0, "fp32"
        a2.state, a2.theta_max, a2.max_nli, a2.theta_adapt, a2.theta_hi = None, None, None, None, None
        hc = bench_curve(a2)
        out["hard_cube"] = {k: hc[k] for k in ("value", "config", "counters", "roofline", "field_kernels")}
        if "plain_fp64" in hc:
            out["hard_cube"]["plain_fp64"] = hc["plain_fp64"]
        out["hard_cube"]["unit"] = "s"

    if not args.no_cpu and "plain_fp64" in out:
        out["cpu_baseline"] = cpu_baseline_film(args, w, fields, jmax, out["plain_fp64"])
    print(json.dumps(out), flush=True)


def count(stats):
    return {k: int(sum(s[k] for s in stats)) for k in ("evals", "nli", "li", "mi", "restarts", "fallbacks")}


def cpu_baseline_film(args, w, fields, jmax, plain):
    """The oracle (single-threaded C, FP64, Jacobi CG) on the first
    `cpu_fields` fields, `cpu_nli` nonlinear iterations each, each field
    started from the previous one's end. Its cost is a sum over work units
    (scalar-potential CG iterations, evaluations, inner preconditioner
    iterations) whose unit costs come from the sample itself: an evaluation
    whose potential is already converged (no CG iteration) and one inner
    solve are timed at the sample's last state; the rest of the sample's time
    is its CG iterations. The whole-curve figure weights those unit costs
    with the plain FP64 GPU curve's counts of the same units."""
    import oracle
    o = oracle.Oracle(w.mesh)
    m = w.m0.copy()
    ns = max(1, min(args.cpu_fields, len(fields)))
    tot = dict(evals=0, mi=0, li=0)
    ta = time.perf_counter()
    for k in range(ns):
        m, E, st, rc = o.minimize(m, fields[k], jmax=jmax, max_nli=args.cpu_nli, theta_max=w.theta_max)
        for q in tot:
            tot[q] += st[q]
    t_sample = time.perf_counter() - ta
    h = o.reduce_field(fields[ns - 1])
    tb = time.perf_counter()
    r = o.eval(m, h)  # the potential is warm: no CG iteration
    t_eval = time.perf_counter() - tb
    assert r["poisson_iters"] == 0, r["poisson_iters"]
    tb = time.perf_counter()
    y, it = o.precond(m, r["lam"], r["g"], jmax)
    t_li = (time.perf_counter() - tb) / max(it, 1)
    t_cg = max(t_sample - t_eval * tot["evals"] - t_li * tot["li"], 0.0) / max(tot["mi"], 1)
    est = t_cg * plain["mi"] + t_eval * plain["evals"] + t_li * plain["li"]
    base = {"value": round(est, 1), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"first {ns} of {len(fields)} field steps, {args.cpu_nli} nonlinear iteration(s) each "
                       f"({t_sample:.1f} s: {tot['evals']} evaluations, {tot['mi']} CG iterations, {tot['li']} "
                       f"inner iterations); unit costs {1e3 * t_cg:.1f} ms per CG iteration, {1e3 * t_eval:.0f} ms "
                       f"per evaluation without CG, {1e3 * t_li:.0f} ms per inner iteration, weighted with the "
                       f"plain FP64 GPU curve's counts"),
            "sample_seconds": round(t_sample, 2)}
    base.update(host_info())
    log(f"cpu baseline: sample {t_sample:.1f}s, estimate {est:.0f}s")
    return base


# ---------------------------------------------------------------------------
# one grain (hard cube) or the polycrystal: whole curves as steps
# ---------------------------------------------------------------------------

def curve_in_pieces(args, ctx, w, fields, opts, m, m0, info, jmax, shape):
    """One curve in pieces of --progress-every fields: the state (m, the next
    field, the curve time so far and the per-field counters) is saved after
    every piece, and a later run resumes from it. The curve time is the sum
    of the pieces' wall times; a resumed run starts its first solve from a
    zero potential (the warm start is not saved)."""
    import numpy as np
    import torch

    keys = ("evals", "nli", "li", "mi", "restarts", "fallbacks", "status")
    if os.path.exists(args.state):
        st = np.load(args.state)
        k0, elapsed, runs = int(st["next_field"]), float(st["elapsed"]), int(st["runs"]) + 1
        m.copy_(torch.from_numpy(st["m"]).to(m.device))
        rows, E, mav = [list(x) for x in st["stats"]], list(st["E"]), [list(x) for x in st["m_avg"]]
        log(f"resumed at field {k0} after {elapsed:.1f}s of curve time ({runs - 1} earlier runs)")
    else:
        k0, elapsed, runs, rows, E, mav = 0, 0.0, 1, [], [], []
        m.copy_(m0)
    ctx.reset_warm_start()
    pe = max(1, args.progress_every)
    t_run = 0.0
    while k0 < len(fields):
        torch.cuda.synchronize()
        tc = time.perf_counter()
        r = ctx.curve(m, fields[k0:k0 + pe], opts=opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - tc
        elapsed += dt
        t_run += dt
        rows += [[s[k] for k in keys] for s in r["stats"]]
        E += list(r["E"])
        mav += [list(x) for x in r["m_avg"]]
        k0 = min(len(fields), k0 + pe)
        tmp = args.state + ".tmp.npz"
        np.savez(tmp, m=m.cpu().numpy(), next_field=k0, elapsed=elapsed, runs=runs, stats=np.array(rows),
                 E=np.array(E), m_avg=np.array(mav))
        os.replace(tmp, args.state)
        log(f"fields ..{k0 - 1} done: {dt:.1f}s, curve time so far {elapsed:.1f}s")
        if args.time_limit and t_run > args.time_limit and k0 < len(fields):
            log(f"time limit reached: state saved at field {k0}")
            return
    tot = {k: int(sum(row[i] for row in rows)) for i, k in enumerate(keys[:-1])}
    out = {
        "metric": METRIC, "value": round(elapsed, 2), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(1e3 * elapsed, 1), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 operators/f64 reductions" if args.precision == "fp32" else "f64",
        "data": "synthetic (seeded Kuhn mesh, tilted +z start)",
        "config": {"workload": f"{args.workload}: whole curve of {len(fields)} fields, jmax {jmax}, tol 1e-6, "
                               f"timed in {runs} runs resumed from the saved state",
                   "precision": args.precision, "poisson_preconditioner": args.poisson_prec,
                   "n_mag": info["n_mag"], "n_pot": info["n_pot"], "nnz_K": info["nnz_K"],
                   "pcg_waves_per_block": shape[0]},
        "counters": dict(tot, worst_status=int(max(row[-1] for row in rows))),
        "per_field": {"nli": [int(row[1]) for row in rows], "E": [float(x) for x in E],
                      "m_avg_z": [float(x[2]) for x in mav]},
    }
    print(json.dumps(out), flush=True)


def bench_curve(args):
    import numpy as np
    import torch

    from paper_1801_03690_amd import binding, inputs

    w = inputs.polycrystal() if args.workload == "polycrystal" else inputs.hard_cube()
    if args.workload == "polycrystal":
        args.no_cpu = True
    fields = w.fields if args.fields <= 0 else w.fields[: args.fields]
    prec = binding.MM_FP32_BULK if args.precision == "fp32" else binding.MM_FP64
    ctx = binding.Context(0)
    t0 = time.time()
    ctx.upload(w.mesh)
    info = ctx.info()
    log(f"setup {time.time() - t0:.1f}s n_mag={info['n_mag']} n_pot={info['n_pot']} nnz_K={info['nnz_K']}")
    m0 = torch.tensor(w.m0, dtype=torch.float64, device="cuda")
    m = torch.empty_like(m0)
    pprec = binding.MM_PREC_AMG if args.poisson_prec == "amg" else binding.MM_PREC_JACOBI
    jmax = w.jmax if args.jmax is None else args.jmax
    extra = {k: v for k, v in (("theta_max", args.theta_max), ("max_nli", args.max_nli),
                               ("theta_adapt", args.theta_adapt), ("theta_hi", args.theta_hi)) if v is not None}
    opts = binding.default_opts(jmax=jmax, precision=prec, poisson_prec=pprec, **extra)
    ctx.set_opts(opts)
    if pprec == binding.MM_PREC_AMG:
        amg = ctx.amg_info()
        log(f"multigrid levels {amg['rows']} (operator entries {amg['nnz_A']}, prolongator entries "
            f"{amg['nnz_P']}) built in {amg['setup_seconds']:.2f}s")
    shape = (16, [1])
    if not args.no_tune:
        nw, spw = tune(ctx, binding, args)
        shape = (nw, spw.tolist())
        log(f"tuned shape: {nw} waves per block, slices per wave {spw.tolist()}")

    if args.state:
        return curve_in_pieces(args, ctx, w, fields, opts, m, m0, info, jmax, shape)

    def one_curve(o):
        m.copy_(m0)
        ctx.reset_warm_start()
        if args.progress_every <= 0:
            return ctx.curve(m, fields, opts=o)
        parts = []
        tc = time.perf_counter()
        for k0 in range(0, len(fields), args.progress_every):
            parts.append(ctx.curve(m, fields[k0:k0 + args.progress_every], opts=o))
            log(f"fields {k0}..{min(len(fields), k0 + args.progress_every) - 1} done, "
                f"{time.perf_counter() - tc:.1f}s")
        return dict(m=m, m_avg=np.concatenate([p["m_avg"] for p in parts]),
                    E=np.concatenate([p["E"] for p in parts]), stats=[x for p in parts for x in p["stats"]],
                    rc=max(p["rc"] for p in parts))

    for i in range(args.warmup):
        r = one_curve(opts)
        log(f"warmup {i} done rc={r['rc']}")

    torch.cuda.synchronize()
    ctx.profile(-1)
    ctx.profile(1)
    ctx.profile_kernels(-1)
    ctx.profile_kernels(1)
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(one_curve(opts))
        log(f"step {i} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile(0)
    kt = ctx.profile_kernels(0)
    sec_per_curve = (t1 - t0) / args.steps
    r = results[-1]
    st = r["stats"]
    worst = max(s["status"] for s in st)
    name = ("hard cube 80 nm, 20^3 cells x6 tets + 3x air box, {n} fields 0..{f:.2f} T, jmax {j}, tol 1e-6"
            if args.workload == "hard_cube" else
            "polycrystal 200 nm, 96^3 cells x6 tets + 3x air box, 27 Voronoi grains with a 2 nm boundary phase, "
            "first {n} of {N} fields 0..{f:.2f} T, jmax {j}, tol 1e-6")
    out = {
        "metric": METRIC, "value": round(sec_per_curve, 4), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * sec_per_curve, 2), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 operators/f64 reductions" if prec == binding.MM_FP32_BULK else "f64",
        "data": "synthetic (seeded Kuhn mesh, tilted +z start)",
        "config": {"workload": name.format(n=len(fields), N=len(w.fields), f=fields[-1][2], j=jmax),
                   "precision": args.precision, "poisson_preconditioner": args.poisson_prec,
                   "n_mag": info["n_mag"], "n_pot": info["n_pot"], "nnz_K": info["nnz_K"],
                   "nnz_C_blocks": info["nnz_C_blocks"], "pcg_waves_per_block": shape[0],
                   "pcg_slices_per_wave": shape[1][0]},
        "counters": dict(count(st), worst_status=worst),
        "roofline": roofline(prof, cg_kernel_label(args.poisson_prec, prec == binding.MM_FP32_BULK),
                             measured_traffic(args.workload, args.precision, args.poisson_prec)),
        "field_kernels": kernel_fracs(kt),
    }

    if not args.no_plain and prec != binding.MM_FP64:
        o64 = binding.default_opts(jmax=jmax, precision=binding.MM_FP64, poisson_prec=pprec, **extra)
        ctx.set_opts(o64)
        if not args.no_tune:
            tune(ctx, binding, args)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rp = one_curve(o64)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ctx.set_opts(opts)
        dE = float(np.max(np.abs(rp["E"] - r["E"]) / np.maximum(np.abs(rp["E"]), 1.0)))
        dmav = float(np.max(np.abs(rp["m_avg"] - r["m_avg"])))
        out["plain_fp64"] = {"seconds": round(tb - ta, 4), **count(rp["stats"]),
                             "max_rel_dE_vs_fp32": dE, "max_dmavg_vs_fp32": dmav}
        log(f"plain fp64 curve {tb - ta:.2f}s")

    if args.poisson_prec == "amg" and not args.no_jacobi:
        # the same curve with the Jacobi-preconditioned CG (one kernel per iteration)
        oj = binding.default_opts(jmax=jmax, precision=prec, poisson_prec=binding.MM_PREC_JACOBI, **extra)
        ctx.set_opts(oj)
        if not args.no_tune:
            tune(ctx, binding, args)
        torch.cuda.synchronize()
        ctx.profile(-1)
        ctx.profile(1)
        ta = time.perf_counter()
        rj = one_curve(oj)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        pj = ctx.profile(0)
        ctx.set_opts(opts)
        out["jacobi_cg"] = {
            "seconds": round(tb - ta, 4), "cg_iterations": int(sum(s["mi"] for s in rj["stats"])),
            "max_rel_dE_vs_amg": float(np.max(np.abs(rj["E"] - r["E"]) / np.maximum(np.abs(r["E"]), 1.0))),
            "roofline": roofline(pj, cg_kernel_label("jacobi", prec == binding.MM_FP32_BULK),
                                 measured_traffic(args.workload, args.precision, "jacobi")),
        }
        log(f"jacobi-preconditioned curve {tb - ta:.2f}s")

    if not args.no_cpu:
        import oracle
        o = oracle.Oracle(w.mesh)
        ns = max(1, min(args.cpu_fields, len(fields)))
        ta = time.perf_counter()
        ro = o.curve(w.m0, fields[:ns], jmax=jmax)
        t_sample = time.perf_counter() - ta
        # scaled with the GPU's own distribution of work over the fields
        gpu_all = sum(s["t_nl"] for s in st)
        gpu_sample = sum(s["t_nl"] for s in st[:ns])
        est = t_sample * gpu_all / max(gpu_sample, 1e-12)
        out["cpu_baseline"] = dict({
            "value": round(est, 2), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"first {ns} of {len(fields)} field steps timed ({t_sample:.2f} s, "
                      f"{sum(s['evals'] for s in ro['stats'])} evals); scaled to the whole curve by the "
                      f"GPU's per-field time distribution",
            "sample_seconds": round(t_sample, 3)}, **host_info())
    ctx.close()
    return out


# ---------------------------------------------------------------------------
# the batched parameter study
# ---------------------------------------------------------------------------

def bench_batch(args):
    """64 independent hard cubes of 8^3..24^3 cells (4 nm cells, K1 3.0-4.9
    MJ/m^3, easy axes in a 15 degree cone), each with its own curve 0 .. -8 T
    in 0.1 T steps, all solved together: every kernel launch serves every
    instance. One step = the whole batch of curves."""
    import numpy as np
    import torch

    from paper_1801_03690_amd import binding, inputs

    ws = inputs.batch_cubes()
    nf = len(ws[0].fields) if args.fields <= 0 else min(args.fields, len(ws[0].fields))
    F = np.stack([w.fields[:nf] for w in ws])
    prec = binding.MM_FP32_BULK if args.precision == "fp32" else binding.MM_FP64
    ctx = binding.Context(0)
    t0 = time.time()
    ctx.upload_batch([w.mesh for w in ws])
    t_setup = time.time() - t0
    infos = ctx.inst_info
    tot_pot = sum(d["n_pot"] for d in infos)
    tot_nnz = sum(d["nnz_K"] for d in infos)
    log(f"setup {t_setup:.1f}s instances={len(ws)} n_mag={ctx.n_mag} n_pot={tot_pot} nnz_K={tot_nnz}")
    pprec = binding.MM_PREC_AMG if args.poisson_prec == "amg" else binding.MM_PREC_JACOBI
    jmax = ws[0].jmax if args.jmax is None else args.jmax
    opts = binding.default_opts(jmax=jmax, precision=prec, poisson_prec=pprec)
    ctx.set_opts(opts)
    if pprec == binding.MM_PREC_AMG:
        # build the hierarchies (untimed, like the assembly) with one solve
        ta = time.time()
        ctx.batch_energy_grad(np.concatenate([w.m0 for w in ws]), np.zeros((len(ws), 3)))
        log(f"multigrid hierarchies built and first solve in {time.time() - ta:.1f}s")
    shape = (16, [1] * len(ws))
    if not args.no_tune:
        nw, spw = tune(ctx, binding, args)
        shape = (nw, spw.tolist())
        log(f"tuned shape: {nw} waves per block, slices per wave {spw.tolist()}")
    m0 = torch.tensor(np.concatenate([w.m0 for w in ws]), dtype=torch.float64, device="cuda")
    m = torch.empty_like(m0)

    def run(o):
        m.copy_(m0)
        ctx.reset_warm_start()
        return ctx.batch_curve(m, F, opts=o)

    for i in range(args.warmup):
        run(opts)
        log(f"warmup {i} done")
    torch.cuda.synchronize()
    ctx.profile(-1)
    ctx.profile(1)
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = run(opts)
        log(f"step {i} done rc={r['rc']}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile(0)
    sec = (t1 - t0) / args.steps
    st = r["stats"]
    tot = {k: int(sum(s[k] for row in st for s in row)) for k in ("evals", "nli", "li", "mi", "restarts",
                                                                   "fallbacks")}
    worst = max(s["status"] for row in st for s in row)
    achieved = prof["bytes"] / prof["seconds"] / 1e9 if prof["seconds"] > 0 else None
    out = {
        "metric": METRIC, "value": round(sec, 4), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * sec, 2), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 operators/f64 reductions" if prec == binding.MM_FP32_BULK else "f64",
        "data": "synthetic (seeded Kuhn meshes, tilted +z starts)",
        "config": {"workload": f"batch of 64 hard cubes 8^3..24^3 cells (4 nm), {nf} fields 0..{F[0, -1, 2]:.2f} T "
                               f"each, jmax {jmax}, tol 1e-6, one launch serves all instances",
                   "precision": args.precision, "poisson_preconditioner": args.poisson_prec, "instances": len(ws),
                   "n_mag": ctx.n_mag, "n_pot": tot_pot, "nnz_K": tot_nnz, "pcg_waves_per_block": shape[0],
                   "pcg_slices_per_wave": sorted(set(shape[1]))},
        "counters": dict(tot, worst_status=worst),
        "roofline": {
            "bound": "hbm", "kernel": cg_kernel_label(args.poisson_prec, prec == binding.MM_FP32_BULK),
            "achieved": None if achieved is None else round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "instance_iterations": prof["iterations"], "seconds": round(prof["seconds"], 4), "bytes": prof["bytes"],
        },
    }
    if not args.no_cpu:
        import oracle
        # the smallest instance's first field step, scaled by the Poisson CG
        # work (iterations x stored nonzeros, counted by the GPU run)
        k = int(np.argmin([d["n_pot"] for d in infos]))
        o = oracle.Oracle(ws[k].mesh)
        ta = time.perf_counter()
        o.curve(ws[k].m0, ws[k].fields[:1], jmax=jmax)
        t_sample = time.perf_counter() - ta
        w_all = sum(s["mi"] * infos[i]["nnz_K"] for i, row in enumerate(st) for s in row)
        w_smp = max(st[k][0]["mi"] * infos[k]["nnz_K"], 1)
        out["cpu_baseline"] = dict({
            "value": round(t_sample * w_all / w_smp, 2), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"instance {k} ({infos[k]['n_pot']} potential nodes), first field step ({t_sample:.2f} s); "
                      f"scaled by the batch's scalar-potential CG work (iterations x nnz(K), GPU counts)",
            "sample_seconds": round(t_sample, 3)}, **host_info())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
