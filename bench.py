#!/usr/bin/env python3
"""Benchmark: demagnetization-curve time-to-solution on one MI355X.

One step = one whole demagnetization curve (every field value, each
minimization run to max |m x h_eff| < 1e-6) of the hard-magnetic cube: edge
80 nm, 20^3 cells x 6 tets, 3x air box for the scalar potential, mu0 Ms =
1.61 T, K1 = 4.3 MJ/m^3, A = 7.7 pJ/m, easy axis z tilted 1 degree toward x,
field along -z from 0 to -8 T in 0.05 T steps (161 values), jmax = 1, in the
FP32-bulk mode (FP32 operators and Poisson CG, FP64 reductions, FP64
magnetization), the scalar-potential CG preconditioned by algebraic multigrid
(as in the paper; --poisson-prec jacobi for the Jacobi-preconditioned CG).
Inputs (mesh operators, the start state) are resident in HBM before the timed
region; assembly and the multigrid set-up are untimed, as in the paper.

Printed (one JSON line): time per curve, the measured bandwidth of the
dominant work, one scalar-potential CG iteration, against the HBM roofline
(HIP events around its launches inside the timed region), the plain FP64
form's and the Jacobi-preconditioned form's times for the same curve, and the
CPU FP64 oracle timed on a bounded sample of the same workload.
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
# counter-measured traffic per CG iteration of the hard cube, by preconditioner:
# (file, kernel source it was measured on)
TRAFFIC = {
    "jacobi": (os.path.join(ROOT, "profiles", "pcg_hard_cube_20_traffic.txt"),
               os.path.join(ROOT, "paper_1801_03690_amd", "csrc", "poisson.hip")),
    "amg": (os.path.join(ROOT, "profiles", "amg_hard_cube_20_traffic.txt"),
            os.path.join(ROOT, "paper_1801_03690_amd", "csrc", "amg.hip")),
}
# preconditioner of the scalar-potential CG per workload when --poisson-prec auto:
# multigrid where it is faster (measured), Jacobi on the thin film (a few dozen
# Jacobi iterations per solve) and in batches (multigrid is single-instance)
AUTO_PREC = {"hard_cube": "amg", "polycrystal": "amg", "film": "jacobi", "batch64": "amg"}


def measured_traffic(precision, pprec):
    """Counter-measured bytes per CG iteration, if taken on the current kernel source."""
    import hashlib
    path, src = TRAFFIC[pprec]
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


def tune(ctx, binding, args):
    """Block shape of the scalar-potential kernels, fixed for the run."""
    if args.tune_cache:
        return ctx.tune(binding.MM_TUNE_CACHE, args.tune_cache)
    return ctx.tune(binding.MM_TUNE_MEASURE)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fields", type=int, default=0, help="truncate the schedule (0 = all 161)")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--jmax", type=int, default=None,
                    help="inner iteration cap of the preconditioner solve (default: the workload's)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 comparison curve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-fields", type=int, default=1, help="field steps of the oracle sample")
    ap.add_argument("--no-tune", action="store_true", help="keep the default block shape (no autotuning)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the plain-vs-learned comparison on a held-out film")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON cache of tuned block shapes (reused when it holds this workload)")
    ap.add_argument("--workload", choices=["hard_cube", "batch64", "film", "polycrystal"], default="hard_cube",
                    help="hard_cube: one 20^3 grain (default); batch64: 64 uneven grains in shared launches; "
                         "film: the 1000 x 1000 x 10 nm soft film, plain FP64 against learned + FP32; "
                         "polycrystal: the 200 nm, 96^3-cell, 27-grain magnet (use --fields to bound it)")
    ap.add_argument("--poisson-prec", choices=["auto", "jacobi", "amg"], default="auto",
                    help="preconditioner of the scalar-potential CG (amg: smoothed-aggregation multigrid; "
                         "auto: the faster one for the workload)")
    ap.add_argument("--no-jacobi", action="store_true",
                    help="skip the Jacobi-preconditioned comparison curve of the multigrid headline")
    ap.add_argument("--progress-every", type=int, default=0,
                    help="run the curve in chunks of this many fields and report each (long curves); "
                         "every chunk starts from the previous one's last minimum, as one curve would")
    ap.add_argument("--calibrate", action="store_true",
                    help="only run a plain copy kernel of known size (for scaling HBM counters)")
    args = ap.parse_args()

    if args.poisson_prec == "auto":
        args.poisson_prec = AUTO_PREC[args.workload]
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1801_03690_amd import binding, inputs

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
    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "film":
        return bench_film(args)
    if args.workload == "polycrystal":
        w = inputs.polycrystal()
        args.no_learned = True
        args.no_cpu = True
    else:
        w = inputs.hard_cube()
    fields = w.fields if args.fields <= 0 else w.fields[: args.fields]
    prec = binding.MM_FP32_BULK if args.precision == "fp32" else binding.MM_FP64

    ctx = binding.Context(0)
    t0 = time.time()
    ctx.upload(w.mesh)
    t_setup = time.time() - t0
    info = ctx.info()
    print(f"# setup {t_setup:.1f}s n_mag={info['n_mag']} n_pot={info['n_pot']} nnz_K={info['nnz_K']}",
          file=sys.stderr, flush=True)
    m0 = torch.tensor(w.m0, dtype=torch.float64, device="cuda")
    m = torch.empty_like(m0)
    pprec = binding.MM_PREC_AMG if args.poisson_prec == "amg" else binding.MM_PREC_JACOBI
    jmax = w.jmax if args.jmax is None else args.jmax
    opts = binding.default_opts(jmax=jmax, precision=prec, poisson_prec=pprec)
    ctx.set_opts(opts)
    if pprec == binding.MM_PREC_AMG:
        amg = ctx.amg_info()
        print(f"# multigrid levels {amg['rows']} built in {amg['setup_seconds']:.2f}s", file=sys.stderr, flush=True)
    # block shape of the scalar-potential kernels: timed once here, untimed
    # like the assembly, and fixed for the run
    shape = (16, [1])
    if not args.no_tune:
        nw, spw = tune(ctx, binding, args)
        shape = (nw, spw.tolist())
        print(f"# tuned shape: {nw} waves per block, slices per wave {spw.tolist()}", file=sys.stderr, flush=True)

    def one_curve(o):
        m.copy_(m0)
        ctx.reset_warm_start()
        if args.progress_every <= 0:
            return ctx.curve(m, fields, opts=o)
        parts = []
        tc = time.perf_counter()
        for k0 in range(0, len(fields), args.progress_every):
            parts.append(ctx.curve(m, fields[k0:k0 + args.progress_every], opts=o))
            print(f"# fields {k0}..{min(len(fields), k0 + args.progress_every) - 1} done, "
                  f"{time.perf_counter() - tc:.1f}s", file=sys.stderr, flush=True)
        return dict(m=m, m_avg=np.concatenate([p["m_avg"] for p in parts]),
                    E=np.concatenate([p["E"] for p in parts]), stats=[x for p in parts for x in p["stats"]],
                    rc=max(p["rc"] for p in parts))

    for i in range(args.warmup):
        r = one_curve(opts)
        print(f"# warmup {i} done rc={r['rc']}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    ctx.profile(-1)
    ctx.profile(1)
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(one_curve(opts))
        print(f"# step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile(0)
    sec_per_curve = (t1 - t0) / args.steps
    r = results[-1]
    st = r["stats"]
    tot = {k: int(sum(s[k] for s in st)) for k in ("evals", "nli", "li", "mi", "restarts", "fallbacks")}
    worst = max(s["status"] for s in st)

    avg_iter = prof["seconds"] / max(prof["iterations"], 1)
    achieved = prof["bytes_per_iteration"] / avg_iter / 1e9 if prof["iterations"] else None

    out = {
        "metric": "demag-curve time-to-solution (s) & SpMV HBM GB/s, plain vs learned+FP32, equal tol",
        "value": round(sec_per_curve, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * sec_per_curve, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 operators/f64 reductions" if prec == binding.MM_FP32_BULK else "f64",
        "data": "synthetic (seeded Kuhn mesh, tilted +z start)",
        "config": {"workload": (f"hard cube 80 nm, 20^3 cells x6 tets + 3x air box, {len(fields)} fields "
                                f"0..{fields[-1][2]:.2f} T, jmax {jmax}, tol 1e-6" if args.workload == "hard_cube" else
                                f"polycrystal 200 nm, 96^3 cells x6 tets + 3x air box, 27 Voronoi grains with a "
                                f"2 nm boundary phase, first {len(fields)} of {len(w.fields)} fields "
                                f"0..{fields[-1][2]:.2f} T, jmax {jmax}, tol 1e-6"),
                   "precision": args.precision, "poisson_preconditioner": args.poisson_prec,
                   "n_mag": info["n_mag"], "n_pot": info["n_pot"],
                   "nnz_K": info["nnz_K"], "pcg_waves_per_block": shape[0], "pcg_slices_per_wave": shape[1][0]},
        "counters": dict(tot, worst_status=worst),
        "roofline": {
            "bound": "hbm",
            "kernel": cg_kernel_label(args.poisson_prec, prec == binding.MM_FP32_BULK),
            "achieved": None if achieved is None else round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (measured_traffic(args.precision, args.poisson_prec) if args.workload == "hard_cube"
                        else None),
            "avg_iteration_us": round(1e6 * avg_iter, 3),
            "iterations": prof["iterations"],
            "bytes_per_iteration": prof["bytes_per_iteration"],
        },
    }

    if not args.no_plain and prec != binding.MM_FP64:
        o64 = binding.default_opts(jmax=jmax, precision=binding.MM_FP64, poisson_prec=pprec)
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
        out["plain_fp64"] = {"seconds": round(tb - ta, 4),
                             "evals": int(sum(s["evals"] for s in rp["stats"])),
                             "nli": int(sum(s["nli"] for s in rp["stats"])),
                             "max_rel_dE_vs_fp32": dE, "max_dmavg_vs_fp32": dmav}
        print(f"# plain fp64 curve {tb - ta:.2f}s", file=sys.stderr, flush=True)

    if args.poisson_prec == "amg" and not args.no_jacobi:
        # the same curve with the Jacobi-preconditioned CG (one kernel per iteration)
        oj = binding.default_opts(jmax=jmax, precision=prec, poisson_prec=binding.MM_PREC_JACOBI)
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
        itj = pj["seconds"] / max(pj["iterations"], 1)
        achj = pj["bytes_per_iteration"] / itj / 1e9 if pj["iterations"] else None
        out["jacobi_cg"] = {
            "seconds": round(tb - ta, 4), "cg_iterations": int(sum(s["mi"] for s in rj["stats"])),
            "max_rel_dE_vs_amg": float(np.max(np.abs(rj["E"] - r["E"]) / np.maximum(np.abs(r["E"]), 1.0))),
            "roofline": {"bound": "hbm", "kernel": cg_kernel_label("jacobi", prec == binding.MM_FP32_BULK),
                         "achieved": None if achj is None else round(achj, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": None if achj is None else round(achj / HBM_PEAK_GBS, 4),
                         "traffic": (measured_traffic(args.precision, "jacobi") if args.workload == "hard_cube"
                                     else None),
                         "avg_iteration_us": round(1e6 * itj, 3), "iterations": pj["iterations"],
                         "bytes_per_iteration": pj["bytes_per_iteration"]},
        }
        print(f"# jacobi-preconditioned curve {tb - ta:.2f}s", file=sys.stderr, flush=True)

    if not args.no_learned:
        out["learned_film"] = bench_learned(args, binding, inputs, np, torch)

    if not args.no_cpu:
        import oracle
        o = oracle.Oracle(w.mesh)
        ns = max(1, min(args.cpu_fields, len(fields)))
        ta = time.perf_counter()
        ro = o.curve(w.m0, fields[:ns], jmax=jmax)
        tb = time.perf_counter()
        t_sample = tb - ta
        # extrapolate with the GPU's own distribution of work over the fields
        gpu_all = sum(s["t_nl"] for s in st)
        gpu_sample = sum(s["t_nl"] for s in st[:ns])
        est = t_sample * gpu_all / max(gpu_sample, 1e-12)
        out["cpu_baseline"] = {
            "value": round(est, 2), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"first {ns} of {len(fields)} field steps timed ({t_sample:.2f} s, "
                      f"{sum(s['evals'] for s in ro['stats'])} evals); scaled to the whole curve by the "
                      f"GPU's per-field time distribution",
            "sample_seconds": round(t_sample, 3),
        }
    print(json.dumps(out), flush=True)


def bench_learned(args, binding, inputs, np, torch):
    """Plain FP64 method against learned start + scaling in the FP32-bulk
    mode on a held-out soft film (seed 901 of the training family: 235 x 270
    nm, 5 nm cells, 2 cells thick, 3x air box, field along x from +50 to -50
    mT in 1 mT steps, jmax 4, same stopping rule), with the parameters
    trained by `python -m paper_1801_03690_amd.learn` (data/gnn_films.npz)."""
    path = os.path.join(ROOT, "paper_1801_03690_amd", "data", "gnn_films.npz")
    from paper_1801_03690_amd import learn
    w = inputs.small_film(901)
    ctx = binding.Context(0)
    ctx.upload(w.mesh)
    graph = binding.Graph(ctx)
    net = learn.load_net(path, ctx)
    res = {}
    for name, mode, prec in (("plain_fp64", 0, binding.MM_FP64), ("learned_fp64", 3, binding.MM_FP64),
                             ("learned_fp32", 3, binding.MM_FP32_BULK)):
        o = binding.default_opts(jmax=4, precision=prec)
        ctx.set_opts(o)
        if not args.no_tune:
            tune(ctx, binding, args)
        ctx.reset_warm_start()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.curve_learned(net, graph, mode, w.m0, w.fields, opts=o)
        dt = time.perf_counter() - t0
        st = r["stats"]
        res[name] = dict(seconds=round(dt, 4), evals=int(sum(x["evals"] for x in st)),
                         nli=int(sum(x["nli"] for x in st)), cg_iterations=int(sum(x["mi"] for x in st)),
                         starts_taken=int(r["accepted"].sum()), rc=int(r["rc"]), _r=r)
        print(f"# film {name}: {dt:.2f}s", file=sys.stderr, flush=True)
    ref = res["plain_fp64"]["_r"]
    for k in res:
        r = res[k].pop("_r")
        d = np.abs(r["m_avg"] - ref["m_avg"]).max(axis=1)
        res[k]["basin_changes_vs_plain"] = int((d > 1e-2).sum())
        res[k]["max_rel_dE_vs_plain"] = float(np.max(np.abs(r["E"] - ref["E"]) / np.abs(ref["E"])))
    res["speedup_learned_fp32_vs_plain_fp64"] = round(res["plain_fp64"]["seconds"] / res["learned_fp32"]["seconds"], 3)
    res["workload"] = (f"held-out film {w.name}: {ctx.n_mag} magnet nodes, {len(w.fields)} fields +50..-50 mT, "
                       f"jmax 4, tol 1e-6")
    net.close()
    graph.close()
    ctx.close()
    return res


def bench_film(args):
    """The 1000 x 1000 x 10 nm soft film (200 x 200 x 2 cells of 5 nm, 3x air
    box, 121,203 magnet nodes), field along x from +50 to -50 mT in 1 mT
    steps, jmax 10, tol 1e-6: learned start + scaling in the FP32-bulk mode
    (the value) against the plain FP64 method and learned FP64, with the
    parameters trained on 400-1000 nm films (data/gnn_films_large.npz). Each
    form runs once after a shared warm-up of one field."""
    import numpy as np
    import torch

    from paper_1801_03690_amd import binding, inputs, learn

    w = inputs.film()
    fields = w.fields if args.fields <= 0 else w.fields[: args.fields]
    jmax = w.jmax if args.jmax is None else args.jmax
    ctx = binding.Context(0)
    t0 = time.time()
    ctx.upload(w.mesh)
    info = ctx.info()
    print(f"# setup {time.time() - t0:.1f}s n_mag={info['n_mag']} n_pot={info['n_pot']} nnz_K={info['nnz_K']}",
          file=sys.stderr, flush=True)
    graph = binding.Graph(ctx)
    net = learn.load_net(os.path.join(ROOT, "paper_1801_03690_amd", "data", "gnn_films_large.npz"), ctx)
    legs = (("plain_fp64", 0, binding.MM_FP64), ("learned_fp64", 3, binding.MM_FP64),
            ("learned_fp32", 3, binding.MM_FP32_BULK))
    pprec = binding.MM_PREC_AMG if args.poisson_prec == "amg" else binding.MM_PREC_JACOBI
    res, shapes, prof = {}, {}, None
    for name, mode, prec in legs:
        o = binding.default_opts(jmax=jmax, precision=prec, poisson_prec=pprec)
        ctx.set_opts(o)
        if not args.no_tune:
            nw, spw = tune(ctx, binding, args)
            shapes[name] = (nw, spw.tolist())
        if args.warmup:
            ctx.reset_warm_start()
            ctx.curve_learned(net, graph, mode, w.m0, fields[:1], opts=o)
        ctx.reset_warm_start()
        torch.cuda.synchronize()
        if name == "learned_fp32":
            ctx.profile(-1)
            ctx.profile(1)
        t0 = time.perf_counter()
        r = ctx.curve_learned(net, graph, mode, w.m0, fields, opts=o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if name == "learned_fp32":
            prof = ctx.profile(0)
        st = r["stats"]
        res[name] = dict(seconds=round(dt, 4), evals=int(sum(x["evals"] for x in st)),
                         nli=int(sum(x["nli"] for x in st)), cg_iterations=int(sum(x["mi"] for x in st)),
                         starts_taken=int(r["accepted"].sum()), rc=int(r["rc"]), _r=r)
        print(f"# film {name}: {dt:.2f}s", file=sys.stderr, flush=True)
    ref = res["plain_fp64"]["_r"]
    for k in res:
        r = res[k].pop("_r")
        d = np.abs(r["m_avg"] - ref["m_avg"]).max(axis=1)
        res[k]["basin_changes_vs_plain"] = int((d > 1e-2).sum())
        res[k]["max_rel_dE_vs_plain"] = float(np.max(np.abs(r["E"] - ref["E"]) / np.abs(ref["E"])))
    sec = res["learned_fp32"]["seconds"]
    avg_iter = prof["seconds"] / max(prof["iterations"], 1)
    achieved = prof["bytes_per_iteration"] / avg_iter / 1e9 if prof["iterations"] else None
    out = {
        "metric": "demag-curve time-to-solution (s) & SpMV HBM GB/s, plain vs learned+FP32, equal tol",
        "value": sec, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
        "ms_per_step": round(1e3 * sec, 2), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 operators/f64 reductions (learned component bf16 MFMA)",
        "data": "synthetic (seeded Kuhn mesh, tilted +x start)",
        "config": {"workload": f"soft film 1000x1000x10 nm, 200x200x2 cells x6 tets + 3x air box, "
                               f"{len(fields)} fields +50..{1e3 * fields[-1][0]:.0f} mT along x, jmax {jmax}, tol 1e-6, "
                               f"learned start + scaling, FP32 bulk",
                   "poisson_preconditioner": args.poisson_prec, "n_mag": info["n_mag"], "n_pot": info["n_pot"], "nnz_K": info["nnz_K"],
                   "pcg_shapes": shapes},
        "forms": res,
        "speedup_learned_fp32_vs_plain_fp64": round(res["plain_fp64"]["seconds"] / sec, 3),
        "roofline": {
            "bound": "hbm", "kernel": ("scalar-potential CG iteration: k_pcg_iter<float> (learned_fp32 form)"
                                       if args.poisson_prec == "jacobi" else
                                       "scalar-potential CG iteration with one multigrid cycle<float> "
                                       "(learned_fp32 form)"),
            "achieved": None if achieved is None else round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "avg_iteration_us": round(1e6 * avg_iter, 3), "iterations": prof["iterations"],
            "bytes_per_iteration": prof["bytes_per_iteration"],
        },
    }
    net.close()
    graph.close()
    ctx.close()
    print(json.dumps(out), flush=True)


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
    print(f"# setup {t_setup:.1f}s instances={len(ws)} n_mag={ctx.n_mag} n_pot={tot_pot} nnz_K={tot_nnz}",
          file=sys.stderr, flush=True)
    pprec = binding.MM_PREC_AMG if args.poisson_prec == "amg" else binding.MM_PREC_JACOBI
    jmax = ws[0].jmax if args.jmax is None else args.jmax
    opts = binding.default_opts(jmax=jmax, precision=prec, poisson_prec=pprec)
    ctx.set_opts(opts)
    if pprec == binding.MM_PREC_AMG:
        # build the hierarchies (untimed, like the assembly) with one solve
        ta = time.time()
        ctx.batch_energy_grad(np.concatenate([w.m0 for w in ws]), np.zeros((len(ws), 3)))
        print(f"# multigrid hierarchies built and first solve in {time.time() - ta:.1f}s", file=sys.stderr,
              flush=True)
    shape = (16, [1] * len(ws))
    if not args.no_tune:
        nw, spw = tune(ctx, binding, args)
        shape = (nw, spw.tolist())
        print(f"# tuned shape: {nw} waves per block, slices per wave {spw.tolist()}", file=sys.stderr, flush=True)
    m0 = torch.tensor(np.concatenate([w.m0 for w in ws]), dtype=torch.float64, device="cuda")
    m = torch.empty_like(m0)

    def run(o):
        m.copy_(m0)
        ctx.reset_warm_start()
        return ctx.batch_curve(m, F, opts=o)

    for i in range(args.warmup):
        run(opts)
        print(f"# warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ctx.profile(-1)
    ctx.profile(1)
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = run(opts)
        print(f"# step {i} done rc={r['rc']}", file=sys.stderr, flush=True)
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
        "metric": "demag-curve time-to-solution (s) & SpMV HBM GB/s, plain vs learned+FP32, equal tol",
        "value": round(sec, 4), "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * sec, 2), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 operators/f64 reductions" if prec == binding.MM_FP32_BULK else "f64",
        "data": "synthetic (seeded Kuhn meshes, tilted +z starts)",
        "config": {"workload": f"batch of 64 hard cubes 8^3..24^3 cells (4 nm), {nf} fields 0..{F[0, -1, 2]:.2f} T "
                               f"each, jmax {jmax}, tol 1e-6, one launch serves all instances",
                   "precision": args.precision, "poisson_preconditioner": args.poisson_prec, "instances": len(ws), "n_mag": ctx.n_mag, "n_pot": tot_pot,
                   "nnz_K": tot_nnz, "pcg_waves_per_block": shape[0],
                   "pcg_slices_per_wave": sorted(set(shape[1]))},
        "counters": dict(tot, worst_status=worst),
        "roofline": {
            "bound": "hbm",
            "kernel": cg_kernel_label(args.poisson_prec, prec == binding.MM_FP32_BULK),
            "achieved": None if achieved is None else round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "instance_iterations": prof["iterations"], "seconds": round(prof["seconds"], 4),
            "bytes": prof["bytes"],
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
        out["cpu_baseline"] = {
            "value": round(t_sample * w_all / w_smp, 2), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"instance {k} ({infos[k]['n_pot']} potential nodes), first field step ({t_sample:.2f} s); "
                      f"scaled by the batch's scalar-potential CG work (iterations x nnz(K), GPU counts)",
            "sample_seconds": round(t_sample, 3),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
