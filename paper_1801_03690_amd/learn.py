"""Training and evaluation of the learned warm start / preconditioner scaling.

Orchestration only: every step runs in the library through its C ABI (plain
demagnetization curves that produce the training trajectories, node features,
the Hutchinson probe of the magnetostatic diagonal, the training targets
(mm_gnn_targets), the feature statistics (mm_gnn_moments), the training
loop with the network's forward and backward kernels and Adam
(mm_gnn_train) and the parameter file (mm_gnn_save / mm_gnn_load)). Device
arrays are torch tensors (memory only).

Training data: for each seeded film, the plain method's minimizers m_k along
its field sweep; one sample per step k -> k+1 with
  X     = features(m_k, h_k -> h_{k+1}),
  dm*   = P_{m_k}(m_{k+1} - m_k),
  s*_a  = 1 + t_a / D_a, t_a the mean of the magnetostatic Hessian diagonal
          (Hutchinson, Rademacher probes) over the two directions normal to
          m_k, D_a the exchange diagonal (the preconditioner's Jacobi).
"""
from __future__ import annotations

import time

import numpy as np

from . import binding as B
from . import inputs


class Film:
    """One film: its context, graph, trajectory and training samples (device)."""

    def __init__(self, work, jmax=4, n_probe=32, probe_seed=0, keep=True, precision=B.MM_FP64):
        import torch
        self.work = work
        self.ctx = B.Context(0).upload(work.mesh)
        self.graph = B.Graph(self.ctx)
        self.n = self.ctx.n_mag
        self.jmax = jmax
        t0 = time.perf_counter()
        r = self.ctx.curve(work.m0, work.fields, jmax=jmax, keep_hist=True, precision=precision)
        self.t_curve = time.perf_counter() - t0
        self.plain = r
        hist = r["hist"]
        z = inputs.rademacher(n_probe, self.n, seed=probe_seed)
        self.diag3 = self.ctx.demag_diag(z, rtol=1e-8)
        F = work.fields
        self.samples = []
        for k in range(len(F) - 1):
            mk = torch.tensor(hist[k], device="cuda")
            X = torch.empty((self.n, 32), dtype=torch.float32, device="cuda")
            self.graph.features(mk, F[k], F[k + 1], out=X)
            dmt = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
            st = torch.empty(self.n, dtype=torch.float64, device="cuda")
            self.graph.targets(mk, hist[k + 1], self.diag3, dm_out=dmt, s_out=st)
            self.samples.append((X, mk, dmt, st))
        self.ctx.reset_warm_start()

    def close(self):
        self.graph.close()
        self.ctx.close()


class Normalizer:
    """Per-column mean and spread of the features and the RMS of dm* over
    the training samples. The network standardizes its raw inputs itself,
    in FP32 before the first BF16 product (set on it by configure()): folding
    the standardization into the first layer instead would round the raw
    features to BF16 first, and features that vary by a few per cent around
    a large mean (|m|-like, diagonal ratios near 1) would lose their
    variation. Training sees targets in units of the RMS step; fold() scales
    the trained heads back to unscaled dm."""

    def __init__(self, films):
        s1, s2 = np.zeros(32), np.zeros(32)
        cnt = 0
        d2, dn = 0.0, 0
        for f in films:
            for X, m, dmt, st in f.samples:
                a, b = f.graph.moments(X)
                s1 += a
                s2 += b
                cnt += X.shape[0]
                d2 += float((dmt * dmt).sum())
                dn += dmt.shape[0]
        mu = s1 / cnt
        var = s2 / cnt - mu * mu
        sd = np.sqrt(np.maximum(var, 0.0))
        self.mu = np.where(sd > 1e-12, mu, 0.0)
        self.sd = np.where(sd > 1e-12, sd, 1.0)
        self.dm_rms = float(np.sqrt(d2 / max(dn, 1)))

    def configure(self, net):
        net.set_input_norm(self.mu, self.sd)
        return net

    def apply(self, films):
        """Scale the targets of `films` in place; per-sample weights make the
        warm-start loss relative to the size of each step."""
        for f in films:
            out = []
            for X, m, dmt, st in f.samples:
                dn = (dmt / self.dm_rms).contiguous()
                w = 1.0 / (float((dn * dn).sum(dim=1).mean()) + 1e-4)
                out.append((X, m, dn, st, w))
            f.samples = out

    def fold(self, theta):
        """Parameters whose warm-start head gives unscaled dm."""
        th = np.array(theta, dtype=np.float64)
        n = th.size
        # heads at the end: Wm (64x3), bm (3), Ws (64x1), bs (1)
        o_wm = n - (64 * 3 + 3 + 64 + 1)
        th[o_wm:o_wm + 64 * 3 + 3] *= self.dm_rms
        return th

    def save(self, path, theta, net=None, **meta):
        """npz with the folded parameters, standardization and run facts; with
        `net` also the library's parameter file (path + '.mmgnn')."""
        import json
        th = self.fold(theta)
        np.savez(path, theta=th, mu=self.mu, sd=self.sd, dm_rms=self.dm_rms, meta=json.dumps(meta))
        if net is not None:
            net.set_params(th)
            net.save(str(path) + ".mmgnn")
            net.set_params(theta)


def load_net(path, ctx):
    """A network on `ctx`'s device with the parameters and input
    standardization saved by Normalizer.save (npz) or by mm_gnn_save."""
    net = B.Gnn(ctx)
    if str(path).endswith(".mmgnn"):
        return net.load(path)
    z = np.load(path)
    net.set_params(z["theta"])
    net.set_input_norm(z["mu"], z["sd"])
    return net


def train(films, net, epochs=10, lr=1e-3, w_s=1.0, seed=0, log=None, val=None, stop_at=None, after_epoch=None):
    """Adam over every sample of every film (standardized by Normalizer.apply),
    shuffled each epoch (seeded): one library call (mm_gnn_train) per epoch.
    With stop_at (a time.perf_counter() value) no epoch starts that would end
    after it (judged by the longest epoch so far); after_epoch(ep) runs after
    every epoch (a checkpoint)."""
    samples = [(f.graph, X, m, dmt, st, w) for f in films for (X, m, dmt, st, w) in f.samples]
    hist = []
    longest = 0.0
    for ep in range(epochs):
        if stop_at is not None and ep > 0 and time.perf_counter() + longest > stop_at:
            if log:
                log(dict(stopped_before_epoch=ep))
            break
        t0 = time.perf_counter()
        loss = net.train(samples, 1, lr, w_s=w_s, seed=1000003 * seed + ep)[0]
        rec = dict(epoch=ep, train_loss=float(loss), seconds=time.perf_counter() - t0)
        if val is not None:
            rec["val_dm_loss"] = evaluate(val, net, w_s=0.0)
            rec["val_s_loss"] = evaluate(val, net, w_s=1.0, dm=False)
        hist.append(rec)
        longest = max(longest, time.perf_counter() - t0)
        if log:
            log(rec)
        if after_epoch:
            after_epoch(ep)
    return hist


def evaluate(films, net, w_s=1.0, dm=True):
    """Mean loss over the samples (the warm-start part relative to each
    step's size; dm=False keeps only the scaling part)."""
    tot, cnt = 0.0, 0
    for f in films:
        for X, m, dmt, st, w in f.samples:
            loss, _ = net.loss_grad(f.graph, X, m, dmt, st, inv_dm2=(w if dm else 0.0), w_s=w_s, want_grad=False)
            tot += loss
            cnt += 1
    return tot / max(cnt, 1)


def compare(work, net, jmax=4, modes=(0, 3), ctx=None, precision=B.MM_FP64):
    """Plain (mode 0) against learned curves on one workload, same stopping
    rule. Returns per mode: seconds, evaluations, NCG and CG iterations,
    accepted starts, and the largest difference of <m> from the plain curve
    (a different basin shows as an O(1) difference)."""
    own = ctx is None
    if own:
        ctx = B.Context(0).upload(work.mesh)
    graph = B.Graph(ctx)
    out = {}
    ref = None
    for mode in modes:
        ctx.reset_warm_start()
        t0 = time.perf_counter()
        r = ctx.curve_learned(net, graph, mode, work.m0, work.fields, jmax=jmax, precision=precision)
        dt = time.perf_counter() - t0
        st = r["stats"]
        rec = dict(seconds=dt, evals=int(sum(s["evals"] for s in st)), nli=int(sum(s["nli"] for s in st)),
                   li=int(sum(s["li"] for s in st)), mi=int(sum(s["mi"] for s in st)),
                   accepted=int(r["accepted"].sum()), rc=int(r["rc"]))
        if ref is None:
            ref = r
        rec["max_dmavg_vs_plain"] = float(np.abs(r["m_avg"] - ref["m_avg"]).max())
        rec["basin_mismatches"] = int((np.abs(r["m_avg"] - ref["m_avg"]).max(axis=1) > 1e-2).sum())
        rec["max_rel_dE_vs_plain"] = float(np.max(np.abs(r["E"] - ref["E"]) / np.maximum(np.abs(ref["E"]), 1e-30)))
        out[mode] = rec
    graph.close()
    if own:
        ctx.close()
    return out


def main(argv=None):
    """Train on seeded small films, evaluate on held-out ones, save the
    folded parameters (npz) and a JSON report."""
    import argparse
    import json
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--films", type=int, default=32)
    ap.add_argument("--heldout", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=15)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--probes", type=int, default=32)
    ap.add_argument("--lo", type=float, default=120.0)
    ap.add_argument("--hi", type=float, default=280.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default="gnn_films.npz")
    ap.add_argument("--report", default="gnn_films.json")
    ap.add_argument("--modes", default="0,1,2,3", help="curve modes compared on the held-out films")
    ap.add_argument("--jmax", type=int, default=4, help="inner iteration cap of the curves")
    ap.add_argument("--fp32-data", action="store_true",
                    help="training curves in the FP32-bulk mode (the minima agree with FP64 to round-off level)")
    ap.add_argument("--eval-film", action="store_true",
                    help="also compare plain and learned curves on the 1000 x 1000 x 10 nm film (FP64)")
    ap.add_argument("--train-until", type=float, default=None,
                    help="start no training epoch that would end later than this many seconds after the start "
                         "(the parameters are saved after every epoch)")
    args = ap.parse_args(argv)
    t0 = time.perf_counter()

    def say(*a):
        print(f"[{time.perf_counter() - t0:7.1f}s]", *a, flush=True)

    prec = B.MM_FP32_BULK if args.fp32_data else B.MM_FP64
    films = []
    for i in range(args.films):
        w = inputs.small_film(100 + i, lo=args.lo, hi=args.hi)
        films.append(Film(w, jmax=args.jmax, n_probe=args.probes, probe_seed=500 + i, precision=prec))
        say(f"film {i} {w.name} n={films[-1].n} plain curve {films[-1].t_curve:.2f}s")
    val = []
    for i in range(args.heldout):
        w = inputs.small_film(900 + i, lo=args.lo, hi=args.hi)
        val.append(Film(w, jmax=args.jmax, n_probe=args.probes, probe_seed=1900 + i, precision=prec))
        say(f"held-out {i} {w.name} n={val[-1].n}")
    nz = Normalizer(films)
    nz.apply(films)
    nz.apply(val)
    net = nz.configure(B.Gnn(films[0].ctx))
    net.set_params(inputs.gnn_init(args.seed))
    untrained = dict(val_dm_loss=evaluate(val, net, w_s=0.0), val_s_loss=evaluate(val, net, w_s=1.0, dm=False))
    say("untrained", untrained)
    def checkpoint(ep):
        nz.save(args.out, net.get_params(), net=net, films=args.films, epochs=ep + 1, lr=args.lr, lo=args.lo,
                hi=args.hi, probes=args.probes, seed=args.seed, jmax=args.jmax, fp32_data=args.fp32_data)

    stop_at = None if args.train_until is None else t0 + args.train_until
    hist = train(films, net, epochs=args.epochs, lr=args.lr, seed=args.seed, log=lambda r: say(r), val=val,
                 stop_at=stop_at, after_epoch=checkpoint)
    if not hist:
        checkpoint(-1)
    gains = []
    modes = tuple(int(x) for x in args.modes.split(","))
    for f in val:
        dep = load_net(args.out, f.ctx)
        res = compare(f.work, dep, jmax=args.jmax, modes=modes, ctx=f.ctx)
        say(f.work.name, res)
        gains.append(dict(name=f.work.name, n=f.n, **{f"mode{k}": v for k, v in res.items()}))
        dep.close()
    rep = dict(untrained=untrained, history=hist, heldout=gains)
    if args.eval_film:
        for f in films + val:
            f.close()
        w = inputs.film()
        ctx = B.Context(0).upload(w.mesh)
        dep = load_net(args.out, ctx)
        res = compare(w, dep, jmax=w.jmax, modes=(0, 3), ctx=ctx)
        say(w.name, res)
        rep["film_1000nm"] = {f"mode{k}": v for k, v in res.items()}
        dep.close()
        ctx.close()
    rep["seconds"] = time.perf_counter() - t0
    with open(args.report, "w") as fh:
        json.dump(rep, fh, indent=1)
    say("done")
    return rep


if __name__ == "__main__":
    main()
