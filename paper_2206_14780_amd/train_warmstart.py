"""Train the learned initial guess and evaluate it against the plain start.

  python -m paper_2206_14780_amd.train_warmstart --out weights.npy
  python -m paper_2206_14780_amd.train_warmstart --weights weights.npy --solves 0

Training data: `--solves` open-top boxes of n^3 jittered fluid (default 64^3,
N = 328,300 with walls), viscosity log-uniform in [1, 1e3], dt nu / dp^2
uniform in [10, 200], u a smooth random field plus noise and b = u; the
target of each is the library's FP64 solution to 1e-8 from x0 = u.  Plus
`--channels` lava-like channels of n^3 fluid sites (viscosity contrast e^1
.. e^5, dt nu_max / dp^2 log-uniform in [5, 200]), each run for
`--channel-steps` implicit steps from rest, V_k = A^-1 (V_{k-1} + f): the
samples of step k have u = V_{k-1}, b = V_{k-1} + f and target V_k.
Evaluation: held-out boxes of `--eval-n`^3 (default 160^3, N = 4,491,628),
each solved to `--eval-tol` four ways: plain start (x0 = u) and learned
start, each with the FP64 operator and with the FP32 operator (SPH_MIXED:
FP32 operator and Krylov vectors, FP64 solution).  Prints one JSON line per evaluated
solve and a summary line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--train-n", type=int, default=64)
    ap.add_argument("--solves", type=int, default=200)
    ap.add_argument("--seed0", type=int, default=4000)
    ap.add_argument("--channels", type=int, default=12)
    ap.add_argument("--channel-seed0", type=int, default=6000)
    ap.add_argument("--channel-steps", type=int, default=10)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--weights", default=None, help="start from / evaluate these weights")
    ap.add_argument("--out", default=None, help="write the trained weights here (.npy + .json)")
    ap.add_argument("--eval-n", type=int, default=160)
    ap.add_argument("--eval-solves", type=int, default=20)
    ap.add_argument("--eval-seed0", type=int, default=4500)
    ap.add_argument("--eval-tol", type=float, default=1e-6)
    ap.add_argument("--eval-channel-n", type=int, default=160,
                    help="side of the held-out lava channel whose sequence is evaluated (0 = skip)")
    ap.add_argument("--eval-channel-steps", type=int, default=10)
    a = ap.parse_args(argv)

    import torch
    from . import sph as S
    from . import warmstart as WS
    from . import workloads as W

    def log(msg):
        print(msg, flush=True)

    ctx = S.Context(0)
    params = None
    if a.weights:
        params = torch.as_tensor(WS.load(a.weights)).cuda()
    if a.solves > 0:
        t0 = time.time()
        samples, info = WS.generate(ctx, lambda s: W.warmstart_box(a.train_n, seed=s, tol=1e-8),
                                    range(a.seed0, a.seed0 + a.solves), tol=1e-8, log=log)
        log(f"data: {samples.shape[0]} samples from {a.solves} solves in {time.time() - t0:.0f} s")
        if a.channels > 0:
            t0 = time.time()
            seq, seq_info = WS.generate_sequences(
                ctx, lambda s: W.training_channel(a.train_n, seed=s, tol=1e-8),
                range(a.channel_seed0, a.channel_seed0 + a.channels), a.channel_steps, tol=1e-8, log=log)
            samples = torch.cat([samples, seq])
            info = info + seq_info
            del seq
            log(f"data: {samples.shape[0]} samples with {a.channels} channel sequences "
                f"({time.time() - t0:.0f} s)")
        t1 = time.time()
        p0 = params.cpu().numpy() if params is not None else None
        params, hist = WS.train(ctx, samples, steps=a.steps, batch=a.batch, lr=a.lr, params0=p0,
                                log=log)
        torch.cuda.synchronize()
        log(f"train: {a.steps} steps in {time.time() - t1:.1f} s, final loss {hist[-1][1]:.4e}")
        if a.out:
            WS.save(a.out, params.cpu().numpy(),
                    dict(train_n=a.train_n, solves=a.solves, seed0=a.seed0, channels=a.channels,
                         channel_seed0=a.channel_seed0, channel_steps=a.channel_steps, steps=a.steps,
                         batch=a.batch, lr=a.lr, samples=int(samples.shape[0]),
                         loss=[[int(s), float(l)] for s, l in hist], data=info))
            log(f"wrote {a.out}")
        del samples
    if params is None:
        return 0
    if a.eval_channel_n > 0:
        eval_channel(ctx, params, a.eval_channel_n, a.eval_channel_steps, a.eval_tol, log)
    if a.eval_solves <= 0:
        return 0

    rows = []
    for k in range(a.eval_solves):
        seed = a.eval_seed0 + k
        t0 = time.time()
        w = W.warmstart_box(a.eval_n, seed=seed, tol=a.eval_tol)
        r = WS.Resident(ctx, w)
        row = dict(seed=seed, n=int(w.n), nu=w.meta["nu"], dt_nu_dp2=w.meta["dt_nu_dp2"])
        for name, prec, warm in (("plain_f64", S.SPH_F64, None), ("plain_f32", S.SPH_MIXED, None),
                                 ("learned_f64", S.SPH_F64, params),
                                 ("learned_f32", S.SPH_MIXED, params)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, rep = r.solve(prec, a.eval_tol, warm_params=warm)
            wall = (time.perf_counter() - t) * 1e3
            rel = [float(np.sqrt(rep["true_rr"][c] / rep["bb"][c])) if rep["bb"][c] > 0 else 0.0
                   for c in range(3)]
            row[name] = dict(iters=rep["iters"], status=rep["status"], wall_ms=wall,
                             device_ms=rep["setup_ms"] + rep["iterate_ms"],
                             warm_ms=rep["warm_ms"], warm_used=rep["warm_used"],
                             true_rel_res=max(rel))
            if warm is not None:
                row[name]["rr_ratio"] = [round(float(x / y), 4) if y > 0 else None
                                         for x, y in zip(rep["warm_rr"], rep["plain_rr"])]
        row["speedup_learned_f32_vs_plain_f64"] = (row["plain_f64"]["device_ms"]
                                                   / row["learned_f32"]["device_ms"])
        rows.append(row)
        log(json.dumps(row))
        log(f"eval {k}: {time.time() - t0:.1f} s")
        del r
    sp = [x["speedup_learned_f32_vs_plain_f64"] for x in rows]
    it = {m: float(np.mean([x[m]["iters"] for x in rows]))
          for m in ("plain_f64", "plain_f32", "learned_f64", "learned_f32")}
    ms = {m: float(np.median([x[m]["device_ms"] for x in rows]))
          for m in ("plain_f64", "plain_f32", "learned_f64", "learned_f32")}
    log(json.dumps(dict(summary=True, eval_n=a.eval_n, solves=len(rows), mean_iters=it,
                        median_device_ms=ms, speedup_median=float(np.median(sp)),
                        speedup_min=float(np.min(sp)))))
    return 0


def eval_channel(ctx, params, n, steps, tol, log):
    """The lava channel (seed 5, the benchmark's field at n^3) run as an
    implicit-step sequence from rest; every step is solved with the FP32
    operator (FP64 solution) from the plain previous-step start and from the
    learned start, the trajectory following the plain solves."""
    import torch
    from . import sph as S
    from . import workloads as W
    w = W.lava_channel(n, tol=tol)
    parts = S.device_particles(w)
    nb = ctx.sph_build_neighbors(parts, S.make_domain(w.lo, w.hi, w.periodic, w.h))
    par = S.make_params(w.dt, w.wall, w.avg, True, S.SPH_OP_CACHED)
    fluid = torch.as_tensor(w.ptype == W.FLUID).cuda()
    f = [torch.as_tensor(w.rhs[:, c]).cuda() for c in range(3)]
    V = [torch.zeros(w.n, dtype=torch.float64, device="cuda") for _ in range(3)]
    tot = {"plain_f32": [0.0, 0], "learned_f32": [0.0, 0]}
    used = 0
    for k in range(1, steps + 1):
        B = [torch.where(fluid, V[c] + f[c], torch.zeros_like(f[c])) for c in range(3)]
        row = dict(step=k)
        nxt = None
        for name, warm in (("plain_f32", None), ("learned_f32", params)):
            X = [v.clone() for v in V]
            rep = ctx.sph_visc_solve(nb, None, parts, par, S.SPH_MIXED, B, X,
                                     S.make_opts(tol=tol, x0_given=True, warm_params=warm))
            torch.cuda.synchronize()
            ms = rep["setup_ms"] + rep["iterate_ms"]
            row[name] = dict(iters=rep["iters"], device_ms=round(ms, 3))
            tot[name][0] += ms
            tot[name][1] += rep["iters"]
            if warm is not None:
                row[name]["warm_used"] = rep["warm_used"]
                row[name]["rr_ratio"] = [round(float(a / b), 4) if b > 0 else None
                                         for a, b in zip(rep["warm_rr"], rep["plain_rr"])]
                used += sum(rep["warm_used"])
            else:
                nxt = X
        V = nxt
        log(json.dumps(row))
    log(json.dumps(dict(channel_summary=True, n=int(w.n), steps=steps, device_ms={k: round(v[0], 1) for k, v in
                                                                                      tot.items()},
                        iters={k: v[1] for k, v in tot.items()},
                        speedup=round(tot["plain_f32"][0] / tot["learned_f32"][0], 3),
                        components_on_learned=used, components=3 * steps)))
    nb.free()


if __name__ == "__main__":
    sys.exit(main())
