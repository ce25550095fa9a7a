"""A sequence of implicit viscous steps from rest, V_k = A^-1 (V_{k-1} + f),
solved at every step from three starts: the plain previous-step start with
the FP64 operator, the same with the FP32 operator (SPH_MIXED: FP32 operator
and Krylov vectors, FP64 solution), and the learned start with the FP32
operator.  The trajectory follows the FP64 solutions.

  python -m paper_2206_14780_amd.sequence --workload lava --n 320 --steps 20

Prints one JSON line per step and a summary line (device time per solve from
the library's own events; iterations; true relative residuals)."""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", choices=("lava", "incline", "tank"), default="lava")
    ap.add_argument("--n", type=int, default=320)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--weights", default=None, help="learned-start weights (default: the shipped ones)")
    a = ap.parse_args(argv)

    import torch
    from . import sph as S
    from . import warmstart as WS
    from . import workloads as W

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    make = {"lava": W.lava_channel, "incline": W.incline_papanastasiou, "tank": W.open_box}[a.workload]
    w = make(a.n, tol=a.tol)
    log(f"[sequence] {w.name} n={w.n} generated in {time.time() - t0:.1f} s")
    ctx = S.Context(0)
    parts = S.device_particles(w)
    nb = ctx.sph_build_neighbors(parts, S.make_domain(w.lo, w.hi, w.periodic, w.h))
    par = S.make_params(w.dt, w.wall, w.avg, True, S.SPH_OP_CACHED)
    params = torch.as_tensor(WS.load(a.weights) if a.weights else WS.load()).cuda()
    legs = (("plain_f64", S.SPH_F64, None), ("plain_f32op", S.SPH_MIXED, None),
            ("learned_f32op", S.SPH_MIXED, params))
    V = np.zeros((w.n, 3))
    rows = []
    for k in range(1, a.steps + 1):
        B = w.rhs if k == 1 else W.next_step_rhs(w, V)
        b64 = S.device_vec3(B, S.SPH_F64)
        v64 = S.device_vec3(V, S.SPH_F64)
        row = dict(step=k)
        nxt = None
        for name, prec, warm in legs:
            x = [t.clone() for t in v64]
            o = S.make_opts(tol=a.tol, x0_given=True, warm_params=warm)
            rep = ctx.sph_visc_solve(nb, None, parts, par, prec, b64, x, o)
            torch.cuda.synchronize()
            rel = [float(np.sqrt(t / b)) if b > 0 else 0.0 for t, b in zip(rep["true_rr"], rep["bb"])]
            row[name] = dict(iters=rep["iters"], status=rep["status"],
                             device_ms=round(rep["setup_ms"] + rep["iterate_ms"], 3),
                             true_rel_res=max(rel))
            if warm is not None:
                row[name].update(warm_ms=round(rep["warm_ms"], 3), warm_used=list(rep["warm_used"]))
            if name == "plain_f64":
                nxt = np.stack([t.cpu().numpy() for t in x], axis=1)
        V = nxt
        row["speedup_learned_f32op_vs_plain_f64"] = round(row["plain_f64"]["device_ms"]
                                                          / row["learned_f32op"]["device_ms"], 3)
        rows.append(row)
        log(json.dumps(row))
    tot = {m: float(sum(r[m]["device_ms"] for r in rows)) for m, _, _ in legs}
    its = {m: int(sum(r[m]["iters"] for r in rows)) for m, _, _ in legs}
    log(json.dumps(dict(summary=True, workload=w.name, n=int(w.n), steps=a.steps, tol=a.tol,
                        total_device_ms=tot, total_iters=its,
                        speedup_learned_f32op_vs_plain_f64=tot["plain_f64"] / tot["learned_f32op"],
                        speedup_plain_f32op_vs_plain_f64=tot["plain_f64"] / tot["plain_f32op"],
                        final_max_abs_vx=float(np.abs(V[:, 0]).max()))))
    return 0


if __name__ == "__main__":
    sys.exit(main())
