"""Time steps of the non-Newtonian incline with the semi-implicit
predictor/corrector of the library (sph_semi_implicit_step): per step a
half-step solve, advection, neighbour rebuild, the Papanastasiou viscosity
update from the new velocity, the full-step solve, and the corrector.

  python -m paper_2206_14780_amd.simulate --n 160 --steps 5

The layer starts at rest with the viscosity of the workload's synthetic
shear field; it is driven by the along-slope component of gravity (the
normal component is carried by the pressure, which is outside this path).
Prints one JSON line per step (wall time of the step call, iterations and
device time of both solves, true relative residuals, velocity and viscosity
ranges) and a summary line."""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=160, help="fluid sites per side of the incline")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--dt-factor", type=float, default=20.0,
                    help="time step in units of the workload's dt (dt nu_max/dp^2 = 50 at 1)")
    ap.add_argument("--prec", choices=("mixed", "f64"), default="mixed")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--newtonian", action="store_true", help="keep the viscosity (no update)")
    a = ap.parse_args(argv)

    import torch
    from . import sph as S
    from . import workloads as W

    def log(msg):
        print(msg, flush=True)

    tau0, m, mu0, slope = 100.0, 1000.0, 1.0, 10.0
    t0 = time.time()
    w = W.incline_papanastasiou(a.n, tau0=tau0, m=m, mu0=mu0, slope_deg=slope, tol=a.tol)
    log(f"[simulate] {w.name} n={w.n} generated in {time.time() - t0:.1f} s")
    ctx = S.Context(0)
    p = S.device_particles(w)
    dom = S.make_domain(w.lo, w.hi, w.periodic, w.h)
    dt = a.dt_factor * w.dt
    par = S.make_params(dt, w.wall, w.avg, True, S.SPH_OP_CACHED)
    prec = S.SPH_MIXED if a.prec == "mixed" else S.SPH_F64
    sp = S.make_step_params((math.sin(math.radians(slope)), 0.0, 0.0), None if a.newtonian else (tau0, m, mu0))
    opts = S.make_opts(tol=a.tol)
    u = [torch.zeros(w.n, dtype=torch.float64, device="cuda") for _ in range(3)]
    fluid = torch.as_tensor(w.ptype == W.FLUID, device="cuda")
    rows = []
    for k in range(1, a.steps + 1):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        reps = ctx.sph_semi_implicit_step(dom, p, par, prec, sp, opts, [p.x, p.y, p.z], u, p.mu)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3
        rel = [max(float(np.sqrt(t / b)) for t, b in zip(r["true_rr"], r["bb"]) if b > 0) for r in reps]
        mu_f = p.mu[fluid]
        row = dict(step=k, ms=round(ms, 2), iters=[r["iters"] for r in reps],
                   solve_ms=[round(r["setup_ms"] + r["iterate_ms"], 2) for r in reps],
                   status=[r["status"] for r in reps], true_rel_res=rel,
                   max_ux=float(u[0].max()), mu_range=[float(mu_f.min()), float(mu_f.max())])
        rows.append(row)
        log(json.dumps(row))
        if any(r["status"] != S.SPH_OK for r in reps):
            log("[simulate] a solve did not converge; stopping")
            return 1
    steady = rows[1:] if len(rows) > 1 else rows
    mean_ms = float(np.mean([r["ms"] for r in steady]))
    log(json.dumps(dict(summary=True, workload=w.name, n=int(w.n), steps=a.steps, dt=dt, prec=a.prec,
                        tol=a.tol, viscosity_update=not a.newtonian, mean_step_ms=mean_ms,
                        mean_step_ms_excludes_first=len(rows) > 1,
                        solve_share=float(np.mean([sum(r["solve_ms"]) / r["ms"] for r in steady])),
                        particle_steps_per_s=w.n / (mean_ms * 1e-3),
                        total_iters=int(sum(sum(r["iters"]) for r in rows)))))
    return 0


if __name__ == "__main__":
    sys.exit(main())
