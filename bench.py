#!/usr/bin/env python3
"""Benchmark of the semi-implicit SPH viscous solve on one MI355X.

Headline workload: the lava-like channel, 320^3 jittered fluid sites plus
three wall layers at the bottom and both sides (33,695,360 particles,
periodic along the flow, viscosity nu = 1e4 exp(-0.02 T) over a smooth
temperature field in [1000, 1200], harmonic pair mean, dummy walls,
dt nu_max/dp^2 = 50), run as a sequence of implicit steps from rest,
V_k = A^-1 (V_{k-1} + f) with f the along-slope body force per step (the
operator frozen: the sequence isolates the solve).  One step = the whole hot
path on inputs already in HBM: the right-hand side of the step, the
neighbour build by counting sort, the cached operator build, the learned
start and the robust BiCGSTAB to a 1e-6 relative residual with the FP32
operator and Krylov vectors (FP64 scalars and solution).  The same sequence
is timed beside it from the plain previous-step start, with the FP32 and
with the FP64 operator.

Prints one JSON line: particle-iterations per second of the learned FP32
steps, the roofline of the dominant kernel (the operator launch that
computes A r_star with its dot products, timed with HIP events on the
library's stream over the timed region: every 8th iteration's launch, so
that the event pairs, which leave a few microseconds of idle stream each, do
not slow the timed steps), the FP64 CPU oracle timed on a bounded sample of
the same workload, and, as extra keys, the 100^3 tank, the 160^3
non-Newtonian incline, the plain-versus-learned comparison on held-out 160^3
boxes, the CG against the BiCGSTAB, the Wendland against the Gaussian
kernel, and the paper's all-FP32 solver.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-1e-6 residual per solve, particle-iters/s, HBM GB/s; plain vs learned"
HBM_PEAK_GBS = 8000.0
PROFILE_EVERY = 8  # time the A r_star launch of every 8th iteration
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_apply_sell_f32_A2_lava320_hbm.md")


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when the kernel
    sources have changed since the counters were taken."""
    import hashlib
    try:
        txt = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = dict(l.split(": ", 1) for l in txt.splitlines()
                  if l.startswith(("traffic_bytes_per_launch:", "source_sha256:", "source_files:")))
    h = hashlib.sha256()
    for f in fields.get("source_files", "").split():
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != fields.get("source_sha256", "").strip():
        return None
    return int(fields["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed implicit steps of each leg")
    ap.add_argument("--warmup", type=int, default=1, help="untimed steps before them")
    ap.add_argument("--n", type=int, default=320, help="fluid sites per side of the lava channel")
    ap.add_argument("--legs", default="learned_f32op,plain_f32op,plain_f64",
                    help="sequence legs to time (the first is the headline)")
    ap.add_argument("--cpu-sample", type=int, default=16,
                    help="the oracle's timed sample: particles of the first 1/k of the channel (0 = skip)")
    ap.add_argument("--cpu-sample-iters", type=int, default=2,
                    help="BiCGSTAB iterations of the oracle's timed samples")
    ap.add_argument("--tank-n", type=int, default=100, help="side of the tank leg (0 = skip)")
    ap.add_argument("--incline-n", type=int, default=160, help="side of the incline leg (0 = skip)")
    ap.add_argument("--learned-n", type=int, default=160,
                    help="fluid particles per side of the plain-vs-learned boxes (0 = skip)")
    ap.add_argument("--learned-seeds", type=int, default=3, help="held-out boxes compared")
    ap.add_argument("--learned-reps", type=int, default=2, help="timed solves per box and start")
    ap.add_argument("--cg-n", type=int, default=100,
                    help="tank side of the CG-versus-BiCGSTAB comparison on dynamic walls (0 = skip)")
    ap.add_argument("--cg-steps", type=int, default=3, help="timed steps per solver in that comparison")
    ap.add_argument("--kernel-n", type=int, default=100,
                    help="tank side of the Wendland-versus-Gaussian comparison (0 = skip)")
    ap.add_argument("--kernel-steps", type=int, default=3, help="timed steps per kernel in that comparison")
    ap.add_argument("--fp32-n", type=int, default=100,
                    help="tank side of the all-FP32 solver study (0 skips it)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the steps, copy a buffer of this many MiB on the device once "
                         "(a kernel of known traffic to scale hardware byte counters)")
    return ap.parse_args()


def _oracle_rate(w, sample_iters, X0=None, threads=None):
    """Particle-iterations per second of the FP64 oracle (as it stands:
    matrix-free operator) over `sample_iters` robust BiCGSTAB iterations of w;
    the neighbour grid is built first and not counted."""
    import oracle as O
    if threads:
        O.set_num_threads(threads)
    try:
        t0 = time.perf_counter()
        nbr = O.neighbors(w.pos, w.period, w.h, lo=w.lo, method="grid")
        t_nbr = time.perf_counter() - t0
        op = O.Operator.from_workload(w, nbr=nbr)
        t0 = time.perf_counter()
        _, rep, _ = O.solve(op, w.rhs, X0=X0, tol=w.tol, max_iter=sample_iters, true_res_period=0)
        t_solve = time.perf_counter() - t0
        return w.n * max(rep["iters"], 1) / t_solve, max(rep["iters"], 1), t_solve, t_nbr, O.num_threads()
    finally:
        if threads:
            O.set_num_threads(os.cpu_count() or 1)


def cpu_baseline(w, frac, sample_iters):
    """The FP64 oracle on a slab of the same channel (the particles of its
    first 1/frac along the flow), plus single-thread figures on the 16^3
    Poiseuille channel (whole solve) and the 100^3 tank (first iterations)."""
    import numpy as np

    from paper_2206_14780_amd import workloads as W
    import dataclasses
    L = w.hi[0] - w.lo[0]
    keep = w.pos[:, 0] < w.lo[0] + L / frac
    slab = dataclasses.replace(w, name=w.name + f"_slab{frac}", pos=w.pos[keep], mass=w.mass[keep],
                               rho=w.rho[keep], mu=w.mu[keep], ptype=w.ptype[keep], rhs=w.rhs[keep],
                               periodic=np.array([0, 0, 0]), hi=np.array([w.lo[0] + L / frac, w.hi[1], w.hi[2]]))
    rate, iters, t_solve, t_nbr, cores = _oracle_rate(slab, sample_iters)
    out = {"value": rate, "unit": "particle-iters/s", "cores": cores, "kind": "oracle",
           "sample": (f"the first 1/{frac} of the {w.n}-particle lava channel along the flow ({slab.n} particles, "
                      f"same positions, viscosities and rhs; not periodic), FP64 robust BiCGSTAB with the "
                      f"matrix-free operator, first {iters} iterations in {t_solve:.1f} s (neighbour grid "
                      f"{t_nbr:.1f} s not counted)")}
    single = {}
    p16 = W.poiseuille(16, wall=W.WALL_DUMMY)
    r1, it1, t1, _, _ = _oracle_rate(p16, 10000, threads=1)
    single["poiseuille16"] = {"n": int(p16.n), "iterations": it1, "seconds": round(t1, 3),
                              "particle_iters_per_s": round(r1, 1)}
    tank = W.open_box(100)
    r2, it2, t2, _, _ = _oracle_rate(tank, 1, X0=tank.x0, threads=1)
    single["tank100"] = {"n": int(tank.n), "iterations": it2, "seconds": round(t2, 3),
                         "particle_iters_per_s": round(r2, 1)}
    out["single_thread"] = single
    print(f"[bench] cpu baseline: {json.dumps(out)}", flush=True)
    return out


def _rel(rep):
    import numpy as np
    return max(float(np.sqrt(t / b)) for t, b in zip(rep["true_rr"], rep["bb"]) if b > 0)


def lava_sequence(ctx, w, leg, warmup, steps, profile_every):
    """Sequence V_k = A^-1 (V_{k-1} + f) from rest on the device: every step
    forms its rhs, builds the neighbour lists and solves from the previous
    step's solution (leg: learned_f32op / plain_f32op / plain_f64)."""
    import numpy as np
    import torch

    from paper_2206_14780_amd import sph as S
    from paper_2206_14780_amd import warmstart as WS
    from paper_2206_14780_amd import workloads as W

    prec = S.SPH_F64 if leg == "plain_f64" else S.SPH_MIXED
    warm = torch.as_tensor(WS.load()).cuda() if leg.startswith("learned") else None
    parts = S.device_particles(w)
    dom = S.make_domain(w.lo, w.hi, w.periodic, w.h)
    params = S.make_params(w.dt, w.wall, w.avg, jacobi=True, op_mode=S.SPH_OP_CACHED)
    fluid = torch.as_tensor(w.ptype == W.FLUID).cuda()
    f = [torch.as_tensor(w.rhs[:, c]).cuda() for c in range(3)]
    V = [torch.zeros(w.n, dtype=torch.float64, device="cuda") for _ in range(3)]
    B = [torch.empty_like(v) for v in V]
    opts = S.make_opts(tol=w.tol, x0_given=True, profile=profile_every, warm_params=warm)

    def step():
        for c in range(3):
            torch.where(fluid, V[c] + f[c], torch.zeros_like(f[c]), out=B[c])
        nb = ctx.sph_build_neighbors(parts, dom)
        rep = ctx.sph_visc_solve(nb, None, parts, params, prec, B, V, opts)
        nb.free()
        assert rep["status"] == S.SPH_OK, (leg, rep["status"], rep["state"])
        return rep

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    iters = [r["iters"] for r in reps]
    out = {"ms_per_step": round(total * 1e3 / steps, 3), "total_s": round(total, 3),
           "iterations": iters, "total_iterations": int(sum(iters)),
           "particle_iters_per_s": w.n * sum(iters) / total,
           "time_to_tol_ms_median": round(float(np.median([r["setup_ms"] + r["iterate_ms"] for r in reps])), 3),
           "setup_ms_median": round(float(np.median([r["setup_ms"] for r in reps])), 3),
           "launches_per_iteration": round(sum(r["launches"] for r in reps) / max(sum(iters), 1), 3),
           "issued_iterations_executed": round(sum(iters) / max(sum(r["issued_iters"] for r in reps), 1), 4),
           "true_rel_res_max": round(max(_rel(r) for r in reps), 9),
           "final_max_vx": round(float(V[0].abs().max()), 6)}
    if warm is not None:
        out["warm_ms_median"] = round(float(np.median([r["warm_ms"] for r in reps])), 3)
        out["components_on_learned_start"] = int(sum(sum(r["warm_used"]) for r in reps))
        out["components"] = 3 * steps
    out["_reps"] = reps
    del parts, V, B
    return out


def tank_leg(ctx, n, steps):
    """The 100^3 open-top tank (FP32 operator and vectors, FP64 scalars, the
    previous-step start): whole steps (neighbours + operator + solve)."""
    import torch

    from paper_2206_14780_amd import sph as S
    from paper_2206_14780_amd import workloads as W

    w = W.open_box(n=n)
    parts = S.device_particles(w)
    dom = S.make_domain(w.lo, w.hi, w.periodic, w.h)
    rhs = S.device_vec3(w.rhs, S.SPH_F32)
    x0 = S.device_vec3(w.x0, S.SPH_F32)
    x = [t.clone() for t in x0]
    params = S.make_params(w.dt, w.wall, w.avg, jacobi=True, op_mode=S.SPH_OP_CACHED)
    opts = S.make_opts(tol=w.tol, x0_given=True, profile=PROFILE_EVERY)

    def step():
        for a, b in zip(x, x0):
            a.copy_(b)
        nb = ctx.sph_build_neighbors(parts, dom)
        rep = ctx.sph_visc_solve(nb, None, parts, params, S.SPH_F32, rhs, x, opts)
        nb.free()
        assert rep["status"] == S.SPH_OK, rep
        return rep

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    r = reps[-1]
    a_ms = sum(q["apply_ms"] for q in reps) / max(sum(q["apply_launches"] for q in reps), 1)
    out = {"workload": f"open-top tank {n}^3 jittered fluid + 3 wall layers (dummy), nu=10, dt*nu/dp^2=50, "
                       f"u0 ~ N(0, 0.1^2), previous-step start, f32 vectors/operator + f64 scalars, tol 1e-6",
           "n_particles": int(w.n), "ms_per_step": round(total * 1e3 / steps, 3), "iterations": r["iters"],
           "particle_iters_per_s": w.n * sum(q["iters"] for q in reps) / total,
           "time_to_tol_ms": round(r["setup_ms"] + r["iterate_ms"], 3), "setup_ms": round(r["setup_ms"], 3),
           "launches_per_iteration": round(r["launches"] / max(r["iters"], 1), 3),
           "issued_iterations_executed": round(sum(q["iters"] for q in reps) /
                                               max(sum(q["issued_iters"] for q in reps), 1), 4),
           "true_rel_res": round(_rel(r), 9), "avg_apply_launch_ms": round(a_ms, 4),
           "mat_nnz": int(r["mat_nnz"]), "mat_slots": int(r["mat_slots"])}
    print(f"[bench] tank: {json.dumps(out)}", flush=True)
    return out


def incline_leg(ctx, n):
    """The 160^3 non-Newtonian incline (Papanastasiou viscosity over three
    decades, harmonic mean), one solve from rest to 1e-6: plain start with the
    FP64 operator, plain and learned starts with the FP32 operator."""
    import torch

    from paper_2206_14780_amd import sph as S
    from paper_2206_14780_amd import warmstart as WS
    from paper_2206_14780_amd import workloads as W

    w = W.incline_papanastasiou(n)
    r = WS.Resident(ctx, w)
    warm = torch.as_tensor(WS.load()).cuda()
    out = {"workload": f"incline {n}^3 jittered fluid, periodic x-y, 3 bottom wall layers (dummy), 10 deg, "
                       f"Papanastasiou mu over {w.meta['mu_min']:.0f}..{w.meta['mu_max']:.0f}, harmonic mean, "
                       f"dt*mu_max/dp^2=50, from rest, tol 1e-6", "n_particles": int(w.n)}
    for name, prec, wp in (("plain_f64", S.SPH_F64, None), ("plain_f32op", S.SPH_MIXED, None),
                           ("learned_f32op", S.SPH_MIXED, warm)):
        r.solve(prec, 1e-6, from_u=False, warm_params=wp)
        _, rep = r.solve(prec, 1e-6, from_u=False, warm_params=wp)
        assert rep["status"] == S.SPH_OK, (name, rep["status"])
        out[name] = {"time_to_tol_ms": round(rep["setup_ms"] + rep["iterate_ms"], 3), "iterations": rep["iters"],
                     "particle_iters_per_s": w.n * rep["iters"] / ((rep["setup_ms"] + rep["iterate_ms"]) * 1e-3),
                     "true_rel_res": round(_rel(rep), 9)}
        if wp is not None:
            out[name]["warm_used"] = rep["warm_used"]
    print(f"[bench] incline: {json.dumps(out)}", flush=True)
    del r
    return out


def plain_vs_learned(ctx, n, seeds, reps):
    """Time to tolerance of plain and learned starts on held-out boxes."""
    import numpy as np
    import torch

    from paper_2206_14780_amd import sph as S
    from paper_2206_14780_amd import warmstart as WS
    from paper_2206_14780_amd import workloads as W

    params = torch.as_tensor(WS.load()).cuda()
    legs = (("plain_f64", S.SPH_F64, None), ("plain_f32op", S.SPH_MIXED, None),
            ("learned_f32op", S.SPH_MIXED, params))
    rows = []
    for seed in range(4500, 4500 + seeds):
        w = W.warmstart_box(n, seed=seed, tol=1e-6)
        r = WS.Resident(ctx, w)
        row = {"seed": seed, "dt_nu_dp2": round(w.meta["dt_nu_dp2"], 2), "nu": round(w.meta["nu"], 3)}
        for name, prec, warm in legs:
            r.solve(prec, 1e-6, warm_params=warm)  # warm-up
            wall, dev = [], []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, rep = r.solve(prec, 1e-6, warm_params=warm)
                wall.append((time.perf_counter() - t0) * 1e3)
                dev.append(rep["setup_ms"] + rep["iterate_ms"])
                assert rep["status"] == S.SPH_OK, (name, rep["status"])
            row[name] = {"ms": round(float(np.median(wall)), 2),
                         "device_ms": round(float(np.median(dev)), 2), "iters": rep["iters"],
                         "true_rel_res": round(max(float(np.sqrt(t / b)) for t, b in
                                                   zip(rep["true_rr"], rep["bb"]) if b > 0), 9)}
            if warm is not None:
                row[name]["warm_ms"] = round(rep["warm_ms"], 3)
                row[name]["warm_used"] = rep["warm_used"]
        row["speedup"] = round(row["plain_f64"]["ms"] / row["learned_f32op"]["ms"], 3)
        rows.append(row)
        print(f"[bench] learned box seed {seed}: {json.dumps(row)}", flush=True)
        del r
    return {"workload": f"open-top box {n}^3 jittered fluid + 3 wall layers (dummy), "
                        f"N={w.n}, held-out seeds {4500}..{4500 + seeds - 1}, b = u, x0 = u, tol 1e-6",
            "baseline": "plain previous-step start, FP64 operator and vectors",
            "learned": "learned start (BF16-MFMA MLP) + FP32 operator/Krylov vectors, FP64 solution",
            "speedup_median": round(float(np.median([r["speedup"] for r in rows])), 3),
            "speedup_min": round(float(np.min([r["speedup"] for r in rows])), 3),
            "boxes": rows}


def cg_vs_bicgstab(ctx, n, steps, prec_name):
    """Whole steps (neighbour build + operator build + solve) of the robust
    BiCGSTAB and of the rotated CG on the symmetric variant of the tank
    (dynamic walls, uniform mass), FP32 operator and vectors, to 1e-6."""
    import numpy as np
    import torch

    from paper_2206_14780_amd import sph as S
    from paper_2206_14780_amd import workloads as W

    prec = S.SPH_F32 if prec_name == "f32" else S.SPH_F64
    esz = 4 if prec == S.SPH_F32 else 8
    w = W.open_box(n=n, wall=W.WALL_DYNAMIC)
    parts = S.device_particles(w)
    dom = S.make_domain(w.lo, w.hi, w.periodic, w.h)
    rhs = S.device_vec3(w.rhs, prec)
    x0 = S.device_vec3(w.x0, prec)
    x = [t.clone() for t in x0]
    params = S.make_params(w.dt, w.wall, w.avg, jacobi=True, op_mode=S.SPH_OP_CACHED)
    out = {"workload": f"open-top tank {n}^3 jittered fluid + 3 wall layers (dynamic), uniform mass, nu=10, "
                       f"dt*nu/dp^2=50, {prec_name} vectors/operator + f64 scalars, cached operator, "
                       f"previous-step start, tol 1e-6; whole step (neighbours + matrix + solve)",
           "n_particles": w.n}
    for name, variant, applies in (("bicgstab", S.SPH_ROBUST, 2), ("cg", S.SPH_CG, 1)):
        opts = S.make_opts(tol=w.tol, x0_given=True, profile=PROFILE_EVERY, variant=variant)

        def step():
            for a, b in zip(x, x0):
                a.copy_(b)
            nb = ctx.sph_build_neighbors(parts, dom)
            rep = ctx.sph_visc_solve(nb, None, parts, params, prec, rhs, x, opts)
            nb.free()
            assert rep["status"] == S.SPH_OK, (name, rep)
            return rep

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = [step() for _ in range(steps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        r = reps[-1]
        a_ms = sum(q["apply_ms"] for q in reps) / max(sum(q["apply_launches"] for q in reps), 1)
        nslices = (w.n + 63) // 64
        # as the headline roofline, plus the CG's FP64 weight per row
        alg = r["mat_nnz"] * (4 + esz) + w.n * (7 * esz) + nslices * 8 + (w.n * 8 if variant == S.SPH_CG else 0)
        out[name] = {"ms_per_step": round(ms, 3), "iterations": r["iters"],
                     "applies_per_solve": r["iters"] * applies,
                     "time_to_tol_ms": round(float(np.median([q["setup_ms"] + q["iterate_ms"] for q in reps])), 3),
                     "true_rel_res": round(max(float(np.sqrt(t / b)) for t, b in zip(r["true_rr"], r["bb"]) if b > 0), 9),
                     "timed_kernel": "k_apply_sell<" + ("float" if esz == 4 else "double") + (
                         ", kDotCG>" if variant == S.SPH_CG else ", kDotA2>"),
                     "avg_launch_ms": round(a_ms, 4),
                     "hbm_frac": round(alg / (a_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if a_ms > 0 else None}
        print(f"[bench] {name} on dynamic walls: {json.dumps(out[name])}", flush=True)
    out["cg_speedup"] = round(out["bicgstab"]["ms_per_step"] / out["cg"]["ms_per_step"], 3)
    out["paper_context"] = "the paper reports the CG about 10% faster than the BiCGSTAB with dynamic walls"
    return out


def kernel_comparison(ctx, n, steps, prec_name):
    """Whole steps on the benchmark tank with the Wendland kernel (support 2h,
    ~80 neighbours) and the truncated Gaussian (support 3h, ~250), robust
    BiCGSTAB, FP32 operator and vectors, to 1e-6."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2206_14780_amd import sph as S
    from paper_2206_14780_amd import workloads as W

    prec = S.SPH_F32 if prec_name == "f32" else S.SPH_F64
    esz = 4 if prec == S.SPH_F32 else 8
    out = {"workload": f"open-top tank {n}^3 jittered fluid + 3 wall layers (dummy), nu=10, dt*nu/dp^2=50, "
                       f"{prec_name} vectors/operator + f64 scalars, cached operator, robust BiCGSTAB to 1e-6; "
                       f"whole step (neighbours + matrix + solve)"}
    for name, kern in (("wendland", W.KERNEL_WENDLAND), ("gaussian", W.KERNEL_GAUSSIAN)):
        w = dataclasses.replace(W.open_box(n=n), kernel=kern)
        parts = S.device_particles(w)
        dom = S.make_domain(w.lo, w.hi, w.periodic, w.h, kern)
        rhs = S.device_vec3(w.rhs, prec)
        x0 = S.device_vec3(w.x0, prec)
        x = [t.clone() for t in x0]
        params = S.make_params(w.dt, w.wall, w.avg, jacobi=True, op_mode=S.SPH_OP_CACHED)
        opts = S.make_opts(tol=w.tol, x0_given=True, profile=PROFILE_EVERY)

        def step():
            for a, b in zip(x, x0):
                a.copy_(b)
            nb = ctx.sph_build_neighbors(parts, dom)
            rep = ctx.sph_visc_solve(nb, None, parts, params, prec, rhs, x, opts)
            nb.free()
            assert rep["status"] == S.SPH_OK, (name, rep)
            return rep

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = [step() for _ in range(steps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        r = reps[-1]
        a_ms = sum(q["apply_ms"] for q in reps) / max(sum(q["apply_launches"] for q in reps), 1)
        alg = r["mat_nnz"] * (4 + esz) + w.n * (7 * esz) + ((w.n + 63) // 64) * 8
        out[name] = {"ms_per_step": round(ms, 3), "iterations": r["iters"],
                     "setup_ms": round(float(np.median([q["setup_ms"] for q in reps])), 3),
                     "nnz_per_row": round(r["mat_nnz"] / w.n, 1), "slots_per_row": round(r["mat_slots"] / w.n, 1),
                     "avg_launch_ms": round(a_ms, 4),
                     "hbm_frac": round(alg / (a_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if a_ms > 0 else None,
                     "true_rel_res": round(max(float(np.sqrt(t / b)) for t, b in zip(r["true_rr"], r["bb"]) if b > 0), 9)}
        print(f"[bench] {name} kernel: {json.dumps(out[name])}", flush=True)
        del parts, rhs, x0, x
    out["gaussian_cost_per_launch"] = round(out["gaussian"]["avg_launch_ms"] / out["wendland"]["avg_launch_ms"], 3)
    out["gaussian_step_ratio"] = round(out["gaussian"]["ms_per_step"] / out["wendland"]["ms_per_step"], 3)
    out["paper_context"] = ("the paper estimates the Gaussian kernel about 4x as expensive to evaluate, with about "
                            "twice the neighbour-list memory, partly repaid by fewer iterations")
    return out


def fp32_paper_study(ctx, n):
    """Single-precision solvers (FP32 vectors and operator, FP32 scalars, no
    residual restarts) against the library's default (FP64 scalars,
    periodic true-residual restarts), robust and textbook variants, to 1e-6
    and to the FP32 epsilon 2^-23, on: the benchmark tank from the
    previous-step start; a 64^3 plane channel from rest; and the same channel
    with a transverse component of noise of order 1e-8 (the situation in
    which the paper observes single-precision stalls: a velocity component
    that is analytically zero, its threshold near FLT_MIN).  Two
    single-precision arithmetics: `f32s` rounds FP64-accumulated inner
    products to FP32 (fp32_scalars), `paper32` is the paper's (FP32 matrix
    from cell-relative positions, compensated FP32 gemv and inner products)."""
    import numpy as np
    import torch

    from paper_2206_14780_amd import sph as S
    from paper_2206_14780_amd import workloads as W

    f32s = dict(fp32_scalars=True, true_res_period=0, restart_drop=0.0)
    p32 = dict(true_res_period=0, restart_drop=0.0)
    runs = [("default_f64_scalars", S.SPH_ROBUST, {}, S.SPH_OP_CACHED),
            ("f32s_robust", S.SPH_ROBUST, f32s, S.SPH_OP_CACHED),
            ("f32s_standard", S.SPH_STANDARD, f32s, S.SPH_OP_CACHED),
            ("paper32_robust", S.SPH_ROBUST, p32, S.SPH_OP_PAPER32),
            ("paper32_standard", S.SPH_STANDARD, p32, S.SPH_OP_PAPER32)]
    out = {"workload": f"open-top tank {n}^3 (dummy walls) from the previous-step start; plane channel 64^3 "
                       f"(dummy walls) from rest, and the same with a transverse rhs of N(0, 1e-8^2) noise; "
                       f"FP32 vectors, cached operator, max 3000 iterations",
           "stall_note": "stalls: iterations in which a component with a nonzero right-hand side broke down"}
    chan = W.poiseuille(64, wall=W.WALL_DUMMY)
    noisy = W.poiseuille(64, wall=W.WALL_DUMMY)
    rng = np.random.default_rng(64)
    noisy.rhs = noisy.rhs.copy()
    fl = noisy.ptype == W.FLUID
    noisy.rhs[fl, 1] = 1e-8 * rng.normal(size=int(fl.sum()))
    for wname, w, use_x0 in (("tank", W.open_box(n=n), True), ("channel64", chan, False),
                             ("channel64_transverse_noise", noisy, False)):
        parts = S.device_particles(w)
        dom = S.make_domain(w.lo, w.hi, w.periodic, w.h)
        nb = ctx.sph_build_neighbors(parts, dom)
        rhs = S.device_vec3(w.rhs, S.SPH_F32)
        start = w.x0 if use_x0 else np.zeros((w.n, 3))
        x0 = S.device_vec3(start, S.SPH_F32)
        live = [c for c in range(3) if np.any(w.rhs[:, c] != 0)]
        res = {}
        for tol_name, tol in (("tol_1e-6", 1e-6), ("tol_2^-23", 2.0 ** -23)):
            for name, var, extra, mode in runs:
                params = S.make_params(w.dt, w.wall, w.avg, jacobi=True, op_mode=mode)
                x = [t.clone() for t in x0]
                o = S.make_opts(tol=tol, x0_given=use_x0, max_iter=3000, variant=var, **extra)
                rep = ctx.sph_visc_solve(nb, None, parts, params, S.SPH_F32, rhs, x, o)
                torch.cuda.synchronize()
                res[f"{tol_name}/{name}"] = {
                    "status": rep["status"], "iterations": rep["iters"],
                    "solve_ms": round(rep["setup_ms"] + rep["iterate_ms"], 3),
                    "stalls": [rep["stall_count"][c] for c in live],
                    "states": [rep["state"][c] for c in live],
                    "true_rel_res": [float(f"{np.sqrt(rep['true_rr'][c] / rep['bb'][c]):.4e}") for c in live]}
        nb.free()
        out[wname] = res
        print(f"[bench] fp32 study {wname}: {json.dumps(res)}", flush=True)
        del parts, rhs, x0
    return out

def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the solver has no "
              "multi-GPU domain decomposition.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2206_14780_amd import sph as S
    from paper_2206_14780_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.time()
    w = W.lava_channel(args.n)
    print(f"[bench] workload {w.name} n={w.n} generated in {time.time() - t0:.1f} s", flush=True)
    ctx = S.Context(0)
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    legs = [l for l in args.legs.split(",") if l]
    seq = {}
    for leg in legs:
        seq[leg] = lava_sequence(ctx, w, leg, args.warmup, args.steps, PROFILE_EVERY)
        print(f"[bench] lava {leg}: " + json.dumps({k: v for k, v in seq[leg].items() if k != "_reps"}),
              flush=True)
    head = seq[legs[0]]
    reps = head.pop("_reps")
    for leg in legs[1:]:
        seq[leg].pop("_reps")

    # dominant kernel: the A r_star operator launch (one per iteration)
    a_ms = sum(r["apply_ms"] for r in reps) / max(sum(r["apply_launches"] for r in reps), 1)
    esz = 8 if legs[0] == "plain_f64" else 4
    nnz, slots = reps[-1]["mat_nnz"], reps[-1]["mat_slots"]
    nslices = (w.n + 63) // 64
    # algorithmic bytes per launch: every stored nonzero (column index +
    # coefficient), x (3 values) and y (3 values) and the diagonal per row,
    # one slice pointer per 64 rows
    alg_bytes = nnz * (4 + esz) + w.n * (7 * esz) + nslices * 8
    roofline = None
    if a_ms > 0:
        achieved = alg_bytes / (a_ms * 1e-3) / 1e9
        traffic = measured_traffic() if (args.n == 320 and esz == 4) else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": f"k_apply_sell<{'float' if esz == 4 else 'double'}, kDotA2>",
                    "avg_launch_ms": round(a_ms, 4), "alg_bytes_per_launch": int(alg_bytes),
                    "mat_nnz": int(nnz), "mat_slots": int(slots)}
        if traffic:
            roofline["traffic_rate_gbs"] = round(traffic / (a_ms * 1e-3) / 1e9, 1)
            roofline["traffic_frac"] = round(traffic / (a_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    extras = {}
    if args.tank_n > 0:
        print("[bench] tank", flush=True)
        extras["tank100"] = tank_leg(ctx, args.tank_n, 5)
    if args.incline_n > 0:
        print("[bench] incline", flush=True)
        extras["incline160"] = incline_leg(ctx, args.incline_n)
    if args.learned_n > 0 and args.learned_seeds > 0:
        print("[bench] plain vs learned (held-out boxes)", flush=True)
        extras["plain_vs_learned"] = plain_vs_learned(ctx, args.learned_n, args.learned_seeds, args.learned_reps)
    if args.cg_n > 0:
        print("[bench] CG vs BiCGSTAB (dynamic walls)", flush=True)
        extras["cg_vs_bicgstab"] = cg_vs_bicgstab(ctx, args.cg_n, args.cg_steps, "f32")
    if args.kernel_n > 0:
        print("[bench] Wendland vs Gaussian kernel", flush=True)
        extras["kernel_comparison"] = kernel_comparison(ctx, args.kernel_n, args.kernel_steps, "f32")
    if args.fp32_n > 0:
        print("[bench] all-FP32 solver study", flush=True)
        extras["fp32_paper"] = fp32_paper_study(ctx, args.fp32_n)
    cpu = None
    if args.cpu_sample > 0:
        print("[bench] cpu baseline (oracle)", flush=True)
        cpu = cpu_baseline(w, args.cpu_sample, args.cpu_sample_iters)

    plain = seq.get("plain_f64")
    out = {
        "metric": METRIC,
        "value": head["particle_iters_per_s"],
        "unit": "particle-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if legs[0] == "plain_f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"lava-like channel {args.n}^3 jittered fluid + 3 wall layers (dummy, bottom and "
                               f"sides), periodic x, nu = 1e4 exp(-0.02 T) over a smooth T field in [1000, 1200], "
                               f"harmonic mean, dt*nu_max/dp^2=50; sequence of implicit steps from rest "
                               f"V_k = A^-1 (V_(k-1) + f), each step: rhs, neighbour build, operator build, "
                               f"{legs[0].replace('_', ' ')} start, robust BiCGSTAB to 1e-6"
                               + ("" if legs[0] == "plain_f64" else ", f32 operator and Krylov vectors, "
                                  "f64 scalars and solution"),
                   "n_particles": int(w.n), "tol": w.tol, "scalar_dtype": "f64"},
        "iterations": head["iterations"],
        "time_to_tol_ms": head["time_to_tol_ms_median"],
        "launches_per_iteration": head["launches_per_iteration"],
        "issued_iterations_executed": head["issued_iterations_executed"],
        "true_rel_res_max": head["true_rel_res_max"],
        "roofline": roofline,
        "sequence": seq,
        "speedup_vs_plain_f64": (round(plain["ms_per_step"] / head["ms_per_step"], 3) if plain else None),
        "speedup_vs_plain_f32op": (round(seq["plain_f32op"]["ms_per_step"] / head["ms_per_step"], 3)
                                   if "plain_f32op" in seq and legs[0] != "plain_f32op" else None),
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
