"""Full-size cases: the benchmark tank, the non-Newtonian incline, the learned
start at 4.5M particles and the 33.7M-particle lava channel, solved on the GPU
as the benchmark runs them, and compared with the FP64 oracle.

The tank (1.16M rows) and the incline (4.17M rows) are solved whole by the
oracle (its operator assembled once on the neighbour pattern, FP64, eps =
1e-12): the GPU's FP64 solve at 1e-12 must match it within 1e-10 relative L2,
the FP32 operator with an FP64 solution (SPH_MIXED) at 1e-8 within 1e-5, and
the FP32 path at the benchmark's 1e-6 is reported (its distance is set by the
tolerance, as an FP64 solve to 1e-6 shows).

For every case the oracle also evaluates 2,048 sampled rows exactly (the
cell-grid search restricted to those rows): on them the GPU's FP64 and FP32
cached operators applied to the GPU's solution agree with the oracle's rows
within the elementwise rounding bound, and so does each entry of the scaled
residual b - A x that the GPU's FP64 operator gives; the norm of that
residual over all rows meets the tolerance and equals the solver's report."""
import time

import numpy as np
import pytest

import oracle as O
from paper_2206_14780_amd import sph as S
from paper_2206_14780_amd import warmstart as WS
from paper_2206_14780_amd import workloads as W
from oracle import mlp as OM
from oracle import warmstart as OW

from gpu_util import F32_U, F64_U, GpuCase, apply_bound, rel_l2, to_np

pytestmark = pytest.mark.gpu
NSAMPLE = 2048


@pytest.fixture(scope="module")
def ctx():
    return S.Context(0)


def _rows(w, seed):
    return np.sort(np.random.default_rng(seed).choice(w.n, size=NSAMPLE, replace=False))


def _oracle_rows(w, rows, jacobi=True):
    nbr = O.neighbors_rows(w.pos, w.period, w.h, rows, lo=w.lo)
    return O.Operator.from_workload(w, jacobi=jacobi, nbr=nbr)


def _check_solution(g, w, B, X, rep, rows, tag, prec=S.SPH_F64):
    """The solve converged; on the sampled rows the GPU's FP64 and FP32
    operators and each entry of its scaled residual match the oracle; the
    residual over all rows meets the tolerance and equals the report.  An
    SPH_F32 solve takes its right-hand side in FP32, so its residual is that
    of the rounded B."""
    assert rep["status"] == S.SPH_OK, (tag, rep["state"])
    if prec == S.SPH_F32:
        B = B.astype(np.float32).astype(np.float64)
    rel = [np.sqrt(t / b) if b > 0 else 0.0 for t, b in zip(rep["true_rr"], rep["bb"])]
    print(f"[{tag}] iters {rep['iters']} true rel res {rel}", flush=True)
    assert max(rel) <= w.tol * (1.0 + 1e-9)
    op = _oracle_rows(w, rows)
    d = op.diag()[rows]
    op_u = _oracle_rows(w, rows, jacobi=False)
    du = op_u.diag()[rows]
    Yo = op.apply(X)[rows]
    Yg = g.apply(X, S.SPH_F64, jacobi=True)
    bound = apply_bound(du, X, F64_U, True)
    assert np.all(np.abs(Yg[rows] - Yo) <= bound[:, None]), tag
    # the FP32 cached operator (coefficients rounded once) on X rounded to FP32
    X32 = X.astype(np.float32).astype(np.float64)
    Yo32 = op.apply(X32)[rows]
    Yg32 = g.apply(X32, S.SPH_F32, jacobi=True)[rows]
    bound32 = apply_bound(du, X32, F32_U, True)
    assert np.all(np.abs(Yg32 - Yo32) <= bound32[:, None]), tag + " (FP32 operator)"
    # the scaled residual: 1/D is the row sum of the scaled fluid rows (A 1 = 1
    # there) and 1 on wall rows; every sampled entry against the oracle's
    dinv = g.apply(np.ones((w.n, 3)), S.SPH_F64, jacobi=True)[:, 0]
    dinv[w.ptype != W.FLUID] = 1.0
    assert np.all(np.abs(dinv[rows] * d - 1.0) <= 1e-13), tag
    rg = B * dinv[:, None] - Yg
    ro = B[rows] / d[:, None] - Yo
    rbound = bound + 2.0 * F64_U * np.abs(B[rows] / d[:, None]).max(axis=1)
    assert np.all(np.abs(rg[rows] - ro) <= rbound[:, None]), tag + " (residual entries)"
    # over all rows: the norm meets the tolerance and is the reported one
    bh = B * dinv[:, None]
    rr = (rg * rg).sum(axis=0)
    bb = (bh * bh).sum(axis=0)
    assert np.all(rr <= np.maximum(w.tol ** 2 * bb, np.asarray(rep["tau2"])) * (1.0 + 1e-6)), tag
    assert np.allclose(rr, rep["true_rr"], rtol=1e-6, atol=1e-30 * bb.max()), (tag, rr, rep["true_rr"])
    worst = np.abs(ro).max(axis=0) / np.sqrt(np.where(bb > 0, bb, 1.0))
    print(f"[{tag}] largest sampled residual entry / |b|: {worst}", flush=True)
    return rel


def _oracle_whole(w, X0=None, tol=1e-12):
    """The oracle's FP64 solution of the whole system (operator assembled once,
    restart policy of the library's default: a true-residual check every 20
    iterations and a restart after a 10x drop)."""
    op = O.Operator.from_workload(w, jacobi=True).assemble()
    t = time.time()
    X, rep, _ = O.solve(op, w.rhs, X0=X0, tol=tol, true_res_period=20, restart_drop=0.1)
    print(f"[oracle] {w.name}: {rep['iters']} iterations to {tol:g} in {time.time() - t:.1f} s "
          f"on {O.num_threads()} threads", flush=True)
    assert rep["status"] == 0
    return X


def _solve(g, B, prec, tol, X0=None):
    X, rep = g.solve(B, prec, X0=X0, tol=tol, history=False, true_res_period=20, restart_drop=-1.0)
    assert rep["status"] == S.SPH_OK
    return X


@pytest.mark.timeout(900)
def test_tank_100_against_the_whole_oracle_solution(ctx):
    # the benchmark's workload, from the previous-step start
    w = W.open_box(100)
    print(f"[tank] n={w.n}", flush=True)
    g = GpuCase(ctx, w)
    Xo = _oracle_whole(w, X0=w.x0)
    X64 = _solve(g, w.rhs, S.SPH_F64, 1e-12, w.x0)
    e64 = rel_l2(X64, Xo)
    Xm = _solve(g, w.rhs, S.SPH_MIXED, 1e-8, w.x0)
    em = rel_l2(Xm, Xo)
    X, rep = g.solve(w.rhs, S.SPH_F32, X0=w.x0, history=False, true_res_period=20, restart_drop=-1.0)
    ef = rel_l2(X, Xo)
    ef64 = rel_l2(_solve(g, w.rhs, S.SPH_F64, w.tol, w.x0), Xo)
    emax = np.abs(Xm - Xo).max() / np.abs(Xo).max()
    # the all-FP32 path (FP32 solution) solved as tight as FP32 storage of x
    # allows on this system (2^-23) meets the 1e-5 gate of the FP32 path
    X23 = _solve(g, w.rhs, S.SPH_F32, 2.0 ** -23, w.x0)
    e23 = rel_l2(X23, Xo)
    print(f"[tank] rel L2 to the oracle (eps 1e-12): FP64 at 1e-12 {e64:.2e}; FP32 operator + FP64 "
          f"solution at 1e-8 {em:.2e} (largest entry {emax:.2e}); FP32 at 2^-23 {e23:.2e}; FP32 at 1e-6 "
          f"{ef:.2e}, FP64 at 1e-6 {ef64:.2e}", flush=True)
    assert e64 < 1e-10
    assert em < 1e-5 and emax < 1e-5
    assert e23 < 1e-5
    assert ef <= 2.0 * ef64 + 1e-6
    _check_solution(g, w, w.rhs, X, rep, _rows(w, 1), "tank100 f32", S.SPH_F32)


@pytest.mark.timeout(900)
def test_incline_160_against_the_whole_oracle_solution(ctx):
    # non-Newtonian layer (Papanastasiou viscosity over 3 decades, harmonic
    # mean): FP32 operator and Krylov vectors, FP64 scalars and solution
    w = W.incline_papanastasiou(160)
    print(f"[incline] n={w.n} mu {w.meta['mu_min']:.3g}..{w.meta['mu_max']:.3g}", flush=True)
    g = GpuCase(ctx, w)
    Xo = _oracle_whole(w)
    X64 = _solve(g, w.rhs, S.SPH_F64, 1e-12)
    e64 = rel_l2(X64, Xo)
    Xm8 = _solve(g, w.rhs, S.SPH_MIXED, 1e-8)
    em8 = rel_l2(Xm8, Xo)
    X, rep = g.solve(w.rhs, S.SPH_MIXED, history=False, true_res_period=20, restart_drop=-1.0)
    em = rel_l2(X, Xo)
    ef64 = rel_l2(_solve(g, w.rhs, S.SPH_F64, w.tol), Xo)
    print(f"[incline] rel L2 to the oracle (eps 1e-12): FP64 at 1e-12 {e64:.2e}; FP32 operator + FP64 "
          f"solution at 1e-8 {em8:.2e}, at 1e-6 {em:.2e} (FP64 at 1e-6 {ef64:.2e})", flush=True)
    assert e64 < 1e-10
    assert em8 < 1e-5
    assert em <= 2.0 * ef64 + 1e-6
    _check_solution(g, w, w.rhs, X, rep, _rows(w, 2), "incline160 mixed")


def test_learned_start_160(ctx):
    # the trained network on a held-out 160^3 box: the GPU's start on the
    # sampled fluid rows against the oracle's (features from the exact rows,
    # BF16 network), then the learned FP32-operator solve
    import torch
    w = W.warmstart_box(160, seed=4500)
    print(f"[learned] n={w.n}", flush=True)
    g = GpuCase(ctx, w)
    p = WS.load()
    par = S.make_params(w.dt, w.wall, w.avg, True, S.SPH_OP_CACHED)
    x0 = S.device_vec3(np.zeros((w.n, 3)), S.SPH_F64)
    U = ctx.sph_mlp_warmstart(g.nb, g.parts, par, S.SPH_F64, S.device_vec3(w.x0, S.SPH_F64),
                              S.device_vec3(w.rhs, S.SPH_F64), torch.as_tensor(p).cuda(), x0)
    torch.cuda.synchronize()
    xg = to_np(x0)
    rows = _rows(w, 3)
    rows = rows[w.ptype[rows] == W.FLUID]
    op = _oracle_rows(w, rows, jacobi=False)
    So, Uo = OW.samples(op, w.x0, w.rhs, w.mu, w.rho, w.ptype)
    assert abs(U - Uo) <= 1e-6 * Uo
    Sr = So.reshape(w.n, 3, 8)[rows].reshape(-1, 8).astype(np.float32).astype(np.float64)
    _, pred, _ = OM.forward(p, Sr, bf=True)
    xo = Uo * pred.reshape(-1, 3)
    e = rel_l2(xg[rows], xo)
    print(f"[learned] start rel L2 on {rows.size} fluid rows {e:.3e}", flush=True)
    assert e < 1e-4
    its = {}
    for name, prec, warm in (("plain f64", S.SPH_F64, None), ("learned f64", S.SPH_F64, p),
                             ("plain mixed", S.SPH_MIXED, None), ("learned mixed", S.SPH_MIXED, p)):
        o = dict(history=False, true_res_period=20, restart_drop=-1.0)
        if warm is not None:
            o["warm_params"] = torch.as_tensor(warm).cuda()
        X, rep = g.solve(w.rhs, prec, X0=w.x0, **o)
        _check_solution(g, w, w.rhs, X, rep, rows, name)
        its[name] = rep["iters"]
        if warm is not None:
            # what the trained network gains: a start whose FP64 true
            # residual is several times smaller than the plain start's on
            # every component (measured: 0.06 of it on this machine)
            ratio = [float(np.sqrt(a / b)) for a, b in zip(rep["warm_rr"], rep["plain_rr"])]
            print(f"[learned] {name}: residual of the learned start / plain start {ratio}, "
                  f"components on the learned start {rep['warm_used']}", flush=True)
            assert all(u == 1 for u in rep["warm_used"]) and max(ratio) < 0.25
    print(f"[learned] iterations {its}", flush=True)


def test_lava_320_two_steps(ctx):
    # lava-like channel, temperature-dependent viscosity over ~50x, harmonic
    # mean: two implicit steps (V_k = A^-1 (V_{k-1} + f), V_0 = 0), the
    # second from the plain start V_1 and from the learned start
    import torch
    w = W.lava_channel(320)
    print(f"[lava] n={w.n}", flush=True)
    g = GpuCase(ctx, w)
    rows = _rows(w, 5)
    X1, rep = g.solve(w.rhs, S.SPH_MIXED, history=False, true_res_period=20, restart_drop=-1.0)
    _check_solution(g, w, w.rhs, X1, rep, rows, "lava step 1")
    B2 = W.next_step_rhs(w, X1)
    p = torch.as_tensor(WS.load()).cuda()
    for name, warm in (("lava step 2 plain", None), ("lava step 2 learned", p)):
        o = dict(history=False, true_res_period=20, restart_drop=-1.0)
        if warm is not None:
            o["warm_params"] = warm
        X2, rep = g.solve(B2, S.SPH_MIXED, X0=X1, **o)
        _check_solution(g, w, B2, X2, rep, rows, name)
        if warm is not None:
            ratio = [float(a / b) if b > 0 else None for a, b in zip(rep["warm_rr"], rep["plain_rr"])]
            print(f"[lava] components on the learned start: {rep['warm_used']}, true r.r of the learned "
                  f"start / plain start {ratio}", flush=True)
            # the network's viscosity input is relative to the system's mean,
            # so the channel's viscosities (far below the training boxes') are
            # within its range: it is kept on the driven component
            assert rep["warm_used"][0] == 1
