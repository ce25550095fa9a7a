"""The two largest configurations against the FP64 oracle, run by hand on a
machine with a GPU (minutes of oracle time on the host cores, so not a
pytest module):

  python tests/oracle_fullsize.py box    # held-out 160^3 learned-start box
  python tests/oracle_fullsize.py lava   # first step of the 320^3 channel

box: the oracle solves the whole 4,491,628-row system to 1e-12 (operator
assembled once on the neighbour pattern; restarted every 25 iterations so
that it reports progress); the GPU solves it as the benchmark does (plain
start with the FP64 operator, learned start with the FP32 operator and an
FP64 solution, both to 1e-6) and with the FP64 operator to 1e-12; printed:
the relative L2 distance of each GPU solution to the oracle's.

lava: the first implicit step of the 33,695,360-row channel from rest, as
the benchmark solves it (learned start, FP32 operator, FP64 solution, 1e-6)
and with the FP64 operator to 1e-6 and 1e-10.  The oracle evaluates the FP64
residual D^-1 B - D^-1 A X of each GPU solution over all rows with its own
neighbour lists and matrix-free operator, then solves the whole system to
1e-12 itself; printed: the residuals and the relative L2 distance of each GPU
solution to the oracle's."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import oracle as O  # noqa: E402
from paper_2206_14780_amd import sph as S  # noqa: E402
from paper_2206_14780_amd import warmstart as WS  # noqa: E402
from paper_2206_14780_amd import workloads as W  # noqa: E402

from gpu_util import GpuCase, rel_l2  # noqa: E402


def log(msg):
    print(msg, flush=True)


def gpu_solve(g, B, prec, tol, X0, warm=None):
    import torch
    o = dict(history=False, true_res_period=20, restart_drop=-1.0)
    if warm is not None:
        o["warm_params"] = torch.as_tensor(warm).cuda()
    X, rep = g.solve(B, prec, X0=X0, tol=tol, **o)
    assert rep["status"] == S.SPH_OK, rep["state"]
    rel = [float(np.sqrt(t / b)) if b > 0 else 0.0 for t, b in zip(rep["true_rr"], rep["bb"])]
    return X, rep["iters"], rel


def oracle_solve(w, X0, tol, chunk=25):
    op = O.Operator.from_workload(w, jacobi=True)
    log(f"[oracle] neighbour lists: {int(op.row_ptr[-1])} entries")
    op.assemble()
    log("[oracle] operator assembled")
    X = np.asarray(X0, dtype=np.float64)
    total = 0
    t = time.time()
    while True:
        X, rep, _ = O.solve(op, w.rhs, X0=X, tol=tol, max_iter=chunk, true_res_period=20, restart_drop=0.1)
        total += rep["iters"]
        rel = [float(np.sqrt(a / b)) if b > 0 else 0.0 for a, b in zip(rep["true_rr"], rep["bb"])]
        log(f"[oracle] {total} iterations, {time.time() - t:.0f} s, true rel res {rel}")
        if rep["status"] == 0:
            return X
        assert rep["status"] == 2, rep  # not converged yet: continue from X


def box():
    w = W.warmstart_box(160, seed=4500)
    log(f"[box] n={w.n}, {O.num_threads()} oracle threads")
    ctx = S.Context(0)
    g = GpuCase(ctx, w)
    p = WS.load()
    sols = {}
    for name, prec, tol, warm in (("plain FP64 operator, 1e-6", S.SPH_F64, 1e-6, None),
                                  ("learned start, FP32 operator + FP64 solution, 1e-6", S.SPH_MIXED, 1e-6, p),
                                  ("plain FP64 operator, 1e-12", S.SPH_F64, 1e-12, None)):
        X, its, rel = gpu_solve(g, w.rhs, prec, tol, w.x0, warm)
        sols[name] = X
        log(f"[box] GPU {name}: {its} iterations, true rel res {rel}")
    Xo = oracle_solve(w, w.x0, 1e-12)
    for name, X in sols.items():
        log(f"[box] rel L2 to the oracle (1e-12): GPU {name}: {rel_l2(X, Xo):.3e}, "
            f"largest entry {np.abs(X - Xo).max() / np.abs(Xo).max():.3e}")


def lava():
    w = W.lava_channel(320)
    log(f"[lava] n={w.n}, {O.num_threads()} oracle threads")
    ctx = S.Context(0)
    g = GpuCase(ctx, w)
    p = WS.load()
    X0 = np.zeros((w.n, 3))
    sols = {}
    for name, prec, tol, warm in (("learned start, FP32 operator + FP64 solution, 1e-6", S.SPH_MIXED, 1e-6, p),
                                  ("plain FP64 operator, 1e-6", S.SPH_F64, 1e-6, None),
                                  ("plain FP64 operator, 1e-10", S.SPH_F64, 1e-10, None)):
        X, its, rel = gpu_solve(g, w.rhs, prec, tol, X0, warm)
        sols[name] = X
        log(f"[lava] GPU {name}: {its} iterations, true rel res (GPU) {rel}")
    del g
    t = time.time()
    op = O.Operator.from_workload(w, jacobi=True)
    log(f"[oracle] neighbour lists: {int(op.row_ptr[-1])} entries in {time.time() - t:.0f} s")
    d = op.diag()
    bh = w.rhs / d[:, None]
    bb = (bh * bh).sum(axis=0)
    for name, X in sols.items():
        t = time.time()
        r = bh - op.apply(X)
        rel = np.sqrt((r * r).sum(axis=0) / np.where(bb > 0, bb, 1.0))
        log(f"[lava] oracle residual of GPU {name}: relative {rel.tolist()} ({time.time() - t:.0f} s)")
    del op
    Xo = oracle_solve(w, X0, 1e-12)
    for name, X in sols.items():
        log(f"[lava] rel L2 to the oracle (1e-12): GPU {name}: {rel_l2(X, Xo):.3e}, "
            f"largest entry {np.abs(X - Xo).max() / np.abs(Xo).max():.3e}")


if __name__ == "__main__":
    {"box": box, "lava": lava}[sys.argv[1]]()
