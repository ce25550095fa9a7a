"""Training and use of the learned initial guess.

Every computation runs in the HIP library through the C ABI: the FP64 solves
that produce the targets (sph_visc_solve), the samples (sph_mlp_samples), the
BF16-MFMA training steps (sph_mlp_train_step) and the start inside the solve
(opts.warm_params).  PyTorch only holds device memory and draws the batch
indices.

The network and its samples are defined in include/sph.h: one sample per
fluid particle and velocity component, features (u/U, d/U, log10 nu,
log10(dt nu / h^2)) with d = (u - A u)/A_rr, output o with start
U (o . (b, u, d)/U).  The
learned start is not part of the paper, which names better initial guesses
as future work (Sections "Conclusions and future work" and "Implementation
notes").
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Callable, Iterable, Optional

import numpy as np

from . import sph as S
from . import workloads as W

NPARAM = S.SPH_MLP_NPARAM
SAMPLE = S.SPH_MLP_SAMPLE
LAYERS = [(4, 64), (64, 64), (64, 64), (64, 3)]  # (in, out), each W [in][out] then b [out]

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "warm_mlp.npy")


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases, last layer scaled by 0.1 so the first
    starts are small; the flat layout of include/sph.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (fi, fo) in enumerate(LAYERS):
        lim = math.sqrt(6.0 / fi) * (0.1 if k == len(LAYERS) - 1 else 1.0)
        parts.append(rng.uniform(-lim, lim, size=fi * fo))
        parts.append(np.zeros(fo))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == NPARAM
    return p


def save(path: str, params, meta: dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.save(path, np.asarray(params, dtype=np.float32))
    with open(os.path.splitext(path)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1, sort_keys=True)


def load(path: str = DEFAULT_WEIGHTS) -> np.ndarray:
    p = np.load(path, allow_pickle=False)
    if p.dtype != np.float32 or p.shape != (NPARAM,):
        raise ValueError(f"{path}: expected {NPARAM} float32 parameters")
    return p


class Resident:
    """One workload resident on the device: particles, neighbour lists, and
    u and b in each precision used (copied once, so solves start from data
    already in HBM)."""

    def __init__(self, ctx: S.Context, w: W.Workload):
        self.ctx, self.w = ctx, w
        self.parts = S.device_particles(w)
        self.nb = ctx.sph_build_neighbors(self.parts, S.make_domain(w.lo, w.hi, w.periodic, w.h))
        self.u = w.x0 if w.x0 is not None else w.rhs
        self.params = S.make_params(w.dt, w.wall, w.avg, True, S.SPH_OP_CACHED)
        self._dev = {}

    def vectors(self, prec: int):
        """(b, u, x) device vectors of the precision; x is the solution buffer."""
        import torch
        if prec not in self._dev:
            b = S.device_vec3(self.w.rhs, prec)
            u = S.device_vec3(self.u, prec)
            self._dev[prec] = (b, u, [torch.empty_like(t) for t in u])
        return self._dev[prec]

    def solve(self, prec: int, tol: float, from_u: bool = True, warm_params=None,
              max_iter: int = 10000):
        """Solve A V = b from x0 = u (from_u) or zero; warm_params: cuda
        tensor or None.  Returns (x, report); x is overwritten by the next
        solve of the same precision."""
        import torch
        b, u, x = self.vectors(prec)
        for xc, uc in zip(x, u):
            if from_u:
                xc.copy_(uc)
        # from_u: u is the initial guess, so warm_u stays null (the library
        # then takes u from x and saves one operator pass)
        o = S.make_opts(tol=tol, max_iter=max_iter, x0_given=from_u, warm_params=warm_params,
                        warm_u=None if from_u or warm_params is None else u)
        rep = self.ctx.sph_visc_solve(self.nb, None, self.parts, self.params, prec, b, x, o)
        torch.cuda.synchronize()
        return x, rep


def generate(ctx: S.Context, make: Callable[[int], W.Workload], seeds: Iterable[int],
             tol: float = 1e-8, log: Optional[Callable[[str], None]] = print):
    """Samples (cuda float32, m x 8, fluid rows only) of the workloads
    make(seed): the target of each is the FP64 solution to `tol` from the
    plain start x0 = u."""
    import torch
    chunks, info = [], []
    for k, seed in enumerate(seeds):
        t0 = time.time()
        w = make(seed)
        r = Resident(ctx, w)
        xs, rep = r.solve(S.SPH_F64, tol)
        if rep["status"] != S.SPH_OK:
            raise RuntimeError(f"training solve {seed} did not converge: {rep['state']}")
        out = torch.empty((3 * w.n, SAMPLE), dtype=torch.float32, device="cuda")
        b64, u64, _ = r.vectors(S.SPH_F64)
        U = ctx.sph_mlp_samples(r.nb, r.parts, r.params, u64, b64, xs, out)
        fl = torch.as_tensor(np.repeat(w.ptype == W.FLUID, 3), device="cuda")
        chunks.append(out[fl])
        rec = {k2: float(v) for k2, v in w.meta.items() if isinstance(v, (int, float))}
        rec.update(seed=int(seed), n=int(w.n), iters=int(rep["iters"]), U=float(U))
        info.append(rec)
        if log:
            log(f"data {k}: seed {seed} n {w.n} iters {rep['iters']} U {U:.3g} "
                f"({time.time() - t0:.1f} s)")
        del r
    return torch.cat(chunks), info


def generate_sequences(ctx: S.Context, make: Callable[[int], W.Workload], seeds: Iterable[int], steps: int,
                       tol: float = 1e-8, log: Optional[Callable[[str], None]] = print):
    """Samples (cuda float32, fluid rows only) of implicit-step sequences from
    rest, V_k = A^-1 (V_{k-1} + f) with f the first step's rhs on fluid rows:
    at step k the current velocity is u = V_{k-1}, the right-hand side
    b = V_{k-1} + f and the target the FP64 solution V_k to `tol` from the
    previous-step start."""
    import torch
    chunks, info = [], []
    for seed in seeds:
        t0 = time.time()
        w = make(seed)
        parts = S.device_particles(w)
        nb = ctx.sph_build_neighbors(parts, S.make_domain(w.lo, w.hi, w.periodic, w.h))
        params = S.make_params(w.dt, w.wall, w.avg, True, S.SPH_OP_CACHED)
        fluid = torch.as_tensor(w.ptype == W.FLUID).cuda()
        f = [torch.as_tensor(w.rhs[:, c]).cuda() for c in range(3)]
        V = [torch.zeros(w.n, dtype=torch.float64, device="cuda") for _ in range(3)]
        fl3 = torch.as_tensor(np.repeat(w.ptype == W.FLUID, 3), device="cuda")
        its = []
        for k in range(steps):
            B = [torch.where(fluid, V[c] + f[c], torch.zeros_like(f[c])) for c in range(3)]
            X = [v.clone() for v in V]
            o = S.make_opts(tol=tol, x0_given=True)
            rep = ctx.sph_visc_solve(nb, None, parts, params, S.SPH_F64, B, X, o)
            if rep["status"] != S.SPH_OK:
                raise RuntimeError(f"training sequence {seed} step {k}: {rep['state']}")
            out = torch.empty((3 * w.n, SAMPLE), dtype=torch.float32, device="cuda")
            ctx.sph_mlp_samples(nb, parts, params, V, B, X, out)
            chunks.append(out[fl3])
            its.append(int(rep["iters"]))
            V = X
        rec = {k2: float(v) for k2, v in w.meta.items() if isinstance(v, (int, float))}
        rec.update(seed=int(seed), n=int(w.n), steps=steps, iters=its)
        info.append(rec)
        if log:
            log(f"sequence {seed}: n {w.n} iters {its} ({time.time() - t0:.1f} s)")
        nb.free()
        del parts
    return torch.cat(chunks), info


def train(ctx: S.Context, samples, steps: int = 6000, batch: int = 65536, lr: float = 2e-3,
          lr_min: float = 1e-5, warmup: int = 100, seed: int = 0, params0=None,
          log_every: int = 500, log: Optional[Callable[[str], None]] = print):
    """Adam on the mean squared error of the start, relative to U; returns
    (params as a cuda tensor, [(step, loss)])."""
    import torch
    m_all = samples.shape[0]
    p0 = init_params(seed) if params0 is None else np.asarray(params0, np.float32)
    params = torch.as_tensor(p0).cuda()
    am = torch.zeros(NPARAM, dtype=torch.float32, device="cuda")
    av = torch.zeros_like(am)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    hist = []
    for step in range(1, steps + 1):
        if step <= warmup:
            rate = lr * step / warmup
        else:
            q = (step - warmup) / max(1, steps - warmup)
            rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * q))
        idx = torch.randint(0, m_all, (batch,), generator=gen, device="cuda", dtype=torch.int32)
        want = step == 1 or step % log_every == 0 or step == steps
        loss = ctx.sph_mlp_train_step(samples, idx, batch, params, am, av, step, rate, want_loss=want)
        if want:
            hist.append((step, loss))
            if log:
                log(f"train step {step} lr {rate:.2e} loss {loss:.4e}")
    return params, hist
