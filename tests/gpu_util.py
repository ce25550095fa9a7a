"""Helpers of the GPU parity tests: run one workload through the HIP library
(C ABI via the binding) and through the oracle on the same seeded inputs."""
import numpy as np

import oracle as O
from paper_2206_14780_amd import sph as S
from paper_2206_14780_amd import workloads as W

F32_U = 2.0 ** -24
F64_U = 2.0 ** -53


def to_np(ts):
    return np.stack([t.detach().double().cpu().numpy() for t in ts], axis=1)


def domain_of(w):
    return S.make_domain(w.lo, w.hi, w.periodic, w.h, getattr(w, "kernel", S.SPH_KERNEL_WENDLAND))


class GpuCase:
    """A workload resident on the GPU with its neighbour handle."""

    def __init__(self, ctx, w):
        self.ctx, self.w = ctx, w
        self.parts = S.device_particles(w)
        self.dom = domain_of(w)
        self.nb = ctx.sph_build_neighbors(self.parts, self.dom)

    def export(self):
        rp, cols = self.ctx.sph_neighbors_export(self.nb)
        return rp.cpu().numpy(), cols.cpu().numpy()

    def apply(self, X, prec, jacobi=True, op_mode=S.SPH_OP_CACHED, wall=None, avg=None, dt=None):
        import torch
        w = self.w
        par = S.make_params(w.dt if dt is None else dt, w.wall if wall is None else wall,
                            w.avg if avg is None else avg, jacobi, op_mode)
        xs = S.device_vec3(X, prec)
        ys = [torch.empty_like(t) for t in xs]
        self.ctx.sph_visc_apply(self.nb, self.parts, par, prec, xs, ys)
        torch.cuda.synchronize()
        return to_np(ys)

    def solve(self, B, prec, X0=None, tol=None, op_mode=S.SPH_OP_CACHED, jacobi=True, history=True,
              **opt):
        import torch
        w = self.w
        par = S.make_params(w.dt, w.wall, w.avg, jacobi, op_mode)
        rhs = S.device_vec3(B, prec)
        xs = S.device_vec3(np.zeros((w.n, 3)) if X0 is None else X0, prec)
        # default: the oracle's policy (check every 50 iterations; FP64 never
        # restarts on a drop, FP32 vectors restart after a 1e-6 drop)
        opt.setdefault("true_res_period", 50)
        opt.setdefault("restart_drop", 0.0 if prec == S.SPH_F64 else 1e-6)
        o = S.make_opts(tol=w.tol if tol is None else tol, x0_given=X0 is not None, **opt)
        rep = self.ctx.sph_visc_solve(self.nb, None, self.parts, par, prec, rhs, xs, o,
                                      history_cap=(o.max_iter + 1) if history else 0)
        torch.cuda.synchronize()
        return to_np(xs), rep


def oracle_op(w, jacobi=True, nbr=None, **over):
    return O.Operator.from_workload(w, jacobi=jacobi, nbr=nbr, **over)


def apply_bound(op_unscaled_diag, X, u, jacobi, wall_rows_bound=2.0, k=130):
    """Elementwise bound of |A x (GPU) - A x (exact)|: the sum over at most k
    terms rounds with error <= (k + 2) u sum |terms|, and sum |terms| <=
    (2 D_b - 1) |x|_inf for an unscaled fluid row (A.1 = 1 with a positive
    diagonal D_b and non-positive off-diagonals), <= 3 |x|_inf after Jacobi
    scaling, and <= 2 |x|_inf on wall rows."""
    xm = np.abs(X).max()
    D = op_unscaled_diag
    if jacobi:
        s = np.full_like(D, 3.0)
    else:
        s = 2.0 * D - 1.0
    s = np.maximum(s, wall_rows_bound)
    return (k + 2) * u * s * xm + 1e-300


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_tank(seed=7, n=(6, 6, 5), wall=W.WALL_DUMMY, avg=W.AVG_HARMONIC, mu_span=1000.0,
               dt_nu=50.0, jitter=0.2, tol=1e-6):
    """Jittered block in a periodic x-y channel between 3-layer walls;
    log-uniform viscosity over mu_span.  n = (6, 6, 5) gives N = 396 (a
    ragged 6 x 64 + 12)."""
    rng = np.random.default_rng(seed)
    pos, pt = W.lattice(n, 1.0, walls=((False, False), (False, False), (True, True)),
                        jitter=jitter, rng=rng)
    N = pos.shape[0]
    mu = 10.0 ** rng.uniform(0.0, np.log10(mu_span), N)
    rho = rng.uniform(0.95, 1.05, N)
    mass = rho * rng.uniform(0.97, 1.03, N)
    perm = rng.permutation(N)
    pos, pt, mu, rho, mass = pos[perm], pt[perm], mu[perm], rho[perm], mass[perm]
    lo = np.array([0.0, 0.0, -3.0])
    hi = np.array([float(n[0]), float(n[1]), n[2] + 3.0])
    B = rng.normal(size=(N, 3))
    B[pt == W.WALL] = 0.0
    return W.Workload(f"tank{n}", pos, mass, rho, mu, pt, lo, hi, np.array([1, 1, 0]), 1.3,
                      dt_nu / mu.max(), wall, avg, B, None, tol)
