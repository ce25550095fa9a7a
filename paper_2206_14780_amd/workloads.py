"""Seeded synthetic particle fields for the implicit viscous solve.

This module only *lays out inputs*: particle lattices, jitter, wall layers,
per-particle viscosity fields and right-hand sides.  It contains none of the
solver's or the operator's arithmetic, so both the HIP library and the CPU
oracle can take their inputs from here without sharing any method code.

The geometries stand in for the paper's analytic test cases (plane Poiseuille
flow, Section "Test case: the plane Poiseuille flow"); there is no public data
set behind them.  Every array is float64 except the particle type (uint8,
0 = fluid, 1 = wall).  Velocities and right-hand sides are (N, 3) arrays in
the original (generator) particle order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

FLUID = 0
WALL = 1

WALL_DYNAMIC = 0
WALL_DUMMY = 1

AVG_ARITH = 0
AVG_HARMONIC = 1
KERNEL_WENDLAND = 0
KERNEL_GAUSSIAN = 1


@dataclass
class Workload:
    """One linear system A(dt) V = B of the semi-implicit viscous step.

    pos     (N,3) positions; mass, rho, mu (N,) mass, density, dynamic viscosity
    ptype   (N,) uint8, 0 fluid / 1 wall
    lo, hi  (3,) domain box; periodic (3,) int flags (period = hi - lo)
    h       smoothing length (support radius 2h, Wendland kernel)
    dt      time step of the viscous system
    wall    WALL_DYNAMIC or WALL_DUMMY; avg AVG_ARITH or AVG_HARMONIC
    rhs     (N,3) right-hand side B; x0 (N,3) initial guess or None (zero)
    tol     relative residual tolerance of the solve
    """

    name: str
    pos: np.ndarray
    mass: np.ndarray
    rho: np.ndarray
    mu: np.ndarray
    ptype: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    periodic: np.ndarray
    h: float
    dt: float
    wall: int
    avg: int
    rhs: np.ndarray
    x0: Optional[np.ndarray]
    tol: float
    meta: dict = field(default_factory=dict)
    kernel: int = 0  # KERNEL_WENDLAND (support 2h) or KERNEL_GAUSSIAN (support 3h)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def period(self) -> np.ndarray:
        """Per-axis period (0 on non-periodic axes)."""
        return np.where(self.periodic != 0, self.hi - self.lo, 0.0)


def lattice(n, dp, origin=(0.0, 0.0, 0.0), walls=((False, False),) * 3, layers=3,
            jitter=0.0, rng=None):
    """Cubic lattice of n[0] x n[1] x n[2] fluid sites plus `layers` wall layers.

    Site (i, j, k) sits at origin + (idx + 1/2) dp.  walls[a] = (low, high) adds
    `layers` wall layers below index 0 / above index n[a]-1 on axis a.  Fluid
    sites are jittered by U(-jitter, jitter) dp per coordinate; walls are not.
    Returns (pos (N,3), ptype (N,)).
    """
    ranges = []
    for a in range(3):
        lo_i = -layers if walls[a][0] else 0
        hi_i = n[a] + layers if walls[a][1] else n[a]
        ranges.append(np.arange(lo_i, hi_i, dtype=np.int64))
    kk, jj, ii = np.meshgrid(ranges[2], ranges[1], ranges[0], indexing="ij")
    idx = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    is_fluid = np.all((idx >= 0) & (idx < np.asarray(n)[None, :]), axis=1)
    pos = np.asarray(origin, dtype=np.float64)[None, :] + (idx.astype(np.float64) + 0.5) * dp
    if jitter > 0.0:
        nf = int(is_fluid.sum())
        pos[is_fluid] += rng.uniform(-jitter * dp, jitter * dp, size=(nf, 3))
    ptype = np.where(is_fluid, FLUID, WALL).astype(np.uint8)
    return pos, ptype


def smooth_field(pos, length, rng, n_modes=16, chunk=1 << 21):
    """Sum of `n_modes` random plane waves (wavelength in [length/4, length],
    random direction, phase and amplitude), min-max normalised to [0, 1]."""
    dirs = rng.normal(size=(n_modes, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    lam = rng.uniform(length / 4.0, length, size=n_modes)
    kvec = dirs * (2.0 * math.pi / lam)[:, None]
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    amp = rng.uniform(0.5, 1.0, size=n_modes)
    out = np.empty(pos.shape[0], dtype=np.float64)
    # the plane-wave sum in FP64 on the CPU; torch's elementwise cos runs on
    # all host cores (numpy's on one)
    import torch
    kt, pt_, at = (torch.from_numpy(np.ascontiguousarray(a)) for a in (kvec.T, phase, amp))
    for s in range(0, pos.shape[0], chunk):
        p = torch.from_numpy(np.ascontiguousarray(pos[s:s + chunk]))
        out[s:s + chunk] = (torch.cos(p @ kt + pt_[None, :]) @ at).numpy()
    lo, hi = out.min(), out.max()
    return (out - lo) / (hi - lo) if hi > lo else np.zeros_like(out)


def _shuffle(rng, *arrays):
    perm = rng.permutation(arrays[0].shape[0])
    return [a[perm] for a in arrays]


def poiseuille(n=16, wall=WALL_DYNAMIC, dt_nu_dp2=10.0, nu=1.0, g=1.0, tol=1e-8,
               shuffle_seed=None):
    """Periodic plane channel (plane Poiseuille flow, Section "Domain
    discretization"): n x n x n fluid sites of spacing dp = 1/n between walls
    at z = -1/2 and z = +1/2, three wall layers on each side, periodic in x and
    y with period 1.  Fluid at z = -1/2 + (k + 1/2) dp, walls at
    +-(1/2 + (j + 1/2) dp).  rho = 1, m = rho dp^3, mu = nu rho,
    dt = dt_nu_dp2 dp^2 / nu, rhs = u0 + dt g with u0 = 0, g = (g, 0, 0) on
    fluid rows and 0 (zero wall velocity) on wall rows; x0 = 0.
    """
    dp = 1.0 / n
    pos, ptype = lattice((n, n, n), dp, origin=(0.0, 0.0, -0.5),
                         walls=((False, False), (False, False), (True, True)))
    N = pos.shape[0]
    rho = np.ones(N)
    mass = rho * dp ** 3
    mu = nu * rho
    dt = dt_nu_dp2 * dp * dp / nu
    rhs = np.zeros((N, 3))
    rhs[ptype == FLUID, 0] = dt * g
    if shuffle_seed is not None:
        pos, ptype, rhs = _shuffle(np.random.default_rng(shuffle_seed), pos, ptype, rhs)
    lo = np.array([0.0, 0.0, -0.5 - 3 * dp])
    hi = np.array([1.0, 1.0, 0.5 + 3 * dp])
    return Workload(f"poiseuille{n}_{'dyn' if wall == WALL_DYNAMIC else 'dummy'}", pos, mass,
                    rho, mu, ptype, lo, hi, np.array([1, 1, 0]), 1.3 * dp, dt, wall,
                    AVG_ARITH, rhs, None, tol,
                    meta=dict(dp=dp, nu=nu, g=g, L=1.0))


def open_box(n=100, seed=2, nu=10.0, dt_nu_dp2=50.0, sigma_u=0.1, wall=WALL_DUMMY, tol=1e-6,
             jitter=0.1):
    """Open-top tank: n^3 fluid sites (dp = 1) jittered by U(-0.1, 0.1) dp,
    three wall layers on the four sides and the bottom, no lid.  Constant
    nu (rho = 1), dt = dt_nu_dp2 / nu, u0 ~ N(0, sigma_u^2) per component on
    fluid rows; rhs = u0 (fluid), 0 (walls); x0 = rhs (previous-step start).
    n = 100 gives N = 1,157,308."""
    rng = np.random.default_rng(seed)
    pos, ptype = lattice((n, n, n), 1.0, walls=((True, True), (True, True), (True, False)),
                         jitter=jitter, rng=rng)
    N = pos.shape[0]
    rho = np.ones(N)
    mass = rho.copy()
    mu = nu * rho
    dt = dt_nu_dp2 / nu
    rhs = np.zeros((N, 3))
    fl = ptype == FLUID
    rhs[fl] = rng.normal(0.0, sigma_u, size=(int(fl.sum()), 3))
    pos, ptype, rhs = _shuffle(rng, pos, ptype, rhs)
    lo = np.array([-3.0, -3.0, -3.0])
    hi = np.array([n + 3.0, n + 3.0, float(n)])
    return Workload(f"open_box{n}", pos, mass, rho, mu, ptype, lo, hi, np.array([0, 0, 0]),
                    1.3, dt, wall, AVG_ARITH, rhs, rhs.copy(), tol,
                    meta=dict(dp=1.0, nu=nu, seed=seed))


def papanastasiou_mu(D, tau0, m, mu0):
    """Regularised Bingham viscosity (eq. papa), evaluated in float64 as
    tau0 * (-expm1(-m D)) / D + mu0 with the D -> 0 limit m tau0 + mu0.
    An input recipe for the viscosity field, not part of the solve."""
    D = np.asarray(D, dtype=np.float64)
    safe = np.where(D > 0.0, D, 1.0)
    y = np.where(D > 0.0, -np.expm1(-m * safe) / safe, m)
    return tau0 * y + mu0


def incline_papanastasiou(n=160, seed=3, tau0=100.0, m=1000.0, mu0=1.0, slope_deg=10.0,
                          dt_numax_dp2=50.0, wall=WALL_DUMMY, tol=1e-6, jitter=0.1):
    """Non-Newtonian layer on an inclined plane: n^3 jittered fluid sites
    (dp = 1), periodic in x and y (period n), three bottom wall layers, open
    top.  The viscosity is the Papanastasiou law of a smooth seeded shear-rate
    field D in [0, 1] (so mu spans [tau0(1-e^-m)+mu0, m tau0 + mu0]), walls
    take the field at their own position; harmonic pairwise average;
    dt = dt_numax_dp2 / mu_max; rhs = dt (sin slope, 0, 0) on fluid rows."""
    rng = np.random.default_rng(seed)
    pos, ptype = lattice((n, n, n), 1.0, walls=((False, False), (False, False), (True, False)),
                         jitter=jitter, rng=rng)
    N = pos.shape[0]
    D = smooth_field(pos, float(n), rng)
    mu = papanastasiou_mu(D, tau0, m, mu0)
    rho = np.ones(N)
    mass = rho.copy()
    mu_max = m * tau0 + mu0
    dt = dt_numax_dp2 / mu_max
    rhs = np.zeros((N, 3))
    rhs[ptype == FLUID, 0] = dt * math.sin(math.radians(slope_deg))
    pos, ptype, rhs, mu = _shuffle(rng, pos, ptype, rhs, mu)
    lo = np.array([0.0, 0.0, -3.0])
    hi = np.array([float(n), float(n), float(n)])
    return Workload(f"incline_papa{n}", pos, mass, rho, mu, ptype, lo, hi,
                    np.array([1, 1, 0]), 1.3, dt, wall, AVG_HARMONIC, rhs, None, tol,
                    meta=dict(dp=1.0, seed=seed, mu_min=float(mu.min()), mu_max=float(mu.max())))


def warmstart_box(n=64, seed=4000, wall=WALL_DUMMY, tol=1e-6, jitter=0.1):
    """Open-top tank for the learned initial guess: constant nu drawn
    log-uniform in [1, 1e3], dt nu / dp^2 uniform in [10, 200], current
    velocity u = smooth vector field (each component scaled to [-1, 1]) plus
    N(0, 0.1^2) noise on fluid rows; rhs = u (fluid), 0 (walls); x0 = rhs.
    n = 64 gives N = 328,300 and n = 160 gives N = 4,491,628."""
    rng = np.random.default_rng(seed)
    pos, ptype = lattice((n, n, n), 1.0, walls=((True, True), (True, True), (True, False)),
                         jitter=jitter, rng=rng)
    N = pos.shape[0]
    nu = float(10.0 ** rng.uniform(0.0, 3.0))
    dtnu = float(rng.uniform(10.0, 200.0))
    dt = dtnu / nu
    fl = ptype == FLUID
    u = np.zeros((N, 3))
    for c in range(3):
        u[:, c] = 2.0 * smooth_field(pos, float(n), rng) - 1.0
    u[fl] += rng.normal(0.0, 0.1, size=(int(fl.sum()), 3))
    u[~fl] = 0.0
    rho = np.ones(N)
    pos, ptype, u = _shuffle(rng, pos, ptype, u)
    lo = np.array([-3.0, -3.0, -3.0])
    hi = np.array([n + 3.0, n + 3.0, float(n)])
    return Workload(f"warmstart_box{n}_s{seed}", pos, rho.copy(), rho, nu * rho, ptype, lo, hi,
                    np.array([0, 0, 0]), 1.3, dt, wall, AVG_ARITH, u, u.copy(), tol,
                    meta=dict(dp=1.0, seed=seed, nu=nu, dt_nu_dp2=dtnu))


def lava_channel(n=320, seed=5, nu0=1e4, b=0.02, T_lo=1000.0, T_hi=1200.0,
                 dt_numax_dp2=50.0, wall=WALL_DUMMY, tol=1e-6, jitter=0.1):
    """Lava-like channel: n^3 jittered fluid sites (dp = 1), periodic in x,
    three wall layers at the bottom and both y sides, open top; temperature
    T = smooth field scaled to [T_lo, T_hi]; nu = nu0 exp(-b T); harmonic
    average; dt = dt_numax_dp2 / nu_max; rhs of the first step = u0 +
    (sin 10 deg, 0, 0) with u0 = 0.  n = 320 gives N = 33,695,360."""
    rng = np.random.default_rng(seed)
    pos, ptype = lattice((n, n, n), 1.0, walls=((False, False), (True, True), (True, False)),
                         jitter=jitter, rng=rng)
    N = pos.shape[0]
    T = T_lo + (T_hi - T_lo) * smooth_field(pos, float(n), rng)
    nu = nu0 * np.exp(-b * T)
    nu_max = nu0 * math.exp(-b * T_lo)
    rho = np.ones(N)
    dt = dt_numax_dp2 / nu_max
    rhs = np.zeros((N, 3))
    rhs[ptype == FLUID, 0] = math.sin(math.radians(10.0))
    lo = np.array([0.0, -3.0, -3.0])
    hi = np.array([float(n), n + 3.0, float(n)])
    return Workload(f"lava_channel{n}", pos, rho.copy(), rho, nu * rho, ptype, lo, hi,
                    np.array([1, 0, 0]), 1.3, dt, wall, AVG_HARMONIC, rhs, None, tol,
                    meta=dict(dp=1.0, seed=seed))


def training_channel(n=64, seed=6000, tol=1e-8):
    """A lava-like channel of the learned start's training set: the generator
    of `lava_channel` at n^3 fluid sites with parameters drawn from the seed:
    temperature span T_hi - T_lo uniform in [50, 250] (viscosity contrast
    e^1 .. e^5 at b = 0.02) and dt nu_max / dp^2 log-uniform in [5, 200]."""
    rng = np.random.default_rng(seed)
    span = float(rng.uniform(50.0, 250.0))
    stiff = float(np.exp(rng.uniform(np.log(5.0), np.log(200.0))))
    w = lava_channel(n, seed=seed, T_lo=1000.0, T_hi=1000.0 + span, dt_numax_dp2=stiff, tol=tol)
    w.name = f"training_channel{n}_s{seed}"
    w.meta.update(T_span=span, dt_numax_dp2=stiff)
    return w


def next_step_rhs(w: Workload, V) -> np.ndarray:
    """Right-hand side of the next implicit step of a sequence started from
    rest, V_k = A^-1 (V_{k-1} + f): the previous solution plus the per-step
    forcing f = the first step's rhs (taken with V_0 = 0) on fluid rows, 0 on
    wall rows."""
    fl = (w.ptype == FLUID)[:, None]
    return np.where(fl, np.asarray(V, dtype=np.float64) + w.rhs, 0.0)


def with_random_order(w: Workload, seed: int) -> Workload:
    """Same system with the particles listed in a seeded random order."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(w.n)
    return Workload(w.name + f"_perm{seed}", w.pos[perm], w.mass[perm], w.rho[perm], w.mu[perm],
                    w.ptype[perm], w.lo, w.hi, w.periodic, w.h, w.dt, w.wall, w.avg,
                    w.rhs[perm], None if w.x0 is None else w.x0[perm], w.tol, dict(w.meta))
