"""FP64 oracle of the learned initial guess: features, start, fallback.

TEST INFRASTRUCTURE ONLY (tests, smoke check).  Numpy plus the C oracle's
operator; nothing is shared with the HIP library.

The learned initial guess is not part of the paper, which names better
initial guesses as future work (Sections "Conclusions and future work" and
"Implementation notes").  Definition used here, one sample per fluid
particle k and velocity component c:

  inc   = u - A u                 (A the unscaled viscous matrix, so inc is
                                   the implicit step's viscous increment
                                   dt * (Laplacian term) of the current u)
  d     = inc / A_kk              (the increment scaled by the row's diagonal:
                                   one Jacobi correction, of the size of u
                                   however stiff the row is)
  U     = RMS of b over fluid rows and components (1 if that is 0)
  L     = mean of log10 nu over fluid rows (nu = mu / rho)
  x     = (u_c / U, d_c / U, log10 nu_k - L, log10(dt nu_k / h^2)): the
          viscosity relative to the system's geometric mean (unchanged when
          every viscosity is scaled), its magnitude through the stiffness
  B     = (b_c / U, u_c / U, d_c / U)
  t     = V_c / U                 (V the converged solution, training only)
  x0_c  = U * (o . B)             with o = MLP(x)
        = o0 b_c + o1 u_c + o2 d_c

Wall rows of the start: a dynamic wall row is the identity, so x0 = b; a
dummy wall row is satisfied exactly, x0_w = b_w - sum_a A_wa x0_a (the
Shepard average of the fluid start, Section "Boundary conditions").  The
fallback keeps, per component, whichever of the learned and the plain start
has the smaller FP64 true residual of the (Jacobi-scaled) system.
"""
from __future__ import annotations

import numpy as np

from . import Operator
from . import mlp

FLUID = 0


def samples(op: Operator, u, b, mu, rho, ptype, target=None):
    """Training / inference samples of one configuration.

    op: the UNSCALED operator (jacobi=False).  Returns (S, U) with S of shape
    (3 n, 8), sample 3 k + c for particle k and component c (all zero on
    wall rows), in FP64 (the GPU stores them rounded to FP32)."""
    if op.jacobi:
        raise ValueError("features use the unscaled operator")
    u = np.asarray(u, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = u.shape[0]
    fl = np.asarray(ptype) == FLUID
    inc = u - op.apply(u)
    d = inc / op.diag()[:, None]
    nfl = int(fl.sum())
    U = float(np.sqrt(np.sum(b[fl] ** 2) / (3.0 * nfl))) if nfl else 0.0
    if not (U > 0.0 and np.isfinite(U)):
        U = 1.0
    nu = np.broadcast_to(np.asarray(mu, np.float64), (n,)) / np.broadcast_to(np.asarray(rho, np.float64), (n,))
    S = np.zeros((n, 3, 8))
    S[:, :, 0] = u / U
    S[:, :, 1] = d / U
    L = float(np.mean(np.log10(nu[fl]))) if nfl else 0.0
    S[:, :, 2] = (np.log10(nu) - L)[:, None]
    S[:, :, 3] = np.log10(op.dt * nu / (op.h * op.h))[:, None]
    S[:, :, 4] = b / U
    S[:, :, 5] = u / U
    S[:, :, 6] = d / U
    if target is not None:
        S[:, :, 7] = np.asarray(target, dtype=np.float64) / U
    S[~fl] = 0.0
    return S.reshape(3 * n, 8), U


def learned_start(op: Operator, params, S, U, b, ptype):
    """x0 (n, 3) from the MLP (BF16 weights, as on the GPU) on the FP32
    samples S; op is the unscaled operator (its wall model decides the wall
    rows)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    fl = np.asarray(ptype) == FLUID
    S32 = np.asarray(S, dtype=np.float32).astype(np.float64)
    _, pred, _ = mlp.forward(params, S32, bf=True)
    x0 = np.zeros((n, 3))
    x0[fl] = U * pred.reshape(n, 3)[fl]
    if op.wall == 0:  # dynamic walls: identity rows
        x0[~fl] = b[~fl]
    else:  # dummy walls: satisfy the wall row given the fluid start
        y = op.apply(x0)  # wall rows: 0 + sum_a A_wa x0_a
        x0[~fl] = b[~fl] - y[~fl]
    return x0


def residual_rr(op_scaled: Operator, b, x):
    """Per-component r . r of the FP64 true residual D^-1 b - D^-1 A x (or
    b - A x without Jacobi scaling)."""
    b = np.asarray(b, dtype=np.float64)
    bh = b / op_scaled.diag()[:, None] if op_scaled.jacobi else b
    r = bh - op_scaled.apply(x)
    return np.sum(r * r, axis=0)


def select(op_scaled: Operator, b, x_plain, x_learn):
    """Per component, the start with the smaller true residual (ties go to
    the plain start).  Returns (x0, used_learned[3], rr_learned, rr_plain)."""
    rr_p = residual_rr(op_scaled, b, x_plain)
    rr_l = residual_rr(op_scaled, b, x_learn)
    use = rr_l < rr_p
    x0 = np.where(use[None, :], x_learn, x_plain)
    return x0, use, rr_l, rr_p


def fixed_blend_params(o):
    """MLP parameters whose output is the constant o (W4 = 0, b4 = o): the
    start is then the fixed blend o0 b + o1 u + o2 d."""
    p = np.zeros(mlp.NPARAM, dtype=np.float32)
    p[mlp.NPARAM - 3:] = np.asarray(o, dtype=np.float32)
    return p
