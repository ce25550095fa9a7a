"""Single-precision BiCGSTAB (TEST INFRASTRUCTURE ONLY: used by the test
suite; the product path never imports it).

The paper's all-FP32 solver (Section "Restructuring the stabilized
biconjugate gradient method", appendix "Implementation notes"): vectors,
operator results and every scalar in FP32, inner products compensated.  Plain
numpy float32 arrays.  Two forms of the inner products:
  dots="kahan"  the paper's: every product rounded to FP32, the products
                added in index order by Kahan's compensated FP32 summation
                (`oracle.kahan_dot_f32`);
  dots="f64"    the FP64 sum of the FP32 operands' exact products, rounded
                once to FP32: more accurate than the paper's arithmetic where
                the products cancel (it keeps their low bits), the form of
                the library's fp32_scalars = 1.
The operator is the oracle's FP64 operator applied to the FP32 vector and
rounded once to FP32 (coefficients evaluated in FP64, as in the library).
Robust and textbook variants, three systems sharing the matrix, the
three-state stopping rule and tau^2 = max(eps^2 b.b, FLT_MIN), as
`orc_bicgstab`, without true-residual restarts (the paper's iteration).  The
rotated CG (Section "Restructuring the Conjugate Gradient") likewise, as
`orc_cg`: Jacobi-weighted products <u, v>_D = sum D_i u_i v_i (the FP64
diagonal times the FP32 products, summed in FP64, rounded once), wall rows
started at their exact value.
"""
from __future__ import annotations

import numpy as np

from . import CONVERGED, FLUID_TYPE, PROGRESSING, ROBUST, STALLED, Operator, kahan_dot_f32

F32 = np.float32
FLT_MIN = F32(np.finfo(np.float32).tiny)
WALL_DYNAMIC = 0


_DOTS = ("f64", "kahan")


def _dot(a, b, dots="f64"):
    """Per-component inner products (3,) of (n, 3) FP32 arrays."""
    if dots == "kahan":
        return np.array([kahan_dot_f32(a[:, c], b[:, c]) for c in range(a.shape[1])], dtype=F32)
    return (a.astype(np.float64) * b.astype(np.float64)).sum(axis=0).astype(F32)


def _div(a, b):
    """Componentwise a / b in FP32, 0 where b is 0 or the quotient is not finite."""
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        q = np.where(b != 0, a / np.where(b != 0, b, F32(1)), F32(0)).astype(F32)
    return np.where(np.isfinite(q), q, F32(0)).astype(F32)


def _dot_w(D, a, b, dots="f64"):
    """Per-component <a, b>_D (D None: Euclidean): the FP64 sum rounded once,
    or (kahan) the compensated FP32 sum of the FP32 products (D a) b with D
    rounded to FP32."""
    if D is None:
        return _dot(a, b, dots)
    if dots == "kahan":
        Df = np.asarray(D, dtype=F32)
        return np.array([kahan_dot_f32(a[:, c], b[:, c], Df) for c in range(a.shape[1])], dtype=F32)
    return (D[:, None] * a.astype(np.float64) * b.astype(np.float64)).sum(axis=0).astype(F32)


def _rhs(op: Operator, B):
    b = np.asarray(B, dtype=np.float64)
    return b / op.diag()[:, None] if op.jacobi else b


def solve(op: Operator, B, tol=2.0 ** -23, max_iter=2000, variant=ROBUST, force_stall=None, dots="f64"):
    """A V = B (three columns) in single precision.  Returns (X (n, 3) FP32,
    report dict with iters, state, stall_count, rr, tau2, and history
    (iters + 1, 3) of r.r).  dots: "f64" or "kahan" (see the module)."""
    if dots not in _DOTS:
        raise ValueError(dots)

    def dot(a, b):
        return _dot(a, b, dots)

    def A(v):
        return op.apply(v.astype(np.float64)).astype(F32)

    b = _rhs(op, B).astype(F32)
    x = np.zeros_like(b)
    r = b.copy()
    rh = r.copy()
    bb = dot(b, b)
    tau2 = np.maximum((F32(tol) * F32(tol)) * bb, FLT_MIN).astype(F32)
    rr = dot(r, r)
    gam = dot(rh, r)
    p = np.zeros_like(b)
    Ap = np.zeros_like(b)
    alphap = np.zeros(3, F32)
    beta = np.zeros(3, F32)
    gprev = np.ones(3, F32)
    alpha = np.ones(3, F32)
    omega = np.ones(3, F32)
    state = np.where(rr < tau2, CONVERGED, PROGRESSING)
    stalls = np.zeros(3, np.int64)
    hist = [rr.copy()]
    it = 0
    fi, fc = force_stall if force_stall is not None else (-1, -1)
    while np.any(state == PROGRESSING) and it < max_iter:
        it += 1
        stall = np.zeros(3, bool)
        if variant == ROBUST:
            # p = (r + beta p) - alpha' A p, each operation rounded to FP32
            p = ((r + beta * p) - alphap * Ap).astype(F32)
        else:
            g = dot(rh, r)
            bt = (_div(g, gprev) * _div(alpha, omega)).astype(F32)
            bt = np.where((gprev != 0) & (omega != 0), bt, F32(0)).astype(F32)
            stall |= g == 0
            gam = g
            beta = bt
            p = (r + bt * (p - omega * Ap)).astype(F32)
        Ap = A(p)
        delta = dot(rh, Ap)
        if it == fi:
            delta[fc] = F32(0)
        alpha = _div(gam, delta)
        stall |= (alpha == 0) | (delta == 0)
        s = (r - alpha * Ap).astype(F32)
        As = A(s)
        tt = dot(As, As)
        ts = dot(As, s)
        w = _div(ts, tt)
        stall |= w == 0
        if variant != ROBUST:
            w = np.where(dot(s, s) < tau2, F32(0), w).astype(F32)
        omega = w
        x = (x + alpha * p + w * s).astype(F32)
        r = (s - w * As).astype(F32)
        if variant == ROBUST:
            g = dot(rh, r)
            ap = np.where(stall, F32(0), _div(g, delta)).astype(F32)
            bt = np.where(stall, F32(0), _div(ap, omega)).astype(F32)
            stall |= g == 0
            gam, alphap, beta = g, ap, bt
        else:
            gprev = gam
        rr = dot(r, r)
        stalls += stall
        state = np.where(rr < tau2, CONVERGED, np.where(stall, STALLED, PROGRESSING))
        hist.append(rr.copy())
    rep = dict(iters=it, state=[int(v) for v in state], stall_count=[int(v) for v in stalls],
               rr=[float(v) for v in rr], tau2=[float(v) for v in tau2], bb=[float(v) for v in bb])
    return x, rep, np.array(hist)


def cg_solve(op: Operator, B, tol=2.0 ** -23, max_iter=2000, force_stall=None, dots="f64"):
    """Rotated CG for the symmetric case (dynamic walls) in single precision.
    Returns (X (n, 3) FP32, report dict as `solve`, history of r.r)."""
    if op.wall != WALL_DYNAMIC:
        raise ValueError("CG needs a symmetric system: dynamic walls")
    if dots not in _DOTS:
        raise ValueError(dots)

    def dot(a, b):
        return _dot(a, b, dots)

    def dot_w(D, a, b):
        return _dot_w(D, a, b, dots)

    def A(v):
        return op.apply(v.astype(np.float64)).astype(F32)

    b64 = _rhs(op, B)
    b = b64.astype(F32)
    D = op.diag() if op.jacobi else None
    x = np.zeros_like(b)
    walls = op._type != FLUID_TYPE
    x[walls] = b[walls]
    # the starting residual in FP64 from the FP32 start, rounded once
    r = (b64 - op.apply(x.astype(np.float64))).astype(F32)
    bb = dot(b, b)
    tau2 = np.maximum((F32(tol) * F32(tol)) * bb, FLT_MIN).astype(F32)
    rr = dot(r, r)
    rho = dot_w(D, r, r)
    beta = np.zeros(3, F32)
    p = np.zeros_like(b)
    state = np.where(rr < tau2, CONVERGED, PROGRESSING)
    stalls = np.zeros(3, np.int64)
    hist = [rr.copy()]
    it = 0
    fi, fc = force_stall if force_stall is not None else (-1, -1)
    while np.any(state == PROGRESSING) and it < max_iter:
        it += 1
        p = (r + beta * p).astype(F32)
        Ap = A(p)
        pap = dot_w(D, p, Ap)
        if it == fi:
            pap[fc] = F32(0)
        alpha = _div(rho, pap)
        stall = alpha == 0
        x = (x + alpha * p).astype(F32)
        r = (r - alpha * Ap).astype(F32)
        rho_new = dot_w(D, r, r)
        beta = np.where(stall, F32(0), _div(rho_new, rho)).astype(F32)
        rho = rho_new
        rr = dot(r, r)
        stalls += stall
        state = np.where(rr < tau2, CONVERGED, np.where(stall, STALLED, PROGRESSING))
        hist.append(rr.copy())
    rep = dict(iters=it, state=[int(v) for v in state], stall_count=[int(v) for v in stalls],
               rr=[float(v) for v in rr], tau2=[float(v) for v in tau2], bb=[float(v) for v in bb])
    return x, rep, np.array(hist)
