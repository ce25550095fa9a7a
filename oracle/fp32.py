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


# ---------------------------------------------------------------------------
# The paper's single-precision matrix (appendix on relative positions,
# appendix "Implementation notes"): pair weights in FP32 from FP32 positions
# relative to cell centres, the cell grid being that of the neighbour
# search (cells of side >= the support, see `cell_grid`); diagonal and
# dummy-wall normalisation as Kahan FP32 sums; the gemv with FP32 products
# summed by Kahan's compensation.
# ---------------------------------------------------------------------------

def cell_grid(lo, hi, periodic, h, support=2.0):
    """(nc, cs, period) per axis: nc = max(1, floor(L / (s (1 + 1e-9)))) cells
    of side L / nc (twice L for a single cell on a non-periodic axis), s the
    support radius; the period is L on periodic axes, else 0."""
    s = float(support) * float(h)
    target = s * (1.0 + 1e-9)
    nc = np.zeros(3, dtype=np.int64)
    cs = np.zeros(3)
    period = np.zeros(3)
    for a in range(3):
        L = float(hi[a]) - float(lo[a])
        n = max(int(np.floor(L / target)), 1)
        nc[a] = n
        cs[a] = L / n if L > 0.0 else 1.0
        if not periodic[a] and n == 1:
            cs[a] = 2.0 * L if L > 0.0 else 1.0
        period[a] = L if periodic[a] else 0.0
    return nc, cs, period


def _disp(d, period):
    return d - period * np.rint(d / period) if period > 0.0 else d


def cell_relative(pos, lo, nc, cs, period):
    """Integer cell coordinates (n, 3) (floor of (x - lo)/cs, wrapped on periodic
    axes, clamped on the others) and the FP32 offsets (n, 3) from the cell
    centres lo + (c + 1/2) cs (minimum image on periodic axes)."""
    pos = np.asarray(pos, dtype=np.float64)
    c = np.zeros(pos.shape, dtype=np.int64)
    r = np.zeros(pos.shape, dtype=F32)
    for a in range(3):
        u = np.floor((pos[:, a] - lo[a]) / cs[a]).astype(np.int64)
        u = np.mod(u, nc[a]) if period[a] > 0.0 else np.clip(u, 0, nc[a] - 1)
        c[:, a] = u
        centre = lo[a] + (u.astype(np.float64) + 0.5) * cs[a]
        r[:, a] = _disp(pos[:, a] - centre, period[a]).astype(F32)
    return c, r


class Paper32Operator:
    """The paper's single-precision matrix of one system (Wendland kernel),
    Jacobi scaled or not, on the oracle's neighbour lists (rows in original
    order, columns ascending).

    Pair (row b, neighbour a), per axis: o = l (c_b - c_a) as the FP32 product
    of the cell side and the integer cell difference (on periodic axes plus
    the multiple of the cell count that the FP64 minimum image takes), then
    d = o + (r'_b - r'_a) in FP32; r2 = (d0^2 + d1^2) + d2^2; q = sqrt(r2) / h;
    F = (105/(128 pi) (q - 2)^3) / h^5 and W = 21/(16 pi) (1 - q/2)^4 (2q + 1)
    / h^3 for q < 2; w = -((2 mubar (m_a / rho_a)) F) / rho_b, 2 mubar = mu_a
    + mu_b or 4 mu_a mu_b / (mu_a + mu_b) -- every operation in FP32 on the
    FP32-rounded particle data.  Fluid row: D = 1 + dt (Kahan sum of w), off
    entries -(dt w), divided by D when scaled; plain diagonal 1 (scaled) or D.
    Dummy-wall row: W / (Kahan sum of W) over fluid neighbours (identity when
    that sum is 0); identity rows otherwise."""

    def __init__(self, op: Operator, lo, hi, periodic):
        if op.kernel != 0:
            raise ValueError("the single-precision matrix is defined for the Wendland kernel")
        from . import lib, _dp
        import ctypes as C
        n = op.n
        pos = np.stack([op._x, op._y, op._z], axis=1)
        nc, cs, period = cell_grid(lo, hi, periodic, op.h, 2.0)
        cell, rel = cell_relative(pos, np.asarray(lo, np.float64), nc, cs, period)
        rp, cols = op.row_ptr, op.cols
        rows = np.repeat(np.arange(n), np.diff(rp))
        a = cols.astype(np.int64)
        d = np.zeros((rows.size, 3), dtype=F32)
        for k in range(3):
            dc = cell[rows, k] - cell[a, k]
            rb, ra = rel[rows, k], rel[a, k]
            if period[k] > 0.0:
                d64 = _disp(pos[rows, k] - pos[a, k], period[k])
                rest = d64 - dc.astype(np.float64) * cs[k] - (rb.astype(np.float64) - ra.astype(np.float64))
                dc = dc + np.rint(rest / period[k]).astype(np.int64) * nc[k]
            o = F32(cs[k]) * dc.astype(F32)
            d[:, k] = o + (rb - ra)
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        hf = F32(op.h)
        inv_h = 1.0 / op.h
        inv_h3 = inv_h * inv_h * inv_h
        inv_h5 = inv_h3 * inv_h * inv_h
        with np.errstate(all="ignore"):
            q = np.sqrt(r2) / hf
            inside = q < F32(2.0)
            t = q - F32(2.0)
            F = np.where(inside, (F32(105.0 / (128.0 * np.pi)) * ((t * t) * t)) * F32(inv_h5), F32(0.0))
            u = F32(1.0) - F32(0.5) * q
            W = np.where(inside, ((F32(21.0 / (16.0 * np.pi)) * (((u * u) * u) * u))
                                  * (F32(2.0) * q + F32(1.0))) * F32(inv_h3), F32(0.0))
            mu = op._mu.astype(F32)
            m = op._mass.astype(F32)
            rho = op._rho.astype(F32)
            mua, mub = mu[a], mu[rows]
            if op.avg == 1:
                ssum = mua + mub
                tm = np.where(ssum > F32(0.0), (F32(4.0) * (mua * mub)) / ssum, F32(0.0))
            else:
                tm = mua + mub
            w = -((tm * (m[a] / rho[a])) * F) / rho[rows]
        w = w.astype(F32)
        W = W.astype(F32)
        fluid = op._type == FLUID_TYPE
        fp = C.POINTER(C.c_float)
        i64p = C.POINTER(C.c_int64)
        L = lib()

        def rowsum(v):
            v = np.ascontiguousarray(v, dtype=F32)
            out = np.zeros(n, dtype=F32)
            L.orc_kahan_rows_f32(n, rp.ctypes.data_as(i64p), v.ctypes.data_as(fp), out.ctypes.data_as(fp))
            return out

        dt = F32(op.dt)
        Sw = rowsum(np.where(fluid[rows], w, F32(0.0)))
        D = np.where(fluid, F32(1.0) + dt * Sw, F32(1.0)).astype(F32)
        Wf = np.where(fluid[a] & ~fluid[rows], W, F32(0.0)).astype(F32)
        SW = rowsum(Wf)
        aba = -(dt * w)
        off = np.where(fluid[rows], aba / D[rows] if op.jacobi else aba, F32(0.0)).astype(F32)
        dummy = (~fluid[rows]) & (op.wall == 1) & (SW[rows] > F32(0.0))
        with np.errstate(all="ignore"):
            off = np.where(dummy, Wf / SW[rows], off).astype(F32)
        self.n, self.row_ptr, self.cols = n, rp, cols
        self.off = np.ascontiguousarray(off, dtype=F32)
        self.D = D                                          # FP32 diagonal 1 + dt sum w (1 on walls)
        self.diag = np.where(fluid & (not op.jacobi), D, F32(1.0)).astype(F32)  # the plain A_bb
        self.jacobi = op.jacobi
        self.cell, self.rel = cell, rel

    def apply(self, X):
        """Y (n, 3) FP32 = the Kahan FP32 gemv of X (rounded to FP32)."""
        from . import lib
        import ctypes as C
        fp = C.POINTER(C.c_float)
        X = np.asarray(X, dtype=F32)
        Y = np.zeros(X.shape, dtype=F32)
        for c in range(3):
            x = np.ascontiguousarray(X[:, c])
            y = np.zeros(self.n, dtype=F32)
            lib().orc_kahan_gemv_f32(self.n, self.row_ptr.ctypes.data_as(C.POINTER(C.c_int64)),
                                     self.cols.ctypes.data_as(C.POINTER(C.c_int32)),
                                     self.diag.ctypes.data_as(fp), self.off.ctypes.data_as(fp),
                                     x.ctypes.data_as(fp), y.ctypes.data_as(fp))
            Y[:, c] = y
        return Y

    def rhs(self, B):
        """The scaled right-hand side FP32(B) / D (rounded once), or FP32(B)."""
        b = np.asarray(B, dtype=F32).astype(np.float64)
        if self.jacobi:
            b = b / self.D.astype(np.float64)[:, None]
        return b.astype(F32)


def _rhs(op: Operator, B):
    b = np.asarray(B, dtype=np.float64)
    return b / op.diag()[:, None] if op.jacobi else b


def solve(op: Operator, B, tol=2.0 ** -23, max_iter=2000, variant=ROBUST, force_stall=None, dots="f64",
          paper32: "Paper32Operator" = None):
    """A V = B (three columns) in single precision.  Returns (X (n, 3) FP32,
    report dict with iters, state, stall_count, rr, tau2, and history
    (iters + 1, 3) of r.r).  dots: "f64" or "kahan" (see the module);
    paper32: the paper's single-precision matrix and gemv instead of the
    FP64 operator rounded to FP32."""
    if dots not in _DOTS:
        raise ValueError(dots)

    def dot(a, b):
        return _dot(a, b, dots)

    if paper32 is not None:
        def A(v):
            return paper32.apply(v)

        b = paper32.rhs(B)
    else:
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
