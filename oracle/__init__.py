"""FP64 CPU oracle for the semi-implicit SPH viscous solve.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the product path never does.  It shares no code
with the HIP library (its own C source, its own neighbour search, its own
operator and solver); only the seeded input generators are common.

What it computes is stated in the C source (`sph_oracle.c`) with the
passages of the paper each function follows.  This module only marshals
numpy arrays into those C functions, plus a dense LU solve (LAPACK through
numpy) that gives a direct answer for small systems.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

CONVERGED, STALLED, PROGRESSING = 0, 1, 2
ROBUST, STANDARD = 0, 1
FLUID_TYPE = 0  # particle type of fluid rows (every other type is a wall)
KERNEL_WENDLAND, KERNEL_GAUSSIAN = 0, 1
SUPPORT = {KERNEL_WENDLAND: 2.0, KERNEL_GAUSSIAN: 3.0}  # support radius in units of h
FLT_MIN = float(np.finfo(np.float32).tiny)
DBL_MIN = float(np.finfo(np.float64).tiny)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        dp, i64p, i32p = C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32)
        L.orc_wendland_w.restype = C.c_double
        L.orc_wendland_w.argtypes = [C.c_double]
        L.orc_wendland_f.restype = C.c_double
        L.orc_wendland_f.argtypes = [C.c_double]
        for f in ("orc_gauss_w", "orc_gauss_f"):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [C.c_double]
        L.orc_neighbors_brute.restype = C.c_int64
        L.orc_neighbors_brute.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_double, i64p, i32p, C.c_int64]
        L.orc_neighbors_grid.restype = C.c_int64
        L.orc_neighbors_grid.argtypes = [C.c_int64, dp, dp, dp, dp, dp, C.c_double, i64p, i32p,
                                         C.c_int64]
        L.orc_neighbors_grid_rows.restype = C.c_int64
        L.orc_neighbors_grid_rows.argtypes = [C.c_int64, dp, dp, dp, dp, dp, C.c_double, i64p, C.c_int64,
                                              i64p, i32p, C.c_int64]
        L.orc_apply.argtypes = [C.POINTER(OrcOp), C.POINTER(dp), C.POINTER(dp)]
        L.orc_diag.argtypes = [C.POINTER(OrcOp), dp]
        L.orc_assemble_dense.argtypes = [C.POINTER(OrcOp), dp]
        L.orc_assemble_csr.argtypes = [C.POINTER(OrcOp), dp, dp]
        L.orc_bicgstab.restype = C.c_int32
        L.orc_bicgstab.argtypes = [C.POINTER(OrcOp), C.c_int32, C.POINTER(dp), C.POINTER(dp),
                                   C.c_double, C.c_int32, C.c_double, C.c_int32, C.c_double,
                                   C.c_int32, C.c_int32, C.POINTER(OrcReport), dp, C.c_int32]
        L.orc_cg.restype = C.c_int32
        L.orc_cg.argtypes = [C.POINTER(OrcOp), C.POINTER(dp), C.POINTER(dp), C.c_double, C.c_int32,
                             C.c_double, C.c_int32, C.c_int32, C.c_int32, C.POINTER(OrcReport), dp,
                             C.c_int32]
        L.orc_ybar.restype = C.c_double
        L.orc_ybar.argtypes = [C.c_double, C.c_double]
        L.orc_papanastasiou.argtypes = [C.POINTER(OrcOp), C.POINTER(dp), C.c_double, C.c_double, C.c_double,
                                        dp, dp]
        fp = C.POINTER(C.c_float)
        L.orc_kahan_sum_f32.restype = C.c_float
        L.orc_kahan_sum_f32.argtypes = [C.c_int64, fp]
        L.orc_kahan_dot_f32.restype = C.c_float
        L.orc_kahan_dot_f32.argtypes = [C.c_int64, fp, fp, fp]
        L.orc_kahan_rows_f32.argtypes = [C.c_int64, i64p, fp, fp]
        L.orc_kahan_gemv_f32.argtypes = [C.c_int64, i64p, i32p, fp, fp, fp, fp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


class OrcOp(C.Structure):
    _fields_ = [("n", C.c_int64), ("row_ptr", C.POINTER(C.c_int64)),
                ("cols", C.POINTER(C.c_int32)), ("x", C.POINTER(C.c_double)),
                ("y", C.POINTER(C.c_double)), ("z", C.POINTER(C.c_double)),
                ("period", C.c_double * 3), ("h", C.c_double),
                ("mass", C.POINTER(C.c_double)), ("rho", C.POINTER(C.c_double)),
                ("mu", C.POINTER(C.c_double)), ("type", C.POINTER(C.c_uint8)),
                ("dt", C.c_double), ("wall", C.c_int32), ("avg", C.c_int32),
                ("jacobi", C.c_int32), ("kernel", C.c_int32),
                ("a_diag", C.POINTER(C.c_double)), ("a_off", C.POINTER(C.c_double))]


class OrcReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("state", C.c_int32 * 3),
                ("stall_count", C.c_int32 * 3), ("rr", C.c_double * 3), ("bb", C.c_double * 3),
                ("tau2", C.c_double * 3), ("true_rr", C.c_double * 3),
                ("n_true_checks", C.c_int32), ("n_replaced", C.c_int32),
                ("history_len", C.c_int32)]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def _fp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_float))


def kahan_sum_f32(v) -> np.float32:
    """Kahan's compensated FP32 sum of v in index order."""
    v = np.ascontiguousarray(v, dtype=np.float32)
    return np.float32(lib().orc_kahan_sum_f32(v.size, _fp(v)))


def kahan_dot_f32(a, b, w=None) -> np.float32:
    """sum_i (w_i) a_i b_i in FP32: products rounded to FP32, then added in
    index order with Kahan's compensation."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float32)
    return np.float32(lib().orc_kahan_dot_f32(a.size, _fp(w), _fp(a), _fp(b)))


def wendland_w(q):
    """w(q) of the Wendland psi_{3,1} kernel (radius 2), elementwise."""
    L = lib()
    q = np.asarray(q, dtype=np.float64)
    return np.vectorize(L.orc_wendland_w, otypes=[np.float64])(q)


def wendland_f(q):
    """f(q) with F(r, h) = f(r/h)/h^5 = (1/r) dW/dr, elementwise."""
    L = lib()
    q = np.asarray(q, dtype=np.float64)
    return np.vectorize(L.orc_wendland_f, otypes=[np.float64])(q)


def gauss_w(q):
    """w(q) of the normalised truncated Gaussian (radius 3), elementwise."""
    return np.vectorize(lib().orc_gauss_w, otypes=[np.float64])(np.asarray(q, dtype=np.float64))


def gauss_f(q):
    """f(q) = w'(q)/q of the truncated Gaussian, elementwise."""
    return np.vectorize(lib().orc_gauss_f, otypes=[np.float64])(np.asarray(q, dtype=np.float64))


def _soa(pos):
    pos = np.asarray(pos, dtype=np.float64)
    return [np.ascontiguousarray(pos[:, a]) for a in range(3)]


def neighbors(pos, period, h, lo=None, method="grid", support=2.0):
    """CSR neighbour lists (row_ptr int64 [n+1], cols int32 ascending) of
    N(i) = {j != i : |r_i - r_j|^2 < (support h)^2}, minimum image on axes
    whose period is > 0.  method = "brute" (all pairs) or "grid" (cell grid)."""
    L = lib()
    x, y, z = _soa(pos)
    n = x.shape[0]
    per = np.ascontiguousarray(np.asarray(period, dtype=np.float64))
    lo_ = np.ascontiguousarray(np.zeros(3) if lo is None else np.asarray(lo, dtype=np.float64))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cap = max(1, n * (96 if support <= 2.0 else 300))
    while True:
        cols = np.zeros(cap, dtype=np.int32)
        args = [n, _dp(x), _dp(y), _dp(z)]
        if method == "grid":
            args.append(_dp(lo_))
        args += [_dp(per), float(support) * float(h), row_ptr.ctypes.data_as(C.POINTER(C.c_int64)),
                 cols.ctypes.data_as(C.POINTER(C.c_int32)), cap]
        fn = L.orc_neighbors_grid if method == "grid" else L.orc_neighbors_brute
        nnz = int(fn(*args))
        if nnz <= cap:
            return row_ptr, cols[:nnz].copy()
        cap = nnz


def neighbors_rows(pos, period, h, rows, lo=None, support=2.0):
    """CSR lists (row_ptr int64 [n+1], cols int32 ascending) holding the
    neighbour set of `rows` only (every other row empty): the cell-grid search
    of `neighbors` restricted to a sample of rows, so that an Operator built
    on it gives exact rows of A for systems too large for full lists."""
    L = lib()
    x, y, z = _soa(pos)
    n = x.shape[0]
    rows = np.unique(np.asarray(rows, dtype=np.int64))
    if rows.size and (rows[0] < 0 or rows[-1] >= n):
        raise ValueError("row out of range")
    per = np.ascontiguousarray(np.asarray(period, dtype=np.float64))
    lo_ = np.ascontiguousarray(np.zeros(3) if lo is None else np.asarray(lo, dtype=np.float64))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cap = max(1, rows.size * (128 if support <= 2.0 else 320))
    while True:
        cols = np.zeros(cap, dtype=np.int32)
        nnz = int(L.orc_neighbors_grid_rows(n, _dp(x), _dp(y), _dp(z), _dp(lo_), _dp(per),
                                            float(support) * float(h),
                                            rows.ctypes.data_as(C.POINTER(C.c_int64)), rows.size,
                                            row_ptr.ctypes.data_as(C.POINTER(C.c_int64)),
                                            cols.ctypes.data_as(C.POINTER(C.c_int32)), cap))
        if nnz <= cap:
            return row_ptr, cols[:nnz].copy()
        cap = nnz


class Operator:
    """The viscous matrix A(dt) of one particle system (optionally Jacobi
    scaled), backed by the C oracle.  Keeps every array it hands to C alive."""

    def __init__(self, pos, mass, rho, mu, ptype, period, h, dt, wall, avg, jacobi=True,
                 nbr=None, lo=None, kernel=KERNEL_WENDLAND):
        pos = np.asarray(pos, dtype=np.float64)
        self.n = pos.shape[0]
        self.period = np.asarray(period, dtype=np.float64)
        self.h = float(h)
        self.kernel = int(kernel)
        if nbr is None:
            nbr = neighbors(pos, self.period, h, lo=lo, method="grid", support=SUPPORT[self.kernel])
        self.row_ptr, self.cols = nbr
        self._x, self._y, self._z = _soa(pos)
        self._mass = np.ascontiguousarray(np.broadcast_to(np.asarray(mass, np.float64), (self.n,)))
        self._rho = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, np.float64), (self.n,)))
        self._mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, np.float64), (self.n,)))
        self._type = np.ascontiguousarray(np.asarray(ptype, dtype=np.uint8))
        s = OrcOp()
        s.n = self.n
        s.row_ptr = self.row_ptr.ctypes.data_as(C.POINTER(C.c_int64))
        s.cols = self.cols.ctypes.data_as(C.POINTER(C.c_int32))
        s.x, s.y, s.z = _dp(self._x), _dp(self._y), _dp(self._z)
        for a in range(3):
            s.period[a] = float(self.period[a])
        s.h = self.h
        s.mass, s.rho, s.mu = _dp(self._mass), _dp(self._rho), _dp(self._mu)
        s.type = self._type.ctypes.data_as(C.POINTER(C.c_uint8))
        s.dt = float(dt)
        s.wall = int(wall)
        s.avg = int(avg)
        s.jacobi = int(bool(jacobi))
        s.kernel = self.kernel
        self.s = s
        self.dt, self.wall, self.avg, self.jacobi = float(dt), int(wall), int(avg), bool(jacobi)

    @classmethod
    def from_workload(cls, w, jacobi=True, nbr=None, **over):
        kw = dict(pos=w.pos, mass=w.mass, rho=w.rho, mu=w.mu, ptype=w.ptype, period=w.period,
                  h=w.h, dt=w.dt, wall=w.wall, avg=w.avg, kernel=getattr(w, "kernel", KERNEL_WENDLAND))
        kw.update(over)
        return cls(jacobi=jacobi, nbr=nbr, lo=w.lo, **kw)

    def apply(self, X):
        """Y = A X (or D^-1 A X), X and Y of shape (n, 3)."""
        X = np.asarray(X, dtype=np.float64)
        xs = [np.ascontiguousarray(X[:, c]) for c in range(3)]
        ys = [np.zeros(self.n) for _ in range(3)]
        xa = (C.POINTER(C.c_double) * 3)(*[_dp(a) for a in xs])
        ya = (C.POINTER(C.c_double) * 3)(*[_dp(a) for a in ys])
        lib().orc_apply(C.byref(self.s), xa, ya)
        return np.stack(ys, axis=1)

    def diag(self):
        d = np.zeros(self.n)
        lib().orc_diag(C.byref(self.s), _dp(d))
        return d

    def dense(self):
        A = np.zeros((self.n, self.n))
        lib().orc_assemble_dense(C.byref(self.s), _dp(A))
        return A

    def entries(self):
        """(diag (n,), off (nnz,)): the entries of A (or D^-1 A) on the
        neighbour pattern (row_ptr, cols), as the dense assembly forms them."""
        d = np.zeros(self.n)
        e = np.zeros(max(int(self.row_ptr[-1]), 1))
        lib().orc_assemble_csr(C.byref(self.s), _dp(d), _dp(e))
        return d, e[:int(self.row_ptr[-1])]

    def assemble(self):
        """Stores the entries once; every later apply (and solve) on this
        operator then multiplies by them instead of re-evaluating each pair
        weight.  Returns self."""
        self._a_diag, self._a_off = self.entries()
        if self._a_off.size == 0:
            self._a_off = np.zeros(1)
        self.s.a_diag = _dp(self._a_diag)
        self.s.a_off = _dp(self._a_off)
        return self


def solve(op: Operator, B, X0=None, tol=1e-8, max_iter=10000, variant=ROBUST, floor=DBL_MIN,
          true_res_period=50, force_stall=None, history_cap=None, restart_drop=0.0):
    """BiCGSTAB solve of A V = B (three columns) with the oracle.

    Returns (X (n,3), report dict, history (len,3) of r.r per iteration)."""
    B = np.asarray(B, dtype=np.float64)
    n = op.n
    bs = [np.ascontiguousarray(B[:, c]) for c in range(3)]
    X0 = np.zeros((n, 3)) if X0 is None else np.asarray(X0, dtype=np.float64)
    xs = [np.ascontiguousarray(X0[:, c]).copy() for c in range(3)]
    cap = int(history_cap or (max_iter + 2))
    hist = np.zeros((cap, 3))
    rep = OrcReport()
    ba = (C.POINTER(C.c_double) * 3)(*[_dp(a) for a in bs])
    xa = (C.POINTER(C.c_double) * 3)(*[_dp(a) for a in xs])
    fi, fc = force_stall if force_stall is not None else (-1, -1)
    lib().orc_bicgstab(C.byref(op.s), int(variant), ba, xa, float(tol), int(max_iter),
                       float(floor), int(true_res_period), float(restart_drop), int(fi), int(fc),
                       C.byref(rep), _dp(hist), cap)
    report = dict(iters=rep.iters, status=rep.status, state=list(rep.state),
                  stall_count=list(rep.stall_count), rr=list(rep.rr), bb=list(rep.bb),
                  tau2=list(rep.tau2), true_rr=list(rep.true_rr),
                  n_true_checks=rep.n_true_checks, n_replaced=rep.n_replaced,
                  history_len=rep.history_len)
    return np.stack(xs, axis=1), report, hist[:rep.history_len].copy()


def cg_solve(op: Operator, B, X0=None, tol=1e-8, max_iter=10000, floor=DBL_MIN, true_res_period=50,
             force_stall=None, history_cap=None):
    """Rotated CG solve of A V = B (three columns) with the oracle, for the
    symmetric case (dynamic walls, uniform mass); the wall rows of the start
    are set to their exact value.  Raises ValueError for dummy walls.

    Returns (X (n,3), report dict, history (len,3) of r.r per iteration)."""
    B = np.asarray(B, dtype=np.float64)
    n = op.n
    bs = [np.ascontiguousarray(B[:, c]) for c in range(3)]
    X0 = np.zeros((n, 3)) if X0 is None else np.asarray(X0, dtype=np.float64)
    xs = [np.ascontiguousarray(X0[:, c]).copy() for c in range(3)]
    cap = int(history_cap or (max_iter + 2))
    hist = np.zeros((cap, 3))
    rep = OrcReport()
    ba = (C.POINTER(C.c_double) * 3)(*[_dp(a) for a in bs])
    xa = (C.POINTER(C.c_double) * 3)(*[_dp(a) for a in xs])
    fi, fc = force_stall if force_stall is not None else (-1, -1)
    st = lib().orc_cg(C.byref(op.s), ba, xa, float(tol), int(max_iter), float(floor), int(true_res_period),
                      int(fi), int(fc), C.byref(rep), _dp(hist), cap)
    if st == -1:
        raise ValueError("CG needs a symmetric system: dynamic walls")
    report = dict(iters=rep.iters, status=rep.status, state=list(rep.state),
                  stall_count=list(rep.stall_count), rr=list(rep.rr), bb=list(rep.bb),
                  tau2=list(rep.tau2), true_rr=list(rep.true_rr),
                  n_true_checks=rep.n_true_checks, n_replaced=rep.n_replaced,
                  history_len=rep.history_len)
    return np.stack(xs, axis=1), report, hist[:rep.history_len].copy()


def ybar(D, m):
    """The regularised yield term Ybar(D) of the Papanastasiou law (scalar)."""
    return float(lib().orc_ybar(float(D), float(m)))


def papanastasiou(op: Operator, U, tau0, m, mu0):
    """Viscosity from the velocity field U (n, 3): returns (mu, D), mu updated
    on fluid rows (tau0 Ybar(D) + mu0), the operator's own mu on wall rows."""
    U = np.asarray(U, dtype=np.float64)
    us = [np.ascontiguousarray(U[:, c]) for c in range(3)]
    ua = (C.POINTER(C.c_double) * 3)(*[_dp(a) for a in us])
    mu = np.zeros(op.n)
    D = np.zeros(op.n)
    lib().orc_papanastasiou(C.byref(op.s), ua, float(tau0), float(m), float(mu0), _dp(mu), _dp(D))
    return mu, D


def dense_solve(op: Operator, B):
    """Direct answer of A V = B by LU (LAPACK dgesv through numpy)."""
    A = op.dense()
    B = np.asarray(B, dtype=np.float64)
    if op.jacobi:
        B = B / op.diag()[:, None]
    return np.linalg.solve(A, B)
