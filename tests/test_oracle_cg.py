"""Pins of the oracle's rotated CG (Section "Restructuring the Conjugate
Gradient") for the symmetric case (dynamic walls, uniform mass): a direct LU
answer, the textbook CG and the textbook Jacobi-preconditioned CG written
out here in their unrotated form, the Galerkin property that characterises
the CG iterate, finite termination, and the stopping rules."""
import numpy as np
import pytest

import oracle as O
from paper_2206_14780_amd import workloads as W

from test_oracle_operator import _tank


def _sym_tank(n=(6, 6, 5), avg=W.AVG_HARMONIC, mu_span=100.0, dt_nu=10.0, seed=7):
    # uniform mass keeps A symmetric on the fluid rows; density and
    # viscosity still vary per particle (both enter the pair weight
    # symmetrically)
    kw, pt = _tank(seed=seed, n=n, wall=W.WALL_DYNAMIC, avg=avg, mu_span=mu_span, dt_nu=dt_nu)
    kw["mass"] = np.full(pt.size, 1.0)
    return kw, pt


def _rhs(pt, seed, walls=True):
    B = np.random.default_rng(seed).normal(size=(pt.size, 3))
    if not walls:
        B[pt != W.FLUID] = 0.0
    return B


def test_fluid_block_is_symmetric():
    # the premise of the CG (Section "Linear system properties and
    # resolution"): with dynamic walls and uniform mass the fluid-fluid
    # block of the unscaled matrix is symmetric, the full matrix is not
    kw, pt = _sym_tank()
    A = O.Operator(jacobi=False, **kw).dense()
    f = pt == W.FLUID
    Aff = A[np.ix_(f, f)]
    assert np.abs(Aff - Aff.T).max() <= 1e-15 * np.abs(Aff).max()
    assert np.abs(A - A.T).max() > 1e-3 * np.abs(A[f][:, ~f]).max()


@pytest.mark.parametrize("jacobi", [True, False])
@pytest.mark.parametrize("avg", [W.AVG_ARITH, W.AVG_HARMONIC])
def test_matches_dense_lu(jacobi, avg):
    kw, pt = _sym_tank(avg=avg)
    op = O.Operator(jacobi=jacobi, **kw)
    B = _rhs(pt, 11)
    X, rep, _ = O.cg_solve(op, B, tol=1e-13)
    Xd = O.dense_solve(op, B)
    assert rep["status"] == 0 and rep["state"] == [O.CONVERGED] * 3
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < 1e-10
    # identity wall rows: the start takes their exact value and keeps it
    w = pt != W.FLUID
    assert np.array_equal(X[w], B[w])


def _textbook_cg(A, b, x0, iters, d=None):
    """The unrotated CG of the paper's listing on A x = b (d: Jacobi
    preconditioner z = r / d, the textbook PCG), in the unscaled system.
    Returns the iterates x_1..x_iters."""
    x = x0.copy()
    r = b - A @ x
    z = r if d is None else r / d
    p = z.copy()
    rz = r @ z
    out = []
    for _ in range(iters):
        Ap = A @ p
        a = rz / (p @ Ap)
        x = x + a * p
        r = r - a * Ap
        z = r if d is None else r / d
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        out.append(x.copy())
    return out


@pytest.mark.parametrize("jacobi", [False, True])
def test_equals_textbook_cg(jacobi):
    # without scaling the rotated CG is the printed textbook CG reordered;
    # with the Jacobi scaling it is the textbook Jacobi-preconditioned CG
    # (the D-weighted inner product): same iterates in FP64
    kw, pt = _sym_tank(mu_span=30.0, dt_nu=20.0)
    op = O.Operator(jacobi=jacobi, **kw)
    A = O.Operator(jacobi=False, **kw).dense()
    d = np.diag(A).copy() if jacobi else None
    B = _rhs(pt, 3)
    f = pt == W.FLUID
    w = ~f
    for k in (1, 2, 5, 9):
        X, rep, _ = O.cg_solve(op, B, tol=0.0, max_iter=k, true_res_period=0)
        assert rep["iters"] == k
        for c in range(3):
            # reduced system on the fluid rows, wall values moved to the rhs
            bf = B[f, c] - A[np.ix_(f, w)] @ B[w, c]
            xs = _textbook_cg(A[np.ix_(f, f)], bf, np.zeros(f.sum()), k, None if d is None else d[f])
            ref = xs[-1]
            assert np.linalg.norm(X[f, c] - ref) <= 1e-9 * np.linalg.norm(ref)


def test_galerkin_property():
    # the k-th CG iterate is the Galerkin solution on the Krylov space
    # K_k = span{r0, M r0, ..., M^(k-1) r0} of the preconditioned operator
    # M = D^-1 A: x_k - x0 lies in K_k and A x_k - b is orthogonal to K_k
    # (for SPD A this is the minimum of the A-norm of the error over x0 + K_k)
    kw, pt = _sym_tank(n=(5, 5, 4), mu_span=10.0, dt_nu=30.0, seed=9)
    op = O.Operator(jacobi=True, **kw)
    A = O.Operator(jacobi=False, **kw).dense()
    f = pt == W.FLUID
    Aff = A[np.ix_(f, f)]
    d = np.diag(Aff)
    B = _rhs(pt, 8, walls=False)
    X0 = np.random.default_rng(4).normal(scale=0.1, size=(pt.size, 3))
    X0[~f] = 0.0
    for k in (2, 4, 6):
        X, rep, _ = O.cg_solve(op, B, X0=X0, tol=0.0, max_iter=k, true_res_period=0)
        for c in range(3):
            r0 = B[f, c] - Aff @ X0[f, c]
            K = np.empty((f.sum(), k))
            v = r0 / d
            for j in range(k):
                K[:, j] = v / np.linalg.norm(v)
                v = (Aff @ v) / d
            Q, _ = np.linalg.qr(K)
            step = X[f, c] - X0[f, c]
            off = step - Q @ (Q.T @ step)
            assert np.linalg.norm(off) <= 1e-8 * np.linalg.norm(step)
            res = B[f, c] - Aff @ X[f, c]
            assert np.linalg.norm(Q.T @ res) <= 1e-9 * np.linalg.norm(r0)


def test_finite_termination():
    # in exact arithmetic CG ends within as many iterations as the fluid
    # block has rows; in FP64 a tiny system gets there to ~1e-13
    kw, pt = _sym_tank(n=(2, 2, 2), mu_span=1.0, dt_nu=5.0)
    nf = int((pt == W.FLUID).sum())
    op = O.Operator(jacobi=True, **kw)
    B = _rhs(pt, 5)
    X, rep, _ = O.cg_solve(op, B, tol=1e-12)
    assert rep["status"] == 0 and rep["iters"] <= nf
    Xd = O.dense_solve(op, B)
    assert np.linalg.norm(X - Xd) <= 1e-11 * np.linalg.norm(Xd)


def test_zero_rhs_and_exact_start():
    kw, pt = _sym_tank()
    op = O.Operator(jacobi=True, **kw)
    X, rep, _ = O.cg_solve(op, np.zeros((pt.size, 3)), tol=1e-8)
    assert rep["iters"] == 0 and np.all(X == 0.0) and rep["state"] == [O.CONVERGED] * 3
    B = _rhs(pt, 6)
    Xd = O.dense_solve(op, B)
    X, rep, _ = O.cg_solve(op, B, X0=Xd, tol=1e-8)
    assert rep["iters"] == 0 and rep["status"] == 0


def test_forced_stall_recovers():
    # alpha forced to zero at iteration 3 on component 1: that iteration is a
    # no-op for it (stalled, beta = 0), the next restarts the direction from
    # r and the solve still converges to the LU answer
    kw, pt = _sym_tank()
    op = O.Operator(jacobi=True, **kw)
    B = _rhs(pt, 12)
    _, rep0, h0 = O.cg_solve(op, B, tol=1e-10)
    X, rep, h = O.cg_solve(op, B, tol=1e-10, force_stall=(3, 1))
    assert rep["stall_count"] == [0, 1, 0] and rep["status"] == 0
    assert np.array_equal(h[3, 1], h[2, 1])  # no change at the stalled iteration
    assert rep["iters"] > rep0["iters"]
    Xd = O.dense_solve(op, B)
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < 1e-8


def test_periodic_true_residual_keeps_result():
    # periodic FP64 true-residual checks do not change an FP64 solve
    kw, pt = _sym_tank()
    op = O.Operator(jacobi=True, **kw)
    B = _rhs(pt, 13)
    X1, r1, _ = O.cg_solve(op, B, tol=1e-10, true_res_period=0)
    X2, r2, _ = O.cg_solve(op, B, tol=1e-10, true_res_period=3)
    assert r1["iters"] == r2["iters"] and r2["n_true_checks"] > 1 and r2["n_replaced"] == 0
    assert np.array_equal(X1, X2)


def test_refuses_dummy_walls():
    kw, pt = _tank(wall=W.WALL_DUMMY)
    op = O.Operator(jacobi=True, **kw)
    with pytest.raises(ValueError):
        O.cg_solve(op, _rhs(pt, 1))


def test_more_iterations_fewer_applies_than_bicgstab():
    # the paper's observation on dynamic walls: the CG needs more iterations
    # than the BiCGSTAB, each with one apply instead of two
    kw, pt = _sym_tank(n=(10, 10, 8), mu_span=1.0, dt_nu=50.0)
    op = O.Operator(jacobi=True, **kw)
    B = _rhs(pt, 3)
    Xc, rc, _ = O.cg_solve(op, B, tol=1e-8)
    Xb, rb, _ = O.solve(op, B, tol=1e-8)
    assert rc["status"] == 0 and rb["status"] == 0
    assert rb["iters"] < rc["iters"] < 2 * rb["iters"]
    assert np.linalg.norm(Xc - Xb) <= 1e-6 * np.linalg.norm(Xb)
