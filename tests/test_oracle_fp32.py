"""Pins of the oracle's single-precision BiCGSTAB (the paper's all-FP32
solver): everything stays FP32, it reaches FP32 accuracy against the LU
answer, its first iterates follow the FP64 iteration within FP32 rounding,
the two variants agree in their first iterates, and a forced stall stays in
its component."""
import numpy as np
import pytest

import oracle as O
from oracle import fp32 as OF
from paper_2206_14780_amd import workloads as W

from test_oracle_operator import _tank


def _case(seed=7, **kw):
    k, pt = _tank(seed=seed, **kw)
    op = O.Operator(jacobi=True, **k)
    B = np.random.default_rng(seed).normal(size=(pt.size, 3))
    return op, B


@pytest.mark.parametrize("variant", [O.ROBUST, O.STANDARD])
def test_fp32_solution_and_types(variant):
    op, B = _case(mu_span=100.0, dt_nu=10.0)
    X, rep, h = OF.solve(op, B, tol=1e-6, variant=variant)
    assert X.dtype == np.float32 and h.dtype == np.float32
    assert rep["state"] == [O.CONVERGED] * 3
    assert all(np.float32(v) == v for v in rep["rr"] + rep["tau2"])
    Xd = O.dense_solve(op, B)
    # FP32 storage and a 1e-6 residual: within a few 1e-6 of the exact answer
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < 2e-5


@pytest.mark.parametrize("variant", [O.ROBUST, O.STANDARD])
def test_first_iterates_follow_fp64(variant):
    op, B = _case(seed=3, mu_span=30.0, dt_nu=20.0)
    # r.r falls by about 1e7 over the first five iterations of this system;
    # until cancellation sets in the FP32 iterates track the FP64 ones to
    # FP32 rounding amplified by that fall (measured: 3e-8, 8e-8, 2e-6, 1e-5,
    # 5e-5 relative; 3e-3 at the sixth)
    _, r32, h32 = OF.solve(op, B, tol=0.0, max_iter=4, variant=variant)
    _, r64, h64 = O.solve(op, B, tol=1e-30, max_iter=4, variant=variant, true_res_period=0)
    assert r32["iters"] == r64["iters"] == 4
    d = np.abs(h32 / h64 - 1.0).max(axis=1)
    assert d[0] < 1e-7 and d[1] < 1e-6 and np.all(d < 1e-4)


def test_variants_agree_early():
    op, B = _case(seed=5, mu_span=30.0, dt_nu=20.0)
    _, _, hr = OF.solve(op, B, tol=0.0, max_iter=4, variant=O.ROBUST)
    _, _, hs = OF.solve(op, B, tol=0.0, max_iter=4, variant=O.STANDARD)
    assert np.allclose(hr, hs, rtol=1e-3, atol=0)


def test_forced_stall_stays_in_its_component():
    op, B = _case(seed=9, mu_span=30.0, dt_nu=20.0)
    _, r0, h0 = OF.solve(op, B, tol=1e-6)
    _, r1, h1 = OF.solve(op, B, tol=1e-6, force_stall=(2, 1))
    assert r0["stall_count"] == [0, 0, 0] and r1["stall_count"][1] >= 1
    assert r1["stall_count"][0] == 0 and r1["stall_count"][2] == 0
    n = min(len(h0), len(h1))
    assert np.array_equal(h0[:n, 0], h1[:n, 0]) and np.array_equal(h0[:n, 2], h1[:n, 2])


# --- rotated CG in single precision (symmetric case: dynamic walls, uniform mass)

def _sym_case(seed=7, jacobi=True):
    from test_oracle_cg import _rhs, _sym_tank
    kw, pt = _sym_tank(seed=seed)
    return O.Operator(jacobi=jacobi, **kw), _rhs(pt, seed), pt


@pytest.mark.parametrize("jacobi", [True, False])
def test_fp32_cg_solution_and_types(jacobi):
    op, B, pt = _sym_case(jacobi=jacobi)
    X, rep, h = OF.cg_solve(op, B, tol=1e-6)
    assert X.dtype == np.float32 and h.dtype == np.float32
    assert rep["state"] == [O.CONVERGED] * 3
    assert all(np.float32(v) == v for v in rep["rr"] + rep["tau2"])
    b = B / op.diag()[:, None] if jacobi else B
    wr = pt != W.FLUID
    # wall rows start at their value rounded to FP32; the FP64 starting
    # residual keeps only that rounding, so they move by at most about it
    assert np.all(np.abs(X[wr] - b[wr]) <= 2.0 ** -22 * np.abs(b[wr]))
    Xd = O.dense_solve(op, B)
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < 2e-5


@pytest.mark.parametrize("jacobi", [True, False])
def test_fp32_cg_first_iterates_follow_fp64(jacobi):
    op, B, _ = _sym_case(seed=3, jacobi=jacobi)
    _, r32, h32 = OF.cg_solve(op, B, tol=0.0, max_iter=4)
    _, r64, h64 = O.cg_solve(op, B, tol=1e-30, max_iter=4, true_res_period=0)
    assert r32["iters"] == r64["iters"] == 4
    d = np.abs(h32 / h64 - 1.0).max(axis=1)
    assert d[0] < 1e-6 and np.all(d < 1e-4)


def test_fp32_cg_forced_stall_and_dummy_walls_refused():
    op, B, _ = _sym_case(seed=9)
    _, r0, h0 = OF.cg_solve(op, B, tol=1e-6)
    _, r1, h1 = OF.cg_solve(op, B, tol=1e-6, force_stall=(2, 1))
    assert r0["stall_count"] == [0, 0, 0] and r1["stall_count"] == [0, 1, 0]
    assert r1["state"] == [O.CONVERGED] * 3
    n = min(len(h0), len(h1))
    assert np.array_equal(h0[:n, 0], h1[:n, 0]) and np.array_equal(h0[:n, 2], h1[:n, 2])
    kw, _ = _tank(wall=W.WALL_DUMMY)
    with pytest.raises(ValueError):
        OF.cg_solve(O.Operator(jacobi=True, **kw), B)


# --- the paper's compensated single-precision sums (appendix "Implementation
# notes": Kahan's summation for every multi-term sum) -------------------------

def test_kahan_dot_rounds_each_product_to_fp32():
    # (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24 lies half-way between two FP32
    # neighbours and rounds to the even one, 1 + 2^-11, which the second
    # product cancels exactly: the paper's arithmetic gives 0.  The FP64 sum of
    # the exact products keeps the 2^-24 that the rounding dropped.
    a = np.array([1.0 + 2.0 ** -12, -1.0], dtype=np.float32)
    b = np.array([1.0 + 2.0 ** -12, 1.0 + 2.0 ** -11], dtype=np.float32)
    assert O.kahan_dot_f32(a, b) == np.float32(0.0)
    A, B = a[:, None], b[:, None]
    assert OF._dot(A, B, "kahan")[0] == np.float32(0.0)
    assert OF._dot(A, B, "f64")[0] == np.float32(2.0 ** -24)


def test_kahan_sum_keeps_what_plain_fp32_drops():
    # 1 followed by 2^20 terms of 2^-24 (half a unit in the last place of 1):
    # a plain FP32 sum rounds each addition back to 1 (ties to even); the
    # exact sum 1 + 2^-4 is representable and Kahan's compensation reaches it.
    v = np.concatenate([[1.0], np.full(1 << 20, 2.0 ** -24)]).astype(np.float32)
    plain = np.float32(1.0)
    for t in (v[1], v[2], v[3]):
        plain = np.float32(plain + t)
    assert plain == np.float32(1.0)
    assert O.kahan_sum_f32(v) == np.float32(1.0625)
    ones = np.ones_like(v)
    assert O.kahan_dot_f32(v, ones) == np.float32(1.0625)


def test_kahan_dot_within_its_error_bound():
    # |Kahan - exact| <= (2u + 2 n u^2) sum |p_i| over the FP32 products p_i
    # (u = 2^-24), the exact sum of the products taken in rational arithmetic;
    # a plain FP32 running sum of the same products errs far more on this data.
    from fractions import Fraction
    rng = np.random.default_rng(17)
    n = 20000
    a = (rng.normal(size=n) * 10.0 ** rng.uniform(-3, 3, n)).astype(np.float32)
    b = rng.normal(size=n).astype(np.float32)
    p = a * b  # FP32 products, each correctly rounded
    exact = sum(Fraction(float(t)) for t in p)
    mag = float(np.abs(p.astype(np.float64)).sum())
    u = 2.0 ** -24
    k = O.kahan_dot_f32(a, b)
    err_k = abs(float(Fraction(float(k)) - exact))
    assert err_k <= (2 * u + 2 * n * u * u) * mag
    plain = np.float32(0.0)
    for t in p:
        plain = np.float32(plain + t)
    err_p = abs(float(Fraction(float(plain)) - exact))
    assert err_p > 10.0 * err_k
    w = rng.uniform(0.5, 2.0, n).astype(np.float32)
    pw = (w * a) * b
    exact_w = sum(Fraction(float(t)) for t in pw)
    kw = O.kahan_dot_f32(a, b, w)
    assert abs(float(Fraction(float(kw)) - exact_w)) <= (2 * u + 2 * n * u * u) * float(np.abs(pw.astype(np.float64)).sum())


@pytest.mark.parametrize("variant", [O.ROBUST, O.STANDARD])
def test_kahan_form_solves_and_differs_from_the_rounded_once_form(variant):
    op, B = _case(mu_span=100.0, dt_nu=10.0)
    X, rep, h = OF.solve(op, B, tol=1e-6, variant=variant, dots="kahan")
    assert X.dtype == np.float32 and h.dtype == np.float32
    assert rep["state"] == [O.CONVERGED] * 3
    assert all(np.float32(v) == v for v in rep["rr"] + rep["tau2"])
    Xd = O.dense_solve(op, B)
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < 2e-5
    _, _, h64 = OF.solve(op, B, tol=1e-6, variant=variant, dots="f64")
    # the same iteration: the first residuals agree to FP32 rounding ...
    assert np.allclose(h[:3], h64[:3], rtol=1e-4, atol=0)
    # ... but it is a different arithmetic, not the other form under a new name
    k = min(len(h), len(h64))
    assert not np.array_equal(h[:k], h64[:k])


def test_kahan_form_cg():
    k, pt = _tank(seed=4, wall=W.WALL_DYNAMIC, avg=W.AVG_HARMONIC, mu_span=1.0, dt_nu=20.0)
    k["mass"] = np.ones(pt.size)
    op = O.Operator(jacobi=True, **k)
    B = np.random.default_rng(4).normal(size=(pt.size, 3))
    X, rep, h = OF.cg_solve(op, B, tol=1e-6, dots="kahan")
    assert rep["state"] == [O.CONVERGED] * 3
    Xd = O.dense_solve(op, B)
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < 2e-5


# --- the paper's single-precision matrix (appendix on relative positions) ---

def _paper_case(seed=7, uniform=False, wall=W.WALL_DUMMY, jacobi=True, **kw):
    k, pt = _tank(seed=seed, uniform=uniform, wall=wall, **kw)
    op = O.Operator(jacobi=jacobi, **k)
    lo = np.array([0.0, 0.0, -3.0])
    hi = np.array([6.0, 6.0, 8.0])
    return op, OF.Paper32Operator(op, lo, hi, [1, 1, 0]), pt, lo, hi


def test_cell_relative_positions_rebuild_the_positions():
    op, P, pt, lo, hi = _paper_case()
    nc, cs, period = OF.cell_grid(lo, hi, [1, 1, 0], op.h)
    assert np.all(cs >= 2.0 * op.h) and np.all(nc >= 1)
    pos = np.stack([op._x, op._y, op._z], axis=1)
    centre = lo + (P.cell + 0.5) * cs
    back = centre + P.rel.astype(np.float64)
    for a in range(3):
        d = back[:, a] - pos[:, a]
        if period[a] > 0:
            d = d - period[a] * np.rint(d / period[a])
        # the offset is the FP32 rounding of the exact one (|r'| <= a cell)
        assert np.all(np.abs(d) <= 2.0 ** -24 * cs[a])
    inside = (pos[:, 2] >= lo[2]) & (pos[:, 2] < hi[2])
    assert np.all(np.abs(P.rel[inside]) <= 0.5 * cs * (1 + 1e-6))


def test_grouped_displacement_gives_a_symmetric_fp32_matrix():
    # uniform mass, density and viscosity, no scaling: the fluid block is
    # symmetric, and with the displacement grouped as o' + (r'_b - r'_a) the
    # FP32 entries are equal bit for bit for (b, a) and (a, b)
    op, P, pt, _, _ = _paper_case(uniform=True, jacobi=False)
    n = op.n
    rows = np.repeat(np.arange(n), np.diff(P.row_ptr))
    fl = pt == W.FLUID
    ff = fl[rows] & fl[P.cols]
    M = {}
    for b, a, v in zip(rows[ff], P.cols[ff], P.off[ff]):
        M[(b, a)] = v
    assert len(M) > 1000
    assert all(M[(a, b)] == v for (b, a), v in M.items())


@pytest.mark.parametrize("wall", [W.WALL_DYNAMIC, W.WALL_DUMMY])
@pytest.mark.parametrize("jacobi", [True, False])
def test_fp32_entries_round_the_fp64_matrix(wall, jacobi):
    op, P, pt, _, _ = _paper_case(wall=wall, jacobi=jacobi, mu_span=100.0, dt_nu=20.0)
    d64, e64 = op.entries()
    u = 2.0 ** -24
    rows = np.repeat(np.arange(op.n), np.diff(P.row_ptr))
    rowmax = np.zeros(op.n)
    np.maximum.at(rowmax, rows, np.abs(e64))
    # each entry is ~15 FP32 operations from the particle data; (q - 2)^3
    # loses relative accuracy near the support edge, so the bound is on the
    # row's largest entry
    assert np.all(np.abs(P.off.astype(np.float64) - e64) <= 64 * u * rowmax[rows] + 1e-45)
    assert np.allclose(P.diag.astype(np.float64), d64, rtol=8 * u, atol=0)
    D64 = op.diag()
    assert np.allclose(P.D.astype(np.float64), D64, rtol=8 * u * 100, atol=0)


def test_kahan_gemv_within_its_bound():
    op, P, pt, _, _ = _paper_case(mu_span=1000.0, dt_nu=50.0)
    X = np.random.default_rng(4).normal(size=(op.n, 3)).astype(np.float32)
    Y = P.apply(X)
    # the same FP32 matrix applied in exact-enough FP64 arithmetic
    rows = np.repeat(np.arange(op.n), np.diff(P.row_ptr))
    Xd = X.astype(np.float64)
    Ye = P.diag.astype(np.float64)[:, None] * Xd
    np.add.at(Ye, rows, P.off.astype(np.float64)[:, None] * Xd[P.cols])
    mag = np.abs(P.diag.astype(np.float64))[:, None] * np.abs(Xd)
    np.add.at(mag, rows, np.abs(P.off.astype(np.float64))[:, None] * np.abs(Xd[P.cols]))
    u = 2.0 ** -24
    # FP32 rounding of each product (u) plus Kahan's 2u on the sum
    assert np.all(np.abs(Y.astype(np.float64) - Ye) <= 4 * u * mag + 1e-37)


@pytest.mark.parametrize("variant", [O.ROBUST, O.STANDARD])
def test_paper_single_precision_solve(variant):
    op, P, pt, _, _ = _paper_case(mu_span=100.0, dt_nu=10.0)
    B = np.random.default_rng(7).normal(size=(op.n, 3))
    X, rep, h = OF.solve(op, B, tol=1e-6, variant=variant, dots="kahan", paper32=P)
    assert X.dtype == np.float32 and h.dtype == np.float32
    assert rep["state"] == [O.CONVERGED] * 3
    Xd = O.dense_solve(op, B)
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < 2e-5
