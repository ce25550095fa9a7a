"""Pins of the oracle's single-precision BiCGSTAB (the paper's all-FP32
solver): everything stays FP32, it reaches FP32 accuracy against the LU
answer, its first iterates follow the FP64 iteration within FP32 rounding,
the two variants agree in their first iterates, and a forced stall stays in
its component."""
import numpy as np
import pytest

import oracle as O
from oracle import fp32 as OF

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
