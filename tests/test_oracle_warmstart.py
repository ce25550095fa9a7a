"""Pins of the warm-start oracle (features, learned start, fallback) against
what linear algebra fixes: fixed blends reproduce b and u exactly, the
increment u - A u vanishes on constant fields (rows of A sum to one), the
blend u + D^-1 (u - A u) is one Jacobi sweep from u (error against
(I + dt L)^-1 u of second order in dt where u alone errs to first order),
the Jacobi blend on a single-site system is exact, dummy wall rows are
satisfied exactly, and the fallback keeps the smaller true residual."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
from oracle import warmstart as WS
from paper_2206_14780_amd import workloads as W


def _case(wall=W.WALL_DUMMY, dt_nu=20.0, seed=11, n=(6, 6, 6)):
    rng = np.random.default_rng(seed)
    pos, pt = W.lattice(n, 1.0, walls=((False, False), (False, False), (True, True)),
                        jitter=0.15, rng=rng)
    N = pos.shape[0]
    fl = pt == W.FLUID
    nu = 3.0
    rho = np.ones(N)
    mu = nu * rho
    u = np.zeros((N, 3))
    u[fl] = rng.normal(size=(int(fl.sum()), 3))
    kw = dict(pos=pos, mass=rho.copy(), rho=rho, mu=mu, ptype=pt,
              period=np.array([n[0], n[1], 0.0]), h=1.3, dt=dt_nu / nu, wall=wall,
              avg=W.AVG_ARITH)
    return kw, pt, u, nu


@pytest.mark.parametrize("wall", [W.WALL_DYNAMIC, W.WALL_DUMMY])
def test_fixed_blends_reproduce_b_and_u(wall):
    kw, pt, u, _ = _case(wall=wall)
    op = O.Operator(jacobi=False, **kw)
    fl = pt == W.FLUID
    b = u + 0.3
    b[~fl] = np.random.default_rng(5).normal(size=(int((~fl).sum()), 3))
    S, U = WS.samples(op, u, b, kw["mu"], kw["rho"], pt)
    x_b = WS.learned_start(op, WS.fixed_blend_params([1, 0, 0]), S, U, b, pt)
    x_u = WS.learned_start(op, WS.fixed_blend_params([0, 1, 0]), S, U, b, pt)
    # the start is U * (o . B) evaluated on FP32 samples: FP32 rounding only
    assert np.allclose(x_b[fl], b[fl], rtol=2e-7, atol=0)
    assert np.allclose(x_u[fl], u[fl], rtol=2e-7, atol=0)
    r = b - op.apply(x_b)
    if wall == W.WALL_DYNAMIC:
        assert np.array_equal(x_b[~fl], b[~fl])
    # wall rows of the unscaled system hold exactly (to rounding)
    assert np.max(np.abs(r[~fl])) < 1e-12 * np.max(np.abs(b))


def test_increment_vanishes_on_constant_fields():
    kw, pt, _, _ = _case(wall=W.WALL_DUMMY)
    op = O.Operator(jacobi=False, **kw)
    u = np.tile([1.5, -2.0, 0.25], (pt.size, 1))
    S, _ = WS.samples(op, u, u, kw["mu"], kw["rho"], pt)
    fl = np.repeat(pt == W.FLUID, 3)
    assert np.max(np.abs(S[fl, 1])) < 1e-13
    assert np.max(np.abs(S[fl, 6])) < 1e-13
    assert np.all(S[~fl] == 0.0)


def test_scalar_features_are_the_workload_parameters():
    # constant viscosity: the relative-viscosity feature is 0, the stiffness
    # feature is log10(dt nu / h^2)
    kw, pt, u, nu = _case(dt_nu=37.0)
    op = O.Operator(jacobi=False, **kw)
    S, _ = WS.samples(op, u, u, kw["mu"], kw["rho"], pt)
    fl = np.repeat(pt == W.FLUID, 3)
    assert np.allclose(S[fl, 2], 0.0, rtol=0, atol=1e-15)
    assert np.allclose(S[fl, 3], np.log10(37.0 / 1.3 ** 2), rtol=0, atol=1e-14)


def test_viscosity_feature_is_scale_free():
    # variable viscosity: feature 2 = log10 nu_k minus its mean over fluid
    # rows (zero mean, the same when every viscosity is multiplied by 10),
    # while the stiffness feature moves by exactly log10 10 = 1
    kw, pt, u, nu = _case(dt_nu=20.0)
    rng = np.random.default_rng(8)
    mu = 10.0 ** rng.uniform(0.0, 2.0, pt.size)
    kw = dict(kw, mu=mu)
    op = O.Operator(jacobi=False, **kw)
    S, _ = WS.samples(op, u, u, mu, kw["rho"], pt)
    fl = pt == W.FLUID
    f2 = S.reshape(-1, 3, 8)[fl, 0, 2]
    assert abs(f2.mean()) < 1e-12
    lognu = np.log10(mu / kw["rho"])[fl]
    assert np.allclose(f2, lognu - lognu.mean(), rtol=0, atol=1e-13)
    op10 = O.Operator(jacobi=False, **dict(kw, mu=10.0 * mu))
    S10, _ = WS.samples(op10, u, u, 10.0 * mu, kw["rho"], pt)
    assert np.allclose(S10[:, 2], S[:, 2], rtol=0, atol=1e-13)
    f3 = S.reshape(-1, 3, 8)[fl, 0, 3]
    assert np.allclose(S10.reshape(-1, 3, 8)[fl, 0, 3], f3 + 1.0, rtol=0, atol=1e-13)


def test_jacobi_blend_is_second_order_in_dt():
    # x* = (I + dt L)^-1 u: the start u errs by O(dt); u + D^-1 (u - A u)
    # = u - D^-1 dt L u with D = 1 + O(dt) errs by O(dt^2).  Halving dt must
    # halve the first error and quarter the second (periodic fluid, no walls,
    # so A = I + dt L exactly).
    rng = np.random.default_rng(3)
    pos, pt = W.lattice((6, 6, 6), 1.0, jitter=0.15, rng=rng)
    N = pos.shape[0]
    u = rng.normal(size=(N, 3))
    errs = []
    for dt in (0.02, 0.01):
        kw = dict(pos=pos, mass=np.ones(N), rho=np.ones(N), mu=np.ones(N), ptype=pt,
                  period=np.array([6.0, 6.0, 6.0]), h=1.3, dt=dt, wall=W.WALL_DUMMY,
                  avg=W.AVG_ARITH)
        op = O.Operator(jacobi=False, **kw)
        xs = O.dense_solve(op, u)
        S, U = WS.samples(op, u, u, kw["mu"], kw["rho"], pt)
        x1 = WS.learned_start(op, WS.fixed_blend_params([0, 1, 1]), S, U, u, pt)
        errs.append((np.linalg.norm(u - xs), np.linalg.norm(x1 - xs)))
    (e0u, e0n), (e1u, e1n) = errs
    assert 1.8 < e0u / e1u < 2.2
    assert 3.5 < e0n / e1n < 4.5
    assert e0n < 0.2 * e0u


def test_targets_and_blend_loss():
    # with t = x*/U the loss of the network is the mean squared relative error
    # of the start it produces
    kw, pt, u, _ = _case()
    op = O.Operator(jacobi=False, **kw)
    xs = O.dense_solve(op, u)
    S, U = WS.samples(op, u, u, kw["mu"], kw["rho"], pt, target=xs)
    fl = pt == W.FLUID
    p = WS.fixed_blend_params([0, 1, 1])
    x0 = WS.learned_start(op, p, S, U, u, pt)
    Sf = S[np.repeat(fl, 3)]
    loss, _ = M.loss_grad(p, Sf.astype(np.float32).astype(np.float64), bf=True)
    ref = np.mean(((x0[fl] - xs[fl]) / U) ** 2)
    assert abs(loss - ref) <= 1e-6 * ref


@pytest.mark.parametrize("wall", [W.WALL_DYNAMIC, W.WALL_DUMMY])
def test_fallback_keeps_the_smaller_residual(wall):
    kw, pt, u, _ = _case(wall=wall)
    op_s = O.Operator(jacobi=True, **kw)
    b = u.copy()
    xs = O.dense_solve(op_s, b)
    bad = xs.copy()
    bad[:, 1] += 10.0  # component 1: the learned start is far off
    x0, use, rr_l, rr_p = WS.select(op_s, b, u, bad)
    assert list(use) == [True, False, True]
    assert rr_l[0] < 1e-20 and rr_l[2] < 1e-20
    assert np.array_equal(x0[:, 1], u[:, 1])
    assert np.array_equal(x0[:, 0], bad[:, 0])


@pytest.mark.parametrize("wall", [W.WALL_DYNAMIC, W.WALL_DUMMY])
def test_blend_011_is_one_jacobi_sweep(wall):
    # with b = u the blend o = (0, 1, 1) is x0 = u + D^-1 (b - A u) on fluid
    # rows: one Jacobi sweep from u, checked against the dense matrix
    kw, pt, u, _ = _case(wall=wall, dt_nu=150.0)
    op = O.Operator(jacobi=False, **kw)
    A = op.dense()
    fl = pt == W.FLUID
    S, U = WS.samples(op, u, u, kw["mu"], kw["rho"], pt)
    x0 = WS.learned_start(op, WS.fixed_blend_params([0, 1, 1]), S, U, u, pt)
    jac = u + (u - A @ u) / np.diag(A)[:, None]
    assert np.allclose(x0[fl], jac[fl], rtol=1e-6, atol=1e-6 * np.abs(jac).max())
    assert np.abs(np.diag(A)[fl]).min() > 10.0  # a stiff case: D matters
