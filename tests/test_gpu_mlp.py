"""GPU parity of the learned initial guess against the oracle: the BF16-MFMA
MLP forward, gradient and Adam step, the samples of a configuration, the
learned start itself, and the solve that chooses between learned and plain
starts.  All calls go through the C ABI.

Tolerances.  Both sides use the same BF16-rounded weights and the same
BF16-rounded layer inputs; the GPU accumulates in FP32 (MFMA) where the
oracle uses FP64.  A 64-term FP32 dot product errs by at most about
64 * 2^-24 = 4e-6 of the sum of its absolute terms, and a pre-activation
that lands within that distance of a BF16 rounding boundary may round to
the neighbouring BF16 value on one side only (a change of 2^-8 relative in
one of 64 inputs of the next layer).  Outputs are therefore compared in
relative L2 at 1e-4 and pointwise at 2^-8 of the output scale; the gradient
(a sum over the batch of such terms) in relative L2 at 1e-3."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
from oracle import warmstart as WS
from paper_2206_14780_amd import sph as S
from paper_2206_14780_amd import workloads as W

from gpu_util import GpuCase, rel_l2, small_tank, to_np

pytestmark = pytest.mark.gpu

FWD_REL = 1e-4
FWD_ABS = 2.0 ** -8
GRAD_REL = 1e-3


@pytest.fixture(scope="module")
def ctx():
    return S.Context(0)


def _params(seed=3, noise=0.05):
    p = M.init_params(seed).astype(np.float64)
    p += np.random.default_rng(seed + 100).normal(scale=noise, size=p.shape)
    p[M.NPARAM - 3:] = [0.4, 0.5, 0.8]
    return p.astype(np.float32)


def _samples(m, seed=0):
    rng = np.random.default_rng(seed)
    S_ = np.zeros((m, M.SAMPLE))
    S_[:, 0] = rng.normal(size=m)
    S_[:, 1] = rng.normal(scale=0.3, size=m)
    S_[:, 2] = rng.uniform(0.0, 3.0, m)
    S_[:, 3] = rng.uniform(0.7, 2.1, m)
    S_[:, 4] = S_[:, 0] + rng.normal(scale=0.1, size=m)
    S_[:, 5] = S_[:, 0]
    S_[:, 6] = S_[:, 1]
    S_[:, 7] = S_[:, 0] + 0.7 * S_[:, 1]
    return S_.astype(np.float32)


def _cuda(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


@pytest.mark.parametrize("m", [1, 15, 16, 17, 1000, 4099, 70001])
def test_forward_matches_oracle(ctx, m):
    import torch
    Sm = _samples(m, seed=m)
    p = _params()
    out = torch.empty((m, 4), dtype=torch.float32, device="cuda")
    print(f"forward m={m}", flush=True)
    ctx.sph_mlp_forward(_cuda(Sm), m, _cuda(p), out)
    torch.cuda.synchronize()
    g = out.cpu().double().numpy()
    o, pred, _ = M.forward(p.astype(np.float64), Sm.astype(np.float64), bf=True)
    scale = np.abs(o).max()
    assert rel_l2(g[:, :3], o) < FWD_REL
    assert np.max(np.abs(g[:, :3] - o)) <= FWD_ABS * scale
    assert rel_l2(g[:, 3], pred) < FWD_REL


def test_forward_rejects_misaligned_arrays(ctx):
    # the inference kernel moves samples and outputs as 16-byte vectors
    import torch
    p = _cuda(_params())
    buf = torch.zeros(17 * 8 + 4, dtype=torch.float32, device="cuda")
    out = torch.zeros(17 * 4 + 4, dtype=torch.float32, device="cuda")
    with pytest.raises(S.SphError):
        ctx.sph_mlp_forward(buf[1:], 16, p, out)
    with pytest.raises(S.SphError):
        ctx.sph_mlp_forward(buf, 16, p, out[1:])
    ctx.sph_mlp_forward(buf[4:], 16, p, out[4:])  # 16-byte offsets are fine
    torch.cuda.synchronize()


@pytest.mark.parametrize("batch", [1, 37, 4101, 65536])
def test_gradient_matches_oracle(ctx, batch):
    import torch
    pool = _samples(20000, seed=7)
    idx = np.random.default_rng(batch).integers(0, pool.shape[0], size=batch).astype(np.int32)
    p = _params(5)
    grad = torch.empty(M.NPARAM, dtype=torch.float32, device="cuda")
    print(f"grad batch={batch}", flush=True)
    loss = ctx.sph_mlp_grad(_cuda(pool), _cuda(idx), batch, _cuda(p), grad)
    torch.cuda.synchronize()
    lo, go = M.loss_grad(p.astype(np.float64), pool[idx].astype(np.float64), bf=True)
    gg = grad.cpu().double().numpy()
    assert abs(loss - lo) <= 1e-4 * lo
    assert rel_l2(gg, go) < GRAD_REL
    # every parameter block on its own
    o = 0
    for name, shape in M.SIZES:
        k = int(np.prod(shape))
        assert rel_l2(gg[o:o + k], go[o:o + k]) < 5 * GRAD_REL, name
        o += k


def test_adam_steps_match_oracle(ctx):
    import torch
    pool = _samples(5000, seed=9)
    idx = _cuda(np.arange(4096, dtype=np.int32))
    p0 = _params(6)
    params = _cuda(p0.copy())
    m = torch.zeros(M.NPARAM, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    grad = torch.empty_like(m)
    pool_d = _cuda(pool)
    lr = 1e-3
    pm, mm, vm = p0.astype(np.float64), np.zeros(M.NPARAM), np.zeros(M.NPARAM)
    for step in (1, 2, 3):
        ctx.sph_mlp_grad(pool_d, idx, 4096, params, grad)
        g = grad.cpu().double().numpy()
        ctx.sph_mlp_train_step(pool_d, idx, 4096, params, m, v, step, lr)
        torch.cuda.synchronize()
        pm, mm, vm = M.adam(pm, g, mm, vm, step, lr)
        pg = params.cpu().double().numpy()
        # FP32 master weights: one rounding of p per step, FP32 moments
        assert np.max(np.abs(pg - pm)) <= 1e-3 * lr + 4 * 2.0 ** -24 * np.max(np.abs(pm))
        pm = pg
        mm = m.cpu().double().numpy()
        vm = v.cpu().double().numpy()


def test_training_lowers_the_loss(ctx):
    import torch
    pool = _samples(50000, seed=11)
    pool_d = _cuda(pool)
    params = _cuda(M.init_params(1))
    m = torch.zeros(M.NPARAM, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    gen = np.random.default_rng(0)
    losses = []
    for step in range(1, 301):
        idx = _cuda(gen.integers(0, pool.shape[0], size=2048).astype(np.int32))
        losses.append(ctx.sph_mlp_train_step(pool_d, idx, 2048, params, m, v, step, 3e-3))
    # target t = B0 + 0.7 B2 - 0.1 noise: a fixed blend the network can represent
    assert np.mean(losses[-20:]) < 0.05 * np.mean(losses[:5])


# --- samples and the learned start ------------------------------------------------

def _state(w, seed=1):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(w.n, 3))
    u[w.ptype != W.FLUID] = 0.0
    b = u + 0.05 * rng.normal(size=(w.n, 3))
    b[w.ptype != W.FLUID] = rng.normal(size=(int((w.ptype != W.FLUID).sum()), 3))
    return u, b


@pytest.mark.parametrize("wall", [W.WALL_DYNAMIC, W.WALL_DUMMY])
@pytest.mark.parametrize("op_mode", [S.SPH_OP_CACHED, S.SPH_OP_ONTHEFLY])
def test_samples_match_oracle(ctx, wall, op_mode):
    import torch
    w = small_tank(wall=wall)
    u, b = _state(w)
    t = np.random.default_rng(3).normal(size=(w.n, 3))
    case = GpuCase(ctx, w)
    par = S.make_params(w.dt, w.wall, w.avg, True, op_mode)
    out = torch.empty((3 * w.n, M.SAMPLE), dtype=torch.float32, device="cuda")
    print(f"samples wall={wall} op_mode={op_mode}", flush=True)
    U = ctx.sph_mlp_samples(case.nb, case.parts, par, S.device_vec3(u, S.SPH_F64),
                            S.device_vec3(b, S.SPH_F64), S.device_vec3(t, S.SPH_F64), out)
    torch.cuda.synchronize()
    g = out.cpu().double().numpy()
    op = O.Operator.from_workload(w, jacobi=False)
    So, Uo = WS.samples(op, u, b, w.mu, w.rho, w.ptype, target=t)
    assert abs(U - Uo) <= 1e-13 * Uo
    ref = So.astype(np.float32).astype(np.float64)
    # FP64 on both sides, then one rounding to FP32: at most one FP32 ulp apart
    # (plus 1e-12 of the column's scale where cancellation leaves a tiny value)
    floor = 1e-12 * np.abs(ref).max(axis=0, keepdims=True)
    assert np.all(np.abs(g - ref) <= 2.0 ** -23 * np.abs(ref) + floor)


@pytest.mark.parametrize("prec", [S.SPH_F64, S.SPH_F32])
@pytest.mark.parametrize("wall", [W.WALL_DYNAMIC, W.WALL_DUMMY])
@pytest.mark.parametrize("op_mode", [S.SPH_OP_CACHED, S.SPH_OP_ONTHEFLY])
def test_learned_start_matches_oracle(ctx, prec, wall, op_mode):
    import torch
    w = small_tank(wall=wall, seed=8)
    u, b = _state(w, seed=2)
    if prec == S.SPH_F32:  # both sides see the same FP32 inputs
        u = u.astype(np.float32).astype(np.float64)
        b = b.astype(np.float32).astype(np.float64)
    p = _params(4)
    case = GpuCase(ctx, w)
    par = S.make_params(w.dt, w.wall, w.avg, True, op_mode)
    x0 = S.device_vec3(np.zeros((w.n, 3)), prec)
    print(f"learned start prec={prec} wall={wall} op_mode={op_mode}", flush=True)
    U = ctx.sph_mlp_warmstart(case.nb, case.parts, par, prec, S.device_vec3(u, prec),
                              S.device_vec3(b, prec), _cuda(p), x0)
    torch.cuda.synchronize()
    g = to_np(x0)
    op = O.Operator.from_workload(w, jacobi=False)
    So, Uo = WS.samples(op, u, b, w.mu, w.rho, w.ptype)
    xo = WS.learned_start(op, p, So, Uo, b, w.ptype)
    assert abs(U - Uo) <= 1e-6 * Uo
    fl = w.ptype == W.FLUID
    assert rel_l2(g[fl], xo[fl]) < FWD_REL
    assert rel_l2(g, xo) < FWD_REL
    # wall rows of the unscaled system hold for the GPU's own start: the
    # wall value is an FP64-accurate sum rounded once to the precision
    r = b - op.apply(g)
    u_p = 2.0 ** -24 if prec == S.SPH_F32 else 2.0 ** -53
    bound = u_p * np.abs(g[~fl]) + 1e-12 * np.abs(g).max()
    assert np.all(np.abs(r[~fl]) <= bound)


def _solve_pair(ctx, w, prec, p, X0, tol):
    """GPU solve with the learned start; the oracle's start, choice and solve."""
    import torch
    u = w.rhs
    case = GpuCase(ctx, w)
    pd = _cuda(p)
    ud = S.device_vec3(u, prec)
    Xg, rep = case.solve(w.rhs, prec, X0=X0, tol=tol, warm_params=pd, warm_u=ud)
    torch.cuda.synchronize()
    opu = O.Operator.from_workload(w, jacobi=False)
    ops = O.Operator.from_workload(w, jacobi=True)
    So, Uo = WS.samples(opu, u, w.rhs, w.mu, w.rho, w.ptype)
    xl = WS.learned_start(opu, p, So, Uo, w.rhs, w.ptype)
    xp = np.zeros((w.n, 3)) if X0 is None else X0
    x0, use, rr_l, rr_p = WS.select(ops, w.rhs, xp, xl)
    return Xg, rep, x0, use, rr_l, rr_p, ops


@pytest.mark.parametrize("x0_given", [False, True])
def test_solve_with_learned_start_fp64(ctx, x0_given):
    w = small_tank(seed=12, tol=1e-12)
    w.rhs[w.ptype != W.FLUID] = 0.0
    p = WS.fixed_blend_params([0.0, 1.0, 1.0])  # one Jacobi sweep from u
    X0 = w.rhs.copy() if x0_given else None
    Xg, rep, x0, use, rr_l, rr_p, ops = _solve_pair(ctx, w, S.SPH_F64, p, X0, 1e-12)
    assert rep["status"] == S.SPH_OK
    assert rep["warm_used"] == [int(v) for v in use]
    assert np.allclose(rep["warm_rr"], rr_l, rtol=1e-6)
    assert np.allclose(rep["plain_rr"], rr_p, rtol=1e-9)
    Xo, orep, _ = O.solve(ops, w.rhs, X0=x0, tol=1e-13, max_iter=2000)
    assert rel_l2(Xg, Xo) < 1e-10


def test_bad_network_falls_back_to_the_plain_start(ctx):
    # a start 50 b is far worse than b itself: every component keeps the plain
    # start and the iteration is bitwise the plain solve's
    w = small_tank(seed=13, tol=1e-8)
    p = WS.fixed_blend_params([50.0, 0.0, 0.0])
    case = GpuCase(ctx, w)
    X0 = w.rhs * 0.5
    Xa, ra = case.solve(w.rhs, S.SPH_F64, X0=X0, tol=1e-8)
    Xb, rb = case.solve(w.rhs, S.SPH_F64, X0=X0, tol=1e-8, warm_params=_cuda(p))
    assert rb["warm_used"] == [0, 0, 0]
    assert ra["iters"] == rb["iters"]
    assert np.array_equal(Xa, Xb)
    assert ra["history"] == rb["history"]


@pytest.mark.parametrize("wall", [W.WALL_DYNAMIC, W.WALL_DUMMY])
def test_solve_with_learned_start_fp32(ctx, wall):
    w = small_tank(seed=14, wall=wall, tol=1e-6)
    w.rhs[w.ptype != W.FLUID] = 0.0
    p = _params(9, noise=0.01)
    p[M.NPARAM - 3:] = [0.1, 0.9, 0.9]
    Xg, rep, x0, use, rr_l, rr_p, ops = _solve_pair(ctx, w, S.SPH_F32, p, w.rhs.copy(), 1e-6)
    assert rep["status"] == S.SPH_OK
    Xo, _, _ = O.solve(ops, w.rhs, X0=x0, tol=1e-12, max_iter=2000)
    assert rel_l2(Xg, Xo) < 1e-5


@pytest.mark.parametrize("op_mode", [S.SPH_OP_CACHED, S.SPH_OP_ONTHEFLY])
def test_solve_with_learned_start_mixed(ctx, op_mode):
    # FP32 operator, FP64 solution: the learned start (computed with the FP32
    # operator) enters the FP64 solution vector
    w = small_tank(seed=15, tol=1e-6)
    w.rhs[w.ptype != W.FLUID] = 0.0
    p = WS.fixed_blend_params([0.0, 1.0, 1.0])
    case = GpuCase(ctx, w)
    Xg, rep = case.solve(w.rhs, S.SPH_MIXED, X0=w.rhs.copy(), tol=1e-6, op_mode=op_mode,
                         warm_params=_cuda(p), warm_u=S.device_vec3(w.rhs, S.SPH_MIXED))
    assert rep["status"] == S.SPH_OK
    ops = O.Operator.from_workload(w, jacobi=True)
    Xo, _, _ = O.solve(ops, w.rhs, tol=1e-12, max_iter=2000)
    assert rel_l2(Xg, Xo) < 1e-5
    opu = O.Operator.from_workload(w, jacobi=False)
    So, Uo = WS.samples(opu, w.rhs, w.rhs, w.mu, w.rho, w.ptype)
    xl = WS.learned_start(opu, p, So, Uo, w.rhs, w.ptype)
    _, use, rr_l, rr_p = WS.select(ops, w.rhs, w.rhs, xl)
    assert rep["warm_used"] == [int(v) for v in use]
    assert np.allclose(rep["plain_rr"], rr_p, rtol=1e-9)
    assert np.allclose(rep["warm_rr"], rr_l, rtol=1e-3)


@pytest.mark.parametrize("prec", [S.SPH_F64, S.SPH_MIXED])
def test_start_from_x0_matches_explicit_u(ctx, prec):
    # warm_u null with x0_given takes u = x0 and forms the plain start's
    # residual inside the feature pass; it must equal the separate path
    # (u given explicitly) bit for bit
    w = small_tank(seed=16, tol=1e-8)
    w.rhs[w.ptype != W.FLUID] = 0.0
    p = WS.fixed_blend_params([0.2, 0.8, 0.9])
    case = GpuCase(ctx, w)
    X0 = w.rhs * 0.9
    Xa, ra = case.solve(w.rhs, prec, X0=X0, tol=1e-8, warm_params=_cuda(p))
    Xb, rb = case.solve(w.rhs, prec, X0=X0, tol=1e-8, warm_params=_cuda(p),
                        warm_u=S.device_vec3(X0, prec))
    assert ra["status"] == rb["status"] == S.SPH_OK
    # the residual vectors are identical; their norms are reduced over two
    # different grids (last-bit differences only)
    assert ra["warm_used"] == rb["warm_used"]
    assert np.allclose(ra["plain_rr"], rb["plain_rr"], rtol=1e-13, atol=0)
    assert ra["history"] == rb["history"]
    assert np.array_equal(Xa, Xb)
