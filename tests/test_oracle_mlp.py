"""Pins of the MLP oracle: finite differences of the exact FP64 network,
bfloat16 rounding and Adam against PyTorch's CPU implementations, and the
blend structure pred = o . B."""
import numpy as np
import torch

from oracle import mlp as M


def _samples(m=50, seed=0):
    rng = np.random.default_rng(seed)
    S = rng.normal(size=(m, M.SAMPLE))
    S[:, 2] = rng.uniform(0, 3, m)
    S[:, 3] = rng.uniform(0, 2.5, m)
    return S


def test_parameter_count():
    assert M.NPARAM == 4 * 64 + 64 + 2 * (64 * 64 + 64) + 64 * 3 + 3 == 8835


def test_gradient_matches_central_differences():
    p = M.init_params(3).astype(np.float64)
    p += np.random.default_rng(1).normal(scale=0.05, size=p.shape)  # non-zero biases
    S = _samples()
    loss, g = M.loss_grad(p, S, bf=False)
    idx = np.random.default_rng(2).choice(M.NPARAM, 80, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = eps
        fd = (M.loss_grad(p + e, S, bf=False)[0] - M.loss_grad(p - e, S, bf=False)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd), abs(g[i])) + 1e-10, (i, fd, g[i])


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(4).normal(scale=10.0, size=10000)
    x = np.concatenate([x, [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=20)
    t = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2)
    p, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    for step in range(1, 6):
        g = rng.normal(size=20)
        opt.zero_grad()
        t.grad = torch.tensor(g)
        opt.step()
        p, m, v = M.adam(p, g, m, v, step, 1e-2)
    assert np.allclose(p, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_prediction_blends_the_basis():
    d = M.unpack(np.zeros(M.NPARAM))
    d = {k: v.copy() for k, v in d.items()}
    d["b4"][:] = [0.25, -1.0, 2.0]
    S = _samples(7)
    o, pred, _ = M.forward(M.pack(d), S)
    assert np.allclose(o, [0.25, -1.0, 2.0])
    assert np.allclose(pred, S[:, 4:7] @ np.array([0.25, -1.0, 2.0]))
