"""FP64 oracle of the per-particle MLP that gives the solver its initial guess.

TEST INFRASTRUCTURE ONLY (tests, smoke check).  Plain numpy, sharing nothing
with the HIP kernels.

The learned initial guess is not part of the paper (which names better
initial guesses as future work, Sections "Conclusions and future work" and
"Implementation notes"); the network is defined here:

  sample = (features x[4], basis B[3], target t) for one fluid particle and
           one velocity component;
  z1 = x W1 + b1,  h1 = relu(z1)                       (4 -> 64)
  z2 = h1 W2 + b2, h2 = relu(z2)                       (64 -> 64)
  z3 = h2 W3 + b3, h3 = relu(z3)                       (64 -> 64)
  o  = h3 W4 + b4                                      (64 -> 3)
  pred = o . B,  loss = mean over samples of (pred - t)^2

Parameters are one flat FP32 vector (W1 4x64, b1, W2 64x64, b2, W3 64x64, b3,
W4 64x3, b4; matrices row-major as [in][out]).  With `bf16=True` the oracle
rounds, to bfloat16 (nearest-even), exactly the quantities the GPU kernels
feed to their BF16 products: every weight matrix, the layer inputs h1, h2 of
the two 64x64 products, and the gradient signals dz2, dz3 that enter the
backward products.  With `bf16=False` it is the exact FP64 network, which the
finite-difference test pins.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 4, 64, 3
SIZES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("W3", (N_H, N_H)), ("b3", (N_H,)), ("W4", (N_H, N_OUT)), ("b4", (N_OUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
SAMPLE = 8  # floats per sample: x[4], B[3], t


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) through FP32, back to FP64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed=0):
    """He-uniform initial weights, zero biases, output layer scaled down."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SIZES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shape[0])
            d[name] = rng.uniform(-lim, lim, size=shape)
        else:
            d[name] = np.zeros(shape)
    d["W4"] *= 0.1
    return pack(d).astype(np.float32)


def forward(p, S, bf=True):
    """Returns (o, pred, cache) for samples S (m x 8)."""
    P = unpack(p)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    x, B = S[:, 0:4].astype(np.float64), S[:, 4:7].astype(np.float64)
    W1, W2, W3, W4 = r(P["W1"]), r(P["W2"]), r(P["W3"]), r(P["W4"])
    z1 = x @ W1 + P["b1"]
    h1 = np.maximum(z1, 0.0)
    a1 = r(h1)
    z2 = a1 @ W2 + P["b2"]
    h2 = np.maximum(z2, 0.0)
    a2 = r(h2)
    z3 = a2 @ W3 + P["b3"]
    h3 = np.maximum(z3, 0.0)
    o = h3 @ W4 + P["b4"]
    pred = np.sum(o * B, axis=1)
    return o, pred, dict(x=x, B=B, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, h3=h3, W2=W2, W3=W3, W4=W4)


def loss_grad(p, S, bf=True):
    """Mean squared error of pred against t and its gradient (flat vector)."""
    o, pred, c = forward(p, S, bf)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    t = S[:, 7].astype(np.float64)
    m = S.shape[0]
    err = pred - t
    loss = np.mean(err ** 2)
    go = (2.0 / m) * err[:, None] * c["B"]
    g = {}
    g["W4"] = c["h3"].T @ go
    g["b4"] = go.sum(axis=0)
    dz3 = (go @ c["W4"].T) * (c["z3"] > 0)
    g["W3"] = c["a2"].T @ r(dz3)
    g["b3"] = dz3.sum(axis=0)
    dz2 = (r(dz3) @ c["W3"].T) * (c["z2"] > 0)
    g["W2"] = c["a1"].T @ r(dz2)
    g["b2"] = dz2.sum(axis=0)
    dz1 = (r(dz2) @ c["W2"].T) * (c["z1"] > 0)
    g["W1"] = c["x"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba), bias-corrected, on FP32 master weights."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
