"""Reference of the surrogate network: forward pass, masked mean-square loss,
its gradient and one Adam step, in float64 numpy.

TEST INFRASTRUCTURE ONLY (imported by tests/ and the benchmark's checks).

The network maps (1000/T, x_H, log10 x_V, E_z/1e7 V/m) to (log10 D_O,
log10 D_H): 4 -> 128 -> 128 -> 2 with SiLU activations.  With emulate=True
the values that the GPU kernels hold in BF16 are rounded to BF16 (round to
nearest even) at the same points: all three weight matrices, the first
hidden activation h1 and the back-propagated dz2 entering the two 128x128
products; everything else is float64 here (float32 on the GPU).  The
gradient is the plain chain rule of that computation.  Pinned by
single-path networks computed by hand (the forward wiring), finite
differences (the gradient, emulate=False), brute-force BF16 rounding and
the closed form of Adam's first step.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 4, 128, 2
SIZES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("W3", (N_H, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def bf16(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), via float32."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def standardise(X, Y, M):
    """Input mean/std (population) over all rows; target mean/std over the
    rows whose mask is set, per output."""
    xm = X.mean(axis=0)
    xs = X.std(axis=0)
    xs = np.where(xs > 1e-12, xs, 1.0)
    ym = np.zeros(N_OUT)
    ys = np.ones(N_OUT)
    for o in range(N_OUT):
        v = Y[M[:, o] != 0, o]
        if v.size:
            ym[o] = v.mean()
            s = v.std()
            ys[o] = s if s > 1e-12 else 1.0
    return xm, xs, ym, ys


def forward(p, Xs, emulate=True):
    """Standardised inputs Xs [n,4] -> outputs [n,2] and the intermediates."""
    w = unpack(p)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, W3 = r(w["W1"]), r(w["W2"]), r(w["W3"])
    z1 = Xs @ W1 + w["b1"]
    h1 = r(silu(z1))
    z2 = h1 @ W2 + w["b2"]
    h2 = silu(z2)
    y = h2 @ W3 + w["b3"]
    return y, dict(W1=W1, W2=W2, W3=W3, z1=z1, h1=h1, z2=z2, h2=h2)


def loss_and_grad(p, Xs, Ts, M, emulate=True):
    """Sum over outputs of the masked mean square error of standardised
    targets Ts, and its gradient with respect to the parameter vector."""
    y, c = forward(p, Xs, emulate)
    cnt = np.maximum(M.sum(axis=0), 1.0)
    e = (y - Ts) * M
    loss = float((e * e / cnt).sum())
    dy = 2.0 * e / cnt
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    g = {}
    g["W3"] = c["h2"].T @ dy
    g["b3"] = dy.sum(axis=0)
    dz2 = (dy @ c["W3"].T) * dsilu(c["z2"])
    g["b2"] = dz2.sum(axis=0)
    dz2r = r(dz2)
    g["W2"] = c["h1"].T @ dz2r
    dh1 = dz2r @ c["W2"].T
    dz1 = dh1 * dsilu(c["z1"])
    g["b1"] = dz1.sum(axis=0)
    g["W1"] = Xs.T @ dz1
    return loss, pack(g)


def adam(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) at step number t (1-based)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def he_init(rng, members=1):
    out = []
    for _ in range(members):
        d = {"W1": rng.normal(0, np.sqrt(2 / N_IN), (N_IN, N_H)), "b1": np.zeros(N_H),
             "W2": rng.normal(0, np.sqrt(2 / N_H), (N_H, N_H)), "b2": np.zeros(N_H),
             "W3": rng.normal(0, np.sqrt(2 / N_H), (N_H, N_OUT)), "b3": np.zeros(N_OUT)}
        out.append(pack(d))
    return np.stack(out)
