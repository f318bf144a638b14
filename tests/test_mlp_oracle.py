"""Pins of the surrogate network's reference (oracle/mlp_oracle.py):
finite differences of the float64 loss, brute-force BF16 rounding, the
closed form of Adam's first step, and standardisation."""
import numpy as np

from oracle import mlp_oracle as R


def _data(rng, n=37):
    X = rng.normal(size=(n, 4))
    Y = rng.normal(size=(n, 2))
    M = (rng.random((n, 2)) > 0.2).astype(float)
    return X, Y, M


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = R.he_init(rng)[0] * 0.5
    X, Y, M = _data(rng)
    loss, g = R.loss_and_grad(p, X, Y, M, emulate=False)
    idx = np.concatenate([rng.choice(R.N_PARAMS, 60, replace=False),
                          [0, 511, 512, 640, 640 + 16383, R.N_PARAMS - 1]])
    h = 1e-6
    for k in idx:
        e = np.zeros(R.N_PARAMS)
        e[k] = h
        lp, _ = R.loss_and_grad(p + e, X, Y, M, emulate=False)
        lm, _ = R.loss_and_grad(p - e, X, Y, M, emulate=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_bf16_rounding_is_nearest_even():
    rng = np.random.default_rng(1)
    f = np.concatenate([rng.normal(size=5000).astype(np.float32) * 10 ** rng.uniform(-3, 3, 5000),
                        np.array([1.0 + 2**-8, 1.0 + 3 * 2**-8, -1.0 - 2**-8, 0.0], np.float32)])
    r = R.bf16(f)
    for x, y in zip(f.astype(np.float64), r):
        u = np.float32(x).view(np.uint32)
        lo = np.uint32(u & 0xFFFF0000).view(np.float32).astype(np.float64)
        step = np.uint32((u & 0xFFFF0000) + 0x10000).view(np.float32).astype(np.float64)
        cands = sorted({lo, step}, key=lambda c: (abs(c - x), int(np.float32(c).view(np.uint32) >> 16) & 1))
        assert y == cands[0], (x, y, cands)


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(2)
    p = rng.normal(size=50)
    g = rng.choice([-1.0, 1.0], 50) * rng.uniform(0.1, 10.0, 50)   # |g| >> eps
    q, m, v = R.adam(p, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    np.testing.assert_allclose(p - q, 1e-3 * np.sign(g), rtol=1e-6)


def test_standardisation_moments():
    rng = np.random.default_rng(3)
    X, Y, M = _data(rng, 500)
    X = X * [1, 2, 3, 4] + [5, -1, 0, 2]
    xm, xs, ym, ys = R.standardise(X, Y, M)
    Z = (X - xm) / xs
    np.testing.assert_allclose(Z.mean(0), 0, atol=1e-12)
    np.testing.assert_allclose(Z.std(0), 1, atol=1e-12)
    for o in range(2):
        t = (Y[M[:, o] != 0, o] - ym[o]) / ys[o]
        assert abs(t.mean()) < 1e-12 and abs(t.std() - 1) < 1e-12


def test_forward_single_paths_match_hand_computation():
    """A network with one nonzero weight per layer computes one scalar path,
    written out here with math.exp: an input, hidden or output index taken
    from the wrong axis (a transposed operand) sends the signal elsewhere."""
    import math
    rng = np.random.default_rng(4)
    X = rng.normal(size=(9, 4)) * 2.0
    for i, j, k, o in ((2, 17, 101, 1), (0, 127, 3, 0), (3, 64, 64, 1)):
        d = {name: np.zeros(shape) for name, shape in R.SIZES}
        a, b, c = 0.75, -1.5, 2.25
        d["W1"][i, j] = a
        d["W2"][j, k] = b
        d["W3"][k, o] = c
        d["b3"][:] = (0.3, -0.7)
        y, _ = R.forward(R.pack(d), X, emulate=False)
        for n in range(X.shape[0]):
            z1 = X[n, i] * a
            h1 = z1 / (1.0 + math.exp(-z1))
            z2 = h1 * b
            h2 = z2 / (1.0 + math.exp(-z2))
            want = [0.3, -0.7]
            want[o] += h2 * c
            assert abs(y[n, o] - want[o]) <= 1e-14 * max(1.0, abs(want[o])), (i, j, k, o, n)
            assert y[n, 1 - o] == want[1 - o]
