"""The FP64 surrogate-network reference: backward pinned to the forward by
central finite differences, and the forward to a hand-evaluated tiny case."""
import numpy as np

from oracle import mlp


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = rng.normal(scale=0.3, size=mlp.N_PARAMS)
    X = rng.normal(size=(37, 2))
    t = rng.normal(size=37)
    L, g = mlp.loss_grad(p, X, t)
    idx = np.concatenate([np.arange(0, 200), rng.choice(mlp.N_PARAMS, 300, replace=False), [mlp.N_PARAMS - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_grad(p + e, X, t)[0] - mlp.loss_grad(p - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), i


def test_forward_by_hand():
    # one active path: W1[0] = (1, 0), W2[0, 0] = 1, w3[0] = 1, everything else 0
    W1 = np.zeros((64, 2)); W1[0, 0] = 1.0
    W2 = np.zeros((64, 64)); W2[0, 0] = 1.0
    w3 = np.zeros(64); w3[0] = 1.0
    p = mlp.pack(W1, np.zeros(64), W2, np.zeros(64), w3, 0.5)
    x = 0.7
    s = lambda z: z / (1 + np.exp(-z))  # noqa: E731
    y, _ = mlp.forward(p, np.array([[x, -3.0]]))
    # the other 63 hidden units see z = 0 and silu(0) = 0
    assert abs(y[0] - (s(s(x)) + 0.5)) < 1e-15


def test_bf16_rounding():
    # bfloat16 keeps 8 significant bits: the spacing at 1 is 2^-7
    v = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, 1.0 + 3 * 2**-9, 1.0 + 2**-9, 3.14159265, -2.5e-3])
    r = mlp.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                 # tie -> even significand (1.0)
    assert r[2] == 1.0 + 2 * 2**-7     # tie -> even significand (1 + 2^-6)
    assert r[3] == 1.0 + 2**-7         # above the midpoint
    assert r[4] == 1.0                 # below the midpoint
    assert abs(r[5] / v[5] - 1) < 2**-8 and abs(r[6] / v[6] - 1) < 2**-8
