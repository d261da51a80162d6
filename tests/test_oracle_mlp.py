"""Pins for the fp64 reference of the variant-cost network (oracle/mlp.py):
finite differences, closed forms, the linear regime, Adam's first step and a
hand-computed feature vector."""
import numpy as np

from oracle import mlp


def _rand_problem(seed, n=37):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.3, mlp.N_PARAMS)
    x = rng.normal(0.0, 1.0, (n, mlp.N_IN))
    t = rng.normal(0.0, 1.0, (n, mlp.N_OUT))
    m = (rng.random((n, mlp.N_OUT)) < 0.7).astype(np.float64)
    return p, x, t, m


def test_gradient_matches_central_differences():
    p, x, t, m = _rand_problem(1)
    g = mlp.grad(p, x, t, m)
    h = 1e-6
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.N_PARAMS, 300, replace=False)
    # every parameter block is probed
    bounds = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SHAPES])
    idx = np.unique(np.concatenate([idx, bounds[:-1], bounds[1:] - 1]))
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        num = (mlp.loss(p + e, x, t, m) - mlp.loss(p - e, x, t, m)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, num, g[i])


def test_zero_last_layer_closed_form():
    p, x, t, m = _rand_problem(3)
    w = mlp.unpack(p)
    w["W3"][:] = 0.0
    w["b3"][:] = np.arange(mlp.N_OUT) * 0.25
    p = mlp.pack(w)
    y, _ = mlp.forward(p, x)
    assert np.array_equal(y, np.broadcast_to(w["b3"], y.shape))
    cnt = m.sum()
    assert np.isclose(mlp.loss(p, x, t, m), (m * (w["b3"] - t) ** 2).sum() / cnt, rtol=1e-14)
    g = mlp.unpack(mlp.grad(p, x, t, m))
    assert np.allclose(g["b3"], (2 * m * (w["b3"] - t)).sum(axis=0) / cnt, rtol=1e-13)
    for k in ("W1", "b1", "W2", "b2"):
        assert not g[k].any()


def test_linear_regime_is_the_composed_affine_map():
    rng = np.random.default_rng(4)
    w = {"W1": rng.random((12, 64)), "b1": rng.random(64), "W2": rng.random((64, 64)), "b2": rng.random(64),
         "W3": rng.normal(size=(64, 6)), "b3": rng.normal(size=6)}
    x = rng.random((9, 12))  # all pre-activations positive: both ReLUs are the identity
    y, _ = mlp.forward(mlp.pack(w), x)
    lin = x @ w["W1"] @ w["W2"] @ w["W3"] + (w["b1"] @ w["W2"] + w["b2"]) @ w["W3"] + w["b3"]
    assert np.allclose(y, lin, rtol=1e-12)


def test_empty_mask_gives_zero_loss_and_gradient():
    p, x, t, _ = _rand_problem(5)
    m = np.zeros_like(t)
    assert mlp.loss(p, x, t, m) == 0.0
    assert not mlp.grad(p, x, t, m).any()


def test_adam_first_step_moves_by_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p, m, v = mlp.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), step=1, lr=0.01, eps=1e-12)
    assert np.allclose(p[:3], -0.01 * np.sign(g[:3]), rtol=1e-6)
    assert p[3] == 0.0
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_closed_form():
    # With the same gradient g at every step, m_t = (1 - b1^t) g and
    # v_t = (1 - b2^t) g^2, so the bias-corrected moments are exactly g and g^2
    # at every step and each step moves by -lr g / (|g| + eps). A correction
    # that used the wrong step, the wrong beta, or none at all breaks this from
    # step 2 on.
    g = np.array([3.0, -0.5, 1e-3, 2.0e-2])
    lr, eps = 0.01, 1e-8
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 11):
        p, m, v = mlp.adam(p, g, m, v, step=t, lr=lr, eps=eps)
        assert np.allclose(p, -t * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-12)
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12)


def test_adam_alternating_gradient_closed_form():
    # g_t = (-1)^(t+1) g: the squares stay constant (v_hat = g^2) while the
    # first moment is a geometric sum,
    #   m_t = (1 - b1) g (-1)^(t+1) (1 - (-b1)^t) / (1 + b1),
    # so the step t update is -lr (m_t / (1 - b1^t)) / (|g| + eps).
    b1 = 0.9
    g = np.array([1.5, -0.25])
    lr, eps = 1e-3, 1e-8
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    exp_p = np.zeros(2)
    for t in range(1, 9):
        gt = g if t % 2 == 1 else -g
        p, m, v = mlp.adam(p, gt, m, v, step=t, lr=lr, eps=eps)
        mt = (1 - b1) * g * (-1) ** (t + 1) * (1 - (-b1) ** t) / (1 + b1)
        assert np.allclose(m, mt, rtol=1e-12)
        exp_p = exp_p - lr * (mt / (1 - b1 ** t)) / (np.abs(g) + eps)
        assert np.allclose(p, exp_p, rtol=1e-12)


def test_features_hand_example():
    # an array of 1000 values against a bitset of 32768 (Fig. 1's first and third containers)
    f = mlp.features(1, 2, 1000, 32768, 0, 0, 0)
    exp = np.zeros(12)
    exp[0] = 1.0
    exp[4] = 1.0
    exp[6] = np.log2(1001) / 16
    exp[7] = np.log2(32769) / 16
    exp[10] = np.log2(32.768) / 16
    assert np.allclose(f, exp, rtol=1e-15)
    # run container (c=300, r=3, Fig. 1's second) against itself, op = ANDNOT
    f = mlp.features(3, 3, 300, 300, 3, 3, 3)
    assert f[2] == 1.0 and f[5] == 1.0 and f[8] == 2.0 / 16 and f[10] == 0.0 and f[11] == 1.0
