"""Pins of the reference MLP (the learned terminator is not in the paper; these pin
the oracle to calculus and to the published Adam rule, not to itself)."""
import numpy as np

from oracle import mlp


def _data(seed=0, n=6):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(rng)
    x = rng.standard_normal((n, 64))
    t = rng.standard_normal((n, 448))
    return rng, p, x, t


def test_parameter_count():
    assert mlp.n_params() == 263360


def test_gradient_matches_central_differences():
    rng, p, x, t = _data()
    loss, g = mlp.loss_and_grad(p, x, t)
    idx = rng.choice(p.size, 40, replace=False)
    # include biases and every layer
    idx = np.concatenate([idx, [0, 64 * 256 + 3, 16384 + 256 + 5, p.size - 1, p.size - 449]])
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp = p.copy()
        pp[i] += h
        lp = mlp.loss_and_grad(pp, x, t)[0]
        pp[i] -= 2 * h
        lm = mlp.loss_and_grad(pp, x, t)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])


def test_first_adam_step_is_sign_step():
    """Kingma & Ba: after bias correction the first step is lr * g / (|g| + eps)."""
    _, p, x, t = _data(1)
    _, g = mlp.loss_and_grad(p, x, t)
    p1, m, v = mlp.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, 1e-3)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + mlp.ADAM_EPS), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_encode_decode_round_trip():
    rng = np.random.default_rng(3)
    a = rng.uniform(0.2, 1.4, (4, 300))
    b = rng.uniform(0.05, 0.3, (4, 300))
    x, t, c, s = mlp.encode(a, b)
    assert x.shape == (4, 64) and t.shape == (4, 448)
    ae, be = mlp.decode(t, a, b, c, s)
    assert np.allclose(ae, a[:, :256], rtol=0, atol=1e-14)
    assert np.allclose(be, b[:, :256], rtol=1e-14, atol=0)
    assert np.allclose(c, a[:, 16:32].mean(axis=1)) and np.allclose(s, b[:, 16:32].mean(axis=1))


def _fd_mismatch(p, x, t, g, idx):
    """Largest |finite difference - g| / max(|g|, 1e-3) over the parameters idx."""
    worst = 0.0
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp = p.copy()
        pp[i] += h
        lp = mlp.loss_and_grad(pp, x, t)[0]
        pp[i] -= 2 * h
        lm = mlp.loss_and_grad(pp, x, t)[0]
        worst = max(worst, abs((lp - lm) / (2 * h) - g[i]) / max(abs(g[i]), 1e-3))
    return worst


def test_planted_gradient_mistakes_are_caught():
    """The finite-difference pin must reject plausible backward-pass mistakes, planted here in
    a copy of the oracle's gradient: a sign flip in one layer's weights and a dropped bias
    gradient."""
    rng, p, x, t = _data(2)
    _, g = mlp.loss_and_grad(p, x, t)
    w2 = slice(64 * 256 + 256, 64 * 256 + 256 + 256 * 256)
    idx_w2 = rng.choice(np.arange(w2.start, w2.stop), 8, replace=False)
    assert _fd_mismatch(p, x, t, g, idx_w2) <= 1e-6
    bad = g.copy()
    bad[w2] *= -1.0
    assert _fd_mismatch(p, x, t, bad, idx_w2) > 0.5
    b4 = slice(p.size - 448, p.size)
    bad = g.copy()
    bad[b4] = 0.0
    assert _fd_mismatch(p, x, t, bad, np.arange(b4.start, b4.start + 8)) > 0.5


def test_zero_network_extends_with_the_constant_chain():
    """With every parameter zero the network outputs 0, which decodes to a_n = c and
    b_n = s for n >= 32: the constant chain the square-root terminator assumes."""
    rng = np.random.default_rng(5)
    a = rng.uniform(0.2, 1.4, (3, 32))
    b = rng.uniform(0.05, 0.3, (3, 32))
    x, _, c, s = mlp.encode(a, b)
    y, _ = mlp.forward(np.zeros(mlp.n_params()), x)
    ae, be = mlp.decode(y, a, b, c, s)
    assert np.array_equal(ae[:, :32], a) and np.array_equal(be[:, :32], b)
    assert np.allclose(ae[:, 32:], c[:, None], rtol=0, atol=1e-15)
    assert np.allclose(be[:, 32:], s[:, None], rtol=1e-15, atol=0)


def test_weighted_loss_gradient_matches_central_differences():
    """Per-output weights: the gradient of sum_j w_j (y_j - t_j)^2 / n against central
    differences, unit weights give the plain loss, and a gradient that forgets the weights
    (planted in a copy) fails the check."""
    rng, p, x, t = _data(4)
    w = rng.uniform(0.1, 3.0, 448)
    loss, g = mlp.loss_and_grad(p, x, t, w)
    idx = np.concatenate([rng.choice(p.size, 24, replace=False), [p.size - 1, p.size - 449]])
    worst = 0.0
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp = p.copy()
        pp[i] += h
        lp = mlp.loss_and_grad(pp, x, t, w)[0]
        pp[i] -= 2 * h
        lm = mlp.loss_and_grad(pp, x, t, w)[0]
        worst = max(worst, abs((lp - lm) / (2 * h) - g[i]) / max(abs(g[i]), 1e-3))
    assert worst <= 1e-6
    l1, g1 = mlp.loss_and_grad(p, x, t, np.ones(448))
    l0, g0 = mlp.loss_and_grad(p, x, t)
    assert abs(l1 - l0) <= 1e-15 * l0 and np.array_equal(g1, g0)
    _, g_unw = mlp.loss_and_grad(p, x, t)            # the planted mistake: weights dropped
    b4 = np.arange(p.size - 448, p.size - 440)
    bad = 0.0
    for i in b4:
        h = 1e-6
        pp = p.copy()
        pp[i] += h
        lp = mlp.loss_and_grad(pp, x, t, w)[0]
        pp[i] -= 2 * h
        lm = mlp.loss_and_grad(pp, x, t, w)[0]
        bad = max(bad, abs((lp - lm) / (2 * h) - g_unw[i]) / max(abs(g_unw[i]), 1e-3))
    assert bad > 0.05
