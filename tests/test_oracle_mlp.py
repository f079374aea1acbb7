"""Pins of the warm-start network oracle (CPU).  The analytic gradient is
checked against central finite differences of the loss, which share none of
its code; the loss against closed-form cases."""
import numpy as np

from oracle import mlp


def _problem(Q=3, hidden=5, N=7, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, Q, Q)) + 1j * rng.standard_normal((N, Q, Q))
    G = A @ np.conj(np.transpose(A, (0, 2, 1)))
    nb = mlp.gauge_fix(rng.standard_normal((N, Q)) + 1j * rng.standard_normal((N, Q)))
    c = rng.standard_normal((N, Q)) + 1j * rng.standard_normal((N, Q))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    theta = 0.5 * rng.standard_normal(mlp.param_count(Q, hidden))
    return G, nb, c, theta


def test_gradient_matches_finite_differences():
    Q, hidden = 3, 5
    G, nb, c, theta = _problem(Q, hidden)
    bound = 4.0
    L0, grad = mlp.batch_loss_and_grad(theta, G, nb, c, bound, Q, hidden)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp = mlp.batch_loss_and_grad(tp, G, nb, c, bound, Q, hidden)[0]
        lm = mlp.batch_loss_and_grad(tm, G, nb, c, bound, Q, hidden)[0]
        fd[i] = (lp - lm) / (2 * h)
    assert 0.0 < L0 < 1.0
    assert np.abs(grad - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


def test_loss_closed_forms():
    rng = np.random.default_rng(1)
    c = rng.standard_normal((4, 6)) + 1j * rng.standard_normal((4, 6))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    assert np.allclose(mlp.loss(c, c), 0.0, atol=1e-15)
    # any phase and scale of the target direction scores zero
    ph = np.exp(1j * rng.uniform(0, 6, 4))[:, None] * rng.uniform(0.1, 5, 4)[:, None]
    assert np.allclose(mlp.loss(ph * c, c), 0.0, atol=1e-14)
    # a vector orthogonal to the target scores one
    w = rng.standard_normal((4, 6)) + 1j * rng.standard_normal((4, 6))
    w -= np.sum(np.conj(c) * w, axis=1, keepdims=True) * c
    assert np.allclose(mlp.loss(w, c), 1.0, atol=1e-14)
    # cos^2 law: c_hat = cos t c + sin t w_unit -> L = sin^2 t
    wu = w / np.linalg.norm(w, axis=1, keepdims=True)
    t = np.array([0.1, 0.5, 1.0, 1.4])[:, None]
    assert np.allclose(mlp.loss(np.cos(t) * c + np.sin(t) * wu, c), np.sin(t[:, 0]) ** 2)


def test_zero_network_returns_the_neighbour():
    Q, hidden = 4, 8
    G, nb, _, _ = _problem(Q, hidden, seed=2)
    theta = np.zeros(mlp.param_count(Q, hidden))
    c_hat, _ = mlp.forward(theta, mlp.features(G, nb, 5.0), nb, Q, hidden)
    assert np.array_equal(c_hat, nb)


def test_features_layout():
    Q = 3
    G = np.zeros((1, Q, Q), complex)
    G[0] = [[1, 2 + 3j, 4 - 1j], [2 - 3j, 5, 6 + 2j], [4 + 1j, 6 - 2j, 7]]
    nb = np.array([[1 + 2j, 3 - 4j, 0.5j]])
    z = mlp.features(G, nb, 2.0)
    assert z.shape == (1, Q * Q + 2 * Q)
    assert np.allclose(z[0], [0.5, 2.5, 3.5, 1.0, 1.5, 2.0, -0.5, 3.0, 1.0,
                              1, 2, 3, -4, 0, 0.5])


def test_gauge_fix():
    rng = np.random.default_rng(4)
    v = rng.standard_normal((9, 5)) + 1j * rng.standard_normal((9, 5))
    f = mlp.gauge_fix(v)
    k = np.argmax(np.abs(v), axis=1)
    top = f[np.arange(9), k]
    assert np.allclose(top.imag, 0.0, atol=1e-15) and np.all(top.real > 0)
    assert np.allclose(np.abs(f), np.abs(v))
    assert np.allclose(mlp.gauge_fix(f), f)


def test_adam_first_step_is_a_sign_step():
    """With bias correction the first Adam step is -lr g / (|g| + eps)."""
    g = np.array([3.0, -0.2, 1e-3, -50.0])
    th, m, v = mlp.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, 0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
