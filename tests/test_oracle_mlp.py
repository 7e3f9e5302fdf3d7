"""Pins of the float64 network reference: the chain-rule gradient against
central differences, the features against their definition's invariances."""
import numpy as np

from oracle import mlp


def _params(seed=0):
    rng = np.random.default_rng(seed)
    P = rng.normal(scale=0.4, size=1325)
    P[1313:1319] = rng.normal(scale=0.1, size=6)
    P[1319:1325] = rng.uniform(0.5, 2.0, size=6)
    return P


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    P = _params()
    x = rng.normal(size=(37, 6))
    t = rng.normal(size=37)
    g = mlp.loss_grad(P, x, t)
    h = 1e-6
    for k in list(range(0, 1313, 7)) + [1312, 191, 223, 1247, 1279]:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (mlp.loss(Pp, x, t) - mlp.loss(Pm, x, t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * (1 + abs(fd)), (k, fd, g[k])


def test_features_invariances():
    """Galilean shift and scalings (rho, u, p) -> (A rho, B u, A B^2 p) move the
    velocity features by a shift/scale only; the thermodynamic ones are
    invariant."""
    rng = np.random.default_rng(2)
    WL = np.stack([rng.uniform(0.1, 5, 50), rng.uniform(-2, 2, 50), rng.uniform(0.1, 5, 50)], 1)
    WR = np.stack([rng.uniform(0.1, 5, 50), rng.uniform(-2, 2, 50), rng.uniform(0.1, 5, 50)], 1)
    x, pbar = mlp.features(WL, WR)
    A, B = 2.5, 0.3
    sc = np.array([A, B, A * B * B])
    xs, pbs = mlp.features(WL * sc, WR * sc)
    np.testing.assert_allclose(xs, x, atol=1e-12)
    np.testing.assert_allclose(pbs, A * B * B * pbar, rtol=1e-14)
    assert np.all(np.abs(x[:, 0:2]).max() < 10)


def test_adam_first_step_moves_by_lr():
    P = _params()
    g = np.random.default_rng(3).normal(size=1313)
    P2, m, v = mlp.adam(P, g, np.zeros(1313), np.zeros(1313), 1, lr=1e-3)
    # first bias-corrected step is lr * sign(g) up to eps
    np.testing.assert_allclose(P2[:1313] - P[:1313], -1e-3 * np.sign(g), rtol=1e-4, atol=1e-9)
    np.testing.assert_array_equal(P2[1313:], P[1313:])
