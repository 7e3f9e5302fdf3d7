"""Pins of the float64 network reference: the forward pass against closed
forms of single-path parameter blocks, the features against a hand-computed
case and their definition's invariances, the chain-rule gradients against
central differences."""
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


# Offsets of the parameter block (the layout the C header documents).
W1, B1, W2, B2, W3, B3, MEAN, STD = 0, 192, 224, 1248, 1280, 1312, 1313, 1319


def _one_path_block(k, j1, j2, a, b, c, d, e, f, mu, sigma):
    """Parameters with a single active path: input slot k -> hidden unit j1 of
    layer 1 -> hidden unit j2 of layer 2 -> output."""
    P = np.zeros(1325)
    P[STD:STD + 6] = 1.0
    P[W1 + 6 * j1 + k] = a        # W1[j1][k]
    P[B1 + j1] = b
    P[W2 + 32 * j2 + j1] = c      # W2[j2][j1]
    P[B2 + j2] = d
    P[W3 + j2] = e
    P[B3] = f
    P[MEAN + k] = mu
    P[STD + k] = sigma
    return P


def test_forward_closed_form_per_input_slot():
    """With one active unit per layer the network is the scalar composition
    y = e tanh(c tanh(a (x_k - mu)/sigma + b) + d) + f, whatever the other
    inputs are.  One block per input slot fixes the weight layout (a transposed
    W1 or W2 reads a zero), the direction of standardisation ((x - mu)/sigma,
    not (x - mu) sigma) and which feature slot feeds which column."""
    rng = np.random.default_rng(11)
    x = rng.normal(size=(9, 6))
    for k in range(6):
        j1, j2 = (5 * k + 3) % 32, (7 * k + 11) % 32
        a, b, c, d, e, f, mu, sigma = 0.7, -0.2, 1.3, 0.1, -0.9, 0.25, 0.3, 2.5
        P = _one_path_block(k, j1, j2, a, b, c, d, e, f, mu, sigma)
        want = [e * np.tanh(c * np.tanh(a * (xs[k] - mu) / sigma + b) + d) + f for xs in x]
        np.testing.assert_allclose(mlp.forward(P, x), want, rtol=1e-14, atol=1e-15)
    # the bias-only network ignores its input: y = e tanh(c tanh(b) + d) + f
    P = _one_path_block(0, 4, 9, 0.0, 0.5, -1.1, 0.3, 2.0, -0.4, 0.0, 1.0)
    np.testing.assert_allclose(mlp.forward(P, x), 2.0 * np.tanh(-1.1 * np.tanh(0.5) + 0.3) - 0.4,
                               rtol=1e-14)


def test_features_of_a_hand_computed_case():
    """rho_L = 3, rho_R = 1 (mean 2), p_L = 1, p_R = 3 (mean 2), gamma = 1.4 so
    cbar = sqrt(1.4 * 2 / 2) = sqrt(1.4); u_L = 2 sqrt(1.4), u_R = -sqrt(1.4)/2.
    Features: ln(3/2), ln(1/2), ln(1/2), ln(3/2), 2, -1/2, in that order."""
    s = np.sqrt(1.4)
    x, pbar = mlp.features([[3.0, 2.0 * s, 1.0]], [[1.0, -0.5 * s, 3.0]], gamma=1.4)
    np.testing.assert_allclose(x[0], [0.4054651081081644, -0.6931471805599453, -0.6931471805599453,
                                      0.4054651081081644, 2.0, -0.5], rtol=1e-14, atol=1e-15)
    assert pbar[0] == 2.0


def test_backward_matches_central_differences_of_the_weighted_output():
    """backward(P, x, dy) is the gradient of sum_s dy_s y_s."""
    rng = np.random.default_rng(12)
    P = _params(5)
    x = rng.normal(size=(23, 6))
    dy = rng.normal(size=23)
    g = mlp.backward(P, x, dy)
    h = 1e-6
    for k in list(range(0, 1313, 11)) + [191, 223, 1247, 1279, 1311, 1312]:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (dy @ mlp.forward(Pp, x) - dy @ mlp.forward(Pm, x)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * (1 + abs(fd)), (k, fd, g[k])


def test_loss_gradient_is_backward_of_the_residual():
    rng = np.random.default_rng(13)
    P = _params(6)
    x = rng.normal(size=(31, 6))
    t = rng.normal(size=31)
    dy = 2.0 * (mlp.forward(P, x) - t) / len(t)
    np.testing.assert_allclose(mlp.loss_grad(P, x, t), mlp.backward(P, x, dy), rtol=1e-13, atol=1e-16)
