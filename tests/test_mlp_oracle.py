"""Pins of the FP64 reference of the learned root-solve guess (oracle/mlp_oracle.c)
against facts fixed outside it: central finite differences of its own loss,
a hand-evaluated forward pass with asymmetric weight placement (catches
transposed or shifted weight indices and wrong feature definitions), the
bracket property, and the closed form of Adam under a constant gradient."""
import math

import numpy as np
import pytest

import oracle as O

NH = 32
OW1, OB1, OW2, OB2, OW3, OB3 = 0, 128, 160, 1184, 1216, 1248


def _samples(n, seed):
    rng = np.random.default_rng(seed)
    E = np.exp(rng.uniform(math.log(1e-3), math.log(60.0), n))
    r = rng.uniform(0.0, 0.995, n)
    M = r * E
    lo = np.maximum(0.0, E - M * M / E)
    eps = lo + rng.uniform(0.0, 1.0, n) * (E - lo)
    return E, M, eps


def _params(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, O.mlp_nparam())


def test_layout_size():
    assert O.mlp_nparam() == NH * 4 + NH + NH * NH + NH + NH + 1 == 1249


def test_gradient_matches_central_differences():
    E, M, eps = _samples(40, 1)
    p = _params(2)
    L, g = O.mlp_loss_grad(p, E, M, eps)
    h = 1e-6
    fd = np.empty_like(p)
    for k in range(p.size):
        q = p.copy()
        q[k] += h
        lp, _ = O.mlp_loss_grad(q, E, M, eps)
        q[k] -= 2 * h
        lm, _ = O.mlp_loss_grad(q, E, M, eps)
        fd[k] = (lp - lm) / (2 * h)
    err = np.abs(fd - g).max() / np.abs(g).max()
    assert err < 1e-6, err
    assert L > 0


def test_loss_is_mean_squared_relative_error():
    E, M, eps = _samples(25, 3)
    p = _params(4)
    guess = O.mlp_forward(p, E, M)
    L, _ = O.mlp_loss_grad(p, E, M, eps)
    assert L == pytest.approx(np.mean(((guess - eps) / E) ** 2), rel=1e-12)


def test_forward_hand_evaluated():
    """Only hidden unit 5 of layer 1 and unit 3 of layer 2 are live, linked by
    W2[3][5]; a transposed W2, a W1 stored [4][32], or a wrong feature changes z."""
    p = np.zeros(O.mlp_nparam())
    w1 = np.array([0.7, -1.3, 0.4, 2.1])
    p[OW1 + 5 * 4: OW1 + 5 * 4 + 4] = w1
    p[OB1 + 5] = 0.25
    p[OW2 + 3 * NH + 5] = 1.7
    p[OB2 + 3] = -0.2
    p[OW3 + 3] = 2.5
    p[OB3] = -0.3
    E = np.array([0.05, 1.0, 7.5, 48.0])
    M = np.array([0.01, 0.6, 7.0, 10.0])
    out = O.mlp_forward(p, E, M)
    for k in range(E.size):
        r = M[k] / E[k]
        lo = max(0.0, E[k] - M[k] ** 2 / E[k])
        f = np.array([math.log(E[k]) / 5.0, r, r * r, math.log(max(lo / E[k], 1e-30)) / 10.0])
        h1 = math.tanh(0.25 + float(w1 @ f))
        h2 = math.tanh(-0.2 + 1.7 * h1)
        z = -0.3 + 2.5 * h2
        want = lo + (E[k] - lo) / (1.0 + math.exp(-z))
        assert out[k] == pytest.approx(want, rel=1e-14)


def test_guess_stays_in_the_bracket():
    E, M, _ = _samples(500, 5)
    M[:20] = 0.0                 # no flow: lo = E, the guess is the root E itself
    M[20:40] = 1.5 * E[20:40]    # M > E: lo = 0
    g = O.mlp_forward(_params(6, scale=3.0), E, M)
    lo = np.maximum(0.0, E - M * M / E)
    assert np.all(g >= lo) and np.all(g <= E)
    np.testing.assert_array_equal(g[:20], E[:20])


@pytest.mark.parametrize("lr,b1,b2", [(1e-3, 0.9, 0.999), (5e-2, 0.5, 0.9)])
def test_adam_constant_gradient_closed_form(lr, b1, b2):
    """With a constant gradient g the bias-corrected moments equal g and g^2 at
    every step, so each step moves a parameter by lr g / (|g| + epsilon)."""
    rng = np.random.default_rng(7)
    n = O.mlp_nparam()
    p0 = rng.normal(size=n)
    g = rng.normal(size=n)
    g[:5] = 0.0
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    eps = 1e-8
    for t in (1, 2, 3):
        O.mlp_adam(p, g, m, v, t, lr=lr, b1=b1, b2=b2, epsilon=eps)
        want = p0 - t * lr * g / (np.abs(g) + eps)
        np.testing.assert_allclose(p, want, rtol=0, atol=1e-12)
    assert np.all(p[:5] == p0[:5])


def test_adam_reduces_the_loss():
    # learnable targets: the root for P = e/3, e = -E + sqrt(4E^2 - 3M^2)
    E, M, _ = _samples(400, 8)
    eps = -E + np.sqrt(4 * E * E - 3 * M * M)
    p = _params(9, scale=0.3)
    m, v = np.zeros_like(p), np.zeros_like(p)
    L0, _ = O.mlp_loss_grad(p, E, M, eps)
    for t in range(1, 201):
        _, g = O.mlp_loss_grad(p, E, M, eps)
        O.mlp_adam(p, g, m, v, t, lr=1e-2)
    L1, _ = O.mlp_loss_grad(p, E, M, eps)
    assert L1 < 0.1 * L0, (L0, L1)
