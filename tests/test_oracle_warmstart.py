"""Pins for the oracle's warm-start pieces: hand-computed features, a network
with a closed-form output, and finite differences of the loss."""

import math

import numpy as np

import gen
import oracle
from oracle import warmstart as ows


def test_features_on_a_weighted_path():
    """Path 0-1-2 with w01 = 2, w12 = -1: C = -L/4 has S01 = 0.5, S12 = -0.25,
    d = (-0.5, -0.25, 0.25)."""
    g = gen.Graph(3, np.array([0, 1]), np.array([1, 2]), np.array([2.0, -1.0]))
    f = ows.features(oracle.maxcut_sdp(g))
    l1, l2 = math.log(2.0), math.log(3.0)
    expect = np.array([
        [l1, 0.5, 0.5, -0.5, -1.0, l2, l2, 0.75],
        [l2, 0.75, 0.25, -0.25, -1.0, l1, l1, 0.375],
        [l1, 0.25, -0.25, 0.25, 0.0, l2, l2, 0.75],
    ])
    np.testing.assert_allclose(f, expect, rtol=0, atol=1e-15)


def test_features_isolated_vertex_is_zero_apart_from_diagonal():
    g = gen.Graph(4, np.array([0]), np.array([1]), np.array([1.0]))
    f = ows.features(oracle.maxcut_sdp(g))
    assert np.all(f[2:] == 0.0)


def test_mlp_forward_closed_form():
    """n_in = 2, h = 2, W1 = I, b1 = 0, W2 = [[1,0],[0,0]], b2 = (0, 0.5),
    W3 = (2, 3), b3 = -1: x = (3, -4) -> 2*3 + 3*0.5 - 1 = 6.5 and
    x = (-1, 2) -> 3*0.5 - 1 = 0.5."""
    params = np.array([1, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0.5, 2, 3, -1], dtype=float)
    assert params.size == ows.param_count(2, 2)
    out = ows.mlp_forward(params, 2, 2, np.zeros(8), np.ones(8), np.array([[3.0, -4.0], [-1.0, 2.0]]))
    np.testing.assert_allclose(out, [6.5, 0.5], rtol=0, atol=1e-15)


def test_mlp_gradient_central_differences():
    rng = np.random.default_rng(0)
    nin, h, n = 3, 4, 25
    params = rng.standard_normal(ows.param_count(nin, h)) * 0.7
    mu = rng.standard_normal(8)
    isd = 0.5 + rng.random(8)
    X = rng.standard_normal((n, nin))
    T = rng.standard_normal(n)
    loss, grad = ows.mlp_loss_grad(params, nin, h, mu, isd, X, T)
    assert math.isclose(loss, np.mean((ows.mlp_forward(params, nin, h, mu, isd, X) - T) ** 2), rel_tol=1e-14)
    eps = 1e-6
    fd = np.zeros_like(params)
    for k in range(params.size):
        e = np.zeros_like(params)
        e[k] = eps
        lp, _ = ows.mlp_loss_grad(params + e, nin, h, mu, isd, X, T)
        lm, _ = ows.mlp_loss_grad(params - e, nin, h, mu, isd, X, T)
        fd[k] = (lp - lm) / (2 * eps)
    assert np.linalg.norm(grad - fd) <= 1e-7 * np.linalg.norm(grad)
