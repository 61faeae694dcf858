"""Pins of the oracle's negative-curvature step (Alg. 1, Sec. 5): the small PSD
subproblem over S for directions V, and solves that raise the rank by blocks.

The step is checked against things fixed independently of its own formula:
the closed-form one-direction step, the change of the augmented Lagrangian
itself (oracle.objective on the expanded factor), optimality under PSD
perturbations and a brute-force grid (both through that objective), and the
closed-form SDP values of cycles and complete graphs.
"""

import math

import numpy as np
import pytest

import gen
import oracle


def _point(kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "maxcut":
        p = oracle.maxcut_sdp(gen.er_graph(60, 200, seed, "gauss"))
        sigma = 1.7
    else:
        p = oracle.lovasz_sdp(gen.er_graph(40, 120, seed, "unit"))
        sigma = np.full(p.m, 5.0)
        sigma[0] = 2.0
    R = rng.standard_normal((p.n, 3)) / math.sqrt(p.n)
    y = rng.standard_normal(p.m)
    w = y - sigma * (oracle.amap(p, R) - p.b)
    return p, R, y, sigma, w


def _change(p, R, y, sigma, cols):
    """Augmented Lagrangian of [R, cols] minus that of R (the objective itself)."""
    return oracle.objective(p, np.concatenate([R, cols], axis=1), y, sigma) - oracle.objective(p, R, y, sigma)


def _sqrt_cols(V, S):
    lam, U = np.linalg.eigh(0.5 * (S + S.T))
    keep = lam > 0
    return V @ (U[:, keep] * np.sqrt(lam[keep]))


@pytest.mark.parametrize("kind", ["maxcut", "lovasz"])
def test_single_direction_is_the_closed_form(kind):
    p, R, y, sigma, w = _point(kind, 3)
    theta, v = oracle.min_eig(p, w, want_vector=True)
    assert theta < 0
    S, phi, cols = oracle.curvature_step(p, w, sigma, v[:, None])
    a = oracle.amap(p, v[:, None])
    s = max(0.0, -theta / float(np.dot(np.broadcast_to(sigma, a.shape) * a, a)))
    assert math.isclose(S[0, 0], s, rel_tol=1e-10)
    assert math.isclose(phi, 0.5 * theta * s, rel_tol=1e-9)  # theta s + kappa s^2 / 2 at s = -theta / kappa


@pytest.mark.parametrize("kind,q", [("maxcut", 3), ("lovasz", 4)])
def test_model_is_the_change_of_the_augmented_lagrangian(kind, q):
    p, R, y, sigma, w = _point(kind, 5)
    thetas, V = oracle.min_eigs(p, w, q)
    assert np.all(thetas < 0)
    S, phi, cols = oracle.curvature_step(p, w, sigma, V)
    d = _change(p, R, y, sigma, cols)
    f0 = oracle.objective(p, R, y, sigma)
    assert abs(d - phi) <= 1e-9 * (1.0 + abs(f0))
    assert phi < 0


@pytest.mark.parametrize("kind,q", [("maxcut", 3), ("lovasz", 3)])
def test_step_is_optimal_under_psd_perturbations(kind, q):
    p, R, y, sigma, w = _point(kind, 7)
    _, V = oracle.min_eigs(p, w, q)
    S, phi, cols = oracle.curvature_step(p, w, sigma, V)
    base = _change(p, R, y, sigma, cols)
    scale = 1e-9 * (1.0 + abs(oracle.objective(p, R, y, sigma)))
    rng = np.random.default_rng(11)
    trials = [S * (1 + 1e-3), S * (1 - 1e-3)]
    for _ in range(20):
        B = rng.standard_normal((q, q))
        trials.append(S + 1e-3 * np.trace(S) * (B @ B.T) / q)
        M = S + 1e-3 * np.trace(S) * 0.5 * (B + B.T)
        lam, U = np.linalg.eigh(M)
        trials.append((U * np.maximum(lam, 0)) @ U.T)
    for T in trials:
        assert _change(p, R, y, sigma, _sqrt_cols(V, T)) >= base - scale


def test_brute_force_grid_two_directions():
    p, R, y, sigma, w = _point("maxcut", 9)
    _, V = oracle.min_eigs(p, w, 2)
    S, phi, cols = oracle.curvature_step(p, w, sigma, V)
    amax = 2.0 * max(S[0, 0], S[1, 1]) + 1e-12
    best = math.inf
    for a in np.linspace(0, amax, 25):
        for c in np.linspace(0, amax, 25):
            lim = math.sqrt(a * c)
            for b in np.linspace(-lim, lim, 9):
                T = np.array([[a, b], [b, c]])
                best = min(best, _change(p, R, y, sigma, _sqrt_cols(V, T)))
    f0 = abs(oracle.objective(p, R, y, sigma))
    assert best >= phi - 1e-9 * (1.0 + f0)     # nothing on the grid beats the step
    assert best <= phi + 0.02 * abs(phi)        # and the grid gets close to it


@pytest.mark.parametrize("kind", ["maxcut", "lovasz"])
def test_more_directions_never_decrease_less(kind):
    p, R, y, sigma, w = _point(kind, 13)
    _, V = oracle.min_eigs(p, w, 4)
    phis = [oracle.curvature_step(p, w, sigma, V[:, :q])[1] for q in (1, 2, 4)]
    assert phis[1] <= phis[0] + 1e-12 and phis[2] <= phis[1] + 1e-12


def _solve_value(p, r, eps, **kw):
    opts = oracle.SolveOptions(eps_kkt=eps, r_max=max(r, p.n), max_outer=400, max_inner=2000, **kw)
    out = oracle.solve(p, gen.init_factor(p.n, r, 1), opts=opts)
    assert out["status"] == "converged", out["kkt"]
    return -out["kkt"]["pobj"], out


@pytest.mark.parametrize("n", [7, 9])
def test_block_rank_steps_reach_odd_cycle_values(n):
    val, out = _solve_value(oracle.maxcut_sdp(gen.cycle_graph(n)), 1, 1e-7, rank_block=3)
    assert math.isclose(val, n * (1 + math.cos(math.pi / n)) / 2, rel_tol=1e-6)


def test_block_rank_steps_complete_graph_and_lovasz():
    val, _ = _solve_value(oracle.maxcut_sdp(gen.complete_graph(6)), 1, 1e-7, rank_block=4)
    assert math.isclose(val, 9.0, rel_tol=1e-6)
    val, _ = _solve_value(oracle.lovasz_sdp(gen.cycle_graph(5)), 1, 1e-6, rank_block=2, sigma_edges=5.0)
    assert math.isclose(val, math.sqrt(5.0), rel_tol=1e-5)
