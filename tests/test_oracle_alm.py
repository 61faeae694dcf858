"""Pins for the oracle's solve path: the quartic line search, and solve values
against closed forms (MaxCut on cycles/complete/bipartite graphs, Lovasz theta
of cycles/complete/edgeless graphs), brute-force max cuts, an independent dense
convex ALM, and the ALM theory invariants of Sec. 2.3."""

import math

import numpy as np
import pytest

import gen
import oracle
from oracle.dense_alm import dense_alm


def _problems():
    rng = np.random.default_rng(5)
    g = gen.er_graph(10, 18, 2, "gauss")
    yield oracle.maxcut_sdp(g), rng
    yield oracle.lovasz_sdp(gen.er_graph(9, 12, 3)), rng
    mats = []
    for _ in range(4):
        A = rng.standard_normal((8, 8))
        mats.append(A + A.T)
    yield oracle.generic_sdp(np.diag(rng.standard_normal(8)), mats, rng.standard_normal(4)), rng


def test_quartic_coefficients_reproduce_objective_along_the_ray():
    for p, rng in _problems():
        R = rng.standard_normal((p.n, 3))
        y = rng.standard_normal(p.m)
        sigma = 1.3
        f, G, a, P = oracle.objective_grad(p, R, y, sigma)
        k = oracle.line_search_coeffs(p, R, G, y, sigma, P, a)
        for t in [0.0, 0.01, 0.1, 0.37, 1.0]:
            direct = oracle.objective(p, R - t * G, y, sigma)
            poly = sum(k[i] * t ** i for i in range(5))
            assert math.isclose(poly, direct, rel_tol=1e-11, abs_tol=1e-11 * (1 + abs(direct)))
        # phi'(0) is the directional derivative <grad, -G> = -||G||^2
        assert math.isclose(k[1], -np.sum(G * G), rel_tol=1e-11)


def test_quartic_argmin_against_dense_grid():
    rng = np.random.default_rng(11)
    for _ in range(200):
        k = rng.standard_normal(5)
        k[4] = abs(k[4]) + 1e-3
        k[1] = -abs(k[1])
        t = oracle.quartic_argmin(k)
        grid = np.linspace(0.0, 20.0, 200001)
        vals = k[0] + grid * (k[1] + grid * (k[2] + grid * (k[3] + grid * k[4])))
        tg = grid[np.argmin(vals)]
        phi = lambda s: k[0] + s * (k[1] + s * (k[2] + s * (k[3] + s * k[4])))
        assert phi(t) <= phi(tg) + 1e-12 * (1 + abs(phi(tg)))
        assert t >= 0.0


def test_quartic_argmin_degenerate_cases():
    assert oracle.quartic_argmin(np.array([1.0, 0.0, 0.0, 0.0, 0.0])) == 0.0
    # convex quadratic: minimiser -k1/(2 k2)
    assert math.isclose(oracle.quartic_argmin(np.array([0.0, -2.0, 0.5, 0.0, 0.0])), 2.0, rel_tol=1e-14)
    # unbounded below along the ray: no step
    assert oracle.quartic_argmin(np.array([0.0, -1.0, -1.0, 0.0, 0.0])) == 0.0


def _solve_value(p, r, eps=1e-8, seed=1, **kw):
    R0 = gen.init_factor(p.n, r, seed)
    opts = oracle.SolveOptions(eps_kkt=eps, r_max=max(r, p.n), max_outer=400, max_inner=2000, **kw)
    out = oracle.solve(p, R0, opts=opts)
    assert out["status"] == "converged", out["kkt"]
    return -out["kkt"]["pobj"], out


@pytest.mark.parametrize("n", [6, 8, 10])
def test_maxcut_even_cycle(n):
    val, _ = _solve_value(oracle.maxcut_sdp(gen.cycle_graph(n)), 2)
    assert math.isclose(val, n, rel_tol=1e-6)


@pytest.mark.parametrize("n", [5, 7, 9])
def test_maxcut_odd_cycle(n):
    val, _ = _solve_value(oracle.maxcut_sdp(gen.cycle_graph(n)), 2)
    assert math.isclose(val, n * (1 + math.cos(math.pi / n)) / 2, rel_tol=1e-6)


def test_maxcut_complete_graph():
    n = 6
    val, _ = _solve_value(oracle.maxcut_sdp(gen.complete_graph(n)), 3)
    assert math.isclose(val, n * n / 4, rel_tol=1e-6)


def test_maxcut_complete_bipartite():
    g = gen.complete_bipartite_graph(3, 4)
    val, _ = _solve_value(oracle.maxcut_sdp(g), 2)
    assert math.isclose(val, 12.0, rel_tol=1e-6)


def _brute_maxcut(g):
    n = g.n
    best = -math.inf
    for bits in range(1 << (n - 1)):
        s = np.array([1 if (bits >> i) & 1 else -1 for i in range(n)])
        cut = float(np.sum(g.w * (s[g.ei] != s[g.ej])))
        best = max(best, cut)
    return best


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_maxcut_brute_force_sandwich_unit_weights(seed):
    g = gen.er_graph(12, 26, seed, "unit")
    sdp, _ = _solve_value(oracle.maxcut_sdp(g), 4, eps=1e-7)
    mc = _brute_maxcut(g)
    assert mc <= sdp * (1 + 1e-6)
    assert mc >= 0.87856 * sdp


def test_maxcut_brute_force_upper_bound_signed_weights():
    g = gen.er_graph(12, 30, 9, "pm1")
    sdp, _ = _solve_value(oracle.maxcut_sdp(g), 4, eps=1e-7)
    assert _brute_maxcut(g) <= sdp * (1 + 1e-6) + 1e-9


@pytest.mark.parametrize("n,expect", [
    (5, math.sqrt(5.0)),
    (7, 7 * math.cos(math.pi / 7) / (1 + math.cos(math.pi / 7))),
    (6, 3.0),
])
def test_lovasz_theta_cycles(n, expect):
    val, _ = _solve_value(oracle.lovasz_sdp(gen.cycle_graph(n)), 3, eps=1e-6)
    assert math.isclose(val, expect, rel_tol=1e-5)


def test_lovasz_theta_complete_and_edgeless():
    v1, _ = _solve_value(oracle.lovasz_sdp(gen.complete_graph(5)), 3)
    assert math.isclose(v1, 1.0, rel_tol=1e-6)
    v2, _ = _solve_value(oracle.lovasz_sdp(gen.edgeless_graph(6)), 2)
    assert math.isclose(v2, 6.0, rel_tol=1e-6)


def test_dense_alm_closed_forms():
    out = dense_alm(oracle.maxcut_sdp(gen.cycle_graph(5)), eps=1e-9)
    assert math.isclose(-out["pobj"], 5 * (1 + math.cos(math.pi / 5)) / 2, rel_tol=1e-7)
    out = dense_alm(oracle.lovasz_sdp(gen.cycle_graph(5)), eps=1e-9)
    assert math.isclose(-out["pobj"], math.sqrt(5.0), rel_tol=1e-7)


@pytest.mark.parametrize("weights", ["gauss", "pm1"])
def test_bm_solve_matches_dense_convex_alm(weights):
    g = gen.er_graph(14, 30, 4, weights)
    p = oracle.maxcut_sdp(g)
    bm, _ = _solve_value(p, 3, eps=1e-8)
    dn = dense_alm(p, eps=1e-9)
    assert math.isclose(bm, -dn["pobj"], rel_tol=1e-6)


def test_alm_proximity_and_nonexpansiveness_on_even_cycle():
    """Sec. 2.3: for the exact subproblem solution X at y and its dual update z,
    ||A X - b|| <= ||y - y*|| / rho and ||z - y*|| <= ||y - y*||, with y* = -1 for
    the even cycle in minimisation form.  Exact subproblems come from the dense ALM
    run for a single outer step."""
    n = 8
    p = oracle.maxcut_sdp(gen.cycle_graph(n))
    ystar = -np.ones(n)
    rng = np.random.default_rng(3)
    for rho in [0.5, 1.0, 3.0]:
        y = ystar + 0.5 * rng.standard_normal(n)
        out = dense_alm(p, sigma=rho, max_outer=1, y0=y, inner_tol=1e-14)
        X, z = out["X"], out["y"]
        res = np.diag(X) - 1.0
        assert np.linalg.norm(res) <= np.linalg.norm(y - ystar) / rho * (1 + 1e-6)
        assert np.linalg.norm(z - ystar) <= np.linalg.norm(y - ystar) * (1 + 1e-6)


def test_rank_expansion_step_is_exact_minimiser():
    """p = 1 case of the small SDP of Alg. 1: L(X + s v v^T) = L(X) + s theta + (sigma/2) s^2 ||A(vv^T)||^2,
    minimised over s >= 0 at s* = max(0, -theta / (sigma ||A(vv^T)||^2))."""
    g = gen.er_graph(30, 80, 6, "gauss")
    p = oracle.maxcut_sdp(g)
    R = gen.init_factor(30, 2, 4)
    y = np.zeros(30)
    sigma = 1.0
    f, G, a, _ = oracle.objective_grad(p, R, y, sigma)
    w = y - sigma * (a - p.b)
    theta, v = oracle.min_eig(p, w, want_vector=True)
    assert theta < 0
    s_star = max(0.0, -theta / (sigma * oracle.rank_one_norm2(p, v)))

    def L(s):
        return oracle.objective(p, np.concatenate([R, math.sqrt(s) * v[:, None]], axis=1), y, sigma)

    base = oracle.objective(p, R, y, sigma)
    for s in [0.1 * s_star, 0.5 * s_star, s_star, 2 * s_star]:
        pred = base + s * theta + 0.5 * sigma * s * s * oracle.rank_one_norm2(p, v)
        assert math.isclose(L(s), pred, rel_tol=1e-10, abs_tol=1e-10)
    assert L(s_star) <= min(L(0.9 * s_star), L(1.1 * s_star))


def test_quartic_with_one_penalty_per_constraint():
    """With a penalty vector (trace row sigma, edge rows sigma_e) the quartic
    still reproduces sum_i sigma_i/2 res_i^2 along the ray, and phi'(0) = -||G||^2."""
    p = oracle.lovasz_sdp(gen.er_graph(12, 20, 4))
    rng = np.random.default_rng(8)
    R = rng.standard_normal((p.n, 3))
    y = rng.standard_normal(p.m)
    sig = np.full(p.m, 37.0)
    sig[0] = 1.3
    f, G, a, P = oracle.objective_grad(p, R, y, sig)
    k = oracle.line_search_coeffs(p, R, G, y, sig, P, a)
    for t in [0.0, 0.02, 0.1, 0.5]:
        Rt = R - t * G
        at = oracle.amap(p, Rt)
        direct = (float(np.sum(Rt * oracle.cost_apply(p, Rt))) + float(np.dot(y, p.b - at))
                  + 0.5 * float(np.sum(sig * (at - p.b) ** 2)))
        poly = sum(k[i] * t ** i for i in range(5))
        assert math.isclose(poly, direct, rel_tol=1e-11, abs_tol=1e-11 * (1 + abs(direct)))
    assert math.isclose(k[1], -np.sum(G * G), rel_tol=1e-11)


def test_rank_step_with_one_penalty_per_constraint():
    """L(X + s vv^T) = L(X) + s theta + s^2/2 sum_i sigma_i a_i(vv^T)^2, minimised at
    s* = -theta / sum_i sigma_i a_i(vv^T)^2."""
    p = oracle.lovasz_sdp(gen.er_graph(15, 30, 5))
    R = gen.init_factor(15, 2, 3) / math.sqrt(15)
    y = np.zeros(p.m)
    sig = np.full(p.m, 15.0)
    sig[0] = 1.0
    f, G, a, _ = oracle.objective_grad(p, R, y, sig)
    w = y - sig * (a - p.b)
    theta, v = oracle.min_eig(p, w, want_vector=True)
    assert theta < 0
    av = oracle.amap(p, v[:, None])
    curv = float(np.dot(sig * av, av))
    base = oracle.objective(p, R, y, sig)
    for s in [0.3, 1.0, 2.0]:
        s = s * (-theta / curv)
        val = oracle.objective(p, np.concatenate([R, math.sqrt(s) * v[:, None]], axis=1), y, sig)
        assert math.isclose(val, base + s * theta + 0.5 * s * s * curv, rel_tol=1e-10, abs_tol=1e-10)


@pytest.mark.parametrize("n,expect", [
    (5, math.sqrt(5.0)),
    (7, 7 * math.cos(math.pi / 7) / (1 + math.cos(math.pi / 7))),
])
def test_lovasz_theta_cycles_with_edge_penalty(n, expect):
    val, _ = _solve_value(oracle.lovasz_sdp(gen.cycle_graph(n)), 3, eps=1e-6, sigma_edges=float(n))
    assert math.isclose(val, expect, rel_tol=1e-5)


@pytest.mark.parametrize("n", [7, 9])
def test_penalty_schedule_odd_cycle(n):
    """Started at a penalty far too small to move the multipliers, the schedule
    (sigma x10 whenever pinf falls by less than 4x) still reaches the closed
    form, with a non-decreasing penalty; without it the penalty stays put."""
    p = oracle.maxcut_sdp(gen.cycle_graph(n))
    val, out = _solve_value(p, 2, eps=1e-7, sigma=1e-3, sigma_growth=10.0)
    assert math.isclose(val, n * (1 + math.cos(math.pi / n)) / 2, rel_tol=1e-6)
    s = [h["sigma"] for h in out["history"]]
    assert s[0] == 1e-3 and s[-1] > s[0]
    assert all(b >= a for a, b in zip(s, s[1:]))
    _, fixed = _solve_value(p, 2, eps=1e-7)
    assert {h["sigma"] for h in fixed["history"]} == {1.0}


def test_penalty_schedule_keeps_the_edge_ratio():
    """Lovasz theta of C5 with one penalty for the trace row and another for
    the edge rows: the schedule scales both, keeping their ratio (here 5)."""
    val, out = _solve_value(oracle.lovasz_sdp(gen.cycle_graph(5)), 3, eps=1e-6, sigma=0.01, sigma_edges=0.05,
                            sigma_growth=10.0, sigma_max=100.0)
    assert math.isclose(val, math.sqrt(5.0), rel_tol=1e-5)
    s = [h["sigma"] for h in out["history"]]
    assert s[-1] > s[0] and max(s) <= 100.0


@pytest.mark.parametrize("n", [7, 9])
def test_lbfgs_inner_solver_odd_cycles(n):
    """The L-BFGS subproblem solver (exact quartic line search along its
    directions) reaches the same closed forms as gradient descent."""
    val, _ = _solve_value(oracle.maxcut_sdp(gen.cycle_graph(n)), 2, inner_solver="lbfgs")
    assert math.isclose(val, n * (1 + math.cos(math.pi / n)) / 2, rel_tol=1e-6)


def test_lbfgs_inner_solver_complete_graph_and_lovasz():
    val, _ = _solve_value(oracle.maxcut_sdp(gen.complete_graph(6)), 3, inner_solver="lbfgs")
    assert math.isclose(val, 9.0, rel_tol=1e-6)
    val, _ = _solve_value(oracle.lovasz_sdp(gen.cycle_graph(5)), 3, eps=1e-6, sigma_edges=5.0, inner_solver="lbfgs")
    assert math.isclose(val, math.sqrt(5.0), rel_tol=1e-5)


def test_lbfgs_and_gd_solves_agree_on_a_random_graph():
    """Both subproblem solvers reach one SDP value on G(300, 1200) with N(0,1)
    weights, and L-BFGS does not need more gradient evaluations."""
    p = oracle.maxcut_sdp(gen.er_graph(300, 1200, 3, "gauss"))
    vals = {}
    for solver in ("gd", "lbfgs"):
        val, out = _solve_value(p, 4, eps=1e-7, inner_solver=solver)
        vals[solver] = (val, sum(h["inner_iters"] for h in out["history"]))
    assert math.isclose(vals["gd"][0], vals["lbfgs"][0], rel_tol=1e-6)
    assert vals["lbfgs"][1] <= vals["gd"][1]


def test_inner_gradient_descent_tail_is_log_linear():
    """Sec. 4 (local linear convergence of gradient descent on the subproblem
    under quadratic growth): started near a solution of the 9-cycle at a nearby
    dual, the gradient norm of the exact-step descent falls by a roughly
    constant factor per 25 steps (each factor < 0.5, largest / smallest < 3)."""
    p = oracle.maxcut_sdp(gen.cycle_graph(9))
    sol = oracle.solve(p, gen.init_factor(9, 2, 1), opts=oracle.SolveOptions(eps_kkt=1e-8, max_outer=400,
                                                                              max_inner=3000))
    assert sol["status"] == "converged"
    rng = np.random.default_rng(1)
    y = sol["y"] + 0.05 * rng.standard_normal(9)
    R0 = sol["R"] + 0.05 * rng.standard_normal(sol["R"].shape)
    g = [oracle.inner_gd(p, R0, y, 1.0, 0.0, k)[1]["gnorm"] for k in (25, 50, 75, 100, 125, 150)]
    ratios = [b / a for a, b in zip(g, g[1:])]
    assert all(q < 0.5 for q in ratios)
    assert max(ratios) / min(ratios) < 3.0
