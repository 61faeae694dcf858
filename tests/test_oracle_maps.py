"""Pins for the oracle's per-call quantities (f, G, A(RR^T), A*, lambda_min, KKT).

Each test checks the oracle against something other than itself: the
definitions written out as explicit matrices, finite differences, the worked
examples of Sec. 3.3 and Sec. 4.3 of the paper, or closed-form spectra.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle


def _rand_sym_sparse(n, density, rng):
    A = sp.random(n, n, density=density, random_state=rng, format="csr")
    A = A + A.T
    A.data = rng.standard_normal(A.data.shape[0])
    A = A + A.T
    return sp.csr_matrix(A)


def _explicit_A(p):
    """A_i written out from the constraint definitions (not from oracle code)."""
    n = p.n
    mats = []
    if p.kind == "diag":
        for i in range(n):
            E = np.zeros((n, n))
            E[i, i] = 1.0
            mats.append(E)
    elif p.kind == "edges":
        mats.append(p.c_tr * np.eye(n))
        for i, j in zip(p.ei, p.ej):
            E = np.zeros((n, n))
            E[i, j] = E[j, i] = 0.5
            mats.append(E)
    else:
        mats = [a.toarray() for a in p.A]
    return mats


def _dense_C(p):
    return p.C.toarray() - p.j_coef * np.ones((p.n, p.n))


def _problems(rng):
    n = 9
    g = gen.er_graph(n, 14, 7, "gauss")
    yield oracle.maxcut_sdp(g)
    Cs = _rand_sym_sparse(n, 0.3, rng)
    yield oracle.edges_sdp(n, Cs, rng.standard_normal(g.m_edges + 1), 0.7, g.ei, g.ej, j_coef=0.3)
    A_list = [np.asarray(_rand_sym_sparse(n, 0.4, rng).todense()) for _ in range(5)]
    yield oracle.generic_sdp(Cs.toarray(), A_list, rng.standard_normal(5))


def test_maps_match_explicit_definitions():
    rng = np.random.default_rng(0)
    for p in _problems(rng):
        R = rng.standard_normal((p.n, 3))
        X = R @ R.T
        mats = _explicit_A(p)
        a_explicit = np.array([np.sum(Ai * X) for Ai in mats])
        np.testing.assert_allclose(oracle.amap(p, R), a_explicit, rtol=1e-13, atol=1e-13)
        w = rng.standard_normal(p.m)
        Astar = sum(wi * Ai for wi, Ai in zip(w, mats))
        np.testing.assert_allclose(oracle.adjoint_apply(p, w, R), Astar @ R, rtol=1e-12, atol=1e-12)
        C = _dense_C(p)
        np.testing.assert_allclose(oracle.cost_apply(p, R), C @ R, rtol=1e-12, atol=1e-12)
        assert math.isclose(oracle.cost_fro_norm(p), np.linalg.norm(C), rel_tol=1e-12)
        y = rng.standard_normal(p.m)
        sigma = 1.7
        f_explicit = np.sum(C * X) + y @ (p.b - a_explicit) + 0.5 * sigma * np.sum((a_explicit - p.b) ** 2)
        assert math.isclose(oracle.objective(p, R, y, sigma), f_explicit, rel_tol=1e-12, abs_tol=1e-12)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    for p in _problems(rng):
        R = rng.standard_normal((p.n, 3))
        y = rng.standard_normal(p.m)
        sigma = 0.9
        f, G, a, P = oracle.objective_grad(p, R, y, sigma)
        h = 1e-6
        Gfd = np.zeros_like(R)
        for i in range(R.shape[0]):
            for j in range(R.shape[1]):
                E = np.zeros_like(R)
                E[i, j] = h
                Gfd[i, j] = (oracle.objective(p, R + E, y, sigma) - oracle.objective(p, R - E, y, sigma)) / (2 * h)
        assert np.linalg.norm(G - Gfd) <= 1e-7 * np.linalg.norm(G)


def test_quadratic_growth_counterexample_value():
    """Sec. 3.3, prop. on the necessity of localness for quadratic growth:
    C = 0, A_1 = E_11, A_2 = E_22, b = (0, 1), y = (-eps, 0); for
    X = [[delta, sqrt(delta)], [sqrt(delta), 1]] = R R^T with R = (sqrt(delta), 1)^T,
    L(X, y) - L(X*, y) = eps*delta + rho*delta^2/2 exactly."""
    C = sp.csr_matrix((2, 2))
    p = oracle.SDP(n=2, kind="diag", b=np.array([0.0, 1.0]), C=C)
    Rstar = np.array([[0.0], [1.0]])
    for eps, rho, delta in [(0.3, 1.0, 0.25), (0.01, 2.5, 0.04), (0.0, 0.7, 0.09)]:
        y = np.array([-eps, 0.0])
        R = np.array([[math.sqrt(delta)], [1.0]])
        d = oracle.objective(p, R, y, rho) - oracle.objective(p, Rstar, y, rho)
        assert math.isclose(d, eps * delta + rho * delta ** 2 / 2, rel_tol=1e-13, abs_tol=1e-15)


def _high_rank_example(r, n):
    """The SDP of the prop. on the necessity of localness for low-rankness (Sec. 3.3):
    C = diag(0_r, 1_{n-r}); A_ij = (e_i e_j^T + e_j e_i^T)/2 for i < j <= r;
    A_ii = e_i e_i^T for i < r and A_rr = diag(I_r, 0); b_11 = b_rr = 1, else 0.
    Returns the problem and the index list of (i, j) pairs."""
    pairs = [(i, j) for i in range(r) for j in range(i, r)]
    mats, b = [], []
    for (i, j) in pairs:
        E = np.zeros((n, n))
        if i == j and i < r - 1:
            E[i, i] = 1.0
        elif i == j:
            E[:r, :r] = np.eye(r)
        else:
            E[i, j] = E[j, i] = 0.5
        mats.append(E)
        b.append(1.0 if (i == j and (i == 0 or i == r - 1)) else 0.0)
    C = np.diag(np.concatenate([np.zeros(r), np.ones(n - r)]))
    return oracle.generic_sdp(C, mats, np.array(b)), pairs


def test_two_by_two_rank_example():
    """n = 2, m = 3 instance: X_11 = 1, X_12 = 0, X_11 + X_22 = 1, C = 0.
    At rho = 1 and y = (-3/4, 0, -1/2) the subproblem minimiser is diag(1/4, 1/4)
    with value -13/32, and the dual update returns y+ = 0."""
    mats = [np.array([[1.0, 0.0], [0.0, 0.0]]), np.array([[0.0, 0.5], [0.5, 0.0]]), np.eye(2)]
    p = oracle.generic_sdp(np.zeros((2, 2)), mats, np.array([1.0, 0.0, 1.0]))
    y = np.array([-0.75, 0.0, -0.5])
    R = np.diag([0.5, 0.5])
    f, G, a, _ = oracle.objective_grad(p, R, y, 1.0)
    assert math.isclose(f, -13.0 / 32.0, rel_tol=1e-15)
    assert np.max(np.abs(G)) == 0.0
    y_new, _ = oracle.dual_update(p, a, 1.0, y)
    assert np.max(np.abs(y_new)) == 0.0
    # global optimality of the subproblem: grad_X L = C - A*(y+) is PSD
    assert oracle.min_eig(p, y_new) >= -1e-15
    # and gradient descent from a random factor reaches the same value
    R0 = gen.init_factor(2, 2, 3)
    Rf, info = oracle.inner_gd(p, R0, y, 1.0, 1e-12, 5000)
    assert math.isclose(oracle.objective(p, Rf, y, 1.0), -13.0 / 32.0, rel_tol=1e-9)
    np.testing.assert_allclose(Rf @ Rf.T, np.diag([0.25, 0.25]), atol=1e-6)


@pytest.mark.parametrize("r,n", [(2, 4), (3, 5), (4, 6)])
def test_general_rank_example(r, n):
    """General-r instance (same prop.): at rho = 1 and y_11 = 1/(2r) - 1,
    y_ii = 1/(2r) (1 < i < r), y_rr = -1/2, the minimiser is diag(1/(2r) 1_r, 0)
    with dual update y+ = 0 and Z(y+) = diag(0_r, 1_{n-r})."""
    p, pairs = _high_rank_example(r, n)
    y = np.zeros(len(pairs))
    for k, (i, j) in enumerate(pairs):
        if i == j == 0:
            y[k] = 1.0 / (2 * r) - 1.0
        elif i == j and i < r - 1:
            y[k] = 1.0 / (2 * r)
        elif i == j:
            y[k] = -0.5
    R = np.zeros((n, r))
    R[:r, :r] = np.eye(r) / math.sqrt(2 * r)
    f, G, a, _ = oracle.objective_grad(p, R, y, 1.0)
    assert np.max(np.abs(G)) <= 1e-15
    y_new, _ = oracle.dual_update(p, a, 1.0, y)
    assert np.max(np.abs(y_new)) <= 1e-15
    Z = oracle.slack_dense(p, y_new)
    np.testing.assert_allclose(Z, np.diag(np.concatenate([np.zeros(r), np.ones(n - r)])), atol=1e-15)


def test_spurious_stationary_point_dual_nonlocal():
    """Sec. 4.3, prop. on the necessity of dual localness, with d = 5, k = 3,
    rho = 1, eta = 1, a = eta^2 k = 3, eps = 0.1 < rho eta^2 / 4:
    A_i = (e_i e_d^T + e_d e_i^T)/2 (i < d), A_d = eps I, C = eps diag(2 I, 1),
    b = eps a e_d, y = 2 e_d, F = eta [I_k; 0].  Then A(FF^T) = b, the gradient
    vanishes and C - A*y = eps diag(0, ..., 0, -1), so lambda_min = -eps.
    Written in the edge family: trace row first with c_tr = eps, edges (i, d)."""
    d, k, rho, eta, eps = 5, 3, 1.0, 1.0, 0.1
    a_val = eta ** 2 * k
    ei = np.arange(d - 1)
    ej = np.full(d - 1, d - 1)
    C = sp.diags(eps * np.concatenate([2.0 * np.ones(d - 1), [1.0]]))
    b = np.zeros(d)
    b[0] = eps * a_val
    p = oracle.edges_sdp(d, C, b, eps, ei, ej)
    y = np.zeros(d)
    y[0] = 2.0
    F = np.zeros((d, k))
    F[:k, :k] = eta * np.eye(k)
    f, G, a, _ = oracle.objective_grad(p, F, y, rho)
    np.testing.assert_allclose(a, b, atol=1e-15)
    assert np.max(np.abs(G)) <= 1e-15
    lam = oracle.min_eig(p, y)
    assert math.isclose(lam, -eps, rel_tol=1e-12)
    np.testing.assert_allclose(oracle.slack_dense(p, y), np.diag([0, 0, 0, 0, -eps]), atol=1e-15)


def test_spurious_stationary_point_primal_nonlocal():
    """Sec. 4.3, prop. on the necessity of primal localness: C = 0,
    A_i = (e_i e_d^T + e_d e_i^T)/2 (i < d), A_d = eps I, A_{d+1} = eps diag(2 I, 1),
    b = eps a (0, ..., 0, 1, 1), y* = (0, ..., 0, rho, -rho), F = eta [I_k; 0] with
    eta^2 = 4/(eps k), a = 7/eps.  Then grad_X L = eps rho diag(0, ..., 0, -2) and
    the factor gradient vanishes."""
    d, k, rho = 6, 3, 1.3
    eps = 0.5 / math.sqrt(2 * k)
    eta2 = 4.0 / (eps * k)
    a_val = 7.0 / eps
    mats = []
    for i in range(d - 1):
        E = np.zeros((d, d))
        E[i, d - 1] = E[d - 1, i] = 0.5
        mats.append(E)
    mats.append(eps * np.eye(d))
    mats.append(eps * np.diag(np.concatenate([2.0 * np.ones(d - 1), [1.0]])))
    b = np.zeros(d + 1)
    b[d - 1] = b[d] = eps * a_val
    p = oracle.generic_sdp(np.zeros((d, d)), mats, b)
    y = np.zeros(d + 1)
    y[d - 1], y[d] = rho, -rho
    F = np.zeros((d, k))
    F[:k, :k] = math.sqrt(eta2) * np.eye(k)
    f, G, a, _ = oracle.objective_grad(p, F, y, rho)
    assert np.max(np.abs(G)) <= 1e-12 * math.sqrt(eta2)
    w = y - rho * (a - b)
    expected = np.zeros((d, d))
    expected[d - 1, d - 1] = -2.0 * eps * rho
    np.testing.assert_allclose(oracle.slack_dense(p, w), expected, atol=1e-12)


@pytest.mark.parametrize("n", [5, 6, 7, 8, 9])
def test_cycle_spectrum_closed_form(n):
    """C = -L/4 on the cycle C_n has eigenvalues -(2 - 2 cos(2 pi k/n))/4; with
    uniform y the slack C - diag(y) shifts them by -y."""
    p = oracle.maxcut_sdp(gen.cycle_graph(n))
    yv = 0.37
    lam = oracle.min_eig(p, np.full(n, yv))
    expect = min(-(2 - 2 * math.cos(2 * math.pi * k / n)) / 4 for k in range(n)) - yv
    assert math.isclose(lam, expect, rel_tol=1e-13, abs_tol=1e-14)


def test_cycle_spectrum_large_uses_arpack():
    n = 5001
    p = oracle.maxcut_sdp(gen.cycle_graph(n))
    lam = oracle.min_eig(p, np.full(n, -0.2))
    expect = min(-(2 - 2 * math.cos(2 * math.pi * k / n)) / 4 for k in (n // 2, n // 2 + 1)) + 0.2
    assert math.isclose(lam, expect, rel_tol=1e-10)


def test_neg_ones_spectrum():
    """-J has eigenvalues -n (once) and 0; with the trace row, A*(y) = c_tr y_0 I."""
    g = gen.edgeless_graph(7)
    p = oracle.lovasz_sdp(g)
    lam = oracle.min_eig(p, np.array([0.25]))
    assert math.isclose(lam, -7.0 - 0.25, rel_tol=1e-13)


def test_kkt_zero_at_known_optimum_even_cycle():
    """Even cycle: X* = v v^T with v alternating +-1 and y* = -1 (min form) are
    optimal (S = I - L/4 is PSD since lambda_max(L) = 4); every KKT term vanishes
    and the SDP value is n."""
    n = 8
    p = oracle.maxcut_sdp(gen.cycle_graph(n))
    v = np.array([(-1.0) ** i for i in range(n)])[:, None]
    info = oracle.kkt(p, v, -np.ones(n))
    assert info["kkt"] <= 1e-14
    assert math.isclose(-info["pobj"], n, rel_tol=1e-15)


def test_dual_update_and_pinf():
    p = oracle.maxcut_sdp(gen.cycle_graph(4))
    a = np.array([1.5, 1.0, 0.5, 1.0])
    y = np.array([0.1, 0.2, 0.3, 0.4])
    y_new, pinf = oracle.dual_update(p, a, 2.0, y)
    # y + sigma (b - a) with b = 1
    np.testing.assert_allclose(y_new, [0.1 - 1.0, 0.2, 0.3 + 1.0, 0.4], rtol=0, atol=1e-15)
    assert math.isclose(pinf, math.sqrt(0.5) / 3.0, rel_tol=1e-15)
