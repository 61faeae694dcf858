"""More pins of the oracle, each against something other than the function
under test: the row-by-row MaxCut evaluator against closed forms and the
pinned full evaluator, the relative KKT measure of Sec. 6 against hand-worked
values at a point where all three terms are nonzero, and the ARPACK branch of
the eigen-solvers against exact spectra with a repeated eigenvalue."""

import math

import numpy as np
import pytest

import gen
import oracle


# ---------------------------------------------------------------- rows evaluator


def test_rows_evaluator_isolated_vertex_and_edge_closed_forms():
    """Rows of C R for C = -L/4 written out by hand: an isolated vertex has
    (CR)_i = 0, so G_i = -2 w_i R_i with w_i = y_i - sigma (||R_i||^2 - 1); on a
    single edge {0, 1} of weight w, (CR)_0 = w (R_1 - R_0) / 4."""
    g = gen.Graph(3, np.array([0]), np.array([1]), np.array([2.0]))  # vertex 2 isolated
    R = np.array([[1.0, 2.0], [0.5, -1.0], [3.0, 0.25]])
    y = np.array([0.3, -0.7, 1.1])
    sigma = 1.7
    G, a = oracle.maxcut_objective_grad_rows(g, R, y, sigma, [2, 0])
    w2 = y[2] - sigma * (R[2] @ R[2] - 1.0)
    np.testing.assert_allclose(G[0], -2.0 * w2 * R[2], rtol=1e-15)
    cr0 = 2.0 * (R[1] - R[0]) / 4.0
    w0 = y[0] - sigma * (R[0] @ R[0] - 1.0)
    np.testing.assert_allclose(G[1], 2.0 * (cr0 - w0 * R[0]), rtol=1e-15)
    np.testing.assert_allclose(a, [R[2] @ R[2], R[0] @ R[0]], rtol=1e-15)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_rows_evaluator_matches_full_evaluator(seed):
    """Random row sets (first, last, isolated and repeated-degree rows) of the
    row evaluator against objective_grad (itself pinned by explicit matrices
    and finite differences)."""
    rng = np.random.default_rng(seed)
    n = 400
    g = gen.er_graph(n, 300, seed, "gauss")  # sparse enough to leave isolated vertices
    deg = np.bincount(np.concatenate([g.ei, g.ej]), minlength=n)
    iso = np.flatnonzero(deg == 0)
    assert iso.size > 0
    rows = np.unique(np.concatenate([[0, n - 1], iso[:5], rng.choice(n, 40, replace=False)]))
    rng.shuffle(rows)
    R = rng.standard_normal((n, 5))
    y = rng.standard_normal(n)
    sigma = 0.9
    G_r, a_r = oracle.maxcut_objective_grad_rows(g, R, y, sigma, rows)
    _, G, a, _ = oracle.objective_grad(oracle.maxcut_sdp(g), R, y, sigma)
    np.testing.assert_allclose(G_r, G[rows], rtol=0, atol=1e-13 * np.abs(G).max())
    np.testing.assert_allclose(a_r, a[rows], rtol=1e-15)


# ---------------------------------------------------------------- KKT measure


def test_kkt_hand_worked_four_cycle_all_terms_nonzero():
    """Sec. 6 measure on the 4-cycle (unit weights), C = -L/4, X = R R^T with
    R = 1.5 (1, -1, 1, -1)^T and y = -0.5 * 1, worked by hand:
      A(X) = 2.25 * 1, ||A(X) - b|| = 2.5, ||b|| = 2         -> pinf = 2.5 / 3
      <C, X> = -2.25 * v^T L v / 4 = -2.25 * 16 / 4 = -9,  b^T y = -2
                                                              -> gap = 7 / 12
      lambda_min(C + 0.5 I) = -1 + 0.5 (L's top eigenvalue is 4),
      ||C||_F = sqrt(4 * 4 + 8) / 4                           -> dinf = 0.5 / (1 + sqrt(24) / 4)."""
    g = gen.cycle_graph(4)
    p = oracle.maxcut_sdp(g)
    R = 1.5 * np.array([[1.0], [-1.0], [1.0], [-1.0]])
    y = np.full(4, -0.5)
    k = oracle.kkt(p, R, y)
    assert math.isclose(k["pinf"], 2.5 / 3.0, rel_tol=1e-14)
    assert math.isclose(k["gap"], 7.0 / 12.0, rel_tol=1e-14)
    assert math.isclose(k["dinf"], 0.5 / (1.0 + math.sqrt(24.0) / 4.0), rel_tol=1e-12)
    assert math.isclose(k["pobj"], -9.0, rel_tol=1e-14) and math.isclose(k["dobj"], -2.0, rel_tol=1e-14)
    assert k["kkt"] == max(k["pinf"], k["dinf"], k["gap"])
    # a supplied lambda_min is used as given
    k2 = oracle.kkt(p, R, y, lam_min=-3.0)
    assert math.isclose(k2["dinf"], 3.0 / (1.0 + math.sqrt(24.0) / 4.0), rel_tol=1e-14)
    assert oracle.kkt(p, R, y, lam_min=0.25)["dinf"] == 0.0


def _dense_kkt(C, A_list, b, R, y):
    """The three terms from dense matrices: X = R R^T, <A_i, X> by trace, the
    slack C - sum y_i A_i assembled and passed to LAPACK."""
    X = R @ R.T
    a = np.array([np.trace(A @ X) for A in A_list])
    pinf = np.linalg.norm(a - b) / (1.0 + np.linalg.norm(b))
    Z = C - sum(yi * A for yi, A in zip(y, A_list))
    lam = np.linalg.eigvalsh(Z)[0]
    dinf = abs(min(0.0, lam)) / (1.0 + np.linalg.norm(C))
    pobj, dobj = np.trace(C @ X), b @ y
    gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    return pinf, dinf, gap


@pytest.mark.parametrize("kind", ["maxcut", "lovasz"])
def test_kkt_against_dense_terms_at_a_non_optimal_point(kind):
    rng = np.random.default_rng(5)
    if kind == "maxcut":
        g = gen.er_graph(12, 25, 3, "gauss")
        p = oracle.maxcut_sdp(g)
        C = p.C.toarray()
        A_list = []
        for i in range(p.n):
            E = np.zeros((p.n, p.n))
            E[i, i] = 1.0
            A_list.append(E)
    else:
        g = gen.er_graph(10, 15, 4, "unit")
        p = oracle.lovasz_sdp(g)
        C = -np.ones((p.n, p.n))
        A_list = [np.eye(p.n)]
        for i, j in zip(g.ei, g.ej):
            E = np.zeros((p.n, p.n))
            E[i, j] = E[j, i] = 0.5
            A_list.append(E)
    R = rng.standard_normal((p.n, 3))
    y = rng.standard_normal(p.m)
    pinf, dinf, gap = _dense_kkt(C, A_list, p.b, R, y)
    assert pinf > 1e-3 and dinf > 1e-3 and gap > 1e-3
    k = oracle.kkt(p, R, y)
    assert math.isclose(k["pinf"], pinf, rel_tol=1e-12)
    assert math.isclose(k["dinf"], dinf, rel_tol=1e-10)
    assert math.isclose(k["gap"], gap, rel_tol=1e-12)


# ---------------------------------------------------------------- ARPACK branch


def test_min_eigs_arpack_branch_double_eigenvalue_closed_form():
    """n = 4500 > the dense limit, so ARPACK runs.  With no edges C = 0 and
    Z(y) = -Diag(y): its spectrum is -y exactly.  y puts a simple eigenvalue
    -5 and a double one -4 at the bottom (eigenvectors e_0 and span{e_1, e_2})."""
    n = 4500
    g = gen.edgeless_graph(n)
    p = oracle.maxcut_sdp(g)
    rng = np.random.default_rng(9)
    y = rng.uniform(0.0, 1.0, n)
    y[[17, 1234, 4000]] = [5.0, 4.0, 4.0]
    vals, V = oracle.min_eigs(p, y, 3)
    np.testing.assert_allclose(vals, [-5.0, -4.0, -4.0], rtol=0, atol=1e-9)
    np.testing.assert_allclose(abs(V[17, 0]), 1.0, atol=1e-8)
    P = V[:, 1:] @ V[:, 1:].T  # projector onto the double eigenspace
    E = np.zeros((n, 2))
    E[1234, 0] = E[4000, 1] = 1.0
    np.testing.assert_allclose(P, E @ E.T, atol=1e-8)
    np.testing.assert_allclose(V.T @ V, np.eye(3), atol=1e-10)
    lam, v = oracle.min_eig(p, y, want_vector=True)
    assert abs(lam + 5.0) <= 1e-9 and abs(abs(v[17]) - 1.0) <= 1e-8


@pytest.mark.parametrize("n", [40, 41])
def test_min_eigs_arpack_branch_cycle_spectrum(n):
    """The ARPACK branch forced on cycles (dense_limit below n): C = -L/4 and
    y = c 1 give eigenvalues -(2 - 2 cos(2 pi k / n)) / 4 - c, k = 0..n-1;
    for odd n the smallest is double (k and n - k)."""
    g = gen.cycle_graph(n)
    p = oracle.maxcut_sdp(g)
    c = 0.3
    y = np.full(n, c)
    k = np.arange(n)
    spec = np.sort(-(2.0 - 2.0 * np.cos(2.0 * np.pi * k / n)) / 4.0 - c)
    vals, V = oracle.min_eigs(p, y, 3, dense_limit=10)
    np.testing.assert_allclose(vals, spec[:3], rtol=0, atol=1e-10)
    Z = oracle.slack_dense(p, y)
    np.testing.assert_allclose(Z @ V, V * vals, atol=1e-9)
    if n % 2:
        assert abs(vals[0] - vals[1]) <= 1e-10
    assert abs(oracle.min_eig(p, y, dense_limit=10) - spec[0]) <= 1e-10


# ---------------------------------------------------------------- penalty moments


@pytest.mark.parametrize("kind", ["maxcut", "lovasz"])
def test_penalty_moments_quadratic_form_equals_penalty_of_the_step(kind):
    """For symmetric S, sum_{abcd} S_ab S_cd M[pair(a,b), pair(c,d)] must equal
    sum_i w_i A_i(V S V^T)^2 with A applied to the dense matrix V S V^T through
    the explicit constraint matrices (another route than the pair images)."""
    rng = np.random.default_rng(11)
    if kind == "maxcut":
        p = oracle.maxcut_sdp(gen.er_graph(30, 80, 2, "gauss"))
        mats = []
        for i in range(p.n):
            E = np.zeros((p.n, p.n))
            E[i, i] = 1.0
            mats.append(E)
    else:
        g = gen.er_graph(25, 60, 3, "unit")
        p = oracle.lovasz_sdp(g)
        mats = [np.eye(p.n)]
        for i, j in zip(g.ei, g.ej):
            E = np.zeros((p.n, p.n))
            E[i, j] = E[j, i] = 0.5
            mats.append(E)
    q = 3
    V = np.linalg.qr(rng.standard_normal((p.n, q)))[0]
    wts = rng.uniform(0.5, 2.0, p.m)
    M = oracle.penalty_moments(p, V, wts)
    pairs = [(a, b) for a in range(q) for b in range(a, q)]
    for _ in range(3):
        S = rng.standard_normal((q, q))
        S = S + S.T
        X = V @ S @ V.T
        direct = sum(wi * np.sum(A * X) ** 2 for wi, A in zip(wts, mats))
        # expand the sum over all (a, b, c, d) through the pair numbering
        full = 0.0
        for i1, (a, b) in enumerate(pairs):
            for i2, (c, d) in enumerate(pairs):
                m1 = 1.0 if a == b else 2.0
                m2 = 1.0 if c == d else 2.0
                full += m1 * m2 * S[a, b] * S[c, d] * M[i1, i2]
        assert math.isclose(full, direct, rel_tol=1e-12)
