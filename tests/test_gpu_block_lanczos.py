"""Block Lanczos (alm_bm_lanczos_block, GPU only) against the oracle's exact
eigensolvers: a double eigenvalue is captured with its whole eigenspace (one
Krylov vector cannot), Ritz values bound the eigenvalues from above and agree
within their residuals, the vectors are orthonormal and the reported residuals
are those of the returned vectors, for the MaxCut family and for the trace +
edge family (whose slack carries the -J term)."""

import math

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _almbm():
    import paper_2505_15775_amd as m

    return m


def test_odd_cycle_double_eigenvalue_and_its_eigenspace():
    """C = -L/4 of the 41-cycle and y = c 1: the spectrum of Z is
    -(2 - 2 cos(2 pi k / n)) / 4 - c, whose smallest value is double for odd n
    (k = (n - 1) / 2 and (n + 1) / 2).  Block size 3 returns both vectors of the
    double eigenspace (the projector equals the oracle's) and the next value."""
    n = 41
    g = gen.cycle_graph(n)
    po = oracle.maxcut_sdp(g)
    prob = _almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=8, lanczos_kmax=60, device=DEV)
    c = 0.3
    y = torch.full((n,), c, dtype=torch.float64, device=DEV)
    th, V, rs, m = prob.lanczos_block(y, 3, max_iter=60, seed=5)
    k = np.arange(n)
    spec = np.sort(-(2.0 - 2.0 * np.cos(2.0 * np.pi * k / n)) / 4.0 - c)
    print(f"n={n} basis {m}: theta {th} exact {spec[:3]} resid {rs}")
    assert abs(spec[0] - spec[1]) <= 1e-12 and spec[2] - spec[1] > 1e-3
    np.testing.assert_allclose(th, spec[:3], rtol=0, atol=1e-10)
    Vh = V.cpu().numpy()
    np.testing.assert_allclose(Vh.T @ Vh, np.eye(3), atol=1e-10)
    vals, W = oracle.min_eigs(po, y.cpu().numpy(), 2)
    np.testing.assert_allclose(Vh[:, :2] @ Vh[:, :2].T, W @ W.T, atol=1e-8)
    assert np.all(rs <= 1e-8)
    prob.close()


def test_planted_double_eigenvalue_in_a_small_krylov_space():
    """No edges, so Z = -Diag(y) and its spectrum is -y.  y plants a double
    eigenvalue -5 (vertices 17 and 1234) and -4 (vertex 4000) below a bulk in
    [-1, 0]; n = 4500 and a 61-column basis.  The block of 3 returns -5, -5, -4
    and spans {e_17, e_1234} for the double value; a single Krylov vector's
    Ritz values miss the second copy of -5."""
    n = 4500
    g = gen.edgeless_graph(n)
    prob = _almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=8, lanczos_kmax=60, device=DEV)
    rng = np.random.default_rng(9)
    yh = rng.uniform(0.0, 1.0, n)
    yh[[17, 1234, 4000]] = [5.0, 5.0, 4.0]
    y = torch.from_numpy(yh).to(DEV)
    th, V, rs, m = prob.lanczos_block(y, 3, max_iter=60, seed=3)
    print(f"basis {m}: theta {th} resid {rs}")
    np.testing.assert_allclose(th, [-5.0, -5.0, -4.0], rtol=0, atol=1e-9)
    Vh = V.cpu().numpy()
    P = Vh[:, :2] @ Vh[:, :2].T
    E = np.zeros((n, 2))
    E[17, 0] = E[1234, 1] = 1.0
    np.testing.assert_allclose(P, E @ E.T, atol=1e-7)
    assert abs(abs(Vh[4000, 2]) - 1.0) <= 1e-7
    # one Krylov vector: its space holds a single direction of the -5 eigenspace
    th1, v1, _, _ = prob.lanczos_min_eig(y, max_iter=60, tol=1e-12)
    assert abs(th1 + 5.0) <= 1e-9
    v1h = v1.cpu().numpy()
    assert abs(v1h[17] ** 2 + v1h[1234] ** 2 - 1.0) <= 1e-8
    prob.close()


@pytest.mark.parametrize("q", [1, 4])
def test_er_graph_separated_bottom_against_dense_spectrum(q):
    """ER cost with a bulk dual y ~ -0.5 and four planted entries (12, 11.5, 11,
    10.5) that put four eigenvalues of Z below the bulk: the q smallest Ritz
    pairs equal the dense spectrum's, are orthonormal, bound the eigenvalues from
    above, and their reported residuals are those of the returned vectors."""
    g = gen.er_graph(3000, 15000, 12, "gauss")
    po = oracle.maxcut_sdp(g)
    prob = _almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=8, lanczos_kmax=100, device=DEV)
    rng = np.random.default_rng(3)
    y = -0.5 + 0.2 * rng.standard_normal(g.n)
    y[[5, 700, 1500, 2999]] = [12.0, 11.5, 11.0, 10.5]
    th, V, rs, m = prob.lanczos_block(torch.from_numpy(y).to(DEV), q, max_iter=100, seed=7)
    lam = np.linalg.eigvalsh(oracle.slack_dense(po, y))[:q]
    print(f"q={q} basis {m}: theta {th} exact {lam} resid {rs}")
    Vh = V.cpu().numpy()
    np.testing.assert_allclose(Vh.T @ Vh, np.eye(q), atol=1e-10)
    assert np.all(th >= lam - 1e-10)
    np.testing.assert_allclose(th, lam, rtol=0, atol=1e-9)
    for k in range(q):
        r = oracle.slack_matvec(po, y, Vh[:, k]) - th[k] * Vh[:, k]
        assert math.isclose(np.linalg.norm(r), rs[k], rel_tol=1e-6, abs_tol=1e-12)
    prob.close()


def test_lovasz_slack_with_the_j_term():
    """Trace + edge family, C = -J: Z(y) = -J - y_0 I - sum_e y_e (E_ij + E_ji)/2,
    whose smallest eigenvalue (about -n, along 1) is far below the rest.  The
    block's products carry 1^T q of each basis column for the -J term; the
    smallest Ritz value matches the dense spectrum, all bound from above, and the
    residuals are those of the returned vectors."""
    g = gen.er_graph(400, 1600, 5, "unit")
    po = oracle.lovasz_sdp(g)
    prob = _almbm().Problem.lovasz(g.n, g.ei, g.ej, precision="f64", r_max=8, lanczos_kmax=120, device=DEV)
    rng = np.random.default_rng(4)
    y = rng.standard_normal(po.m)
    th, V, rs, m = prob.lanczos_block(torch.from_numpy(y).to(DEV), 3, max_iter=120, seed=2)
    lam = np.linalg.eigvalsh(oracle.slack_dense(po, y))[:3]
    print(f"lovasz basis {m}: theta {th} exact {lam} resid {rs}")
    assert np.all(th >= lam - 1e-9)
    assert abs(th[0] - lam[0]) <= 1e-9 * abs(lam[0])
    Vh = V.cpu().numpy()
    np.testing.assert_allclose(Vh.T @ Vh, np.eye(3), atol=1e-10)
    for k in range(3):
        r = oracle.slack_matvec(po, y, Vh[:, k]) - th[k] * Vh[:, k]
        assert math.isclose(np.linalg.norm(r), rs[k], rel_tol=1e-6, abs_tol=1e-11)
    prob.close()


def test_argument_checks():
    m = _almbm()
    g = gen.cycle_graph(6)
    prob = m.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=4, lanczos_kmax=10, device=DEV)
    y = torch.zeros(6, dtype=torch.float64, device=DEV)
    for q, it in [(0, 5), (9, 5), (2, 0), (2, 11), (6, 10)]:
        with pytest.raises(m.AlmBmError):
            prob.lanczos_block(y, q, max_iter=it)
    prob.close()
