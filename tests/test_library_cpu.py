"""CPU-side checks of the HIP library: it loads, exports every symbol declared
in include/alm_bm.h, its struct layouts match the binding, and its host-only
helpers behave (no device compute)."""

import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "alm_bm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(alm_bm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2505_15775_amd import _lib

    declared = _declared_functions()
    assert "alm_bm_solve" in declared and "alm_bm_objective_grad" in declared
    for name in declared:
        assert hasattr(_lib.lib, name), f"{name} declared in alm_bm.h but not exported"
    assert sorted(_lib.EXPORTS) == declared


def test_abi_struct_sizes_match():
    from paper_2505_15775_amd import _lib

    sizes = (C.c_int64 * 3)()
    _lib.lib.alm_bm_abi_sizes(sizes)
    assert tuple(sizes) == (C.sizeof(_lib.Desc), C.sizeof(_lib.Options), C.sizeof(_lib.Result))


def test_default_options():
    from paper_2505_15775_amd import default_options

    o = default_options()
    assert o.eps_kkt == 1e-6 and o.sigma == 1.0 and o.max_inner == 500 and o.graph_unroll == 8
    assert o.inner_tol_decay == 0.7 and o.lanczos_tol_rel == 0.1


def test_maxcut_cost_matches_laplacian_definition():
    """C = -L/4 (Sec. 6.1) from the library's host builder against a scipy
    Laplacian built here from the definition L_ij = -w_ij, L_ii = sum_k w_ik."""
    import gen
    from paper_2505_15775_amd import maxcut_cost

    g = gen.er_graph(300, 1200, 3, "gauss")
    rp, ci, cv, dg = maxcut_cost(g.n, g.ei, g.ej, g.w)
    S = sp.csr_matrix((cv, ci, rp), shape=(g.n, g.n)).toarray()
    W = np.zeros((g.n, g.n))
    W[g.ei, g.ej] = g.w
    W[g.ej, g.ei] = g.w
    L = np.diag(W.sum(1)) - W
    np.testing.assert_allclose(S + np.diag(dg), -L / 4, rtol=0, atol=1e-15)
    # columns ascending within rows, no diagonal stored in S
    for i in range(g.n):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0) and not np.any(row == i)


def test_maxcut_cost_merges_duplicates_and_unsorted_input():
    from paper_2505_15775_amd import maxcut_cost

    ei = np.array([3, 0, 1, 0], dtype=np.int32)
    ej = np.array([1, 2, 3, 2], dtype=np.int32)
    w = np.array([1.0, 2.0, 3.0, 0.5])
    rp, ci, cv, dg = maxcut_cost(4, ei, ej, w)
    S = sp.csr_matrix((cv, ci, rp), shape=(4, 4)).toarray()
    expect = np.zeros((4, 4))
    expect[1, 3] = expect[3, 1] = (1.0 + 3.0) / 4
    expect[0, 2] = expect[2, 0] = (2.0 + 0.5) / 4
    np.testing.assert_allclose(S, expect)
    np.testing.assert_allclose(dg, -expect.sum(1))


def test_maxcut_cost_rejects_bad_edges():
    from paper_2505_15775_amd import AlmBmError, maxcut_cost

    with pytest.raises(AlmBmError):
        maxcut_cost(3, np.array([0], np.int32), np.array([0], np.int32), np.array([1.0]))
    with pytest.raises(AlmBmError):
        maxcut_cost(3, np.array([0], np.int32), np.array([5], np.int32), np.array([1.0]))


def test_create_rejects_bad_arguments_before_any_launch():
    """Argument checks run on the host and return INVALID_ARG without touching a device."""
    from paper_2505_15775_amd import _lib

    d = _lib.Desc()
    d.n = 10
    d.m = 10
    d.r_max = 0  # invalid
    d.b = 0
    h = C.c_void_p()
    st = _lib.lib.alm_bm_create(C.byref(d), None, C.byref(h))
    assert st == -1
    d.r_max = 8
    st = _lib.lib.alm_bm_create(C.byref(d), None, C.byref(h))
    assert st == -1 and b"b is null" in _lib.lib.alm_bm_last_error()
    st = _lib.lib.alm_bm_objective_grad(None, 4, None, None, 1.0, None, None, None, None)
    assert st == -1


def test_objective_grad_noalloc_rejects_bad_arguments_before_any_launch():
    """The no-allocation objective/gradient call checks its descriptor on the
    host (nothing is dereferenced or launched before the checks pass)."""
    from paper_2505_15775_amd import _lib

    fake = C.c_void_p(0x1000)  # never dereferenced: every call below fails its checks first
    d = _lib.Desc()
    d.n, d.m, d.b, d.precision, d.cons_kind = 10, 10, 0x1000, 0, 0
    lib = _lib.lib
    assert lib.alm_bm_objective_grad_noalloc(None, 4, fake, fake, 1.0, fake, None, None, None) == -1
    assert lib.alm_bm_objective_grad_noalloc(C.byref(d), 4, None, fake, 1.0, fake, None, None, None) == -1
    assert lib.alm_bm_objective_grad_noalloc(C.byref(d), 129, fake, fake, 1.0, fake, None, None, None) == -1
    assert b"r must be" in lib.alm_bm_last_error()
    d.precision = 1
    assert lib.alm_bm_objective_grad_noalloc(C.byref(d), 4, fake, fake, 1.0, fake, None, None, None) == -6
    d.precision, d.cons_kind = 0, 1
    assert lib.alm_bm_objective_grad_noalloc(C.byref(d), 4, fake, fake, 1.0, fake, None, None, None) == -6
    d.cons_kind, d.j_coef = 0, 1.0
    assert lib.alm_bm_objective_grad_noalloc(C.byref(d), 4, fake, fake, 1.0, fake, None, None, None) == -6
    d.j_coef, d.m = 0.0, 9
    assert lib.alm_bm_objective_grad_noalloc(C.byref(d), 4, fake, fake, 1.0, fake, None, None, None) == -1
    d.m, d.nnz, d.ell_width = 10, 7, 2  # ELL needs nnz = n * ell_width
    assert lib.alm_bm_objective_grad_noalloc(C.byref(d), 4, fake, fake, 1.0, fake, None, None, None) == -1


def test_set_tiles_rejects_bad_values_without_device():
    from paper_2505_15775_amd import _lib

    assert _lib.lib.alm_bm_set_tiles(None, 0, 0) == -1
    assert _lib.lib.alm_bm_batch_autotune(None, 3, None, None, None, None) == -1
    assert _lib.lib.alm_bm_lanczos_block(None, None, 2, 5, 1, None, None, None, None, None) == -1
    assert _lib.lib.alm_bm_ladder_factor(None, 4, None, None) == -1


def _pairs(q):
    return [(a, b) for a in range(q) for b in range(a, q)]


@pytest.mark.parametrize("kind,q", [("maxcut", 1), ("maxcut", 3), ("maxcut", 5), ("lovasz", 2), ("lovasz", 4)])
def test_psd_step_matches_the_oracle_curvature_step(kind, q):
    """The host solver of the block rank step's q x q PSD subproblem against the
    oracle's curvature step, on exact eigenvectors of the slack (so that
    V^T Z V = diag(theta)); M4 is the penalty's quadratic form of A(V S V^T)
    built from its definition (rows for MaxCut; edge rows weighted by the edge
    penalty ratio plus the trace row for Lovasz)."""
    import gen
    import oracle
    import paper_2505_15775_amd as m

    rng = np.random.default_rng(17 + q)
    if kind == "maxcut":
        po = oracle.maxcut_sdp(gen.er_graph(80, 300, 5, "gauss"))
        sigma, rho = 1.3, 1.0
    else:
        po = oracle.lovasz_sdp(gen.er_graph(50, 150, 6, "unit"))
        sigma, rho = 2.0, 4.0
    sig_vec = np.full(po.m, sigma * rho)
    sig_vec[0] = sigma if kind == "lovasz" else sigma * rho
    R = rng.standard_normal((po.n, 2)) / np.sqrt(po.n)
    y = rng.standard_normal(po.m)
    if kind == "lovasz":
        y[0] = 5.0  # the trace multiplier shifts the slack down: several negative eigenvalues
    w = y - sig_vec * (oracle.amap(po, R) - po.b)
    theta, V = oracle.min_eigs(po, w, q)
    assert np.all(theta < 0)
    P = _pairs(q)
    if kind == "maxcut":
        K = np.column_stack([V[:, a] * V[:, b] for a, b in P])            # rows of A(v_a v_b^T)
        M4 = K.T @ K
    else:
        ei, ej = po.ei, po.ej
        K = np.column_stack([0.5 * (V[ei, a] * V[ej, b] + V[ej, a] * V[ei, b]) for a, b in P])
        tr = np.array([1.0 if a == b else 0.0 for a, b in P])              # trace row: c_tr tr(S)
        M4 = rho * (K.T @ K) + po.c_tr ** 2 * np.outer(tr, tr)
    S = m.psd_step(theta, M4, sigma)
    S_o, phi_o, _ = oracle.curvature_step(po, w, sig_vec, V)
    assert np.linalg.norm(S - S_o) <= 1e-7 * max(1.0, np.linalg.norm(S_o))


def test_psd_step_rejects_bad_arguments():
    import paper_2505_15775_amd as m

    with pytest.raises(m.AlmBmError):
        m.psd_step(np.zeros(9), np.eye(45), 1.0)           # q > 8
    with pytest.raises(m.AlmBmError):
        m.psd_step(np.array([-1.0]), np.eye(1), 0.0)       # sigma must be positive
    with pytest.raises(m.AlmBmError):
        m.psd_step(np.array([-1.0]), np.array([[np.nan]]), 1.0)
    with pytest.raises(m.AlmBmError):
        m.psd_step(np.array([np.nan, -1.0]), np.eye(3), 1.0)    # a NaN Ritz value is an error, not S = 0
    with pytest.raises(m.AlmBmError):
        m.psd_step(np.array([-np.inf]), np.eye(1), 1.0)
    # a positive Ritz value gives no step; a negative one the closed form -theta / (sigma M4)
    assert m.psd_step(np.array([0.5]), np.array([[2.0]]), 1.0)[0, 0] == 0.0
    assert abs(m.psd_step(np.array([-0.5]), np.array([[2.0]]), 1.0)[0, 0] - 0.25) <= 1e-12
