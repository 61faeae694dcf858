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


def test_set_tiles_rejects_bad_values_without_device():
    from paper_2505_15775_amd import _lib

    assert _lib.lib.alm_bm_set_tiles(None, 0, 0) == -1
