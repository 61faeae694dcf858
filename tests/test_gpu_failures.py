"""Failure paths and resume (GPU only): a malformed CSR cost (validate = 1)
or edge list is rejected at create with ERR_INVALID_PATTERN, NaN in the start
factor or dual ends the solve with ERR_NUMERIC, and an FP64 solve stopped by
max_outer and resumed from its returned state repeats the uninterrupted solve
bitwise."""

import ctypes as C

import numpy as np
import pytest
import torch

import gen

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _m():
    import paper_2505_15775_amd as m

    return m


def _create(rp, ci, cv, n, ell_width=0, validate=1):
    """alm_bm_create on a hand-made DIAG-family cost; returns (status, handle, arrays)."""
    from paper_2505_15775_amd import _lib

    dev = torch.device(DEV)
    arr = {"ci": torch.tensor(ci, dtype=torch.int32, device=dev), "cv": torch.tensor(cv, dtype=torch.float64,
                                                                                     device=dev),
           "b": torch.ones(n, dtype=torch.float64, device=dev)}
    if rp is not None:
        arr["rp"] = torch.tensor(rp, dtype=torch.int32, device=dev)
    d = _lib.Desc()
    d.n, d.nnz, d.m = n, len(ci), n
    d.row_ptr = arr["rp"].data_ptr() if rp is not None else 0
    d.col_idx, d.val, d.ell_width, d.b = arr["ci"].data_ptr(), arr["cv"].data_ptr(), ell_width, arr["b"].data_ptr()
    d.cons_kind, d.precision, d.r_max, d.lanczos_kmax, d.validate = _lib.CONS_DIAG, 0, 4, 4, validate
    h = C.c_void_p()
    st = _lib.lib.alm_bm_create(C.byref(d), None, C.byref(h))
    return st, h, arr


@pytest.mark.parametrize("case", ["col_out_of_range", "unsorted_row", "bad_row_ptr", "ell_out_of_range"])
def test_malformed_cost_is_rejected_with_invalid_pattern(case):
    from paper_2505_15775_amd import _lib

    n = 4
    rp, ci = [0, 2, 3, 4, 6], [1, 3, 0, 0, 0, 2]
    if case == "col_out_of_range":
        ci = [1, 9, 0, 0, 0, 2]
    elif case == "unsorted_row":
        ci = [3, 1, 0, 0, 0, 2]
    elif case == "bad_row_ptr":
        rp = [0, 3, 2, 4, 6]
    cv = [0.25] * len(ci)
    if case == "ell_out_of_range":
        st, h, _ = _create(None, [1, 2, 0, -1, 3, 0, 2, 1], [0.25] * 8, n, ell_width=2)
    else:
        st, h, _ = _create(rp, ci, cv, n)
    print(f"{case}: status {st}: {_lib.lib.alm_bm_last_error().decode()}")
    assert st == -2
    # the well-formed cost is accepted
    st_ok, h_ok, _ = _create([0, 2, 3, 4, 6], [1, 3, 0, 0, 0, 2], [0.25] * 6, n)
    assert st_ok == 0
    _lib.lib.alm_bm_destroy(h_ok)


@pytest.mark.parametrize("ei,ej", [([0, 2, 1], [1, 3, 2]),      # not sorted by (i, j)
                                   ([0, 1, 1], [1, 1, 3]),      # i = j
                                   ([0, 0, 1], [1, 1, 3])])     # duplicate
def test_malformed_edge_list_is_rejected(ei, ej):
    m = _m()
    with pytest.raises(m.AlmBmError) as e:
        m.Problem.lovasz(4, np.array(ei), np.array(ej), precision="f64", r_max=4, lanczos_kmax=4, device=DEV)
    assert e.value.status == -2


@pytest.mark.parametrize("where", ["R", "y"])
def test_nan_start_ends_with_numeric_error(where):
    m = _m()
    g = gen.er_graph(300, 1200, 2, "gauss")
    prob = m.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=16, lanczos_kmax=40, device=DEV)
    R0 = gen.init_factor(g.n, 4, 1)
    y0 = np.zeros(g.n)
    if where == "R":
        R0[17, 2] = np.nan
    else:
        y0[5] = np.nan
    with pytest.raises(m.AlmBmError) as e:
        prob.solve(R0, y0, eps_kkt=1e-6, max_outer=50)
    print(f"NaN in {where}: {e.value}")
    assert e.value.status == -5
    # the handle stays usable
    st, res, _, _ = prob.solve(gen.init_factor(g.n, 4, 1), eps_kkt=1e-5, max_outer=200)
    assert st == 0
    prob.close()


@pytest.mark.parametrize("inner", [0, 1])
def test_stop_and_resume_repeats_the_uninterrupted_solve_bitwise(inner):
    m = _m()
    g = gen.er_graph(700, 4000, 21, "gauss")
    prob = m.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=32, lanczos_kmax=80, device=DEV,
                            lbfgs_memory_max=3)
    R0 = gen.init_factor(g.n, 4, 3)
    opts = dict(eps_kkt=1e-6, inner_solver=inner, lbfgs_memory=3)
    st, res, R, y = prob.solve(R0, max_outer=300, **opts)
    assert st == 0 and res["outer"] > 6
    st1, res1, R1, y1 = prob.solve(R0, max_outer=5, **opts)
    assert st1 == 1 and res1["outer"] == 5
    st2, res2, R2, y2 = prob.solve(R1.clone(), y1, max_outer=300, resume_outer=res1["outer"],
                                   resume_inner_tol=res1["inner_tol"], resume_pinf=res1["pinf"], **opts)
    print(f"inner solver {inner}: uninterrupted outer {res['outer']} rank {res['rank']}; "
          f"resumed outer {res2['outer']} rank {res2['rank']}")
    assert st2 == 0 and res2["outer"] == res["outer"] and res2["rank"] == res["rank"]
    assert torch.equal(R2, R) and torch.equal(y2, y)
    prob.close()
