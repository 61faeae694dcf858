"""Matrix completion (Sec. 6) in the oracle: the generator against the sample
counts the paper prints, and the SDP value against the nuclear norm of the
ground truth when the observations determine it (exact recovery)."""

import math

import numpy as np
import pytest

import gen
import oracle

# (r, n = n1 + n2, m as printed for the matrix completion instances of Table 2)
TABLE2 = [(3, 10000, 828659), (3, 20000, 1782453), (3, 50000, 4868248), (3, 100000, 10361604),
          (3, 200000, 21961921), (3, 350000, 40223331), (5, 10000, 2300917), (5, 20000, 4952616),
          (5, 50000, 13522024), (5, 100000, 28777703)]


@pytest.mark.parametrize("r,n,m", TABLE2)
def test_sample_count_matches_table2(r, n, m):
    # the printed counts scatter around ceil(gamma r (n - r)) like realised sample sizes (within 3 sqrt(m))
    assert abs(gen.sample_count(n // 2, n - n // 2, r) - m) <= 3 * math.sqrt(m)


def test_instance_observations_are_entries_of_the_ground_truth():
    inst = gen.completion_instance(40, 30, 2, 3)
    M = inst.U @ inst.V.T
    assert inst.m == gen.sample_count(40, 30, 2)
    keys = inst.rows * 30 + inst.cols
    assert np.all(np.diff(keys) > 0)
    np.testing.assert_allclose(inst.vals, M[inst.rows, inst.cols], rtol=1e-13, atol=1e-13)


def test_completion_sdp_value_is_the_nuclear_norm():
    inst = gen.completion_instance(60, 60, 2, 5)
    p = oracle.completion_sdp(inst)
    nuc = float(np.sum(np.linalg.svd(inst.U @ inst.V.T, compute_uv=False)))
    R0 = gen.init_factor(p.n, 2, 1)
    out = oracle.solve(p, R0, opts=oracle.SolveOptions(eps_kkt=1e-7, r_max=16, max_outer=400, max_inner=3000))
    assert out["status"] == "converged", out["kkt"]
    assert math.isclose(out["kkt"]["pobj"], nuc, rel_tol=1e-5)
    # the recovered block Y = U_hat V_hat^T is the ground truth
    R = out["R"]
    Y = R[:60] @ R[60:].T
    assert np.linalg.norm(Y - inst.U @ inst.V.T) <= 1e-3 * np.linalg.norm(inst.U @ inst.V.T)
