"""Per-call parity of host-result entry points (GPU only): the relative KKT
measure of Sec. 6 (alm_bm_kkt) against the oracle's at the same (R, y,
lambda_min), and the block rank step's penalty quadratic form
(alm_bm_block_moments) against the oracle's penalty_moments, both families."""

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


def _case(kind, **ws):
    m = _almbm()
    if kind == "maxcut":
        g = gen.er_graph(1500, 6000, 4, "gauss")
        return g, oracle.maxcut_sdp(g), m.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=16,
                                                         lanczos_kmax=20, device=DEV, **ws)
    g = gen.er_graph(800, 4000, 5, "unit")
    return g, oracle.lovasz_sdp(g), m.Problem.lovasz(g.n, g.ei, g.ej, precision="f64", r_max=16, lanczos_kmax=20,
                                                     device=DEV, **ws)


@pytest.mark.parametrize("kind", ["maxcut", "lovasz"])
def test_kkt_call_matches_oracle_at_a_non_optimal_point(kind):
    g, po, prob = _case(kind)
    rng = np.random.default_rng(7)
    R = rng.standard_normal((po.n, 5)) / (np.sqrt(po.n) if kind == "lovasz" else 1.0)
    y = rng.standard_normal(po.m)
    for lam in (-0.37, 0.2):
        got = prob.kkt(prob.factor(R), torch.from_numpy(y).to(DEV), lam)
        exp = oracle.kkt(po, R, y, lam_min=lam)
        print(f"{kind} lam {lam}: " + " ".join(f"{k} {got[k]:.6e}/{exp[k]:.6e}" for k in got))
        for k in ("pinf", "dinf", "gap", "kkt", "pobj", "dobj"):
            assert abs(got[k] - exp[k]) <= 1e-10 * max(abs(exp[k]), 1e-300), k
        if lam < 0:
            assert got["pinf"] > 0 and got["dinf"] > 0 and got["gap"] > 0
        else:
            assert got["dinf"] == 0.0
    prob.close()


@pytest.mark.parametrize("kind,q,edge_w", [("maxcut", 1, 1.0), ("maxcut", 3, 1.0), ("maxcut", 6, 1.0),
                                           ("lovasz", 2, 1.0), ("lovasz", 4, 37.5)])
def test_block_moments_match_oracle(kind, q, edge_w):
    g, po, prob = _case(kind, rank_block_max=8)
    rng = np.random.default_rng(q)
    V = np.linalg.qr(rng.standard_normal((po.n, q)))[0]
    M4 = prob.block_moments(torch.from_numpy(V), edge_weight=edge_w)
    wts = np.ones(po.m)
    if kind == "lovasz":
        wts[1:] = edge_w  # edge rows; the trace row keeps weight 1
    M_o = oracle.penalty_moments(po, V, wts)
    e = float(np.linalg.norm(M4 - M_o) / np.linalg.norm(M_o))
    print(f"{kind} q={q} edge weight {edge_w}: rel err {e:.2e}")
    assert M4.shape == M_o.shape and e <= 1e-12
    prob.close()


def test_block_moments_rejects_more_directions_than_reserved():
    _, _, prob = _case("maxcut", rank_block_max=2)
    with pytest.raises(_almbm().AlmBmError):
        prob.block_moments(torch.zeros((prob.n, 3), dtype=torch.float64))
    prob.close()
