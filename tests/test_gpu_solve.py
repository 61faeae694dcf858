"""Solve-level checks of the HIP path (GPU only): closed-form SDP values, the
stored oracle solve of the n = 2000 ER workload, KKT re-evaluated by the oracle
at the GPU's final point, determinism, graph replay against eager launches,
and the not-converged exit."""

import json
import math
import os

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def almbm():
    import paper_2505_15775_amd as m

    return m


def _maxcut(g, prec="f64", r_max=32, kmax=100, **ws):
    return almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision=prec, r_max=r_max, lanczos_kmax=kmax, device=DEV,
                                  **ws)


def _oracle_kkt(po, R, y):
    lam = oracle.min_eig(po, y)
    return oracle.kkt(po, R, y, lam_min=lam)


@pytest.mark.parametrize("n", [10, 9, 64])
def test_solve_cycles_closed_form(n):
    g = gen.cycle_graph(n)
    prob = _maxcut(g, r_max=8, kmax=min(n, 60))
    st, res, R, y = prob.solve(gen.init_factor(n, 2, 1), eps_kkt=1e-8, max_outer=400, max_inner=2000)
    val = -res["pobj"]
    expect = n if n % 2 == 0 else n * (1 + math.cos(math.pi / n)) / 2
    print(f"cycle {n}: status {st} value {val:.12f} expect {expect:.12f} outer {res['outer']} rank {res['rank']}")
    assert st == 0
    assert math.isclose(val, expect, rel_tol=1e-6)
    # the solution's rank is rank(X*) (Sec. 3: 1 for even cycles, 2 for odd ones),
    # whatever width the factor grew to: the numerical rank of R, not its width
    sv = np.linalg.svd(R.cpu().numpy(), compute_uv=False)
    assert int(np.sum(sv > 1e-2 * sv[0])) == (1 if n % 2 == 0 else 2)


def test_solve_complete_graph_closed_form():
    g = gen.complete_graph(8)
    prob = _maxcut(g, r_max=8, kmax=8)
    st, res, R, y = prob.solve(gen.init_factor(8, 3, 2), eps_kkt=1e-8, max_outer=400, max_inner=2000)
    assert st == 0 and math.isclose(-res["pobj"], 16.0, rel_tol=1e-6)


@pytest.mark.parametrize("n,expect", [(5, math.sqrt(5.0)), (6, 3.0)])
def test_solve_lovasz_theta_cycles(n, expect):
    g = gen.cycle_graph(n)
    prob = almbm().Problem.lovasz(n, g.ei, g.ej, precision="f64", r_max=8, lanczos_kmax=n, device=DEV)
    st, res, R, y = prob.solve(gen.init_factor(n, 3, 1), eps_kkt=1e-6, max_outer=400, max_inner=2000)
    print(f"lovasz C{n}: status {st} theta {-res['pobj']:.10f} expect {expect:.10f}")
    assert st == 0 and math.isclose(-res["pobj"], expect, rel_tol=1e-5)


def test_solve_er2000_matches_stored_oracle_solve():
    """The n = 2000 ER workload (unit weights, r0 = 8, sigma = 1, eps = 1e-6)
    against the oracle's own solve (tests/golden/make_golden.py), and the KKT
    measure re-evaluated by the oracle (exact lambda_min) at the GPU's (R, y)."""
    gold = json.load(open(os.path.join(GOLDEN, "maxcut_er2000_solve.json")))
    g = gen.er_graph(2000, 10000, 1, "unit")
    prob = _maxcut(g, r_max=64, kmax=100)
    st, res, R, y = prob.solve(gen.init_factor(2000, 8, 1), eps_kkt=1e-6, sigma=1.0)
    print(f"er2000: status {st} outer {res['outer']} inner {res['inner_total']} rank {res['rank']} "
          f"pobj {res['pobj']:.10f} (oracle {gold['pobj']:.10f}) kkt {res['kkt']:.2e} time {res['time_s']:.2f}s")
    assert st == 0
    assert abs(res["pobj"] - gold["pobj"]) <= 1e-5 * abs(gold["pobj"])
    po = oracle.maxcut_sdp(g)
    k = _oracle_kkt(po, R.cpu().numpy(), y.cpu().numpy())
    print(f"oracle KKT at GPU point: {k}")
    assert k["pinf"] <= 1e-6 and k["gap"] <= 1e-6 and k["dinf"] <= 2e-6


def test_solve_deterministic_and_graph_matches_eager():
    g = gen.er_graph(700, 4000, 21, "gauss")
    outs = []
    for unroll in (8, 8, 0, 3):
        prob = _maxcut(g, r_max=32, kmax=80)
        st, res, R, y = prob.solve(gen.init_factor(700, 4, 3), eps_kkt=1e-5, graph_unroll=unroll, max_outer=300)
        outs.append((st, res["outer"], res["rank"], R.cpu().numpy().copy(), y.cpu().numpy().copy()))
        prob.close()
    for o in outs[1:]:
        assert o[0] == outs[0][0] and o[1] == outs[0][1] and o[2] == outs[0][2]
        assert np.array_equal(o[3], outs[0][3]) and np.array_equal(o[4], outs[0][4])


def test_solve_max_outer_exit_returns_valid_outputs():
    g = gen.er_graph(500, 2500, 5, "unit")
    prob = _maxcut(g, r_max=16, kmax=50)
    st, res, R, y = prob.solve(gen.init_factor(500, 4, 1), eps_kkt=1e-9, max_outer=2, max_inner=5)
    assert st == 1  # NOT_CONVERGED
    assert res["outer"] == 2 and np.all(np.isfinite(R.cpu().numpy())) and np.all(np.isfinite(y.cpu().numpy()))


def test_solve_refuses_ok_without_a_certified_lanczos_value():
    """dinf needs lambda_min of the slack.  A solve restarted at a converged
    point with a 2-vector Krylov space and no restarts measures a KKT value
    below eps, but its Ritz interval [theta - resid, theta + resid] reaches
    below -eps (1 + ||C||_F), so the value is not certified and the solve must
    not return OK; the residual is reported."""
    g = gen.er_graph(700, 4000, 21, "gauss")
    prob = _maxcut(g, r_max=32, kmax=80)
    st, res, R, y = prob.solve(gen.init_factor(700, 4, 3), eps_kkt=1e-5, max_outer=300)
    assert st == 0
    cn = float(np.linalg.norm(oracle.maxcut_sdp(g).C.toarray()))
    ltol = 0.1 * 1e-5 * (1.0 + cn)
    assert res["lanczos_resid"] <= ltol
    st2, res2, _, _ = prob.solve(R.clone(), y, eps_kkt=1e-5, max_outer=3, lanczos_kmax=2, lanczos_restarts=0)
    print(f"kmax 2: status {st2} kkt {res2['kkt']:.3e} lanczos resid {res2['lanczos_resid']:.3e} (tol {ltol:.3e})")
    assert st2 == 1 and res2["lanczos_resid"] > ltol
    assert res2["lanczos_resid"] - res2["lam_min"] > 1e-5 * (1.0 + cn)
    assert res2["kkt"] <= 1e-5  # only the missing certificate keeps it from OK
    prob.close()


def test_certified_stop_at_a_clustered_spectrum_is_sound():
    """At a tight tolerance the bottom of the slack's spectrum is a cluster of
    about rank-many eigenvalues near zero, where the Ritz residual stalls above
    its own tolerance.  The solve stops once the low end of the Ritz interval
    is dual feasible; the oracle's exact lambda_min at the returned dual must
    then meet the tolerance as well, so the stop is sound."""
    g = gen.er_graph(5000, 30000, 23, "gauss")
    po = oracle.maxcut_sdp(g)
    cn = float(np.sqrt(po.C.multiply(po.C).sum()))
    prob = _maxcut(g, r_max=64, kmax=60)
    st, res, R, y = prob.solve(gen.init_factor(g.n, 16, 1), eps_kkt=1e-5, sigma=16.0, max_outer=300)
    print(f"status {st} outer {res['outer']} kkt {res['kkt']:.2e} theta {res['lam_min']:.3e} "
          f"resid {res['lanczos_resid']:.3e} dtol {1e-5 * (1 + cn):.3e}")
    assert st == 0
    assert res["lanczos_resid"] - res["lam_min"] <= 1e-5 * (1.0 + cn) * (1 + 1e-12)
    yh = y.cpu().numpy()
    lam = oracle.min_eig(po, yh)
    k = oracle.kkt(po, R.cpu().numpy(), yh, lam_min=lam)
    print(f"oracle lambda_min {lam:.3e}: kkt {k['kkt']:.2e} (dinf {k['dinf']:.2e})")
    assert k["dinf"] <= 1e-5 and k["kkt"] <= 1.2e-5
    prob.close()


def test_solve_gpu_matches_oracle_trajectory_short():
    """Same start, same options, a few outer iterations: final objective and
    dual agree with the oracle's run (discrete decisions coincide on this case)."""
    g = gen.er_graph(400, 2000, 8, "gauss")
    po = oracle.maxcut_sdp(g)
    R0 = gen.init_factor(400, 6, 2)
    opts = dict(eps_kkt=1e-12, max_outer=3, max_inner=40, rank_policy=1)
    prob = _maxcut(g, r_max=16, kmax=100)
    st, res, R, y = prob.solve(R0, **opts)
    out = oracle.solve(po, R0, opts=oracle.SolveOptions(eps_kkt=1e-12, max_outer=3, max_inner=40,
                                                        rank_policy="fixed", r_max=16))
    Ro, yo = out["R"], out["y"]
    assert abs(res["pobj"] - out["kkt"]["pobj"]) <= 1e-9 * abs(out["kkt"]["pobj"])
    assert np.linalg.norm(y.cpu().numpy() - yo) <= 1e-8 * np.linalg.norm(yo)
    Xg = R.cpu().numpy() @ R.cpu().numpy().T
    assert np.linalg.norm(Xg - Ro @ Ro.T) <= 1e-8 * np.linalg.norm(Ro @ Ro.T)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_solve_mixed_precision_reports_error(prec):
    g = gen.er_graph(2000, 10000, 1, "unit")
    gold = json.load(open(os.path.join(GOLDEN, "maxcut_er2000_solve.json")))
    prob = _maxcut(g, prec=prec, r_max=64, kmax=100)
    st, res, R, y = prob.solve(gen.init_factor(2000, 8, 1), eps_kkt=1e-4, sigma=1.0)
    err = abs(res["pobj"] - gold["pobj"]) / abs(gold["pobj"])
    print(f"{prec}: status {st} outer {res['outer']} kkt {res['kkt']:.2e} rel obj err vs FP64 oracle {err:.2e} "
          f"promoted_at {res['promoted_at_outer']}")
    assert st == 0 and err <= 2e-4


def test_bf16_ladder_factor_is_the_certified_point():
    """A BF16 solve to 1e-5 has to switch to float storage (BF16 rounding of R
    alone moves A(RR^T) by about 2^-9 per row).  Its status and KKT values refer
    to the float factor, which alm_bm_ladder_factor returns: the oracle's KKT
    measure with the exact lambda_min at that factor meets the tolerance, while
    the BF16 copy left in R is farther from feasibility."""
    g = gen.er_graph(2000, 10000, 1, "unit")
    po = oracle.maxcut_sdp(g)
    prob = _maxcut(g, prec="bf16", r_max=64, kmax=100)
    st, res, R, y = prob.solve(gen.init_factor(2000, 8, 1), eps_kkt=1e-5, sigma=1.0, max_outer=400)
    print(f"status {st} outer {res['outer']} promoted at {res['promoted_at_outer']} kkt {res['kkt']:.2e}")
    assert st == 0 and res["promoted_at_outer"] >= 0
    Rf = prob.ladder_factor(res["rank"])
    assert Rf.dtype == torch.float32 and tuple(Rf.shape) == (2000, res["rank"])
    yh = y.cpu().numpy()
    lam = oracle.min_eig(po, yh)
    kf = oracle.kkt(po, Rf.double().cpu().numpy(), yh, lam_min=lam)
    kb = oracle.kkt(po, R.double().cpu().numpy(), yh, lam_min=lam)
    print(f"oracle at the float factor: kkt {kf['kkt']:.2e} (pinf {kf['pinf']:.2e}); "
          f"at the BF16 copy: kkt {kb['kkt']:.2e} (pinf {kb['pinf']:.2e})")
    assert kf["kkt"] <= 1.5e-5
    assert kb["pinf"] > kf["pinf"]
    assert np.allclose(R.float().cpu().numpy(), Rf.to(torch.bfloat16).float().cpu().numpy())
    with pytest.raises(almbm().AlmBmError):
        prob.ladder_factor(res["rank"] + 1)
    prob.close()
    p64 = _maxcut(g, r_max=16, kmax=20)
    with pytest.raises(almbm().AlmBmError):
        p64.ladder_factor(4)
    p64.close()


@pytest.mark.parametrize("n,expect", [(5, math.sqrt(5.0)), (7, 7 * math.cos(math.pi / 7) / (1 + math.cos(math.pi / 7)))])
def test_solve_lovasz_theta_cycles_with_edge_penalty(n, expect):
    g = gen.cycle_graph(n)
    prob = almbm().Problem.lovasz(n, g.ei, g.ej, precision="f64", r_max=8, lanczos_kmax=n, device=DEV)
    st, res, R, y = prob.solve(gen.init_factor(n, 3, 1), eps_kkt=1e-6, sigma_edges=float(n), max_outer=400,
                               max_inner=2000)
    print(f"lovasz C{n} with edge penalty: status {st} theta {-res['pobj']:.10f} expect {expect:.10f}")
    assert st == 0 and math.isclose(-res["pobj"], expect, rel_tol=1e-5)


def test_solve_lovasz_random_graph_with_edge_penalty_oracle_kkt():
    """G(500, 5000): with sigma on the trace row only the solve stays near X = J/n;
    with the edge rows at 10 n sigma it converges, and the oracle's KKT measure
    (exact eigensolver) at the returned point agrees."""
    g = gen.er_graph(500, 5000, 4, "unit")
    prob = almbm().Problem.lovasz(g.n, g.ei, g.ej, precision="f64", r_max=64, lanczos_kmax=60, device=DEV)
    R0 = gen.init_factor(g.n, 16, 4) / math.sqrt(g.n)
    st, res, R, y = prob.solve(R0, eps_kkt=1e-4, sigma_edges=10.0 * g.n, max_outer=600, time_limit_s=100)
    print(f"lovasz G(500,5000): status {st} outer {res['outer']} rank {res['rank']} kkt {res['kkt']:.2e} "
          f"theta {-res['pobj']:.8f} time {res['time_s']:.1f}s")
    assert st == 0
    po = oracle.lovasz_sdp(g)
    k = oracle.kkt(po, R.cpu().numpy(), y.cpu().numpy())
    print(f"oracle KKT at the GPU point: {k}")
    assert k["kkt"] <= 2e-4


@pytest.mark.parametrize("n", [9, 64])
def test_penalty_schedule_cycles_closed_form(n):
    """Penalty schedule from sigma = 1e-3 (x10 whenever pinf falls by less than
    4x): the closed form is reached and the penalty only grew."""
    g = gen.cycle_graph(n)
    prob = _maxcut(g, r_max=8, kmax=min(n, 60))
    st, res, R, y = prob.solve(gen.init_factor(n, 2, 1), eps_kkt=1e-8, sigma=1e-3, sigma_growth=10.0,
                               max_outer=400, max_inner=2000)
    val = -res["pobj"]
    expect = n if n % 2 == 0 else n * (1 + math.cos(math.pi / n)) / 2
    print(f"cycle {n} with schedule: status {st} value {val:.12f} expect {expect:.12f} outer {res['outer']} "
          f"sigma {res['sigma_final']:.1e} ({res['sigma_increases']} increases)")
    assert st == 0
    assert math.isclose(val, expect, rel_tol=1e-6)
    assert res["sigma_increases"] >= 1 and res["sigma_final"] > 1e-3


def test_penalty_schedule_er_workload():
    """G(2000, 10^4): the scheduled solve from sigma = 1e-2 and the fixed
    sigma = 1 solve reach the same objective, and the oracle's KKT at the
    scheduled solve's point meets the tolerance."""
    g = gen.er_graph(2000, 10000, 1, "unit")
    eps = 1e-6
    out = {}
    for name, kw in (("fixed", {}), ("schedule", {"sigma": 1e-2, "sigma_growth": 4.0})):
        prob = _maxcut(g, r_max=48, kmax=100)
        st, res, R, y = prob.solve(gen.init_factor(g.n, 8, 1), eps_kkt=eps, max_outer=500, **kw)
        print(f"ER 2000 {name}: status {st} outer {res['outer']} inner {res['inner_total']} rank {res['rank']} "
              f"pobj {res['pobj']:.12e} sigma {res['sigma_final']:.2e} time {res['time_s']:.2f}s", flush=True)
        assert st == 0
        out[name] = (res, R, y)
    d = abs(out["schedule"][0]["pobj"] - out["fixed"][0]["pobj"]) / abs(out["fixed"][0]["pobj"])
    assert d <= 1e-5
    assert out["schedule"][0]["sigma_increases"] >= 1
    _, R, y = out["schedule"]
    k = _oracle_kkt(oracle.maxcut_sdp(g), R.double().cpu().numpy(), y.cpu().numpy())
    print(f"oracle KKT at the scheduled solve's point: {k['kkt']:.2e}")
    assert k["kkt"] <= 2 * eps


@pytest.mark.parametrize("n,q", [(9, 3), (64, 4)])
def test_block_rank_step_cycles_closed_form(n, q):
    """Rank steps with q directions (Ritz vectors of a full Lanczos pass and the
    small PSD subproblem) from rank 1: the closed forms are reached."""
    g = gen.cycle_graph(n)
    prob = _maxcut(g, r_max=16, kmax=min(n, 60), rank_block_max=q)
    st, res, R, y = prob.solve(gen.init_factor(n, 1, 1), eps_kkt=1e-8, rank_block=q, max_outer=400, max_inner=2000)
    val = -res["pobj"]
    expect = n if n % 2 == 0 else n * (1 + math.cos(math.pi / n)) / 2
    print(f"cycle {n} rank_block {q}: status {st} value {val:.12f} expect {expect:.12f} outer {res['outer']} "
          f"rank {res['rank']} expansions {res['expansions']}", flush=True)
    assert st == 0
    assert math.isclose(val, expect, rel_tol=1e-6)


def test_block_rank_step_er_workload():
    """G(2000, 10^4) from rank 1 with 4 directions per rank step: the same
    objective as the one-vector steps and the oracle's KKT at the returned
    point."""
    g = gen.er_graph(2000, 10000, 1, "unit")
    eps = 1e-6
    out = {}
    for q in (1, 4):
        prob = _maxcut(g, r_max=48, kmax=100, rank_block_max=q)
        st, res, R, y = prob.solve(gen.init_factor(g.n, 1, 1), eps_kkt=eps, rank_block=q, max_outer=500)
        print(f"ER 2000 from rank 1, rank_block {q}: status {st} outer {res['outer']} inner {res['inner_total']} "
              f"rank {res['rank']} pobj {res['pobj']:.12e} time {res['time_s']:.2f}s", flush=True)
        assert st == 0
        out[q] = (res, R, y)
    d = abs(out[4][0]["pobj"] - out[1][0]["pobj"]) / abs(out[1][0]["pobj"])
    assert d <= 1e-5
    _, R, y = out[4]
    k = _oracle_kkt(oracle.maxcut_sdp(g), R.double().cpu().numpy(), y.cpu().numpy())
    print(f"oracle KKT at the block-step solve's point: {k['kkt']:.2e}", flush=True)
    assert k["kkt"] <= 2 * eps


def test_block_rank_step_lovasz_c5():
    """Lovasz theta of C5 (trace row + edge rows, C = -J) from rank 1 with 2
    directions per rank step and the edge penalty: sqrt(5)."""
    g = gen.cycle_graph(5)
    prob = almbm().Problem.lovasz(5, g.ei, g.ej, precision="f64", r_max=8, lanczos_kmax=5, device=DEV, rank_block_max=2)
    st, res, R, y = prob.solve(gen.init_factor(5, 1, 1), eps_kkt=1e-6, sigma_edges=5.0, rank_block=2,
                               max_outer=400, max_inner=2000)
    print(f"lovasz C5 rank_block 2: status {st} value {-res['pobj']:.10f} outer {res['outer']} rank {res['rank']}",
          flush=True)
    assert st == 0
    assert math.isclose(-res["pobj"], math.sqrt(5.0), rel_tol=1e-5)
