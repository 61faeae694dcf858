"""Batched solves (GPU only): every instance of a batch against its own
single-instance solve and against the oracle's KKT measure at the batch's
point, closed forms inside a batch, determinism, and the zero-padding
invariant of the shared row width."""

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


def _instances():
    insts = [(gen.cycle_graph(8), 2), (gen.cycle_graph(9), 2)]
    for (g, r) in gen.batch_instances(6, 3, n_lo=300, n_hi=3000, deg_lo=4, deg_hi=12, ranks=(4, 8)):
        insts.append((g, r))
    return insts


def _problems(insts, prec="f64", r_max=48):
    m = _almbm()
    return [m.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision=prec, r_max=r_max, lanczos_kmax=60, device=DEV)
            for g, _ in insts]


def test_batch_matches_single_solves_and_oracle_kkt():
    insts = _instances()
    probs = _problems(insts)
    stride = 48  # the two largest instances reach rank 31 and 32 at the optimum
    batch = _almbm().Batch(probs, rank_stride=stride)
    factors = [gen.init_factor(g.n, r, 1) for g, r in insts]
    st, sts, res, R, ranks, y = batch.solve(factors, eps_kkt=1e-6, max_outer=400)
    print(f"batch: status {st} per-instance {sts} outer {[x['outer'] for x in res]} ranks {ranks}")
    assert st == 0 and all(s == 0 for s in sts)
    for q, ((g, r), p) in enumerate(zip(insts, probs)):
        s1, r1, Rq1, yq1 = p.solve(factors[q], eps_kkt=1e-6, max_outer=400)
        assert s1 == 0
        Rq, yq = batch.instance(q, R, y, ranks[q])
        po = oracle.maxcut_sdp(g)
        lam = oracle.min_eig(po, yq.cpu().numpy())
        k = oracle.kkt(po, Rq.cpu().numpy(), yq.cpu().numpy(), lam_min=lam)
        print(f"instance {q} n={g.n}: batch pobj {res[q]['pobj']:.10f} single {r1['pobj']:.10f} "
              f"oracle kkt {k['kkt']:.2e}")
        assert abs(res[q]["pobj"] - r1["pobj"]) <= 2e-6 * abs(r1["pobj"])
        assert k["pinf"] <= 1e-6 and k["gap"] <= 1e-6 and k["dinf"] <= 2e-6
    # closed forms of the two cycles
    assert math.isclose(-res[0]["pobj"], 8.0, rel_tol=1e-5)
    assert math.isclose(-res[1]["pobj"], 9 * (1 + math.cos(math.pi / 9)) / 2, rel_tol=1e-5)
    # padding columns stay exactly zero
    for q in range(len(insts)):
        a, b = batch.offsets[q], batch.offsets[q + 1]
        assert float(R[a:b, ranks[q]:].abs().max() if ranks[q] < stride else 0.0) == 0.0


def test_batch_deterministic():
    insts = _instances()[2:6]
    outs = []
    for _ in range(2):
        batch = _almbm().Batch(_problems(insts, prec="f32", r_max=16), rank_stride=16)
        st, sts, res, R, ranks, y = batch.solve([gen.init_factor(g.n, r, 2) for g, r in insts], eps_kkt=1e-5)
        outs.append((R.cpu().numpy().copy(), y.cpu().numpy().copy(), ranks))
        batch.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


def test_batch_rejects_edge_family():
    m = _almbm()
    g = gen.cycle_graph(5)
    lov = m.Problem.lovasz(5, g.ei, g.ej, precision="f64", r_max=8, lanczos_kmax=5, device=DEV)
    with pytest.raises(m.AlmBmError):
        m.Batch([lov], rank_stride=8)


def test_batch_uneven_recipe_32_instances():
    """The first 32 instances of the uneven batch recipe (n log-uniform in
    [1e3, 2e5], average degree uniform in [4, 32], +-1 weights, r in {8, 16};
    sum n = 8.6e5, sum nnz = 1.7e7), FP64, sigma = 16, 1e-4 KKT: every instance
    converges, its objective agrees with its own single solve to what 1e-4 KKT
    fixes, and for n <= 4000 the oracle's KKT measure (exact lambda_min) at the
    batch's point meets the tolerance."""
    insts = gen.batch_instances(32, 3)
    m = _almbm()
    probs = [m.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=64, lanczos_kmax=40, device=DEV,
                              validate=False) for g, _ in insts]
    batch = m.Batch(probs, rank_stride=64)
    factors = [gen.init_factor(g.n, r, 1) for g, r in insts]
    opts = dict(eps_kkt=1e-4, sigma=16.0, max_outer=300)
    st, sts, res, R, ranks, y = batch.solve(factors, **opts)
    print(f"batch of 32: status {st}, outer max {max(x['outer'] for x in res)}, ranks {ranks}", flush=True)
    assert st == 0 and all(s == 0 for s in sts)
    worst = 0.0
    for q, ((g, r), p) in enumerate(zip(insts, probs)):
        s1, r1, _, _ = p.solve(factors[q], **opts)
        assert s1 == 0
        d = abs(res[q]["pobj"] - r1["pobj"]) / abs(r1["pobj"])
        worst = max(worst, d)
        if g.n <= 4000:
            Rq, yq = batch.instance(q, R, y, ranks[q])
            po = oracle.maxcut_sdp(g)
            yh = yq.cpu().numpy()
            k = oracle.kkt(po, Rq.cpu().numpy(), yh, lam_min=oracle.min_eig(po, yh))
            print(f"instance {q} n={g.n}: oracle kkt {k['kkt']:.2e}, objective vs single {d:.1e}", flush=True)
            assert k["kkt"] <= 2e-4
    print(f"largest relative objective difference batch vs single: {worst:.2e}")
    assert worst <= 2e-3
    batch.close()
    for p in probs:
        p.close()


def test_batch_graph_reuse_and_tuned_tiles():
    """A batch with tuned tiles (alm_bm_batch_autotune): the table covers every
    width the stride allows, two solves on the tuned handle agree bitwise, and
    the tuned solve converges to the untuned one's objectives (the variants only
    reorder row sums).  The captured step is reused while the running set and
    widths are unchanged, which the same-handle repeat also exercises."""
    insts = _instances()[2:8]
    m = _almbm()
    factors = [gen.init_factor(g.n, r, 2) for g, r in insts]
    opts = dict(eps_kkt=1e-6, max_outer=300)
    plain = m.Batch(_problems(insts, prec="f64"), rank_stride=48)
    st0, sts0, res0, _, _, _ = plain.solve(factors, **opts)
    plain.close()
    assert st0 == 0
    tuned = m.Batch(_problems(insts, prec="f64"), rank_stride=48)
    table = tuned.autotune(reps=2)
    print(f"tuned variants per width: {table}")
    assert sorted(table) == [4, 8, 16, 32, 48] and all(v in (0, 1, 2) for v in table.values())
    outs = []
    for _ in range(2):
        st, sts, res, R, ranks, y = tuned.solve(factors, **opts)
        assert st == 0 and all(s == 0 for s in sts)
        outs.append((R.cpu().numpy().copy(), y.cpu().numpy().copy(), ranks, [x["pobj"] for x in res]))
    tuned.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    for q in range(len(insts)):
        assert abs(outs[0][3][q] - res0[q]["pobj"]) <= 2e-6 * abs(res0[q]["pobj"])


def test_batch_lbfgs_matches_single_lbfgs_solves_and_oracle_kkt():
    """L-BFGS subproblems inside a batch (per-instance memories, ring regions
    and partial slots from the block table): every instance converges, agrees
    with its own single L-BFGS solve to what 1e-6 KKT fixes, meets the oracle's
    KKT measure, and two batched solves agree bitwise."""
    insts = _instances()
    m = _almbm()

    def probs():
        return [m.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=48, lanczos_kmax=60, device=DEV,
                                 lbfgs_memory_max=4) for g, _ in insts]

    factors = [gen.init_factor(g.n, r, 1) for g, r in insts]
    opts = dict(eps_kkt=1e-6, max_outer=400, inner_solver=1, lbfgs_memory=3, max_inner=100)
    outs = []
    for rep in range(2):
        ps = probs()
        batch = m.Batch(ps, rank_stride=48)
        st, sts, res, R, ranks, y = batch.solve(factors, **opts)
        print(f"batched L-BFGS: status {st} {sts} outer {[x['outer'] for x in res]} "
              f"inner {[x['inner_total'] for x in res]} ranks {ranks}", flush=True)
        assert st == 0 and all(s == 0 for s in sts)
        outs.append((R.cpu().numpy().copy(), y.cpu().numpy().copy()))
        if rep == 0:
            for q, ((g, r), p) in enumerate(zip(insts, ps)):
                s1, r1, _, _ = p.solve(factors[q], **opts)
                assert s1 == 0
                Rq, yq = batch.instance(q, R, y, ranks[q])
                po = oracle.maxcut_sdp(g)
                yh = yq.cpu().numpy()
                k = oracle.kkt(po, Rq.cpu().numpy(), yh, lam_min=oracle.min_eig(po, yh))
                print(f"instance {q} n={g.n}: batch pobj {res[q]['pobj']:.10f} single {r1['pobj']:.10f} "
                      f"inner {res[q]['inner_total']} vs {r1['inner_total']}; oracle kkt {k['kkt']:.2e}", flush=True)
                assert abs(res[q]["pobj"] - r1["pobj"]) <= 2e-6 * abs(r1["pobj"])
                assert k["pinf"] <= 1e-6 and k["gap"] <= 1e-6 and k["dinf"] <= 2e-6
        batch.close()
        for p in ps:
            p.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_batch_lbfgs_rejects_memory_beyond_reservation():
    insts = _instances()[:2]
    m = _almbm()
    batch = m.Batch(_problems(insts), rank_stride=16)  # instances reserve no L-BFGS rings
    with pytest.raises(m.AlmBmError):
        batch.solve([gen.init_factor(g.n, r, 1) for g, r in insts], inner_solver=1, lbfgs_memory=3)
    batch.close()


def test_batch_lbfgs_float_storage_with_bfloat16_rings():
    """FP32 storage (L-BFGS rings in BF16, the line-search product gathering the
    BF16 direction): the batch converges, and each instance's objective agrees
    with its own single FP32 L-BFGS solve to what 1e-5 KKT fixes."""
    insts = _instances()[:6]
    m = _almbm()
    probs = [m.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f32", r_max=48, lanczos_kmax=60, device=DEV,
                              lbfgs_memory_max=3) for g, _ in insts]
    batch = m.Batch(probs, rank_stride=48)
    factors = [gen.init_factor(g.n, r, 1) for g, r in insts]
    opts = dict(eps_kkt=1e-5, max_outer=300, inner_solver=1, lbfgs_memory=3, max_inner=100)
    st, sts, res, R, ranks, y = batch.solve(factors, **opts)
    print(f"f32 batch L-BFGS: status {st} {sts} outer {[x['outer'] for x in res]} ranks {ranks}")
    assert st == 0 and all(s == 0 for s in sts)
    for q, p in enumerate(probs):
        s1, r1, _, _ = p.solve(factors[q], **opts)
        assert s1 == 0
        print(f"instance {q}: batch {res[q]['pobj']:.8f} single {r1['pobj']:.8f}")
        assert abs(res[q]["pobj"] - r1["pobj"]) <= 5e-5 * abs(r1["pobj"])
    batch.close()
    for p in probs:
        p.close()
