"""Benchmark of the ALM-BM hot path on one MI355X.

Workload (default): MaxCut SDP relaxation on an Erdos-Renyi graph with
n = 10,000,000 vertices and M = 40,000,000 edges (average degree 8), N(0,1)
edge weights, rank r = 16, factor stored in BF16 with FP32 arithmetic; inputs
synthetic and resident in HBM before timing.

A step is one inner iteration of the method as run inside the solve: the fused
objective + gradient pass (C R, A(RR^T), adjoint, objective terms), the exact
line search (the product C G and the quartic's roots) and the update R <- R - tG.
Each step is one gradient evaluation, so steps/s = gradient evaluations/s.
The rows evaluated once per outer iteration (dual update, Lanczos matvec and
reorthogonalisation) are timed separately and reported under "per_outer".

Usage: python bench.py [--steps K] [--warmup W] [--precision bf16|f32|f64] [--no-solve]
                       [--n N] [--deg D] [--rank R] [--modes] [--inner lbfgs|gd]
                       [--no-cpu-baseline]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LANCZOS_STEPS = 20
METRIC = "ALM-BM grad evals/sec + HBM GB/s, n=10M MaxCut; wall time to 1e-4 rel KKT"
COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters.json")
KERNEL_SOURCES = ["paper_2505_15775_amd/csrc/diag_kernels.hip", "paper_2505_15775_amd/csrc/spmm_row.hpp",
                  "paper_2505_15775_amd/csrc/common.hpp", "paper_2505_15775_amd/csrc/kernels.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def objgrad_bytes(n, nnz, r, prec):
    """Compulsory HBM bytes of one objective/gradient pass (DIAG family):
    CSR row_ptr + col_idx + values, diagonal, read R once, y, b, write G and A(RR^T)."""
    vb = 8 if prec == "f64" else 4
    rb = {"f64": 8, "f32": 4, "bf16": 2}[prec]
    return (n + 1) * 4 + nnz * (4 + vb) + n * vb + 2 * n * r * rb + 3 * n * 8


def spmm_bytes(n, nnz, r, prec):
    """Compulsory HBM bytes of one cost product P = C X: CSR row_ptr + col_idx +
    values, diagonal, read X once, write P (arithmetic precision)."""
    vb = 8 if prec == "f64" else 4
    rb = {"f64": 8, "f32": 4, "bf16": 2}[prec]
    return (n + 1) * 4 + nnz * (4 + vb) + n * vb + n * r * rb + n * r * vb


def time_events(fn, iters):
    import torch

    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(iters):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / 1000.0


def bench_mode(g, prec, r, steps, warmup, seed, refresh_every=0, lbfgs_memory=0):
    import torch

    import gen
    import paper_2505_15775_amd as almbm

    dev = torch.device("cuda:0")
    t0 = time.time()
    prob = almbm.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision=prec, r_max=r, lanczos_kmax=LANCZOS_STEPS,
                                device=dev, validate=False, lbfgs_memory_max=lbfgs_memory)
    log(f"[bench] {prec}: problem resident in {time.time() - t0:.1f}s (nnz {prob.desc.nnz})")
    R = prob.factor(torch.from_numpy(gen.init_factor(g.n, r, seed)))
    y = torch.zeros(g.n, dtype=torch.float64, device=dev)
    f = torch.empty(1, dtype=torch.float64, device=dev)
    t = torch.empty(1, dtype=torch.float64, device=dev)
    G = torch.empty_like(R)
    Av = torch.empty(g.n, dtype=torch.float64, device=dev)
    sigma = 1.0

    # the solve's inner loop (graph-captured, one sparse product per step between
    # refreshes), run for a fixed number of steps (tolerance 0: never stops early)
    prob.inner_solve(R, y, 0.0, warmup, sigma=sigma, refresh_every=refresh_every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    done, flag, f_last = prob.inner_solve(R, y, 0.0, steps, sigma=sigma, refresh_every=refresh_every)
    el = time.perf_counter() - t1
    assert done == steps and flag == 2, (done, flag)
    log(f"[bench] {prec}: {steps} inner steps in {el:.3f}s, f={f_last:.6e}")
    lb_el = None
    if lbfgs_memory > 0:
        # the same loop with the L-BFGS direction (one gradient evaluation per
        # step plus the streaming of the stored vectors)
        R2 = R.clone()
        lopts = dict(sigma=sigma, refresh_every=refresh_every, inner_solver=1, lbfgs_memory=lbfgs_memory)
        prob.inner_solve(R2, y, 0.0, warmup, **lopts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        done, flag, _ = prob.inner_solve(R2, y, 0.0, steps, **lopts)
        lb_el = time.perf_counter() - t1
        assert done == steps and flag == 2, (done, flag)
        log(f"[bench] {prec}: {steps} L-BFGS steps (memory {lbfgs_memory}) in {lb_el:.3f}s")
        del R2

    # the dominant kernel alone (objective/gradient pass + its one-block finalize)
    from paper_2505_15775_amd import _lib, _ptr, _stream  # noqa: F401

    def og():
        _lib.check(_lib.lib.alm_bm_objective_grad(prob._h, r, _ptr(R), _ptr(y), sigma, _ptr(f), _ptr(G), _ptr(Av),
                                                  _stream()), "objective_grad")

    for _ in range(max(2, warmup)):
        og()
    n_og = max(steps, 10)
    el_og = time_events(og, n_og)
    per_og = el_og / n_og

    # the dominant kernel of an inner step: the sparse cost product (C G in the
    # line search), launched alone through alm_bm_cost_apply on the same stream
    P = torch.empty(R.shape, dtype=torch.float64 if prec == "f64" else torch.float32, device=dev)

    def cp():
        _lib.check(_lib.lib.alm_bm_cost_apply(prob._h, r, _ptr(G), _ptr(P), None, _stream()), "cost_apply")

    for _ in range(max(2, warmup)):
        cp()
    el_cp = time_events(cp, n_og)
    per_cp = el_cp / n_og
    nnz = int(prob.desc.nnz)
    out = {"steps_per_s": steps / el, "ms_per_step": 1000.0 * el / steps,
           "lbfgs_steps_per_s": (steps / lb_el) if lb_el else None,
           "objgrad_ms": 1000.0 * per_og, "objgrad_evals_per_s": 1.0 / per_og,
           "objgrad_bytes": objgrad_bytes(g.n, nnz, r, prec),
           "spmm_ms": 1000.0 * per_cp, "spmm_bytes": spmm_bytes(g.n, nnz, r, prec)}
    out["objgrad_gbs"] = out["objgrad_bytes"] / per_og / 1e9
    out["spmm_gbs"] = out["spmm_bytes"] / per_cp / 1e9
    out["spmm_gathers_per_s"] = nnz / per_cp
    # cache-line requests of one product: every gathered row is a separate
    # request of ceil(row bytes / 128) lines; the streamed arrays add bytes/128
    rb = {"f64": 8, "f32": 4, "bf16": 2}[prec]
    lines = nnz * -(-(r * rb) // 128) + out["spmm_bytes"] / 128.0
    out["spmm_line_requests"] = lines
    out["spmm_line_requests_per_s"] = lines / per_cp
    return prob, R, y, out


def per_outer_rows(prob, y, steps):
    """Dual update and Lanczos (slack matvec + two Gram-Schmidt passes per step,
    host tridiagonal solve every few steps) at full size, FP64."""
    import torch

    Av = torch.ones(prob.n, dtype=torch.float64, device=y.device)
    yy = y.clone()
    el = time_events(lambda: prob.dual_update(Av, 1.0, yy), steps)
    yl = -torch.ones(prob.n, dtype=torch.float64, device=y.device)
    prob.lanczos_min_eig(yl, max_iter=4, tol=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, iters = prob.lanczos_min_eig(yl, max_iter=LANCZOS_STEPS, tol=0.0)
    tl = time.perf_counter() - t0
    return {"dual_update_ms": 1000.0 * el / steps, "lanczos_steps": iters,
            "lanczos_ms_total": 1000.0 * tl, "lanczos_ms_per_step": 1000.0 * tl / max(1, iters)}


def batch_leg(count, eps, sigma, prec, seed=3, loop=True, tune=True, inner="lbfgs"):
    """Uneven MaxCut instances (n log-uniform in [1e3, 2e5], average degree
    uniform in [4, 32], +-1 weights, r in {8, 16}) solved together by one
    batched solve, then one by one with the same options."""
    import torch

    import gen
    import paper_2505_15775_amd as almbm

    insts = gen.batch_instances(count, seed)
    sum_n = sum(g.n for g, _ in insts)
    sum_nnz = sum(2 * g.m_edges for g, _ in insts)
    log(f"[bench] batch: {count} instances, sum n {sum_n}, sum nnz {sum_nnz}")
    lbm = 3 if inner == "lbfgs" else 0
    probs = [almbm.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision=prec, r_max=64, lanczos_kmax=40, device="cuda:0",
                                  validate=False, lbfgs_memory_max=lbm) for g, _ in insts]
    batch = almbm.Batch(probs, rank_stride=64)
    table, t_tune = None, 0.0
    if tune:
        t0 = time.perf_counter()
        table = batch.autotune(reps=3)
        t_tune = time.perf_counter() - t0
        log(f"[bench] batch: tile variants per width {table} (tuned in {t_tune:.2f}s)")
    factors = [gen.init_factor(g.n, r, 1) for g, r in insts]
    opts = dict(eps_kkt=eps, sigma=sigma, max_outer=300)
    if inner == "lbfgs":
        opts.update(inner_solver=1, lbfgs_memory=3, max_inner=100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, sts, res, _, ranks, _ = batch.solve(factors, verbose=1, **opts)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    log(f"[bench] batch: batched solve {tb:.1f}s, {sum(s == 0 for s in sts)}/{count} converged")
    t0 = time.perf_counter()
    nconv = 0
    worst = 0.0
    for q, p in enumerate(probs if loop else []):
        s1, r1, _, _ = p.solve(factors[q], **opts)
        nconv += int(s1 == 0)
        worst = max(worst, abs(r1["pobj"] - res[q]["pobj"]) / abs(r1["pobj"]))
        if q % 8 == 0:
            log(f"[bench] batch loop: instance {q} n={p.n} outer {r1['outer']} {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    if loop:
        log(f"[bench] batch: per-instance loop {tl:.1f}s, {nconv}/{count} converged")
    batch.close()
    for p in probs:
        p.close()
    return {"instances": count, "sum_n": sum_n, "sum_nnz": sum_nnz, "precision": prec, "eps_kkt": eps,
            "sigma": sigma, "inner_solver": inner, "max_inner": opts.get("max_inner", 500), "batched_s": round(tb, 2), "batched_converged": int(sum(s == 0 for s in sts)),
            "loop_s": round(tl, 2) if loop else None, "loop_converged": nconv if loop else None,
            "speedup": round(tl / tb, 3) if loop else None,
            "max_outer_batched": int(max(x["outer"] for x in res)),
            "max_rel_objective_diff": worst if loop else None,
            "tile_variants": {str(k): v for k, v in table.items()} if table else None,
            "tune_s": round(t_tune, 3)}


def kernels_leg(g, reps=20):
    """The rows outside the MaxCut step: the edge family (Lovasz theta,
    G(1e5, 1e6), r = 32, FP32: SDDMM + adjoint product + objective) and the
    warm start's kernels at the full size (features; MLP forward and
    backward, 8 -> 32 -> 32 -> 1, FP32)."""
    import numpy as np
    import torch

    import gen
    import paper_2505_15775_amd as almbm
    from paper_2505_15775_amd import warmstart

    out = {}
    lv = gen.er_graph(100_000, 1_000_000, 4, "unit")
    pl = almbm.Problem.lovasz(lv.n, lv.ei, lv.ej, precision="f32", r_max=32, lanczos_kmax=0, device="cuda:0",
                              validate=False)
    R = pl.factor(torch.from_numpy(gen.init_factor(lv.n, 32, 4) / np.sqrt(lv.n)))
    y = torch.zeros(lv.m_edges + 1, dtype=torch.float64, device="cuda:0")
    for _ in range(3):
        pl.objective_grad(R, y, 1.0)
    t = time_events(lambda: pl.objective_grad(R, y, 1.0), reps) / reps
    E, n, r = lv.m_edges, lv.n, 32
    # pattern (2E ids + 2E edge ids + n+1 row ptr + E upper cols), R read twice (SDDMM, adjoint),
    # G write, y and A(RR^T) per edge (8 B each)
    byts = (2 * E * 4 + 2 * E * 4 + (n + 1) * 4 + E * 4) + 2 * n * r * 4 + n * r * 4 + 2 * (E + 1) * 8
    out["lovasz_objective_grad"] = {"n": n, "edges": E, "r": r, "precision": "f32", "ms": round(1000 * t, 4),
                                    "evals_per_s": round(1.0 / t, 2), "algorithmic_bytes": byts,
                                    "gbs": round(byts / t / 1e9, 1)}
    # the exact line search along a direction (passes 1-3 and their finalizers)
    _, Gd, _ = pl.objective_grad(R, y, 1.0)
    pl.line_search(R, Gd, y, 1.0)
    t = time_events(lambda: pl.line_search(R, Gd, y, 1.0), reps) / reps
    out["lovasz_line_search"] = {"ms": round(1000 * t, 4)}
    pl.close()

    pm = almbm.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f32", r_max=16, lanczos_kmax=0, device="cuda:0",
                              validate=False)
    for _ in range(2):
        F = warmstart.features(pm)
    t = time_events(lambda: warmstart.features(pm), 5) / 5
    nnz = int(pm.desc.nnz)
    out["ws_features"] = {"n": g.n, "ms": round(1000 * t, 3), "algorithmic_bytes": nnz * 8 + g.n * 40,
                          "gbs": round((nnz * 8 + g.n * 40) / t / 1e9, 1)}
    model = warmstart.WarmStartModel(h=32, device="cuda:0")
    model.predict_y0(pm, F)
    t = time_events(lambda: model.predict_y0(pm, F), 5) / 5
    h = 32
    flops = 2.0 * g.n * (8 * h + h * h + h)
    out["ws_mlp_forward"] = {"n": g.n, "h": h, "ms": round(1000 * t, 3), "tflops": round(flops / t / 1e12, 2),
                             "peak_fp32_vector_tflops": 157.3}
    T = torch.zeros(g.n, dtype=torch.float32, device="cuda:0")
    model.loss_grad(F, T)
    t = time_events(lambda: model.loss_grad(F, T), 3) / 3
    out["ws_mlp_loss_grad"] = {"n": g.n, "h": h, "ms": round(1000 * t, 3), "tflops": round(3 * flops / t / 1e12, 2)}
    pm.close()
    return out


# Matrix completion instances of Table 2 (r, n = n1 + n2, the paper's time in s
# to 1e-5 relative KKT on one A100-80GB-PCIe, and with initial rank 1).
TABLE2 = [(3, 10000, 0.379, 0.562), (3, 20000, 0.726, 1.040), (3, 50000, 1.409, 2.344), (3, 100000, 2.944, 3.929),
          (3, 200000, 5.511, 7.937), (3, 350000, 12.759, 14.956), (5, 10000, 0.504, 1.894), (5, 20000, 0.969, 3.349),
          (5, 50000, 3.025, 8.745), (5, 100000, 6.762, 17.297)]


def completion_leg(prec="f64", eps=1e-5, rank_one_upto=20000, sigma=0.03, rows=None):
    """The matrix completion instances of Table 2 (generated with the paper's
    recipe, seeded), solved to its tolerance from rank r (and from rank 1 on
    the smaller ones), beside the paper's A100 times for context.  The paper
    gives no penalty for this workload; sigma = 0.03 was the fastest of
    0.03, 0.1, 0.3 and 1 over these instances (the subproblems' gradient
    steps shrink about tenfold from sigma = 1, for a few more outer steps)."""
    import torch

    import gen
    import paper_2505_15775_amd as almbm

    out = []
    for r, n, t_paper, t_paper_r1 in (TABLE2 if rows is None else rows):
        inst = gen.completion_instance(n // 2, n - n // 2, r, 1)
        p = almbm.Problem.matrix_completion(inst.n1, inst.n2, inst.rows, inst.cols, inst.vals, precision=prec,
                                            r_max=32, lanczos_kmax=60, device="cuda:0", validate=False)
        row = {"r": r, "n": n, "m": inst.m, "sigma": sigma, "paper_a100_s": t_paper, "paper_a100_rank1_s": t_paper_r1}
        starts = [("from_rank_r", r)] + ([("from_rank_1", 1)] if n <= rank_one_upto else [])
        for name, r0 in starts:
            torch.cuda.synchronize()
            st, res, _, _ = p.solve(gen.init_factor(inst.n, r0, 1), eps_kkt=eps, sigma=sigma, max_outer=1000,
                                    time_limit_s=120)
            row[name] = {"status": int(st), "time_s": round(res["time_s"], 3), "outer": res["outer"],
                         "inner": res["inner_total"], "lanczos_s": round(res["time_lanczos_s"], 3),
                         "rank": res["rank"], "kkt": res["kkt"], "objective": res["pobj"]}
        log(f"[bench] completion r={r} n={n} m={inst.m}: {row}")
        out.append(row)
        p.close()
        del p
        torch.cuda.empty_cache()
    return out


def rmat_leg(scale=22, edge_factor=8, r=16, precs=("bf16", "f64"), reps=20):
    """Skewed degrees: MaxCut on an R-MAT graph (2^scale vertices, about
    edge_factor * 2^scale edges, N(0,1) weights).  Times the cost product and
    the objective/gradient pass with the default hub rows and with none."""
    import numpy as np
    import torch

    import gen
    import paper_2505_15775_amd as almbm
    from paper_2505_15775_amd import _lib, _ptr, _stream

    t0 = time.time()
    g = gen.rmat_graph(scale, edge_factor, 7, "gauss")
    deg = np.bincount(np.concatenate([g.ei, g.ej]), minlength=g.n)
    log(f"[bench] R-MAT 2^{scale}: E={g.m_edges} max degree {int(deg.max())} generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    out = {"workload": f"MaxCut SDP on R-MAT 2^{scale} (a,b,c,d = 0.57,0.19,0.19,0.05), E={g.m_edges}, "
                       f"N(0,1) weights, r={r}", "n": g.n, "edges": int(g.m_edges), "max_degree": int(deg.max())}
    for prec in precs:
        prob = almbm.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision=prec, r_max=r, lanczos_kmax=0, device=dev,
                                    validate=False)
        X = prob.factor(torch.from_numpy(gen.init_factor(g.n, r, 1)))
        y = torch.zeros(g.n, dtype=torch.float64, device=dev)
        P = torch.empty(X.shape, dtype=torch.float64 if prec == "f64" else torch.float32, device=dev)
        G = torch.empty_like(X)
        Av = torch.empty(g.n, dtype=torch.float64, device=dev)
        f = torch.empty(1, dtype=torch.float64, device=dev)
        nnz = int(prob.desc.nnz)
        rb = {"f64": 8, "f32": 4, "bf16": 2}[prec]

        def cp():
            _lib.check(_lib.lib.alm_bm_cost_apply(prob._h, r, _ptr(X), _ptr(P), None, _stream()), "cost_apply")

        def og():
            _lib.check(_lib.lib.alm_bm_objective_grad(prob._h, r, _ptr(X), _ptr(y), 1.0, _ptr(f), _ptr(G), _ptr(Av),
                                                      _stream()), "objective_grad")

        row = {}
        for name, thr in (("hubs", 0), ("no_hubs", -1)):
            nh = prob.set_hub_threshold(thr)
            for fn in (cp, og):
                fn()
            per_cp = time_events(cp, reps) / reps
            per_og = time_events(og, reps) / reps
            by = spmm_bytes(g.n, nnz, r, prec)
            lines = nnz * -(-(r * rb) // 128) + by / 128.0
            row[name] = {"hub_rows": nh, "cost_product_ms": round(1000 * per_cp, 4),
                         "objgrad_ms": round(1000 * per_og, 4), "line_requests_per_s": round(lines / per_cp, 0),
                         "cost_product_gbs": round(by / per_cp / 1e9, 1)}
            log(f"[bench] R-MAT {prec} {name}: {row[name]}")
        out[prec] = row
        prob.close()
        del prob
        torch.cuda.empty_cache()
    return out


def gather_probe_leg(rows_list=(500_000, 2_000_000, 10_000_000, 40_000_000), widths=(8, 32, 128), count=80_000_000,
                     reps=5, seed=11):
    """Gathered rows per second of the library's random-row gather probe for
    tables of rows x width bytes (int32 indices uniform over the rows, count
    gathers per launch): the ceiling the sparse cost product runs against.
    Tables above 2.56 GB are skipped."""
    import torch

    from paper_2505_15775_amd import _lib, _ptr, _stream

    dev = torch.device("cuda:0")
    gen_ = torch.Generator(device=dev)
    gen_.manual_seed(seed)
    out = torch.empty(_lib.lib.alm_bm_gather_probe_out_size(), dtype=torch.float32, device=dev)
    res = []
    for rows in rows_list:
        idx = torch.randint(0, rows, (count,), dtype=torch.int32, device=dev, generator=gen_)
        for wb in widths:
            if rows * wb > 2_560_000_000:
                continue
            table = torch.rand(rows * wb // 4, dtype=torch.float32, device=dev, generator=gen_)

            def run():
                _lib.check(_lib.lib.alm_bm_gather_probe(_ptr(table), rows, wb, _ptr(idx), count, _ptr(out),
                                                        _stream()), "gather_probe")

            run()
            t = time_events(run, reps) / reps
            res.append({"table_rows": rows, "row_bytes": wb, "table_mb": round(rows * wb / 1e6, 1),
                        "gathers": count, "ms": round(1000 * t, 4), "rows_per_s": round(count / t, 0),
                        "line_requests_per_s": round(count * -(-wb // 128) / t, 0)})
            log(f"[bench] gather probe: {res[-1]}")
            del table
        del idx
    del out
    torch.cuda.empty_cache()
    return res


def calibrate_copy(nbytes=1 << 30):
    """A plain elementwise copy of known size (read nbytes, write nbytes), for
    scaling the HBM byte counters of a profiled run."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy: {nbytes} bytes read, {nbytes} bytes written")
    del src, dst
    torch.cuda.empty_cache()


def cpu_baseline(n_full, deg, r, seed, evals=2):
    """The FP64 oracle's objective/gradient on a bounded sample of the same
    workload family: an ER graph with n/10 vertices and the same average degree
    and weight law, scaled to the full size by the row count."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import gen
    import oracle

    n_s = max(1000, n_full // 10)
    g = gen.er_graph(n_s, int(n_s * deg / 2), seed + 100, "gauss")
    p = oracle.maxcut_sdp(g)
    R = gen.init_factor(n_s, r, seed)
    y = np.zeros(n_s)
    with threadpool_limits(limits=1):
        oracle.objective_grad(p, R, y, 1.0)
        t0 = time.perf_counter()
        for _ in range(evals):
            oracle.objective_grad(p, R, y, 1.0)
        dt = (time.perf_counter() - t0) / evals
    scale = n_full / n_s
    return {"value": 1.0 / (dt * scale), "unit": "grad_evals/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle.objective_grad (FP64, NumPy/SciPy, 1 thread) on ER n={n_s} M={g.m_edges} "
                      f"N(0,1) weights r={r}, {evals} timed evals of {dt:.2f}s each, scaled by n ratio {scale:.1f}"}


def certified_bracket(pb, Rf, yf, lanczos_steps=200):
    """Bracket on the MaxCut SDP optimum (minimisation form) at a returned
    point, on an FP64 handle pb of the same cost.  Upper end: <C, X^> for X^
    with the rows of R scaled to unit length, a feasible point.  Lower end:
    sum(y) + n * theta, the dual objective of y + theta 1, which is dual
    feasible when theta <= lambda_min(C - Diag(y)); theta is the smallest Ritz
    value of a long Lanczos run, itself an upper bound on lambda_min, so the
    lower end holds as far as theta has converged (its residual is given)."""
    import torch

    Rn = Rf.to(dtype=torch.float64)
    Rn = (Rn / Rn.norm(dim=1, keepdim=True).clamp_min(1e-300)).contiguous()
    zero = torch.zeros(pb.n, dtype=torch.float64, device=Rn.device)
    f, _, _ = pb.objective_grad(Rn, zero, 0.0, want_G=False, want_Av=False)
    yd = yf.to(dtype=torch.float64).contiguous()
    theta, _, resid, iters = pb.lanczos_min_eig(yd, max_iter=lanczos_steps, tol=1e-9, want_vector=False)
    upper = f.item()
    lower = float(yd.sum().item()) + pb.n * theta
    return {"upper": upper, "lower": lower, "rel_width": (upper - lower) / abs(upper), "theta": theta,
            "theta_resid": resid, "lanczos_steps": iters}


def fp64_check(pb, Rf, leg):
    """<C, RR^T> and the primal infeasibility of the returned factor evaluated in
    FP64 (handle pb), against the values the solve reported in its precision."""
    import torch

    R64 = Rf.to(dtype=torch.float64).contiguous()
    zero = torch.zeros(pb.n, dtype=torch.float64, device=R64.device)
    f, _, Av = pb.objective_grad(R64, zero, 0.0, want_G=False)
    pobj = f.item()
    pinf = float(torch.linalg.norm(Av - 1.0).item()) / (1.0 + pb.n ** 0.5)
    return {"pobj": pobj, "rel_pobj_diff_vs_reported": abs(pobj - leg["pobj"]) / abs(pobj), "pinf": pinf}


def solve_legs(g, args):
    """Solves to 1e-4 relative KKT on the benchmark graph (the metric's third
    part): FP64 from the default start (R0 of rank r with unit rows, y = 0),
    the bench precision (BF16 storage, with the ladder to float) from the same
    start, and from the learned warm start.  Each reports wall time, outer and
    inner iterations, rank, the KKT terms, and the objective bracket."""
    import torch

    import gen
    import paper_2505_15775_amd as almbm
    from paper_2505_15775_amd import warmstart

    lbfgs = args.inner == "lbfgs"
    max_inner = args.max_inner or (100 if lbfgs else 500)
    keys = ("outer", "inner_total", "rank", "kkt", "pinf", "dinf", "gap", "pobj", "time_s", "time_lanczos_s",
            "promoted_at_outer", "sigma_final", "sigma_increases", "lam_min", "lanczos_resid")
    legs = {"f64": ("f64_default_start", "f64", False),
            "default": (f"{args.precision}_default_start", args.precision, False),
            "learned": (f"{args.precision}_learned_start", args.precision, True)}
    out, finals = {}, {}
    for leg in [x for x in args.solve_legs.split(",") if x]:
        name, pm, warm = legs[leg]
        log(f"[bench] solve leg {name}")
        ps = almbm.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision=pm, r_max=64, lanczos_kmax=60, device="cuda:0",
                                  validate=False, lbfgs_memory_max=args.lbfgs_memory if lbfgs else 0)
        limit = args.solve_time_limit_f64 if pm == "f64" else args.solve_time_limit
        opts = dict(eps_kkt=1e-4, sigma=args.sigma, max_inner=max_inner, time_limit_s=limit,
                    verbose=1, inner_solver=1 if lbfgs else 0, lbfgs_memory=args.lbfgs_memory)
        if args.sigma_growth != 1.0:
            opts["sigma_growth"] = args.sigma_growth
        if args.refresh_every:
            opts["refresh_every"] = args.refresh_every
        torch.cuda.synchronize()
        if warm:
            model = warmstart.WarmStartModel.load(device="cuda:0")
            st, res, Rf, yf, info = warmstart.solve_warm(ps, model, **opts)
            extra = {"r0": info["r0"], "fallback": info["fallback"], "predict_s": round(info["predict_s"], 3),
                     "total_s": round(info["total_s"], 3)}
        else:
            st, res, Rf, yf = ps.solve(gen.init_factor(g.n, args.rank, args.seed), **opts)
            extra = {}
        out[name] = {"status": int(st), "sigma": args.sigma, "sigma_growth": args.sigma_growth, "max_inner": max_inner,
                     "inner_solver": args.inner, "lbfgs_memory": args.lbfgs_memory if lbfgs else None,
                     **{k: res[k] for k in keys}, **extra}
        log(f"[bench] {name}: {out[name]}")
        if pm == "bf16" and res["promoted_at_outer"] >= 0:
            # the point the solve certified is its float factor (R holds it rounded to BF16)
            finals[name] = (ps.ladder_factor(res["rank"]), yf.clone())
            out[name]["factor"] = "float (after the ladder)"
        else:
            finals[name] = (Rf.clone(), yf.clone())
        ps.close()
        del ps, Rf, yf
        torch.cuda.empty_cache()
    if finals:
        pb = almbm.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=64, lanczos_kmax=200,
                                  device="cuda:0", validate=False)
        for name, (Rf, yf) in finals.items():
            out[name]["bracket"] = certified_bracket(pb, Rf, yf)
            out[name]["fp64_check"] = fp64_check(pb, Rf, out[name])
            log(f"[bench] {name} bracket: {out[name]['bracket']} fp64 check: {out[name]['fp64_check']}")
        pb.close()
        ref = out.get("f64_default_start")
        if ref:
            for name in out:
                if name != "f64_default_start":
                    out[name]["rel_objective_diff_vs_f64"] = abs(out[name]["pobj"] - ref["pobj"]) / abs(ref["pobj"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "f32", "f64"])
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--deg", type=float, default=8.0)
    ap.add_argument("--rank", type=int, default=16)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--modes", action="store_true", default=True,
                    help="also time the other two precisions (default on; --no-modes skips)")
    ap.add_argument("--no-modes", dest="modes", action="store_false")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the solves to 1e-4 relative KKT (FP64 and BF16-ladder default starts, learned start)")
    ap.add_argument("--solve-legs", default="f64,default,learned",
                    help="comma list of solve legs: f64 (FP64 default start), default (bench precision, default "
                         "start), learned (bench precision, learned warm start)")
    ap.add_argument("--solve-time-limit", type=float, default=120.0)
    ap.add_argument("--solve-time-limit-f64", type=float, default=240.0,
                    help="time limit of the FP64 solve leg (its steps at width 64 cost about 2.5x the float ones)")
    ap.add_argument("--sigma", type=float, default=16.0, help="penalty of the --solve leg")
    ap.add_argument("--refresh-every", type=int, default=0,
                    help="inner steps between full sparse evaluations (0: the library default for the precision)")
    ap.add_argument("--sigma-growth", type=float, default=1.0,
                    help="penalty schedule of the --solve legs: sigma x this factor whenever pinf falls by less than 4x")
    ap.add_argument("--max-inner", type=int, default=0,
                    help="gradient steps per subproblem in the solve legs (0: 100 for L-BFGS, 500 for GD)")
    ap.add_argument("--inner", default="lbfgs", choices=["lbfgs", "gd"], help="subproblem solver of the solve legs")
    ap.add_argument("--lbfgs-memory", type=int, default=3, help="L-BFGS pairs kept")
    ap.add_argument("--batch", type=int, default=256,
                    help="batched solve of this many uneven instances (0: skip); --batch-loop adds the per-instance loop")
    ap.add_argument("--batch-eps", type=float, default=1e-4)
    ap.add_argument("--batch-loop", action="store_true",
                    help="also solve the batch's instances one by one (about 150 s at 256 instances)")
    ap.add_argument("--batch-no-loop", action="store_true", help="(default) no per-instance loop")
    ap.add_argument("--only-batch", action="store_true",
                    help="run only the batch leg (--batch N) and print its JSON (profiling; no metric line)")
    ap.add_argument("--batch-no-tune", action="store_true", help="batch leg with the default tiles")
    ap.add_argument("--batch-precision", choices=["f64", "f32"], default="f64",
                    help="storage precision of the batch leg's instances")
    ap.add_argument("--batch-inner", choices=["lbfgs", "gd"], default="lbfgs",
                    help="subproblem solver of the batch leg (both the batch and the loop)")
    ap.add_argument("--kernels", action="store_true", help="also time the edge-family and warm-start kernels")
    ap.add_argument("--completion", action="store_true", help="also the matrix completion instances of Table 2")
    ap.add_argument("--completion-sigma", type=float, default=0.03, help="penalty for the matrix completion solves")
    ap.add_argument("--rmat", type=int, default=0, metavar="SCALE",
                    help="also the skewed-degree leg on an R-MAT graph with 2^SCALE vertices (e.g. 22)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gather-probe", action="store_true", help="skip the random-row gather ceiling sweep")
    ap.add_argument("--calibrate-copy", action="store_true", help="run a 1 GiB copy kernel first (profiling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import gen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        calibrate_copy()
    if args.only_batch:
        if args.batch < 1:
            print("--only-batch needs --batch N", file=sys.stderr)
            sys.exit(2)
        out = batch_leg(args.batch, args.batch_eps, args.sigma, args.batch_precision,
                        loop=args.batch_loop and not args.batch_no_loop,
                        tune=not args.batch_no_tune, inner=args.batch_inner)
        print(json.dumps({"batched_solve": out}))
        return
    t0 = time.time()
    M = int(args.n * args.deg / 2)
    g = gen.er_graph(args.n, M, args.seed, "gauss")
    log(f"[bench] graph n={g.n} M={g.m_edges} generated in {time.time() - t0:.1f}s")

    prob, R, y, main_out = bench_mode(g, args.precision, args.rank, args.steps, args.warmup, args.seed,
                                      args.refresh_every, args.lbfgs_memory)
    per_outer = per_outer_rows(prob, y, 20)
    modes = {}
    if args.modes:
        for pm in ("f64", "f32", "bf16"):
            if pm == args.precision:
                continue
            p2, _, _, o2 = bench_mode(g, pm, args.rank, max(10, args.steps // 2), 2, args.seed)
            modes[pm] = o2
            p2.close()
            torch.cuda.empty_cache()

    # traffic from the committed rocprofv3 counter summary, if it is for this kernel source
    traffic = traffic_og = None
    if os.path.exists(COUNTERS):
        c = json.load(open(COUNTERS))
        key = f"{args.precision}_n{args.n}_r{args.rank}"
        run = c.get("runs", {}).get(key)
        if c.get("kernel_source_hash") == kernel_source_hash() and run:
            traffic = run.get("k_quadq_diag", {}).get("hbm_bytes_per_launch")
            traffic_og = run.get("k_objgrad_diag", {}).get("hbm_bytes_per_launch")

    probe = None if args.no_gather_probe else gather_probe_leg()
    ach = main_out["spmm_gbs"]
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_quadq_diag (sparse cost product C X, one per inner step)",
                "algorithmic_bytes_per_launch": main_out["spmm_bytes"],
                "launch_ms": round(main_out["spmm_ms"], 4),
                "gathered_rows_per_s": round(main_out["spmm_gathers_per_s"], 0),
                "line_requests_per_launch": round(main_out["spmm_line_requests"], 0),
                "line_requests_per_s": round(main_out["spmm_line_requests_per_s"], 0),
                "objgrad": {"kernel": "k_objgrad_diag (full objective/gradient pass)",
                            "achieved": round(main_out["objgrad_gbs"], 1),
                            "frac": round(main_out["objgrad_gbs"] / HBM_PEAK_GBS, 4),
                            "algorithmic_bytes_per_launch": main_out["objgrad_bytes"],
                            "launch_ms": round(main_out["objgrad_ms"], 4), "traffic": traffic_og}}
    if probe:
        # the product's own shape: n rows of r * storage bytes, nnz gathers per launch
        rb = {"f64": 8, "f32": 4, "bf16": 2}[args.precision] * args.rank
        same = [x for x in probe if x["table_rows"] == args.n and x["row_bytes"] == rb]
        if same:
            roofline["gather_ceiling"] = {"probe_rows_per_s": same[0]["rows_per_s"],
                                          "product_rows_per_s": round(main_out["spmm_gathers_per_s"], 0),
                                          "frac": round(main_out["spmm_gathers_per_s"] / same[0]["rows_per_s"], 4)}

    solves = None
    if not args.no_solve:
        prob.close()
        del prob, R, y
        torch.cuda.empty_cache()
        solves = solve_legs(g, args)

    batch = batch_leg(args.batch, args.batch_eps, args.sigma, args.batch_precision,
                      loop=args.batch_loop and not args.batch_no_loop,
                      tune=not args.batch_no_tune, inner=args.batch_inner) if args.batch > 0 else None
    other = kernels_leg(g) if args.kernels else None
    completion = completion_leg(sigma=args.completion_sigma) if args.completion else None
    skewed = rmat_leg(args.rmat) if args.rmat else None

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.n, args.deg, args.rank, args.seed)

    line = {
        "metric": METRIC,
        "value": round(main_out["steps_per_s"], 3),
        "unit": "grad_evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_out["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"MaxCut SDP (C=-L/4, X_ii=1), Erdos-Renyi n={args.n} M={M} (avg degree "
                               f"{args.deg:g}), N(0,1) weights, r={args.rank}, "
                               f"{'BF16 R storage, FP32 arithmetic' if args.precision == 'bf16' else args.precision}",
                   "n": args.n, "nnz": int(2 * M), "r": args.rank, "precision": args.precision},
        "objgrad_evals_per_s": round(main_out["objgrad_evals_per_s"], 3),
        "lbfgs_steps_per_s": (round(main_out["lbfgs_steps_per_s"], 3) if main_out["lbfgs_steps_per_s"] else None),
        "per_outer": per_outer,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if modes:
        line["modes"] = {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                         for k, v in modes.items()}
    if solves:
        line["solve_to_1e-4_kkt"] = solves
    if probe:
        line["gather_probe"] = probe
    if batch is not None:
        line["batched_solve"] = batch
    if other is not None:
        line["other_kernels"] = other
    if completion is not None:
        line["matrix_completion_table2"] = completion
    if skewed is not None:
        line["skewed_degree"] = skewed
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
