"""Learned warm start on the GPU: feature and MLP kernels against the FP64
oracle (and finite differences through it), determinism, Adam, training, and
what the trained network gains over the default start (y = 0) on held-out
generated graphs."""

import math
import os

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import warmstart as ows

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _ws():
    from paper_2505_15775_amd import warmstart

    return warmstart


def _prob(g):
    import paper_2505_15775_amd as almbm

    return almbm.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=32, lanczos_kmax=60, device=DEV)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("g", [gen.er_graph(3001, 20000, 2, "gauss"), gen.torus_graph(30, 41, 3, "pm1"),
                               gen.er_graph(500, 300, 9, "unit")])
def test_features_match_oracle(g):
    prob = _prob(g)
    F = _ws().features(prob).cpu().numpy()
    Fo = ows.features(oracle.maxcut_sdp(g))
    np.testing.assert_allclose(F, Fo, rtol=2e-6, atol=2e-6)
    pool = _ws().pooled(torch.from_numpy(F.astype(np.float32)).to(DEV))
    np.testing.assert_allclose(pool, F.astype(np.float32).astype(np.float64).mean(axis=0), rtol=1e-9)


@pytest.mark.parametrize("h", [16, 32, 64])
def test_mlp_forward_and_gradient_match_oracle(h):
    ws = _ws()
    rng = np.random.default_rng(h)
    n = 5000
    m = ws.WarmStartModel(h=h, device=DEV, seed=h)
    X = rng.standard_normal((n, 8)).astype(np.float32) * 2 + 1
    T = rng.standard_normal(n).astype(np.float32)
    mu = rng.standard_normal(8).astype(np.float32)
    isd = (0.5 + rng.random(8)).astype(np.float32)
    m.mu = torch.from_numpy(mu).to(DEV)
    m.inv_sd = torch.from_numpy(isd).to(DEV)
    params = m.params.cpu().numpy().astype(np.float64)
    Xt, Tt = torch.from_numpy(X).to(DEV), torch.from_numpy(T).to(DEV)

    class P:  # minimal stand-in for a handle in predict_y0
        pass

    prob = P()
    prob.n = n
    out = m.predict_y0(prob, Xt).cpu().numpy()
    out_o = ows.mlp_forward(params, 8, h, mu.astype(np.float64), isd.astype(np.float64), X.astype(np.float64))
    assert rel(out, out_o) <= 2e-5
    loss, grad = m.loss_grad(Xt, Tt)
    loss2, grad2 = m.loss_grad(Xt, Tt)
    assert torch.equal(grad, grad2) and loss.item() == loss2.item()  # deterministic
    lo, go = ows.mlp_loss_grad(params, 8, h, mu.astype(np.float64), isd.astype(np.float64), X.astype(np.float64),
                               T.astype(np.float64))
    print(f"h={h}: loss {loss.item():.6f} oracle {lo:.6f}; grad rel err {rel(grad.cpu().numpy(), go):.2e}")
    assert math.isclose(loss.item(), lo, rel_tol=2e-5)
    assert rel(grad.cpu().numpy(), go) <= 2e-4


def test_adam_step_matches_definition():
    import ctypes as C

    from paper_2505_15775_amd import _ptr, _stream, check, lib

    rng = np.random.default_rng(1)
    k = 1000
    p, g, m, v = (rng.standard_normal(k).astype(np.float32) for _ in range(4))
    v = np.abs(v)
    tp, tg, tm, tv = (torch.from_numpy(a.copy()).to(DEV) for a in (p, g, m, v))
    check(lib.alm_bm_ws_adam(_ptr(tp), _ptr(tg), _ptr(tm), _ptr(tv), k, C.c_float(1e-2), C.c_float(0.9),
                             C.c_float(0.999), C.c_float(1e-8), 3, _stream()), "adam")
    m1 = 0.9 * m + 0.1 * g
    v1 = 0.999 * v + 0.001 * g * g
    p1 = p - 1e-2 * (m1 / (1 - 0.9 ** 3)) / (np.sqrt(v1 / (1 - 0.999 ** 3)) + 1e-8)
    np.testing.assert_allclose(tp.cpu().numpy(), p1, rtol=2e-5, atol=1e-6)


def test_training_reduces_loss():
    ws = _ws()
    g = gen.er_graph(20000, 80000, 4, "gauss")
    prob = _prob(g)
    st, res, R, y = prob.solve(gen.init_factor(g.n, 16, 1), eps_kkt=1e-5, max_outer=200)
    assert st == 0
    F = ws.features(prob)
    model = ws.WarmStartModel(h=32, device=DEV)
    hist = model.fit(F, y.float(), steps=200, batch=8192)
    print(f"training loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}")
    assert hist[-1][1] < 0.5 * hist[0][1]
    y0 = model.predict_y0(prob, F)
    err = float(torch.linalg.norm(y0 - y) / torch.linalg.norm(y))
    print(f"relative error of predicted y0 on the training graph: {err:.3f}")
    assert err < 0.2


@pytest.mark.skipif(not os.path.exists(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                                    "paper_2505_15775_amd", "warmstart_model.npz")),
                    reason="no trained warm-start model in the package")
def test_trained_warm_start_beats_default_start_on_held_out_graphs():
    """Held-out graphs (the first 10 % of the seeded training set, never used in
    training): outer iterations and wall time to 1e-5 relative KKT from the
    learned start against the default start and against the Gershgorin
    dual-feasible start; objectives agree."""
    ws = _ws()
    model = ws.WarmStartModel.load(device=DEV)
    graphs = ws.training_graphs(120, 6)[:4]
    tot_d = tot_w = tot_g = 0
    t_d = t_w = 0.0
    import paper_2505_15775_amd as almbm

    for g in graphs:
        # these graphs reach ranks 39-56 at 1e-5, so the cap must be above that
        prob = almbm.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=64, lanczos_kmax=60, device=DEV)
        st, rd, _, _ = prob.solve(gen.init_factor(g.n, 16, 1), eps_kkt=1e-5, sigma=16.0, max_outer=300)
        stw, rw, _, _, info = ws.solve_warm(prob, model, eps_kkt=1e-5, sigma=16.0, max_outer=300)
        # comparator: the Gershgorin dual-feasible start y0_i = C_ii - sum_j |C_ij| (feature 4)
        yg = ws.features(prob)[:, 4].double().contiguous()
        stg, rg, _, _ = prob.solve(gen.init_factor(g.n, 16, 1), yg, eps_kkt=1e-5, sigma=16.0, max_outer=300)
        assert stg == 0
        tot_g += rg["outer"]
        print(f"n={g.n}: default outer {rd['outer']} ({rd['time_s']:.2f}s) warm outer {rw['outer']} "
              f"({info['total_s']:.2f}s, r0 {info['r0']}, fallback {info['fallback']}) "
              f"pobj {rd['pobj']:.8e} vs {rw['pobj']:.8e}")
        assert st == 0 and stw == 0
        # both meet 1e-5 relative KKT, whose gap term alone allows each objective
        # about 2e-5 relative from its dual bound
        assert abs(rd["pobj"] - rw["pobj"]) <= 3e-5 * abs(rd["pobj"])
        tot_d += rd["outer"]
        tot_w += rw["outer"]
        t_d += rd["time_s"]
        t_w += info["total_s"]
        prob.close()
    print(f"total outer iterations: default {tot_d}, warm {tot_w}, Gershgorin {tot_g}; "
          f"time {t_d:.2f}s vs {t_w:.2f}s")
    assert tot_w < tot_d and tot_w < tot_g


@pytest.mark.parametrize("corrupt", ["nan", "huge"])
def test_warm_start_fallback_on_corrupted_dual(corrupt):
    """A corrupted proposed dual (NaN entries, or 1e6 everywhere) must not stop
    the solve: a NaN start falls back to the default start (y = 0, rank
    min(16, r_max), here below 16), a huge one either recovers or falls back;
    both end at a point whose KKT measure the oracle (exact lambda_min)
    confirms, at the default-start solve's objective."""
    ws = _ws()
    import paper_2505_15775_amd as almbm

    g = gen.er_graph(1500, 6000, 31, "gauss")
    po = oracle.maxcut_sdp(g)
    prob = almbm.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=12, lanczos_kmax=60, device=DEV)
    st_d, rd, _, _ = prob.solve(gen.init_factor(g.n, 8, 1), eps_kkt=1e-6, max_outer=300)
    assert st_d == 0
    y0 = torch.full((g.n,), float("nan") if corrupt == "nan" else 1e6, dtype=torch.float64, device=DEV)
    if corrupt == "nan":
        y0[::2] = 0.0  # NaN in part of the entries
    st, res, R, y, info = ws.solve_from(prob, gen.init_factor(g.n, 8, 1), y0, eps_kkt=1e-6, max_outer=300)
    print(f"{corrupt}: fallback {info['fallback']} ({info.get('reason', '')}) status {st} outer {res['outer']} "
          f"pobj {res['pobj']:.10e} vs default {rd['pobj']:.10e}")
    if corrupt == "nan":
        assert info["fallback"]
    assert st == 0
    yh = y.cpu().numpy()
    kk = oracle.kkt(po, R.cpu().numpy(), yh, lam_min=oracle.min_eig(po, yh))
    assert kk["kkt"] <= 2e-6
    assert abs(res["pobj"] - rd["pobj"]) <= 1e-5 * abs(rd["pobj"])
    prob.close()
