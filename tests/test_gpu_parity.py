"""Per-call parity of the HIP path against the FP64 oracle (GPU only).

FP64 mode: normwise relative error <= 1e-10 for G, A(RR^T), y+ and the line
search coefficients; scalars within 1e-10 relative.  FP32 / BF16 modes report
their error against the FP64 oracle on the same (FP64) input and bound it
loosely (storage rounding: ~1e-7 and ~4e-3 relative per entry).
"""

import math

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def almbm():
    import paper_2505_15775_amd as m

    return m


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def _case_graph(name):
    if name == "er2000":      # the n = 2000, average degree 10 ER workload
        return gen.er_graph(2000, 10000, 1, "unit")
    if name == "er3001g":     # ragged row count, Gaussian weights, several tiles
        return gen.er_graph(3001, 20000, 2, "gauss")
    if name == "torus":       # 30 x 41 torus, +-1 weights, degree 4
        return gen.torus_graph(30, 41, 3, "pm1")
    if name == "edgeless":
        return gen.edgeless_graph(97)
    if name == "single":
        return gen.edgeless_graph(1)
    raise KeyError(name)


DIAG_CASES = [
    ("er2000", 8, False), ("er3001g", 16, False), ("torus", 16, False), ("torus", 16, True),
    ("er3001g", 5, False), ("er3001g", 17, False), ("er2000", 1, False), ("er2000", 32, False),
    ("er3001g", 64, False), ("edgeless", 4, False), ("single", 3, False),
]


@pytest.mark.parametrize("name,r,ell", DIAG_CASES)
def test_objective_grad_diag_f64(name, r, ell):
    g = _case_graph(name)
    print(f"case {name} n={g.n} r={r} ell={ell}", flush=True)
    prob = almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=max(r, 8), lanczos_kmax=0,
                                  device=DEV, ell=ell)
    po = oracle.maxcut_sdp(g)
    rng = np.random.default_rng(7)
    R = gen.init_factor(g.n, r, 4) * (1.0 + 0.2 * rng.standard_normal((g.n, 1)))
    y = rng.standard_normal(g.n)
    sigma = 1.7
    f, G, Av = prob.objective_grad(prob.factor(R), torch.from_numpy(y).to(DEV), sigma)
    torch.cuda.synchronize()
    f_o, G_o, a_o, _ = oracle.objective_grad(po, R, y, sigma)
    assert abs(f.item() - f_o) <= 1e-10 * max(1.0, abs(f_o))
    assert rel(G.cpu(), G_o) <= 1e-10
    assert rel(Av.cpu(), a_o) <= 1e-10


@pytest.mark.parametrize("name,r,ell", DIAG_CASES)
def test_cost_apply_f64(name, r, ell):
    """P = C X and <X, C X> against the oracle's sparse product."""
    g = _case_graph(name)
    prob = almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=max(r, 8), lanczos_kmax=0,
                                  device=DEV, ell=ell)
    po = oracle.maxcut_sdp(g)
    X = np.random.default_rng(11).standard_normal((g.n, r))
    P, xpx = prob.cost_apply(prob.factor(X), want_xpx=True)
    torch.cuda.synchronize()
    P_o = oracle.cost_apply(po, X)
    assert rel(P.cpu(), P_o) <= 1e-10
    x_o = float(np.sum(X * P_o))
    assert abs(xpx.item() - x_o) <= 1e-10 * max(1.0, float(np.sum(np.abs(X * P_o))))


@pytest.mark.parametrize("prec,bound", [("f32", 1e-6), ("bf16", 1e-2)])
def test_cost_apply_reduced_precision(prec, bound):
    g = _case_graph("er3001g")
    prob = almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision=prec, r_max=16, lanczos_kmax=0, device=DEV)
    X = np.random.default_rng(12).standard_normal((g.n, 16))
    Xs = prob.factor(X)
    P = prob.cost_apply(Xs)
    torch.cuda.synchronize()
    assert P.dtype == torch.float32
    # against the oracle on the stored (rounded) factor: only float accumulation differs
    P_o = oracle.cost_apply(oracle.maxcut_sdp(g), Xs.double().cpu().numpy())
    err = rel(P.cpu(), P_o)
    print(f"cost_apply {prec}: rel err vs FP64 product of the stored factor {err:.2e}")
    assert err <= bound


def test_cost_apply_rejects_j_term():
    m = almbm()
    g = gen.cycle_graph(5)
    lov = m.Problem.lovasz(5, g.ei, g.ej, precision="f64", r_max=4, lanczos_kmax=0, device=DEV)
    with pytest.raises(m.AlmBmError):
        lov.cost_apply(lov.factor(np.ones((5, 2))))


@pytest.mark.parametrize("name,r", [("er2000", 8), ("er3001g", 16), ("torus", 5)])
def test_line_search_diag_f64(name, r):
    g = _case_graph(name)
    prob = almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=32, lanczos_kmax=0, device=DEV)
    po = oracle.maxcut_sdp(g)
    rng = np.random.default_rng(9)
    R = gen.init_factor(g.n, r, 5)
    y = -0.5 * np.ones(g.n) + 0.1 * rng.standard_normal(g.n)
    sigma = 1.0
    _, G_o, a_o, P_o = oracle.objective_grad(po, R, y, sigma)
    k_o = oracle.line_search_coeffs(po, R, G_o, y, sigma, P_o, a_o)
    t_o = oracle.quartic_argmin(k_o)
    k, t = prob.line_search(prob.factor(R), prob.factor(G_o), torch.from_numpy(y).to(DEV), sigma)
    torch.cuda.synchronize()
    k = k.cpu().numpy()
    assert np.max(np.abs(k - k_o)) <= 1e-10 * np.max(np.abs(k_o))
    assert abs(t.item() - t_o) <= 1e-8 * max(t_o, 1e-300)
    assert t_o > 0


def test_dual_update_parity():
    g = _case_graph("er3001g")
    prob = almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=8, lanczos_kmax=0, device=DEV)
    po = oracle.maxcut_sdp(g)
    rng = np.random.default_rng(2)
    a = 1.0 + 0.3 * rng.standard_normal(g.n)
    y = rng.standard_normal(g.n)
    y_t = torch.from_numpy(y.copy()).to(DEV)
    pinf = prob.dual_update(torch.from_numpy(a).to(DEV), 2.5, y_t)
    torch.cuda.synchronize()
    y_o, pinf_o = oracle.dual_update(po, a, 2.5, y)
    assert rel(y_t.cpu(), y_o) <= 1e-15
    assert math.isclose(pinf.item(), pinf_o, rel_tol=1e-12)


@pytest.mark.parametrize("name", ["er2000", "torus"])
def test_lanczos_min_eig(name):
    g = _case_graph(name)
    prob = almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=8, lanczos_kmax=400, device=DEV)
    po = oracle.maxcut_sdp(g)
    rng = np.random.default_rng(4)
    deg = np.bincount(np.concatenate([g.ei, g.ej]), minlength=g.n).astype(float)
    y = -deg / 4.0 + 0.3 * rng.standard_normal(g.n)
    lam_o = oracle.min_eig(po, y)
    S = oracle.slack_dense(po, y)
    snorm = np.linalg.norm(S, 2)
    theta, v, resid, iters = prob.lanczos_min_eig(torch.from_numpy(y).to(DEV), max_iter=400, tol=1e-9 * snorm)
    vv = v.cpu().numpy()
    print(f"lanczos {name}: theta {theta:.12e} exact {lam_o:.12e} resid {resid:.2e} iters {iters}")
    assert theta >= lam_o - 1e-10 * snorm          # a Ritz value bounds lambda_min from above
    assert theta - lam_o <= 1e-8 * snorm
    assert abs(np.linalg.norm(vv) - 1.0) <= 1e-10
    # the returned residual is the true one
    assert math.isclose(resid, np.linalg.norm(S @ vv - theta * vv), rel_tol=1e-6, abs_tol=1e-12 * snorm)


# ----------------------------------------------------------------- edge family


def _lovasz_case(n, m, seed):
    g = gen.er_graph(n, m, seed, "unit")
    return g, oracle.lovasz_sdp(g)


@pytest.mark.parametrize("n,m,r", [(300, 1500, 8), (1001, 6000, 32), (257, 900, 3)])
def test_objective_grad_lovasz_f64(n, m, r):
    g, po = _lovasz_case(n, m, 3)
    prob = almbm().Problem.lovasz(g.n, g.ei, g.ej, precision="f64", r_max=max(r, 8), lanczos_kmax=0, device=DEV)
    rng = np.random.default_rng(8)
    R = rng.standard_normal((n, r)) / math.sqrt(n * r)
    y = rng.standard_normal(po.m)
    sigma = 1.4
    f, G, Av = prob.objective_grad(prob.factor(R), torch.from_numpy(y).to(DEV), sigma)
    torch.cuda.synchronize()
    f_o, G_o, a_o, P_o = oracle.objective_grad(po, R, y, sigma)
    assert abs(f.item() - f_o) <= 1e-10 * max(1.0, abs(f_o))
    assert rel(G.cpu(), G_o) <= 1e-10
    assert rel(Av.cpu(), a_o) <= 1e-10
    k_o = oracle.line_search_coeffs(po, R, G_o, y, sigma, P_o, a_o)
    k, t = prob.line_search(prob.factor(R), prob.factor(G_o), torch.from_numpy(y).to(DEV), sigma)
    torch.cuda.synchronize()
    assert np.max(np.abs(k.cpu().numpy() - k_o)) <= 1e-10 * np.max(np.abs(k_o))
    assert abs(t.item() - oracle.quartic_argmin(k_o)) <= 1e-8 * oracle.quartic_argmin(k_o)


def test_edges_with_sparse_cost_and_diag():
    """Edge family with a CSR cost part, a diagonal and a -J term together."""
    n, m = 400, 2000
    g = gen.er_graph(n, m, 12, "unit")
    h = gen.er_graph(n, 1200, 13, "gauss")
    rng = np.random.default_rng(1)
    almbm_ = almbm()
    rp, ci, cv, dg = almbm_.maxcut_cost(n, h.ei, h.ej, h.w)
    dg = dg + rng.standard_normal(n)
    b = rng.standard_normal(m + 1)
    import scipy.sparse as sp
    Cs = sp.csr_matrix((cv, ci, rp), shape=(n, n)) + sp.diags(dg)
    po = oracle.edges_sdp(n, Cs, b, 0.6, g.ei, g.ej, j_coef=0.35)
    prob = almbm_.Problem.edges(n, g.ei, g.ej, b, 0.6, j_coef=0.35, cost_csr=(rp, ci, cv), cost_diag=dg,
                                precision="f64", r_max=16, lanczos_kmax=200, device=DEV)
    R = rng.standard_normal((n, 6))
    y = rng.standard_normal(m + 1)
    f, G, Av = prob.objective_grad(prob.factor(R), torch.from_numpy(y).to(DEV), 0.8)
    torch.cuda.synchronize()
    f_o, G_o, a_o, _ = oracle.objective_grad(po, R, y, 0.8)
    assert abs(f.item() - f_o) <= 1e-10 * max(1.0, abs(f_o))
    assert rel(G.cpu(), G_o) <= 1e-10
    assert rel(Av.cpu(), a_o) <= 1e-10
    lam_o = oracle.min_eig(po, y)
    snorm = np.linalg.norm(oracle.slack_dense(po, y), 2)
    theta, v, resid, iters = prob.lanczos_min_eig(torch.from_numpy(y).to(DEV), max_iter=200, tol=1e-9 * snorm)
    assert lam_o - 1e-10 * snorm <= theta <= lam_o + 1e-8 * snorm


def test_spurious_stationary_point_on_gpu():
    """Sec. 4.3, prop. on the necessity of dual localness (d = 5, k = 3, rho = eta = 1,
    eps = 0.1): the HIP path returns G = 0, A(FF^T) = b and lambda_min = -eps."""
    d, k, eps = 5, 3, 0.1
    ei = np.arange(d - 1)
    ej = np.full(d - 1, d - 1)
    b = np.zeros(d)
    b[0] = eps * k
    diag = eps * np.concatenate([2.0 * np.ones(d - 1), [1.0]])
    prob = almbm().Problem.edges(d, ei, ej, b, eps, cost_diag=diag, precision="f64", r_max=8, lanczos_kmax=5,
                                 device=DEV)
    F = np.zeros((d, k))
    F[:k, :k] = np.eye(k)
    y = np.zeros(d)
    y[0] = 2.0
    yt = torch.from_numpy(y).to(DEV)
    f, G, Av = prob.objective_grad(prob.factor(F), yt, 1.0)
    torch.cuda.synchronize()
    assert float(G.abs().max()) <= 1e-15
    np.testing.assert_allclose(Av.cpu().numpy(), b, atol=1e-15)
    theta, v, resid, iters = prob.lanczos_min_eig(yt, max_iter=5, tol=1e-14)
    assert math.isclose(theta, -eps, rel_tol=1e-12)


# ----------------------------------------------------------------- precision modes


@pytest.mark.parametrize("prec,bound", [("f32", 2e-6), ("bf16", 2e-2)])
@pytest.mark.parametrize("name,r", [("er2000", 8), ("torus", 16)])
def test_precision_modes_error_vs_f64_oracle(prec, bound, name, r):
    """Two comparisons with the FP64 oracle.  (1) At the FP64 factor: the
    error of the mode, dominated in BF16 by rounding the factor (half an ulp
    is 2^-9 relative per entry), reported and bounded loosely.  (2) At the
    factor as stored (the oracle evaluates the rounded values), which isolates
    the kernels' arithmetic: FP32 sums of r-term row products with FP64
    accumulation across rows and FP32 copies of the cost values (2^-24
    relative) give about 1e-7 on f and A(RR^T); G is additionally stored in
    the storage type, at most half an ulp per entry (2^-24 in FP32, 2^-9 in
    BF16), so its bounds are 2e-6 and 2^-9 + 2e-6."""
    g = _case_graph(name)
    prob = almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision=prec, r_max=16, lanczos_kmax=0, device=DEV)
    po = oracle.maxcut_sdp(g)
    rng = np.random.default_rng(7)
    R = gen.init_factor(g.n, r, 4)
    y = -0.6 + 0.1 * rng.standard_normal(g.n)
    Rs = prob.factor(R)
    f, G, Av = prob.objective_grad(Rs, torch.from_numpy(y).to(DEV), 1.0)
    torch.cuda.synchronize()
    f_o, G_o, a_o, _ = oracle.objective_grad(po, R, y, 1.0)
    ef = abs(f.item() - f_o) / abs(f_o)
    eg = rel(G.float().cpu(), G_o)
    ea = rel(Av.cpu(), a_o)
    print(f"precision {prec} {name}: rel err f {ef:.2e} G {eg:.2e} A(RR^T) {ea:.2e}")
    assert ef <= bound and eg <= 5 * bound and ea <= bound
    Rr = Rs.double().cpu().numpy()
    f_r, G_r, a_r, _ = oracle.objective_grad(po, Rr, y, 1.0)
    ef2 = abs(f.item() - f_r) / abs(f_r)
    eg2 = rel(G.double().cpu(), G_r)
    ea2 = rel(Av.cpu(), a_r)
    print(f"  at the stored factor: rel err f {ef2:.2e} G {eg2:.2e} A(RR^T) {ea2:.2e}")
    g_bound = 2e-6 if prec == "f32" else 2.0 ** -9 + 2e-6
    assert ef2 <= 1e-6 and ea2 <= 1e-6 and eg2 <= g_bound


# ----------------------------------------------------------------- inner loop


@pytest.mark.parametrize("name,r,refresh", [("er2000", 8, 0), ("er3001g", 16, 1), ("torus", 7, 5)])
def test_inner_solve_matches_oracle_gradient_descent(name, r, refresh):
    """30 steps of the graph-captured inner loop (carried cost product, refresh
    schedule) against 30 steps of the oracle's gradient descent with exact line
    search from the same start: same iterate up to rounding."""
    g = _case_graph(name)
    prob = almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=32, lanczos_kmax=0, device=DEV)
    po = oracle.maxcut_sdp(g)
    rng = np.random.default_rng(3)
    R0 = gen.init_factor(g.n, r, 6)
    y = -0.5 + 0.2 * rng.standard_normal(g.n)
    Rt = prob.factor(R0)
    done, flag, f_last = prob.inner_solve(Rt, torch.from_numpy(y).to(DEV), 0.0, 30, sigma=1.0,
                                          refresh_every=refresh, graph_unroll=8)
    assert done == 30 and flag == 2
    Ro, info = oracle.inner_gd(po, R0, y, 1.0, 0.0, 30)
    Rg = Rt.cpu().numpy()
    print(f"inner {name} r={r} refresh={refresh}: rel diff R {rel(Rg, Ro):.2e}")
    assert rel(Rg, Ro) <= 1e-9
    assert abs(f_last - oracle.objective(po, Ro, y, 1.0)) <= 1e-9 * abs(f_last)


def test_inner_solve_stops_at_tolerance_like_oracle():
    g = _case_graph("er2000")
    prob = almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=32, lanczos_kmax=0, device=DEV)
    po = oracle.maxcut_sdp(g)
    R0 = gen.init_factor(g.n, 8, 2)
    y = np.full(g.n, -1.5)
    for tol, max_steps in [(1e-2, 500), (3e-3, 400)]:
        Rt = prob.factor(R0)
        done, flag, _ = prob.inner_solve(Rt, torch.from_numpy(y).to(DEV), tol, max_steps, sigma=1.0)
        Ro, info = oracle.inner_gd(po, R0, y, 1.0, tol, max_steps)
        print(f"tol {tol}: gpu steps {done} flag {flag}; oracle steps {info['iters']} converged {info['converged']}")
        assert (flag == 1) == info["converged"] and done == info["iters"]
        assert rel(Rt.cpu().numpy(), Ro) <= 1e-8


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_tile_variants_and_grids_agree(prec):
    g = _case_graph("er3001g")
    prob = almbm().Problem.maxcut(g.n, g.ei, g.ej, g.w, precision=prec, r_max=16, lanczos_kmax=0, device=DEV)
    R = prob.factor(gen.init_factor(g.n, 16, 1))
    y = torch.full((g.n,), -0.7, dtype=torch.float64, device=DEV)
    ref = None
    for v in (0, 1, 2):
        for nb in (8, 64, 368):
            prob.set_tiles(v, nb)
            f, G, Av = prob.objective_grad(R, y, 1.0)
            out = (f.item(), G.double().cpu().numpy(), Av.cpu().numpy())
            if ref is None:
                ref = out
            tol = 1e-13 if prec == "f64" else 1e-5
            assert abs(out[0] - ref[0]) <= tol * abs(ref[0])
            assert rel(out[1], ref[1]) <= (tol if prec != "bf16" else 1e-2)
    v, nb = prob.autotune(16, reps=2)
    assert 0 <= v <= 2 and nb % 8 == 0
