"""GPU test of alm_bm_objective_grad_noalloc, the objective/gradient call with
no handle and no device allocation (its partial sums sit in the library's
static per-GPU scratch array).  Two calls in a row, the second on a smaller
problem with a ragged rank, each checked against alm_bm_objective_grad on a
handle (same kernels and grid, so equal results) and against the FP64 oracle
(eq. AL-BM and its gradient, 1e-10 relative)."""

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2505_15775_amd as almbm

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def test_noalloc_objective_grad_two_calls_match_handle_and_oracle():
    dev = torch.device("cuda:0")
    cases = [(3000, 15000, 21, 16, 0.7), (777, 2500, 22, 5, 2.5)]  # the second call is smaller
    probs, inputs, outs = [], [], []
    for n, m, seed, r, sigma in cases:
        g = gen.er_graph(n, m, seed, "gauss")
        prob = almbm.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=r, lanczos_kmax=0, device=dev)
        rng = np.random.default_rng(seed)
        R = rng.standard_normal((n, r))
        y = rng.standard_normal(n)
        Rt = torch.from_numpy(R).to(dev)
        yt = torch.from_numpy(y).to(dev)
        f = torch.empty(1, dtype=torch.float64, device=dev)
        G = torch.empty((n, r), dtype=torch.float64, device=dev)
        Av = torch.empty(n, dtype=torch.float64, device=dev)
        ref = prob.objective_grad(Rt, yt, sigma)  # handle path, launched first
        probs.append((g, prob))
        inputs.append((R, y, Rt, yt, sigma))
        outs.append((f, G, Av, ref))
    # the first call on a device resolves the scratch array's address, which
    # makes the runtime load that code object (a one-time set-up of about
    # 2 MiB); it runs here on throwaway outputs, before memory is compared
    (g0, prob0), (_, _, Rt0, yt0, sigma0) = probs[0], inputs[0]
    almbm.objective_grad_noalloc(prob0.desc, Rt0, yt0, sigma0, torch.empty(1, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    free_before = torch.cuda.mem_get_info(dev)[0]
    for (g, prob), (_, _, Rt, yt, sigma), (f, G, Av, _) in zip(probs, inputs, outs):
        print(f"noalloc call: n={g.n} r={Rt.shape[1]} sigma={sigma}", flush=True)
        almbm.objective_grad_noalloc(prob.desc, Rt, yt, sigma, f, G, Av)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info(dev)[0] == free_before
    for (g, prob), (R, y, _, _, sigma), (f, G, Av, (f_h, G_h, Av_h)) in zip(probs, inputs, outs):
        assert f.item() == f_h.item()
        assert torch.equal(G, G_h) and torch.equal(Av, Av_h)
        f_o, G_o, a_o, _ = oracle.objective_grad(oracle.maxcut_sdp(g), R, y, sigma)
        ef = abs(f.item() - f_o) / abs(f_o)
        eg = _rel(G.cpu().numpy(), G_o)
        ea = _rel(Av.cpu().numpy(), a_o)
        print(f"n={g.n}: rel err f {ef:.2e} G {eg:.2e} A(RR^T) {ea:.2e}")
        assert ef <= 1e-10 and eg <= 1e-10 and ea <= 1e-10
    for _, prob in probs:
        prob.close()


def test_noalloc_objective_grad_optional_outputs_and_ell():
    """G and Av nullable; an ELL cost (the torus of degree 4)."""
    dev = torch.device("cuda:0")
    g = gen.torus_graph(40, 50, 7, "pm1")
    n, r, sigma = g.n, 8, 1.0
    prob = almbm.Problem.maxcut(n, g.ei, g.ej, g.w, precision="f64", r_max=r, lanczos_kmax=0, device=dev, ell=True)
    rng = np.random.default_rng(8)
    R = rng.standard_normal((n, r))
    y = rng.standard_normal(n)
    Rt = torch.from_numpy(R).to(dev)
    yt = torch.from_numpy(y).to(dev)
    f = torch.empty(1, dtype=torch.float64, device=dev)
    almbm.objective_grad_noalloc(prob.desc, Rt, yt, sigma, f)
    torch.cuda.synchronize()
    f_o, _, _, _ = oracle.objective_grad(oracle.maxcut_sdp(g), R, y, sigma)
    assert abs(f.item() - f_o) <= 1e-10 * abs(f_o)
    prob.close()
