"""Full-size parity (GPU only): the MaxCut workload of the benchmark, Erdos-Renyi
n = 10,000,000, M = 40,000,000, N(0,1) weights, r = 16, in the launch
configuration bench.py times.

* FP64: G and A(RR^T) on 2048 sampled rows against the oracle's row-by-row
  evaluation (1e-10), and f against the oracle's full objective (1e-10).
* BF16 storage: the same sampled rows, error against the FP64 oracle reported
  and bounded (storage rounding).
* Inner loop: after 12 steps with the carried cost product, the objective it
  reports equals a fresh full evaluation at the final factor (a property that
  holds at any size), and the objective decreased.
"""

import time

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N, M, RANK = 10_000_000, 40_000_000, 16


@pytest.fixture(scope="module")
def workload():
    t = time.time()
    g = gen.er_graph(N, M, 5, "gauss")
    rng = np.random.default_rng(17)
    R = gen.init_factor(N, RANK, 5)
    R *= (1.0 + 0.05 * rng.standard_normal((N, 1)))
    y = -0.5 + 0.1 * rng.standard_normal(N)
    rows = np.sort(rng.choice(N, size=2048, replace=False))
    print(f"workload generated in {time.time() - t:.1f}s", flush=True)
    return g, R, y, rows


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _problem(g, prec):
    import paper_2505_15775_amd as almbm

    return almbm.Problem.maxcut(g.n, g.ei, g.ej, g.w, precision=prec, r_max=RANK, lanczos_kmax=0, device=DEV,
                                validate=False)


def test_fullsize_f64_sampled_rows_and_objective(workload):
    g, R, y, rows = workload
    prob = _problem(g, "f64")
    sigma = 1.0
    Rt = prob.factor(R)
    f, G, Av = prob.objective_grad(Rt, torch.from_numpy(y).to(DEV), sigma)
    torch.cuda.synchronize()
    G_rows = G[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    a_rows = Av[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    del G, Av
    G_o, a_o = oracle.maxcut_objective_grad_rows(g, R, y, sigma, rows)
    print(f"full size f64: sampled rel err G {rel(G_rows, G_o):.2e} a {rel(a_rows, a_o):.2e}", flush=True)
    assert rel(G_rows, G_o) <= 1e-10
    assert rel(a_rows, a_o) <= 1e-10
    t = time.time()
    f_o = oracle.objective(oracle.maxcut_sdp(g), R, y, sigma)
    print(f"full size f64: f {f.item():.12e} oracle {f_o:.12e} (oracle {time.time() - t:.1f}s)", flush=True)
    assert abs(f.item() - f_o) <= 1e-10 * abs(f_o)
    prob.close()


def test_fullsize_bf16_sampled_rows(workload):
    g, R, y, rows = workload
    prob = _problem(g, "bf16")
    f, G, Av = prob.objective_grad(prob.factor(R), torch.from_numpy(y).to(DEV), 1.0)
    torch.cuda.synchronize()
    idx = torch.from_numpy(rows).to(DEV)
    G_rows = G[idx].double().cpu().numpy()
    a_rows = Av[idx].cpu().numpy()
    G_o, a_o = oracle.maxcut_objective_grad_rows(g, R, y, 1.0, rows)
    eg, ea = rel(G_rows, G_o), rel(a_rows, a_o)
    print(f"full size bf16 storage: sampled rel err vs FP64 oracle G {eg:.2e} a {ea:.2e}", flush=True)
    assert eg <= 2e-2 and ea <= 1e-2
    prob.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-11), ("f32", 2e-4), ("bf16", 3e-2)])
def test_fullsize_inner_loop_carried_product_consistent(workload, prec, tol):
    g, R, y, rows = workload
    prob = _problem(g, prec)
    Rt = prob.factor(R)
    yt = torch.from_numpy(y).to(DEV)
    f0, _, _ = prob.objective_grad(Rt, yt, 1.0, want_G=False, want_Av=False)
    done, flag, f_last = prob.inner_solve(Rt, yt, 0.0, 12, sigma=1.0)
    f1, _, _ = prob.objective_grad(Rt, yt, 1.0, want_G=False, want_Av=False)
    torch.cuda.synchronize()
    print(f"full size {prec} inner loop: f0 {f0.item():.10e} after 12 steps {f_last:.10e} fresh {f1.item():.10e}",
          flush=True)
    assert done == 12 and flag == 2
    assert f1.item() < f0.item()
    assert abs(f_last - f1.item()) <= tol * abs(f1.item())
    prob.close()
