"""Learned warm start for ALM-BM on MaxCut-type SDPs (diagonal constraints).

A per-vertex MLP (features -> y0_i) proposes the initial dual and a ridge model
on pooled features proposes the initial rank r0; Alg. 1 of the paper starts
from y = 0, and that default start is both the fallback and the reference the
warm start is judged against.  Features, the network's forward and backward
passes and Adam run in the library's HIP kernels (alm_bm_ws_*); this module
only moves tensors and drives the training loop.

Training data are the project's own solves: seeded generated graphs, solved
from the default start, labelled with the final dual y* (per vertex) and the
final rank r* (per graph).

Command line (GPU):
  python -m paper_2505_15775_amd.warmstart train --count 200 --batched --out MODEL.npz
  python -m paper_2505_15775_amd.warmstart curve --count 600 --out MODEL.npz
(curve: held-out errors of models fitted on growing training sets, then
solves of held-out graphs from the default, y0-only, r0-only and full starts)
"""

import argparse
import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import Problem, _lib, _ptr, _stream, check, lib

NFEAT = 8
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warmstart_model.npz")
RANK_CHOICES = (4, 8, 16, 32)


def features(prob):
    """n x 8 float features of the handle's cost (device tensor)."""
    F = torch.empty((prob.n, NFEAT), dtype=torch.float32, device=prob.device)
    scratch = torch.empty(prob.n, dtype=torch.float32, device=prob.device)
    check(lib.alm_bm_ws_features(prob._h, _ptr(F), _ptr(scratch), _stream()), "ws_features")
    return F


def pooled(F):
    """Column means of the features (host numpy, 8 values)."""
    out = torch.empty(NFEAT, dtype=torch.float64, device=F.device)
    work = torch.empty(512, dtype=torch.float64, device=F.device)
    check(lib.alm_bm_ws_pool(_ptr(F), F.shape[0], _ptr(out), _ptr(work), _stream()), "ws_pool")
    return out.cpu().numpy()


def _rank_inputs(pool, n):
    return np.array([math.log(n), pool[0], pool[1], pool[4], pool[5]], dtype=np.float64)


class WarmStartModel:
    def __init__(self, nin=NFEAT, h=32, device="cuda", seed=0):
        self.nin, self.h = nin, h
        self.device = torch.device(device)
        npar = int(lib.alm_bm_ws_param_count(nin, h))
        rng = np.random.default_rng(seed)
        p = np.zeros(npar, dtype=np.float32)
        o = 0
        for fan_in, fan_out in ((nin, h), (None, h), (h, h), (None, h), (h, 1), (None, 1)):
            cnt = (fan_in or 1) * fan_out
            if fan_in is not None:
                lim = math.sqrt(6.0 / fan_in)  # He-uniform for ReLU layers
                p[o:o + cnt] = rng.uniform(-lim, lim, cnt)
            o += cnt
        self.params = torch.from_numpy(p).to(self.device)
        self.mu = torch.zeros(NFEAT, dtype=torch.float32, device=self.device)
        self.inv_sd = torch.ones(NFEAT, dtype=torch.float32, device=self.device)
        self.t_scale = 1.0
        self.rank_coef = None

    # ------------------------------------------------------------ inference

    def predict_y0(self, prob, F=None):
        if F is None:
            F = features(prob)
        out = torch.empty(prob.n, dtype=torch.float64, device=self.device)
        check(lib.alm_bm_ws_forward(_ptr(self.params), self.nin, self.h, _ptr(self.mu), _ptr(self.inv_sd),
                                    prob.n, _ptr(F), _ptr(out), _stream()), "ws_forward")
        return out

    def predict_r0(self, pool, n, r_max=None):
        if self.rank_coef is None:
            return 16
        x = _rank_inputs(pool, n)
        r = float(x @ self.rank_coef[:-1] + self.rank_coef[-1])
        r = int(min(RANK_CHOICES, key=lambda c: abs(c - r)))
        return min(r, r_max) if r_max else r

    # ------------------------------------------------------------ training

    def loss_grad(self, X, T, nblocks=512):
        npar = self.params.numel()
        grad = torch.empty(npar, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        work = torch.empty(int(lib.alm_bm_ws_work_size(self.nin, self.h, nblocks)), dtype=torch.float32,
                           device=self.device)
        check(lib.alm_bm_ws_loss_grad(_ptr(self.params), self.nin, self.h, _ptr(self.mu), _ptr(self.inv_sd),
                                      X.shape[0], _ptr(X), _ptr(T), _ptr(grad), _ptr(loss), _ptr(work), nblocks,
                                      _stream()), "ws_loss_grad")
        return loss, grad

    def fit(self, X, T, steps=400, lr=3e-3, batch=1 << 18, seed=0, log=None):
        """Adam on the mean squared error; X (N x 8 float), T (N float) on the device.
        Minibatches are contiguous slices at seeded random offsets."""
        self.t_scale = float(T.abs().mean().item()) or 1.0
        Ts = (T / self.t_scale).contiguous()
        self.mu = X.mean(dim=0).contiguous()
        self.inv_sd = (1.0 / X.std(dim=0).clamp_min(1e-6)).contiguous()
        npar = self.params.numel()
        m = torch.zeros(npar, dtype=torch.float32, device=self.device)
        v = torch.zeros(npar, dtype=torch.float32, device=self.device)
        rng = np.random.default_rng(seed)
        N = X.shape[0]
        b = min(batch, N)
        hist = []
        for step in range(1, steps + 1):
            off = int(rng.integers(0, N - b + 1))
            loss, grad = self.loss_grad(X[off:off + b], Ts[off:off + b])
            check(lib.alm_bm_ws_adam(_ptr(self.params), _ptr(grad), _ptr(m), _ptr(v), npar, C.c_float(lr),
                                     C.c_float(0.9), C.c_float(0.999), C.c_float(1e-8), step, _stream()), "ws_adam")
            if step % 50 == 0 or step == 1:
                hist.append((step, float(loss.item())))
                if log:
                    log(f"[warmstart] step {step} loss {hist[-1][1]:.5f}")
        # fold the target scale into the output layer so that inference is the
        # forward kernel alone
        o = self.nin * self.h + self.h + self.h * self.h + self.h
        self.params[o:o + self.h + 1] *= self.t_scale
        self.t_scale = 1.0
        return hist

    def fit_rank(self, pools, ns, ranks, lam=1e-3):
        X = np.stack([_rank_inputs(p, n) for p, n in zip(pools, ns)])
        t = np.asarray(ranks, dtype=np.float64)
        coef = np.zeros(X.shape[1] + 1)
        check(lib.alm_bm_ws_ridge_fit(X.ctypes.data, t.ctypes.data, X.shape[0], X.shape[1], lam, coef.ctypes.data),
              "ws_ridge_fit")
        self.rank_coef = coef
        return coef

    # ------------------------------------------------------------ storage

    def save(self, path, meta=None):
        np.savez(path, params=self.params.cpu().numpy(), mu=self.mu.cpu().numpy(), inv_sd=self.inv_sd.cpu().numpy(),
                 t_scale=np.array([self.t_scale]), shape=np.array([self.nin, self.h]),
                 rank_coef=(self.rank_coef if self.rank_coef is not None else np.zeros(0)),
                 meta=np.array([repr(meta or {})]))

    @classmethod
    def load(cls, path=MODEL_PATH, device="cuda"):
        z = np.load(path, allow_pickle=False)
        nin, h = (int(v) for v in z["shape"])
        m = cls(nin, h, device)
        m.params = torch.from_numpy(z["params"]).to(m.device)
        m.mu = torch.from_numpy(z["mu"]).to(m.device)
        m.inv_sd = torch.from_numpy(z["inv_sd"]).to(m.device)
        m.t_scale = float(z["t_scale"][0])
        m.rank_coef = z["rank_coef"] if z["rank_coef"].size else None
        return m


# ---------------------------------------------------------------- solving


def solve_warm(prob, model, r_max=None, fallback_outer=5, seed=1, **opts):
    """Solve from the learned start (predicted y0 and rank r0), with the
    fallback of solve_from.  Returns (status, result, R, y, info)."""
    import gen

    t0 = time.perf_counter()
    F = features(prob)
    y0 = model.predict_y0(prob, F)
    r0 = model.predict_r0(pooled(F), prob.n, r_max or prob.r_max)
    R0 = gen.init_factor(prob.n, r0, seed)
    t_pred = time.perf_counter() - t0
    st, res, R, y, info = solve_from(prob, R0, y0, fallback_outer=fallback_outer, seed=seed, **opts)
    info["r0"] = r0
    info["predict_s"] = t_pred
    info["total_s"] = time.perf_counter() - t0
    return st, res, R, y, info


def solve_from(prob, R0, y0, fallback_outer=5, seed=1, **opts):
    """Solve from a proposed start (R0 host n x r0, y0 device m), falling back
    to the default start (y = 0, rank min(16, r_max) unit rows) when the warm
    run hits a numerical error or a rejected argument, or when after
    `fallback_outer` outer iterations its KKT measure is worse than at its own
    start.  Returns (status, result, R, y, info); info["fallback"] tells
    whether the default start was used."""
    import gen

    opts = dict(opts)
    max_outer = int(opts.pop("max_outer", 1000))
    t0 = time.perf_counter()
    info = {"fallback": False}
    try:
        theta, _, _, _ = prob.lanczos_min_eig(y0, max_iter=min(40, prob.desc.lanczos_kmax), tol=0.0, want_vector=False)
        k0 = prob.kkt(prob.factor(torch.from_numpy(np.ascontiguousarray(R0))), y0, theta)["kkt"]
        if not math.isfinite(k0):
            raise FloatingPointError(f"KKT measure at the proposed start is {k0}")
        st, res, R, y = prob.solve(R0, y0, max_outer=min(fallback_outer, max_outer), **opts)
        if st != 0 and not (res["kkt"] < k0):
            raise FloatingPointError(f"warm start not improving: kkt {res['kkt']:.3e} vs start {k0:.3e}")
        if st != 0 and res["outer"] < max_outer:
            st, res2, R, y = prob.solve(R, y, max_outer=max_outer - res["outer"], **opts)
            res2["outer"] += res["outer"]
            res2["inner_total"] += res["inner_total"]
            res2["time_s"] += res["time_s"]
            res = res2
    except (FloatingPointError, ValueError, _lib.AlmBmError) as e:
        info["fallback"] = True
        info["reason"] = str(e)
        r_fb = min(16, prob.r_max)
        st, res, R, y = prob.solve(gen.init_factor(prob.n, r_fb, seed), None, max_outer=max_outer, **opts)
    info["total_s"] = time.perf_counter() - t0
    return st, res, R, y, info


# ---------------------------------------------------------------- training data


def training_graphs(count, seed, n_lo=1e4, n_hi=1e5, deg_lo=4.0, deg_hi=16.0):
    """Seeded graphs: n log-uniform in [n_lo, n_hi], average degree uniform in
    [deg_lo, deg_hi]; weights N(0,1) for 70 %, +-1 for 15 %, unit for 15 %."""
    import gen

    out = []
    rng = np.random.default_rng(seed)
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d = float(rng.uniform(deg_lo, deg_hi))
        u = rng.random()
        w = "gauss" if u < 0.7 else ("pm1" if u < 0.85 else "unit")
        out.append(gen.er_graph(n, int(round(n * d / 2)), seed * 100003 + k, w))
    return out


def generate_training_set(graphs, eps=1e-5, r0=16, r_max=64, sigma=16.0, device="cuda", log=None):
    import gen

    feats, targets, pools, ns, ranks = [], [], [], [], []
    for k, g in enumerate(graphs):
        prob = Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=r_max, lanczos_kmax=60, device=device,
                              validate=False)
        st, res, R, y = prob.solve(gen.init_factor(g.n, r0, 1), eps_kkt=eps, sigma=sigma, max_outer=300)
        if st != 0:
            if log:
                log(f"[warmstart] graph {k} n={g.n}: not converged (kkt {res['kkt']:.2e}), skipped")
            prob.close()
            continue
        F = features(prob)
        feats.append(F)
        targets.append(y.float())
        pools.append(pooled(F))
        ns.append(g.n)
        ranks.append(res["rank"])
        if log:
            log(f"[warmstart] graph {k} n={g.n} M={g.m_edges}: outer {res['outer']} rank {res['rank']} "
                f"{res['time_s']:.2f}s")
        prob.close()
    return feats, targets, pools, ns, ranks


def generate_training_set_batched(graphs, eps=1e-5, r0=16, r_max=64, sigma=16.0, batch=48, device="cuda",
                                  log=None):
    """As generate_training_set, with the labelling solves run `batch` graphs
    at a time by the batched solver (L-BFGS subproblems of at most 100 steps)."""
    import gen

    from . import Batch

    feats, targets, pools, ns, ranks = [], [], [], [], []
    for start in range(0, len(graphs), batch):
        chunk = graphs[start:start + batch]
        probs = [Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=r_max, lanczos_kmax=60, device=device,
                                validate=False, lbfgs_memory_max=3) for g in chunk]
        b = Batch(probs, rank_stride=r_max)
        t0 = time.time()
        _, sts, res, R, rk, y = b.solve([gen.init_factor(g.n, r0, 1) for g in chunk], eps_kkt=eps, sigma=sigma,
                                        max_outer=300, inner_solver=1, lbfgs_memory=3, max_inner=100)
        for q, (g, p) in enumerate(zip(chunk, probs)):
            if sts[q] != 0:
                if log:
                    log(f"[warmstart] graph {start + q} n={g.n}: not converged (kkt {res[q]['kkt']:.2e}), skipped")
                continue
            _, yq = b.instance(q, R, y, rk[q])
            F = features(p)
            feats.append(F)
            targets.append(yq.float().clone())
            pools.append(pooled(F))
            ns.append(g.n)
            ranks.append(rk[q])
        if log:
            log(f"[warmstart] labelled graphs {start}..{start + len(chunk) - 1} in {time.time() - t0:.1f}s "
                f"(ranks {min(rk)}..{max(rk)})")
        b.close()
        for p in probs:
            p.close()
    return feats, targets, pools, ns, ranks


def _fit(feats, targets, pools, ns, ranks, hidden, seed, steps, log=None):
    model = WarmStartModel(h=hidden, seed=seed)
    X = torch.cat(feats).contiguous()
    T = torch.cat(targets).contiguous()
    hist = model.fit(X, T, steps=steps, log=log)
    model.fit_rank(pools, ns, ranks)
    return model, hist, int(X.shape[0])


def _held_out_errors(model, feats, targets, pools, ns, ranks):
    """Mean relative error of y0 and mean |r0 - r*| over labelled graphs."""
    ey, er = [], []
    for F, T, pl, n, r in zip(feats, targets, pools, ns, ranks):
        out = torch.empty(n, dtype=torch.float64, device=F.device)
        check(lib.alm_bm_ws_forward(_ptr(model.params), model.nin, model.h, _ptr(model.mu), _ptr(model.inv_sd), n,
                                    _ptr(F), _ptr(out), _stream()), "ws_forward")
        t = T.double()
        ey.append(float(torch.linalg.norm(out - t) / torch.linalg.norm(t)))
        er.append(abs(model.predict_r0(pl, n) - r))
    return float(np.mean(ey)), float(np.mean(er))


def ablation(graphs, model, eps=1e-5, sigma=16.0, r_default=16, log=None):
    """Solves of each graph from five starts: the default (y = 0, rank 16), the
    learned y0 at rank 16, y = 0 at the learned r0, both (solve_warm's start,
    without its fallback test), and the Gershgorin dual-feasible start
    y0_i = C_ii - sum_j |C_ij| (feature 4) at rank 16 as a comparator.  L-BFGS
    subproblems of at most 100 steps.  Returns per-start totals of outer
    iterations and seconds."""
    import gen

    opts = dict(eps_kkt=eps, sigma=sigma, max_outer=300, inner_solver=1, lbfgs_memory=3, max_inner=100)
    tot = {k: {"outer": 0, "time_s": 0.0, "converged": 0}
           for k in ("default", "y0_only", "r0_only", "both", "gershgorin")}
    for g in graphs:
        prob = Problem.maxcut(g.n, g.ei, g.ej, g.w, precision="f64", r_max=64, lanczos_kmax=60, validate=False,
                              lbfgs_memory_max=3)
        F = features(prob)
        y0 = model.predict_y0(prob, F)
        r0 = model.predict_r0(pooled(F), g.n, prob.r_max)
        line = f"[warmstart] ablation n={g.n} r0={r0}:"
        y_gersh = F[:, 4].double().contiguous()
        for k, (r, yy) in {"default": (r_default, None), "y0_only": (r_default, y0), "r0_only": (r0, None),
                           "both": (r0, y0), "gershgorin": (r_default, y_gersh)}.items():
            st, res, _, _ = prob.solve(gen.init_factor(g.n, r, 1), yy, **opts)
            tot[k]["outer"] += res["outer"]
            tot[k]["time_s"] += res["time_s"]
            tot[k]["converged"] += int(st == 0)
            line += f" {k} {res['outer']} outer {res['time_s']:.2f}s rank {res['rank']};"
        if log:
            log(line)
        prob.close()
    return tot


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train", help="label seeded graphs with solves and fit the model")
    t.add_argument("--count", type=int, default=120)
    t.add_argument("--seed", type=int, default=6)
    t.add_argument("--steps", type=int, default=600)
    t.add_argument("--hidden", type=int, default=32)
    t.add_argument("--sigma", type=float, default=16.0, help="penalty of the labelling solves")
    t.add_argument("--batched", action="store_true", help="label with the batched solver (L-BFGS subproblems)")
    t.add_argument("--out", default=MODEL_PATH)
    c = sub.add_parser("curve", help="learning curve over training-set sizes, then the start ablation")
    c.add_argument("--count", type=int, default=600)
    c.add_argument("--seed", type=int, default=6)
    c.add_argument("--steps", type=int, default=1200)
    c.add_argument("--hidden", type=int, default=32)
    c.add_argument("--sigma", type=float, default=16.0)
    c.add_argument("--ablation", type=int, default=12, help="held-out graphs solved from the four starts")
    c.add_argument("--out", default=None, help="save the model fitted on the whole training part here")
    a = sub.add_parser("ablation", help="the start ablation alone, for a saved model")
    a.add_argument("--count", type=int, default=600, help="size of the seeded set whose first tenth is held out")
    a.add_argument("--seed", type=int, default=6)
    a.add_argument("--graphs", type=int, default=12)
    a.add_argument("--sigma", type=float, default=16.0)
    a.add_argument("--model", default=MODEL_PATH)
    args = ap.parse_args()

    def log(s):
        print(s, file=sys.stderr, flush=True)

    n_hold = max(1, args.count // 10)
    if args.cmd == "ablation":
        graphs = training_graphs(min(args.graphs, n_hold), args.seed)  # the first graphs are the held-out ones
        abl = ablation(graphs, WarmStartModel.load(args.model), sigma=args.sigma, log=log)
        print(json.dumps({"ablation": abl}), flush=True)
        return
    graphs = training_graphs(args.count, args.seed)
    t0 = time.time()
    if args.cmd == "train":
        gen_set = generate_training_set_batched if args.batched else generate_training_set
        feats, targets, pools, ns, ranks = gen_set(graphs[n_hold:], sigma=args.sigma, log=log)
        log(f"[warmstart] {len(feats)} labelled solves in {time.time() - t0:.1f}s")
        model, hist, nv = _fit(feats, targets, pools, ns, ranks, args.hidden, args.seed, args.steps, log)
        model.save(args.out, meta={"count": args.count, "seed": args.seed, "holdout": n_hold, "vertices": nv,
                                   "loss": hist[-1][1], "sigma": args.sigma})
        log(f"[warmstart] saved {args.out}")
        return
    # learning curve: held-out errors of models fitted on growing prefixes of the training part
    hold = generate_training_set_batched(graphs[:n_hold], sigma=args.sigma, log=log)
    train = generate_training_set_batched(graphs[n_hold:], sigma=args.sigma, log=log)
    log(f"[warmstart] {len(hold[0])} held-out and {len(train[0])} training graphs labelled in {time.time() - t0:.1f}s")
    sizes = [k for k in (10, 25, 50, 100, 200, 400, 800, 1600) if k < len(train[0])] + [len(train[0])]
    curve = []
    model = None
    for k in sizes:
        model, hist, nv = _fit(*(x[:k] for x in train), args.hidden, args.seed, args.steps)
        ey, er = _held_out_errors(model, *hold)
        curve.append({"graphs": k, "vertices": nv, "train_loss": round(hist[-1][1], 6),
                      "held_out_y0_rel_err": round(ey, 4), "held_out_r0_abs_err": round(er, 2)})
        log(f"[warmstart] curve {curve[-1]}")
    if args.out:
        model.save(args.out, meta={"count": args.count, "seed": args.seed, "holdout": n_hold, "graphs": sizes[-1],
                                   "vertices": curve[-1]["vertices"], "loss": curve[-1]["train_loss"],
                                   "sigma": args.sigma, "labels": "batched L-BFGS solves to 1e-5 KKT"})
        log(f"[warmstart] saved {args.out}")
    abl = ablation(graphs[:min(args.ablation, n_hold)], model, sigma=args.sigma, log=log)
    print(json.dumps({"learning_curve": curve, "ablation": abl}), flush=True)


if __name__ == "__main__":
    main()
