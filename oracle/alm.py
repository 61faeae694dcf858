"""ALM-BM solve in FP64 (test infrastructure only).

The loop follows Alg. 1 (ALORA, Sec. 5) in its order: y starts at the given
y0 (zero by default, as Alg. 1 initialises it); each outer iteration
approximately minimises the BM subproblem eq. (AL-BM) by gradient descent
(eq. GD, Sec. 4.2), then looks at the smallest eigenpair of
grad_X L = C - A*(y + sigma (b - A(RR^T))), expands the factor by one column
when that eigenvalue is sufficiently negative (p = 1 case of the rank step of Alg. 1)
or, with rank_block > 1, by the columns of V S^{1/2} for the most negative
eigenvectors V and the small PSD subproblem (curvature_step), then updates y
(eq. ALM) and tests the relative KKT measure of Sec. 6.

Readings where the paper is silent (shared with the HIP path through the
solve options):
* step size: exact minimiser over t >= 0 of the quartic phi(t) = Lbar(R - tG)
  (ties to the smallest t); a fixed step is the alternative;
* inner stop: ||G||_F ||R||_F <= tol_k (1 + |<C, RR^T>|), or max_inner
  iterations, with tol_k = max(eps/10, min(0.1, pinf_{k-1}, kappa tol_{k-1}))
  and kappa = 0.7 (pinf and tol are +inf before the first outer iteration).
  The left side bounds |<grad_X L, RR^T>| = |<G, R>|/2, the subproblem's share
  of the duality-gap term of the KKT measure, so the rule is scale free; the
  tolerance shrinks at least geometrically, as inexact ALM needs;
* rank step with p = 1: s* = max(0, -theta / (sigma ||A(v v^T)||^2)) is the
  exact minimiser over s >= 0 of L(RR^T + s v v^T, y), whose expansion is
  L(X) + s theta + (sigma/2) s^2 ||A(v v^T)||^2; expand iff theta < -tau_rank
  (default eps (1 + ||C||_F)) and r < r_cap = min(r_max, Barvinok-Pataki bound
  floor((sqrt(8m+1)-1)/2) of Sec. 3.3), whether or not the inner solve met its
  tolerance, as Alg. 1 does (an optional gate waits for inner convergence; it
  stalls the rank, hence the dual infeasibility, once max_inner binds);
* penalty sigma fixed by default; the edges family may give its edge rows their
  own penalty sigma_edges (the trace row keeps sigma), one penalty per
  constraint throughout; an optional schedule multiplies every penalty by
  sigma_growth after an outer iteration whose pinf did not fall below
  pinf_reduction times the previous one (the update of the SDPLR solver the
  paper cites in Sec. 2).

Pins: the quartic coefficients against direct evaluation of the objective at
R - tG (tests/test_oracle_alm.py); solve values against closed-form MaxCut and
Lovasz-theta values, brute-force max cuts and an independent dense convex ALM;
the curvature step against the closed-form one-vector step, the objective
change, PSD perturbations and a brute-force grid (tests/test_oracle_rankstep.py).
Trajectory-level agreement with the HIP solve is parity unpinned beyond
final invariants (discrete rank/root decisions may differ near ties).
"""

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .sdp import (amap, amap_uv, cost_apply, cost_fro_norm, kkt, min_eig, min_eigs,
                  objective_grad, rank_one_norm2, slack_matvec)


@dataclass
class SolveOptions:
    eps_kkt: float = 1e-6
    sigma: float = 1.0
    max_outer: int = 1000
    max_inner: int = 500
    step_rule: str = "exact"       # 'exact' | 'fixed'
    eta_fixed: float = 1e-3
    rank_policy: str = "adapt"     # 'adapt' | 'fixed'
    r_max: int = 64
    tau_rank: Optional[float] = None
    inner_tol_scale: float = 0.1   # the 0.1 in min(0.1, pinf_prev, kappa tol_prev)
    inner_tol_decay: float = 0.7   # kappa
    expand_needs_inner: bool = False  # True: expand only after an inner solve met its tolerance
    sigma_edges: Optional[float] = None  # edges family: penalty of the edge rows (trace row keeps sigma)
    # penalty schedule (off at growth 1): after an outer iteration whose pinf is
    # above pinf_reduction times the previous one, sigma *= sigma_growth (every
    # row's penalty, capped at sigma_max for the base penalty).  This is the
    # update of the SDPLR solver the paper cites (Sec. 2); Alg. 1 keeps rho fixed.
    sigma_growth: float = 1.0
    sigma_max: float = 1e6
    pinf_reduction: float = 0.25
    # rank step from the rank_block most negative eigenvectors of the slack at
    # w and the small PSD subproblem of Alg. 1 (curvature_step); 1 = the
    # closed-form one-vector step
    rank_block: int = 1
    # subproblem solver: 'gd' (eq. GD, the paper's) or 'lbfgs' (limited-memory
    # BFGS with the same exact line search, the SDPLR solver of Sec. 2)
    inner_solver: str = "gd"
    lbfgs_memory: int = 8


def line_search_coeffs(p, R, G, y, sigma, P=None, a=None):
    """Coefficients k0..k4 of phi(t) = Lbar_sigma(R - t G, y) = sum_k k_k t^k.

    With c0 = <C, RR^T>, c1 = 2<G, CR>, c2 = <G, CG>, a0 = A(RR^T),
    a1 = A(RG^T + GR^T), a2 = A(GG^T) and e = a0 - b:
      <C, (R-tG)(R-tG)^T> = c0 - t c1 + t^2 c2,
      A((R-tG)(R-tG)^T)   = a0 - t a1 + t^2 a2.
    """
    if P is None:
        P = cost_apply(p, R)
    if a is None:
        a = amap(p, R)
    Q = cost_apply(p, G)
    c0 = float(np.sum(R * P))
    c1 = 2.0 * float(np.sum(G * P))
    c2 = float(np.sum(G * Q))
    a1 = 2.0 * amap_uv(p, R, G)
    a2 = amap(p, G)
    e = a - p.b
    s = sigma  # scalar, or one penalty per constraint
    k0 = c0 + float(np.dot(y, p.b - a)) + 0.5 * float(np.dot(s * e, e))
    k1 = -c1 + float(np.dot(y, a1)) - float(np.dot(s * e, a1))
    k2 = c2 - float(np.dot(y, a2)) + 0.5 * (float(np.dot(s * a1, a1)) + 2.0 * float(np.dot(s * e, a2)))
    k3 = -float(np.dot(s * a1, a2))
    k4 = 0.5 * float(np.dot(s * a2, a2))
    return np.array([k0, k1, k2, k3, k4])


def _phi(k, t):
    return k[0] + t * (k[1] + t * (k[2] + t * (k[3] + t * k[4])))


def quartic_argmin(k):
    """argmin over t >= 0 of the quartic with coefficients k (smallest t on ties).

    Candidates are t = 0 and the real non-negative roots of phi'(t)
    (numpy.roots, i.e. companion-matrix eigenvalues).  Returns 0 when phi is
    unbounded below on t >= 0 (degenerate directions).
    """
    d = np.array([4.0 * k[4], 3.0 * k[3], 2.0 * k[2], k[1]])
    nz = np.flatnonzero(d != 0.0)
    if nz.size == 0:
        return 0.0
    d = d[nz[0]:]
    lead_deg = d.size - 1  # degree of phi' actually present
    # phi unbounded below on t >= 0 when the leading term of phi is negative
    if lead_deg >= 1 and d[0] < 0.0:
        return 0.0
    cands = [0.0]
    if lead_deg >= 1:
        for z in np.roots(d):
            if abs(z.imag) <= 1e-9 * max(1.0, abs(z.real)) and z.real > 0.0:
                cands.append(float(z.real))
    best_t, best_v = 0.0, _phi(k, 0.0)
    for t in sorted(cands):
        v = _phi(k, t)
        if v < best_v:
            best_t, best_v = t, v
    return best_t


def inner_gd(p, R, y, sigma, tol, max_inner, step_rule="exact", eta_fixed=1e-3):
    """Gradient descent R <- R - t G on eq. (AL-BM) until
    ||G||_F ||R||_F <= tol (1 + |<C, RR^T>|)."""
    R = np.array(R, dtype=np.float64, copy=True)
    it = 0
    gnorm = math.inf
    f = math.nan
    for it in range(max_inner):
        f, G, a, P = objective_grad(p, R, y, sigma)
        gnorm = float(np.linalg.norm(G))
        c0 = float(np.sum(R * P))
        if gnorm * float(np.linalg.norm(R)) <= tol * (1.0 + abs(c0)):
            return R, {"iters": it, "f": f, "gnorm": gnorm, "converged": True}
        if step_rule == "exact":
            t = quartic_argmin(line_search_coeffs(p, R, G, y, sigma, P, a))
        else:
            t = eta_fixed
        R = R - t * G
    return R, {"iters": max_inner, "f": f, "gnorm": gnorm, "converged": False}


def _psd_part(M):
    lam, U = np.linalg.eigh(0.5 * (M + M.T))
    return (U * np.maximum(lam, 0.0)) @ U.T


def penalty_moments(p, V, weights=None):
    """The penalty's quadratic form of the negative-curvature subproblem of
    Alg. 1 over the pairs a <= b (row-major) of the columns of V:
        M[pair(a,b), pair(c,d)] = sum_i weights_i A_i(v_a v_b^T) A_i(v_c v_d^T)
    (weights: one per constraint row, default 1), so that for symmetric S
    sum_{a,b,c,d} S_ab S_cd M[pair(a,b), pair(c,d)] = sum_i weights_i A_i(V S V^T)^2."""
    V = np.asarray(V, dtype=np.float64)
    q = V.shape[1]
    wts = np.ones(p.m) if weights is None else np.asarray(weights, dtype=np.float64)
    pairs = [(a, b) for a in range(q) for b in range(a, q)]
    img = [amap_uv(p, V[:, a], V[:, b]) for a, b in pairs]
    return np.array([[float(np.dot(wts * x, z)) for z in img] for x in img])


def curvature_step(p, w, sigma, V, max_iter=200000, tol=1e-12):
    """The negative-curvature subproblem of Alg. 1 (Sec. 5).

    With X = R R^T fixed, w = y - sigma (A(X) - b) and V (n x q) orthonormal
    directions, the augmented Lagrangian of X + V S V^T exceeds that of X by
        phi(S) = <V^T (C - A*(w)) V, S> + 1/2 sum_i sigma_i A_i(V S V^T)^2
    exactly (the penalty is quadratic in X).  This minimises phi over S PSD by
    accelerated projected gradient (FISTA with monotone restarts, step 1/L,
    projection = eigenvalue clipping) until the fixed-point residual
    ||S - P(S - grad/L)||_F is below tol (1 + ||S||_F).  Returns (S, phi(S),
    new columns V S^{1/2} of the factor, n x rank(S)).  When A(V S V^T)
    vanishes for every S the subproblem is linear: S = 0 (no step).
    """
    V = np.asarray(V, dtype=np.float64)
    if V.ndim == 1:
        V = V[:, None]
    n, q = V.shape
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (p.m,))
    G0 = V.T @ np.column_stack([slack_matvec(p, w, V[:, j]) for j in range(q)])
    G0 = 0.5 * (G0 + G0.T)
    # images A(v_k v_l^T) of the matrix units (symmetric in k, l)
    img = {(k, l): amap_uv(p, V[:, k], V[:, l]) for k in range(q) for l in range(k, q)}

    def bmap(S):
        z = np.zeros(p.m)
        for (k, l), a_kl in img.items():
            z += (S[k, l] if k == l else 2.0 * S[k, l]) * a_kl
        return z

    def badj(z):
        M = np.empty((q, q))
        for (k, l), a_kl in img.items():
            M[k, l] = M[l, k] = float(np.dot(z, a_kl))
        return M

    def phi(S):
        z = bmap(S)
        return float(np.sum(G0 * S)) + 0.5 * float(np.dot(sig * z, z))

    def grad(S):
        return G0 + badj(sig * bmap(S))

    # Lipschitz constant: the largest eigenvalue of the Hessian S -> B*(sigma B(S))
    # in an orthonormal basis of the symmetric q x q matrices
    basis = []
    for k in range(q):
        for l in range(k, q):
            E = np.zeros((q, q))
            if k == l:
                E[k, k] = 1.0
            else:
                E[k, l] = E[l, k] = 1.0 / math.sqrt(2.0)
            basis.append(E)
    H = np.array([[float(np.sum(Ei * badj(sig * bmap(Ej)))) for Ej in basis] for Ei in basis])
    L = float(np.max(np.linalg.eigvalsh(0.5 * (H + H.T)))) if basis else 0.0
    if not L > 0.0:
        S = np.zeros((q, q))
        return S, 0.0, np.zeros((n, 0))
    S = np.zeros((q, q))
    Y = S.copy()
    t = 1.0
    f_S = phi(S)
    for _ in range(max_iter):
        S_new = _psd_part(Y - grad(Y) / L)
        f_new = phi(S_new)
        if f_new > f_S:  # restart: plain projected gradient step from S
            Y = S.copy()
            t = 1.0
            S_new = _psd_part(S - grad(S) / L)
            f_new = phi(S_new)
        t_new = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
        Y = S_new + ((t - 1.0) / t_new) * (S_new - S)
        S, f_S, t = S_new, f_new, t_new
        res = np.linalg.norm(S - _psd_part(S - grad(S) / L))
        if res <= tol * (1.0 + np.linalg.norm(S)):
            break
    lam, U = np.linalg.eigh(0.5 * (S + S.T))
    keep = lam > 1e-14 * max(float(np.max(lam)), 1e-300)
    cols = V @ (U[:, keep] * np.sqrt(lam[keep]))
    return S, phi(S), cols


def inner_lbfgs(p, R, y, sigma, tol, max_inner, memory=8):
    """L-BFGS on eq. (AL-BM) with the exact minimiser of the quartic along each
    direction, until ||G||_F ||R||_F <= tol (1 + |<C, RR^T>|) (the stopping
    rule of inner_gd).  Directions by the two-loop recursion over the last
    `memory` pairs (s, g_new - g) with positive curvature, scaled by
    s.y / y.y; a direction that is not a descent direction, or a zero step,
    clears the memory and falls back to -G."""
    R = np.array(R, dtype=np.float64, copy=True)
    S_mem, Y_mem = [], []
    f, G, a, P = objective_grad(p, R, y, sigma)
    for it in range(max_inner):
        gnorm = float(np.linalg.norm(G))
        c0 = float(np.sum(R * P))
        if gnorm * float(np.linalg.norm(R)) <= tol * (1.0 + abs(c0)):
            return R, {"iters": it, "f": f, "gnorm": gnorm, "converged": True}
        # two-loop recursion: D = -H G
        q = G.copy()
        alphas = []
        for s, yv in zip(reversed(S_mem), reversed(Y_mem)):
            rho = 1.0 / float(np.sum(yv * s))
            al = rho * float(np.sum(s * q))
            alphas.append((al, rho))
            q -= al * yv
        if S_mem:
            q *= float(np.sum(S_mem[-1] * Y_mem[-1])) / float(np.sum(Y_mem[-1] * Y_mem[-1]))
        for (al, rho), s, yv in zip(reversed(alphas), S_mem, Y_mem):
            be = rho * float(np.sum(yv * q))
            q += (al - be) * s
        D = -q
        if float(np.sum(D * G)) >= 0.0:
            S_mem, Y_mem = [], []
            D = -G
        t = quartic_argmin(line_search_coeffs(p, R, -D, y, sigma, P, a))
        if t == 0.0 and S_mem:
            S_mem, Y_mem = [], []
            D = -G
            t = quartic_argmin(line_search_coeffs(p, R, G, y, sigma, P, a))
        if t == 0.0:
            return R, {"iters": it, "f": f, "gnorm": gnorm, "converged": False}
        R_new = R + t * D
        f, G_new, a, P = objective_grad(p, R_new, y, sigma)
        s, yv = R_new - R, G_new - G
        if float(np.sum(s * yv)) > 1e-12 * float(np.linalg.norm(s)) * float(np.linalg.norm(yv)):
            S_mem.append(s)
            Y_mem.append(yv)
            if len(S_mem) > memory:
                S_mem.pop(0)
                Y_mem.pop(0)
        R, G = R_new, G_new
    return R, {"iters": max_inner, "f": f, "gnorm": float(np.linalg.norm(G)), "converged": False}


def bp_rank_cap(m):
    """Largest r with r(r+1)/2 <= m (Barvinok-Pataki bound, Sec. 3.3)."""
    return int((math.isqrt(8 * m + 1) - 1) // 2)


def solve(p, R0, y0=None, opts=None, callback=None):
    """ALM-BM with p = 1 rank adaptation (Alg. 1); see the module docstring."""
    opts = opts or SolveOptions()
    R = np.array(R0, dtype=np.float64, copy=True)
    y = np.zeros(p.m) if y0 is None else np.array(y0, dtype=np.float64, copy=True)
    sigma = opts.sigma
    if p.kind == "edges" and opts.sigma_edges:
        # one penalty per constraint: sigma on the trace row, sigma_edges on the edge rows
        sigma = np.full(p.m, float(opts.sigma_edges))
        sigma[0] = opts.sigma
    cnorm = cost_fro_norm(p)
    tau_rank = opts.tau_rank if opts.tau_rank is not None else opts.eps_kkt * (1.0 + cnorm)
    r_cap = min(opts.r_max, bp_rank_cap(p.m))
    pinf_prev = math.inf
    tol_prev = math.inf
    hist = []
    info = None
    status = "not_converged"
    for k in range(opts.max_outer):
        tol = max(opts.eps_kkt / 10.0, min(opts.inner_tol_scale, pinf_prev,
                                                 opts.inner_tol_decay * tol_prev))
        tol_prev = tol
        if opts.inner_solver == "lbfgs":
            R, inner = inner_lbfgs(p, R, y, sigma, tol, opts.max_inner, opts.lbfgs_memory)
        else:
            R, inner = inner_gd(p, R, y, sigma, tol, opts.max_inner, opts.step_rule, opts.eta_fixed)
        a = amap(p, R)
        w = y - sigma * (a - p.b)
        expanded = False
        if opts.rank_policy == "adapt" and opts.rank_block > 1:
            q = min(opts.rank_block, p.n)
            thetas, Vq = min_eigs(p, w, q)
            theta = float(thetas[0])
            gate = inner["converged"] or not opts.expand_needs_inner
            neg = thetas < -tau_rank
            if gate and np.any(neg) and R.shape[1] < r_cap:
                _, _, cols = curvature_step(p, w, sigma, Vq[:, neg])
                cols = cols[:, :r_cap - R.shape[1]]
                if cols.shape[1] > 0:
                    R = np.concatenate([R, cols], axis=1)
                    a = amap(p, R)
                    w = y - sigma * (a - p.b)
                    expanded = True
        elif opts.rank_policy == "adapt":
            theta, v = min_eig(p, w, want_vector=True)
            gate = inner["converged"] or not opts.expand_needs_inner
            if gate and theta < -tau_rank and R.shape[1] < r_cap:
                av = amap(p, v[:, None])
                s = max(0.0, -theta / float(np.dot(sigma * av, av)))
                R = np.concatenate([R, math.sqrt(s) * v[:, None]], axis=1)
                a = amap(p, R)
                w = y - sigma * (a - p.b)
                expanded = True
        else:
            theta = min_eig(p, w)
        y = w
        lam = theta if not expanded else min_eig(p, y)
        info = kkt(p, R, y, lam_min=lam)
        base = float(np.atleast_1d(sigma)[0])
        info.update({"outer": k, "inner_iters": inner["iters"], "rank": R.shape[1],
                     "expanded": expanded, "theta": theta, "f": inner["f"], "sigma": base})
        hist.append(info)
        if callback is not None:
            callback(info)
        pinf_last = pinf_prev
        pinf_prev = info["pinf"]
        if info["kkt"] <= opts.eps_kkt:
            status = "converged"
            break
        if opts.sigma_growth > 1.0 and info["pinf"] > opts.pinf_reduction * pinf_last:
            sigma0 = float(np.atleast_1d(sigma)[0])
            if sigma0 < opts.sigma_max:
                sigma = sigma * (min(opts.sigma_max, sigma0 * opts.sigma_growth) / sigma0)
    return {"R": R, "y": y, "status": status, "history": hist, "kkt": info}
