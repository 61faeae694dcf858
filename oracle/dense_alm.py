"""Dense convex ALM on X for tiny n (test infrastructure only).

A second, factor-free oracle for solve-level values: eq. (ALM) of Sec. 1.2
with each subproblem eq. (AL-P), min over X PSD of L_sigma(X, y), solved by
accelerated projected gradient (FISTA) with the projection onto the PSD cone
done by a full eigendecomposition, step 1/(sigma ||A||^2).  It builds every
A_i as an explicit dense matrix straight from the constraint definitions and
shares nothing with the structured maps in ``sdp.py``, so agreement between
the two is evidence about both.
"""

import numpy as np


def explicit_matrices(p):
    """Dense C and the stack of dense A_i (m x n x n) from the definitions."""
    n = p.n
    C = p.C.toarray() - p.j_coef * np.ones((n, n))
    if p.kind == "diag":
        A = np.zeros((n, n, n))
        A[np.arange(n), np.arange(n), np.arange(n)] = 1.0
    elif p.kind == "edges":
        m = p.m
        A = np.zeros((m, n, n))
        A[0] = p.c_tr * np.eye(n)
        for e, (i, j) in enumerate(zip(p.ei, p.ej)):
            A[e + 1, i, j] = 0.5
            A[e + 1, j, i] = 0.5
    else:
        A = np.stack([a.toarray() for a in p.A])
    return C, A


def _psd_project(X):
    X = 0.5 * (X + X.T)
    vals, vecs = np.linalg.eigh(X)
    vals = np.maximum(vals, 0.0)
    return (vecs * vals) @ vecs.T


def dense_alm(p, sigma=1.0, eps=1e-8, max_outer=2000, max_inner=20000, inner_tol=1e-11, y0=None):
    """Returns dict(X, y, pobj, dobj, kkt, outer)."""
    C, A = explicit_matrices(p)
    m, n = A.shape[0], A.shape[1]
    b = p.b
    Amat = A.reshape(m, n * n)
    opnorm = np.linalg.norm(Amat, 2)
    L = sigma * opnorm ** 2
    step = 1.0 / L
    y = np.zeros(m) if y0 is None else np.array(y0, dtype=np.float64)
    X = np.zeros((n, n))
    cnorm = np.linalg.norm(C)
    info = None
    for k in range(max_outer):
        Z = X.copy()
        Xprev = X.copy()
        tk = 1.0
        for _ in range(max_inner):
            r = Amat @ Z.ravel() - b
            grad = C - (np.tensordot(y - sigma * r, A, axes=1))
            Xn = _psd_project(Z - step * grad)
            tn = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * tk * tk))
            Z = Xn + ((tk - 1.0) / tn) * (Xn - Xprev)
            diff = np.linalg.norm(Xn - Xprev)
            Xprev = Xn
            tk = tn
            if diff <= inner_tol * (1.0 + np.linalg.norm(Xn)):
                break
        X = Xprev
        r = Amat @ X.ravel() - b
        y = y - sigma * r
        S = C - np.tensordot(y, A, axes=1)
        lam = np.linalg.eigvalsh(0.5 * (S + S.T))[0]
        pobj = float(np.sum(C * X))
        dobj = float(b @ y)
        pinf = np.linalg.norm(r) / (1.0 + np.linalg.norm(b))
        dinf = abs(min(0.0, lam)) / (1.0 + cnorm)
        gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
        info = {"pinf": pinf, "dinf": dinf, "gap": gap, "kkt": max(pinf, dinf, gap)}
        if info["kkt"] <= eps:
            break
    return {"X": X, "y": y, "pobj": float(np.sum(C * X)), "dobj": float(b @ y), "kkt": info, "outer": k}
