"""Per-call quantities of the ALM-BM method, in FP64 (test infrastructure only).

Problem (P) of Sec. 1.2: minimise <C, X> subject to A(X) = b, X PSD, with
[A(X)]_i = <A_i, X>.  The Burer-Monteiro factor is R (n x r) and X = R R^T.

Cost matrices handled here have the form C = C_s - j*J, where C_s is a sparse
symmetric matrix (its diagonal included) and J is the all-ones matrix.

Constraint families:

* ``diag``    A_i = e_i e_i^T, m = n (the MaxCut constraints X_ii = b_i, Sec. 6.1)
* ``edges``   A_0 = c_tr * I (trace row) and, for each edge e = {i, j},
              A_e = (e_i e_j^T + e_j e_i^T) / 2, so <A_e, X> = X_ij
              (entry constraints as in the examples of Sec. 3.3 and Sec. 4.3;
              m = |E| + 1).  The Lovasz-theta SDP uses c_tr = 1, b = (1, 0, ...).
* ``generic`` an explicit list of sparse symmetric A_i (tiny examples only).

Pins (tests/test_oracle_*.py): the structured maps against an explicit
<A_i, X> on tiny n; G against central finite differences of f; the worked
examples of Sec. 3.3 (2x2 and general-r rank examples, the quadratic-growth
counter-example) and the stationary points of Sec. 4.3 (G = 0 exactly,
lambda_min < 0); lambda_min against closed-form cycle spectra.
"""

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class SDP:
    n: int
    kind: str                      # 'diag' | 'edges' | 'generic'
    b: np.ndarray                  # length m, float64
    C: sp.csr_matrix               # sparse symmetric part of the cost (diagonal included)
    j_coef: float = 0.0            # cost is C - j_coef * J
    c_tr: float = 0.0              # edges: coefficient of the trace row A_0 = c_tr * I
    ei: Optional[np.ndarray] = None
    ej: Optional[np.ndarray] = None
    A: List[sp.csr_matrix] = field(default_factory=list)  # generic family
    _W_pattern: Optional[sp.csr_matrix] = None

    @property
    def m(self) -> int:
        return int(self.b.shape[0])


def _sym_from_edges(n, ei, ej, vals):
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    rows = np.concatenate([ei, ej])
    cols = np.concatenate([ej, ei])
    v = np.concatenate([vals, vals]).astype(np.float64)
    return sp.csr_matrix((v, (rows, cols)), shape=(n, n))


def maxcut_sdp(graph):
    """MaxCut relaxation of Sec. 6.1 in minimisation form.

    The paper maximises <L, X>/4 over X_ii = 1, X PSD, with L the weighted
    Laplacian (L_ij = -w_ij, L_ii = sum_k w_ik).  Minimising <C, X> with
    C = -L/4 is the same problem; the SDP value is -<C, X*>.
    """
    n = graph.n
    W = _sym_from_edges(n, graph.ei, graph.ej, graph.w)
    deg = np.asarray(W.sum(axis=1)).ravel()
    L = sp.diags(deg) - W
    C = (-0.25 * L).tocsr()
    C.sum_duplicates()
    return SDP(n=n, kind="diag", b=np.ones(n), C=C)


def lovasz_sdp(graph):
    """Lovasz theta in minimisation form: min <-J, X> s.t. tr X = 1 and
    X_ij = 0 for every edge {i, j}; theta(G) = -<C, X*>."""
    n = graph.n
    b = np.zeros(graph.m_edges + 1)
    b[0] = 1.0
    return SDP(n=n, kind="edges", b=b, C=sp.csr_matrix((n, n)), j_coef=1.0, c_tr=1.0,
               ei=np.asarray(graph.ei, np.int64), ej=np.asarray(graph.ej, np.int64))


def edges_sdp(n, C, b, c_tr, ei, ej, j_coef=0.0):
    C = sp.csr_matrix(C, dtype=np.float64)
    return SDP(n=n, kind="edges", b=np.asarray(b, dtype=np.float64), C=C, j_coef=float(j_coef),
               c_tr=float(c_tr), ei=np.asarray(ei, np.int64), ej=np.asarray(ej, np.int64))


def completion_sdp(inst):
    """Matrix completion as an SDP (Sec. 6): min tr(X)/2 over X = [[W1, Y], [Y^T, W2]]
    PSD with Y_ij = M_ij on the observed entries.  X is (n1 + n2) x (n1 + n2);
    entry (i, j) of Y is X_{i, n1 + j}, an entry constraint of the edges family
    with no trace row (c_tr = 0, b_0 = 0).  Its value is the nuclear norm of the
    completed matrix."""
    n = inst.n1 + inst.n2
    b = np.concatenate([[0.0], np.asarray(inst.vals, dtype=np.float64)])
    C = 0.5 * sp.identity(n, format="csr")
    return edges_sdp(n, C, b, 0.0, np.asarray(inst.rows, np.int64), inst.n1 + np.asarray(inst.cols, np.int64))


def generic_sdp(C, A_list, b):
    C = sp.csr_matrix(np.asarray(C, dtype=np.float64) if not sp.issparse(C) else C)
    A = [sp.csr_matrix(np.asarray(a, dtype=np.float64) if not sp.issparse(a) else a) for a in A_list]
    return SDP(n=C.shape[0], kind="generic", b=np.asarray(b, dtype=np.float64), C=C, A=A)


# --------------------------------------------------------------------------- cost


def cost_apply(p, X):
    """C X for C = C_s - j J (X of shape (n,) or (n, k))."""
    Y = p.C @ X
    if p.j_coef != 0.0:
        Y = Y - p.j_coef * np.broadcast_to(np.sum(X, axis=0), np.shape(X))
    return np.asarray(Y)


def cost_fro_norm(p):
    """||C||_F of C = C_s - j J, from ||C_s||^2 - 2 j <C_s, J> + j^2 n^2."""
    cs2 = float(np.sum(p.C.data ** 2))
    s = float(np.sum(p.C.data))
    j = p.j_coef
    return float(np.sqrt(max(cs2 - 2.0 * j * s + j * j * p.n * p.n, 0.0)))


# ---------------------------------------------------------------- constraint map


def amap_uv(p, U, V):
    """A(U V^T) = [<A_i, U V^T>]_i; equal to A((U V^T + V U^T)/2) since A_i is symmetric."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    if U.ndim == 1:
        U = U[:, None]
        V = V[:, None]
    if p.kind == "diag":
        return np.sum(U * V, axis=1)
    if p.kind == "edges":
        a0 = p.c_tr * np.sum(U * V)
        ae = 0.5 * (np.sum(U[p.ei] * V[p.ej], axis=1) + np.sum(U[p.ej] * V[p.ei], axis=1))
        return np.concatenate([[a0], ae])
    if p.kind == "generic":
        return np.array([np.sum(U * (Ai @ V)) for Ai in p.A])
    raise ValueError(p.kind)


def amap(p, R):
    """a = A(R R^T)."""
    return amap_uv(p, R, R)


def _edge_weight_matrix(p, we):
    return _sym_from_edges(p.n, p.ei, p.ej, we)


def adjoint_apply(p, w, X):
    """A*(w) X with A*(w) = sum_i w_i A_i."""
    X = np.asarray(X, dtype=np.float64)
    if p.kind == "diag":
        return (w[:, None] * X) if X.ndim == 2 else w * X
    if p.kind == "edges":
        W = _edge_weight_matrix(p, w[1:])
        return p.c_tr * w[0] * X + 0.5 * np.asarray(W @ X)
    if p.kind == "generic":
        out = np.zeros_like(X)
        for wi, Ai in zip(w, p.A):
            out = out + wi * np.asarray(Ai @ X)
        return out
    raise ValueError(p.kind)


def rank_one_norm2(p, v):
    """||A(v v^T)||^2 (the curvature of the augmented term along v v^T)."""
    a = amap(p, v[:, None])
    return float(np.dot(a, a))


# ------------------------------------------------------------------ objective


def objective(p, R, y, sigma):
    """Lbar_sigma(R, y) = <C, R R^T> + <y, b - A(R R^T)> + sigma/2 ||A(R R^T) - b||^2  (eq. AL-BM).
    sigma may be a scalar or one penalty per constraint (then sum_i sigma_i/2 res_i^2)."""
    P = cost_apply(p, R)
    a = amap(p, R)
    res = a - p.b
    return float(np.sum(R * P) + np.dot(y, p.b - a) + 0.5 * np.dot(sigma * res, res))


def objective_grad(p, R, y, sigma):
    """f, G and a = A(R R^T) at (R, y).

    G = 2 (C - A*(w)) R with w = y - sigma (A(R R^T) - b): the exact gradient of
    eq. (AL-BM); the factor 2 is that of grad h(F) = 2 grad f(X) F (Sec. 4.2).
    Returns (f, G, a, P) with P = C R.
    """
    R = np.asarray(R, dtype=np.float64)
    P = cost_apply(p, R)
    a = amap(p, R)
    res = a - p.b
    w = y - sigma * res
    f = float(np.sum(R * P) + np.dot(y, p.b - a) + 0.5 * np.dot(sigma * res, res))
    G = 2.0 * (P - adjoint_apply(p, w, R))
    return f, G, a, P


def dual_update(p, a, sigma, y):
    """y+ = y + sigma (b - A(X)) (eq. ALM); pinf = ||A(X) - b|| / (1 + ||b||) (Sec. 6)."""
    res = a - p.b
    y_new = y - sigma * res
    pinf = float(np.linalg.norm(res) / (1.0 + np.linalg.norm(p.b)))
    return y_new, pinf


# -------------------------------------------------------------------- spectrum


def slack_matvec(p, y, x):
    """Z(y) x = (C - A*(y)) x (the dual slack map of Sec. 1.2)."""
    return cost_apply(p, x) - adjoint_apply(p, y, x)


def slack_dense(p, y):
    return slack_matvec(p, y, np.eye(p.n))


def min_eig(p, y, want_vector=False, dense_limit=4000):
    """lambda_min(C - A*(y)) and optionally a unit eigenvector.

    Dense LAPACK (numpy.linalg.eigh) up to ``dense_limit``, ARPACK (scipy
    eigsh, smallest algebraic) above it.
    """
    if p.n <= dense_limit:
        S = slack_dense(p, y)
        S = 0.5 * (S + S.T)
        if want_vector:
            vals, vecs = np.linalg.eigh(S)
            return float(vals[0]), vecs[:, 0]
        return float(np.linalg.eigvalsh(S)[0])
    op = spla.LinearOperator((p.n, p.n), matvec=lambda x: slack_matvec(p, y, x), dtype=np.float64)
    rng = np.random.default_rng(12345)
    vals, vecs = spla.eigsh(op, k=1, which="SA", tol=1e-12, v0=rng.standard_normal(p.n),
                            ncv=min(p.n, 64), maxiter=100000)
    if want_vector:
        return float(vals[0]), vecs[:, 0]
    return float(vals[0])


def min_eigs(p, y, q, dense_limit=4000):
    """The q smallest eigenpairs of C - A*(y), ascending: (values, n x q unit
    eigenvectors).  Dense LAPACK up to ``dense_limit``, ARPACK above it."""
    q = int(min(q, p.n))
    if p.n <= dense_limit:
        S = slack_dense(p, y)
        vals, vecs = np.linalg.eigh(0.5 * (S + S.T))
        return vals[:q].copy(), vecs[:, :q].copy()
    op = spla.LinearOperator((p.n, p.n), matvec=lambda x: slack_matvec(p, y, x), dtype=np.float64)
    rng = np.random.default_rng(12345)
    vals, vecs = spla.eigsh(op, k=q, which="SA", tol=1e-12, v0=rng.standard_normal(p.n),
                            ncv=min(p.n, max(64, 4 * q)), maxiter=100000)
    order = np.argsort(vals)
    return vals[order], vecs[:, order]


def kkt(p, R, y, lam_min=None):
    """Relative KKT measure of Sec. 6 at X = R R^T (l2 norms):

    max{ ||A X - b|| / (1 + ||b||),
         |min(0, lambda_min(C - A* y))| / (1 + ||C||_F),
         |<C, X> - b^T y| / (1 + |<C, X>| + |b^T y|) }.
    """
    a = amap(p, R)
    pinf = float(np.linalg.norm(a - p.b) / (1.0 + np.linalg.norm(p.b)))
    if lam_min is None:
        lam_min = min_eig(p, y)
    dinf = abs(min(0.0, lam_min)) / (1.0 + cost_fro_norm(p))
    pobj = float(np.sum(R * cost_apply(p, R)))
    dobj = float(np.dot(p.b, y))
    gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    return {"pinf": pinf, "dinf": dinf, "gap": gap, "kkt": max(pinf, dinf, gap),
            "pobj": pobj, "dobj": dobj, "lam_min": float(lam_min)}


def maxcut_objective_grad_rows(graph, R, y, sigma, rows):
    """G and a = A(RR^T) of the MaxCut SDP (C = -L/4, X_ii = 1) at selected rows
    only, evaluated row by row from the edge list:
      (CR)_i = sum_{j ~ i} w_ij R_j / 4 - (sum_{j ~ i} w_ij) R_i / 4,
      a_i = ||R_i||^2,  G_i = 2 ((CR)_i - (y_i - sigma (a_i - 1)) R_i).
    For parity checks at sizes where assembling the full oracle is slow."""
    rows = np.asarray(rows, dtype=np.int64)
    pos = {int(r): k for k, r in enumerate(rows)}
    sel = np.isin(graph.ei, rows) | np.isin(graph.ej, rows)
    P = np.zeros((rows.shape[0], R.shape[1]))
    deg = np.zeros(rows.shape[0])
    for i, j, wij in zip(graph.ei[sel], graph.ej[sel], graph.w[sel]):
        for u, v in ((int(i), int(j)), (int(j), int(i))):
            k = pos.get(u)
            if k is not None:
                P[k] += 0.25 * wij * R[v]
                deg[k] += wij
    G = np.zeros_like(P)
    a = np.zeros(rows.shape[0])
    for k, i in enumerate(rows):
        P[k] -= 0.25 * deg[k] * R[i]
        a[k] = float(R[i] @ R[i])
        wi = y[i] - sigma * (a[k] - 1.0)
        G[k] = 2.0 * (P[k] - wi * R[i])
    return G, a
