"""FP64 statement of the learned warm start's pieces (test infrastructure only).

The warm start is not in the paper (Alg. 1 starts from y = 0); these functions
write out its definition plainly so that the HIP kernels can be checked:

* ``features``: per-vertex features of a MaxCut-type cost C = S + Diag(d)
  (S off-diagonal): log(1 + deg), sum |S_ij|, sum S_ij, d_i, d_i - sum |S_ij|,
  and over the neighbours j: mean and max of log(1 + deg_j), mean of
  sum_k |S_jk|.
* ``mlp_forward`` / ``mlp_loss_grad``: the n_in -> h -> h -> 1 ReLU network on
  standardised inputs (x - mu) * inv_sd, parameters flattened as W1[n_in][h],
  b1[h], W2[h][h], b2[h], W3[h], b3; loss (1/n) sum (f(x_v) - t_v)^2.

Pins (tests/test_oracle_warmstart.py): hand-computed features on small graphs,
a network whose output is known in closed form, and central finite differences
of the loss for every parameter tensor.
"""

import numpy as np
import scipy.sparse as sp


def features(p):
    """p: a MaxCut-type SDP from oracle.sdp (C holds S and the diagonal)."""
    C = sp.csr_matrix(p.C)
    n = p.n
    d = C.diagonal()
    S = C - sp.diags(d)
    S.eliminate_zeros()
    S = sp.csr_matrix(S)
    deg = np.diff(S.indptr).astype(np.float64)
    absS = abs(S)
    f = np.zeros((n, 8))
    f[:, 0] = np.log1p(deg)
    f[:, 1] = np.asarray(absS.sum(axis=1)).ravel()
    f[:, 2] = np.asarray(S.sum(axis=1)).ravel()
    f[:, 3] = d
    f[:, 4] = d - f[:, 1]
    for i in range(n):
        nb = S.indices[S.indptr[i]:S.indptr[i + 1]]
        if nb.size:
            f[i, 5] = np.mean(f[nb, 0])
            f[i, 6] = np.max(f[nb, 0])
            f[i, 7] = np.mean(f[nb, 1])
    return f


def unpack(params, nin, h):
    params = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = params[o:o + nin * h].reshape(nin, h)
    o += nin * h
    b1 = params[o:o + h]
    o += h
    W2 = params[o:o + h * h].reshape(h, h)
    o += h * h
    b2 = params[o:o + h]
    o += h
    W3 = params[o:o + h]
    o += h
    b3 = params[o]
    return W1, b1, W2, b2, W3, b3


def param_count(nin, h):
    return nin * h + h + h * h + h + h + 1


def mlp_forward(params, nin, h, mu, inv_sd, X):
    W1, b1, W2, b2, W3, b3 = unpack(params, nin, h)
    Z = (np.asarray(X, dtype=np.float64)[:, :nin] - mu[:nin]) * inv_sd[:nin]
    a1 = np.maximum(Z @ W1 + b1, 0.0)
    a2 = np.maximum(a1 @ W2 + b2, 0.0)
    return a2 @ W3 + b3


def mlp_loss_grad(params, nin, h, mu, inv_sd, X, T):
    W1, b1, W2, b2, W3, b3 = unpack(params, nin, h)
    n = X.shape[0]
    Z = (np.asarray(X, dtype=np.float64)[:, :nin] - mu[:nin]) * inv_sd[:nin]
    z1 = Z @ W1 + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2 + b2
    a2 = np.maximum(z2, 0.0)
    out = a2 @ W3 + b3
    e = out - T
    loss = float(np.mean(e * e))
    dout = 2.0 * e / n
    gW3 = a2.T @ dout
    gb3 = np.sum(dout)
    d2 = np.outer(dout, W3) * (z2 > 0)
    gW2 = a1.T @ d2
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2.T) * (z1 > 0)
    gW1 = Z.T @ d1
    gb1 = d1.sum(axis=0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return loss, grad
