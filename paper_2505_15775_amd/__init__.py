"""MI355X-native ALM-BM (augmented Lagrangian Burer-Monteiro) for low-rank SDPs.

Python binding of libalmbm.so (C ABI in include/alm_bm.h).  torch tensors
provide device memory and the HIP stream; every step of the method runs in the
library's HIP kernels.  Names follow arxiv 2505.15775: C, A, b for problem (P)
(Sec. 1.2), R for the factor (F in the paper), sigma for the penalty (rho).
"""

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import AlmBmError, check, default_options, lib  # noqa: F401

__all__ = ["Problem", "Batch", "AlmBmError", "default_options", "maxcut_cost", "objective_grad_noalloc",
           "TORCH_DTYPES"]

TORCH_DTYPES = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def maxcut_cost(n, ei, ej, w):
    """C = -L/4 of the MaxCut relaxation (Sec. 6.1) as CSR (off-diagonal) +
    diagonal, built by the library's host routine.  Returns numpy arrays
    (row_ptr, col_idx, val, diag)."""
    ei = np.ascontiguousarray(ei, dtype=np.int32)
    ej = np.ascontiguousarray(ej, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    m = ei.shape[0]
    rp = np.empty(n + 1, dtype=np.int32)
    ci = np.empty(max(1, 2 * m), dtype=np.int32)
    cv = np.empty(max(1, 2 * m), dtype=np.float64)
    dg = np.empty(n, dtype=np.float64)
    nnz = C.c_int64(0)
    check(lib.alm_bm_maxcut_cost_host(n, m, ei.ctypes.data, ej.ctypes.data, w.ctypes.data, rp.ctypes.data,
                                      ci.ctypes.data, cv.ctypes.data, dg.ctypes.data, C.byref(nnz)),
          "maxcut_cost_host")
    k = nnz.value
    return rp, ci[:k].copy(), cv[:k].copy(), dg


def objective_grad_noalloc(desc, R, y, sigma, f, G=None, Av=None, stream=None):
    """alm_bm_objective_grad_noalloc: eq. (AL-BM) objective, gradient and
    A(RR^T) of a DIAG-family FP64 problem described by ``desc`` (an
    ``_lib.Desc``, e.g. ``Problem.desc``), with no handle and no allocation.
    Every output is caller-owned: f (1 double), G (n x r double, or None), Av
    (n doubles, or None), all on R's device."""
    if R.dtype != torch.float64 or R.dim() != 2 or not R.is_contiguous():
        raise ValueError("R must be a contiguous n x r float64 tensor")
    check(lib.alm_bm_objective_grad_noalloc(C.byref(desc), R.shape[1], _ptr(R), _ptr(y), float(sigma), _ptr(f),
                                            _ptr(G), _ptr(Av), _stream(stream)), "objective_grad_noalloc")


def psd_step(theta, M4, sigma):
    """The block rank step's small PSD subproblem (alm_bm_psd_step, host only):
    theta (q Ritz values), M4 (np x np, np = q(q+1)/2, pairs a <= b row-major),
    sigma.  Returns S (q x q)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    M4 = np.ascontiguousarray(M4, dtype=np.float64)
    q = theta.shape[0]
    S = np.empty((q, q), dtype=np.float64)
    check(lib.alm_bm_psd_step(q, theta.ctypes.data, M4.ctypes.data, float(sigma), S.ctypes.data), "psd_step")
    return S


class Problem:
    """One SDP instance resident on the GPU plus its library handle.

    Build with :meth:`maxcut` or :meth:`edges`; the object keeps every device
    array the handle points at alive.
    """

    def __init__(self, desc_kwargs, arrays, precision, device):
        self.device = torch.device(device)
        self.precision = precision
        self.dtype = TORCH_DTYPES[precision]
        self._arrays = arrays  # keep device arrays alive
        d = _lib.Desc()
        for k, v in desc_kwargs.items():
            setattr(d, k, v)
        self.desc = d
        self.n = int(d.n)
        self.m = int(d.m)
        self.r_max = int(d.r_max)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib.alm_bm_create(C.byref(d), _stream(), C.byref(h)), "create")
        self._h = h

    # ------------------------------------------------------------ constructors

    @classmethod
    def maxcut(cls, n, ei, ej, w, precision="f64", r_max=32, lanczos_kmax=100, device="cuda", ell=False,
               validate=True, rank_block_max=0, lbfgs_memory_max=0, hub_min_degree=0):
        """MaxCut SDP relaxation (Sec. 6.1): min <C, X>, X_ii = 1, X PSD, C = -L/4.
        rank_block_max, lbfgs_memory_max, hub_min_degree: workspace the handle
        reserves for the block rank step, the L-BFGS inner solver and hub rows
        (fields of alm_bm_problem_desc)."""
        rp, ci, cv, dg = maxcut_cost(n, ei, ej, w)
        dev = torch.device(device)
        ell_width = 0
        if ell:
            deg = np.diff(rp)
            ell_width = int(deg.max()) if n else 0
            cols = np.repeat(np.arange(n, dtype=np.int32)[:, None], ell_width, axis=1)
            vals = np.zeros((n, ell_width))
            pos = np.arange(ci.shape[0]) - np.repeat(rp[:-1], deg)
            rows = np.repeat(np.arange(n), deg)
            cols[rows, pos] = ci
            vals[rows, pos] = cv
            ci, cv = cols.ravel(), vals.ravel()
        t_rp = torch.from_numpy(rp).to(dev) if not ell else None
        t_ci = torch.from_numpy(np.ascontiguousarray(ci, dtype=np.int32)).to(dev)
        t_cv = torch.from_numpy(np.ascontiguousarray(cv, dtype=np.float64)).to(dev)
        t_dg = torch.from_numpy(dg).to(dev)
        t_b = torch.ones(n, dtype=torch.float64, device=dev)
        arrays = dict(row_ptr=t_rp, col_idx=t_ci, val=t_cv, diag=t_dg, b=t_b)
        kw = dict(n=n, nnz=int(t_ci.numel()) if ci.shape[0] else 0, row_ptr=t_rp.data_ptr() if t_rp is not None else 0,
                  col_idx=t_ci.data_ptr(), val=t_cv.data_ptr(), ell_width=ell_width, diag=t_dg.data_ptr(),
                  j_coef=0.0, cons_kind=_lib.CONS_DIAG, m=n, b=t_b.data_ptr(), trace_coef=0.0, n_edges=0,
                  edge_i=0, edge_j=0, precision=_lib.PRECISIONS[precision], r_max=r_max,
                  lanczos_kmax=lanczos_kmax, validate=int(validate), rank_block_max=int(rank_block_max),
                  lbfgs_memory_max=int(lbfgs_memory_max), hub_min_degree=int(hub_min_degree))
        return cls(kw, arrays, precision, dev)

    @classmethod
    def edges(cls, n, ei, ej, b, trace_coef, j_coef=0.0, cost_csr=None, cost_diag=None, precision="f64",
              r_max=32, lanczos_kmax=100, device="cuda", validate=True, rank_block_max=0):
        """Trace row + entry constraints: <c_tr I, X> = b[0], X_ij = b[1+e] for the
        sorted edge list (i < j); cost C = S + Diag(d) - j_coef J with S given as
        (row_ptr, col_idx, val) numpy arrays (off-diagonal) or None."""
        dev = torch.device(device)
        ei = np.ascontiguousarray(ei, dtype=np.int32)
        ej = np.ascontiguousarray(ej, dtype=np.int32)
        E = ei.shape[0]
        t_ei = torch.from_numpy(ei if E else np.zeros(1, np.int32)).to(dev)
        t_ej = torch.from_numpy(ej if E else np.zeros(1, np.int32)).to(dev)
        t_b = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)).to(dev)
        arrays = dict(edge_i=t_ei, edge_j=t_ej, b=t_b)
        nnz = 0
        rp_p = ci_p = cv_p = dg_p = 0
        if cost_csr is not None:
            rp, ci, cv = cost_csr
            nnz = int(len(ci))
            if nnz:
                arrays["row_ptr"] = torch.from_numpy(np.ascontiguousarray(rp, np.int32)).to(dev)
                arrays["col_idx"] = torch.from_numpy(np.ascontiguousarray(ci, np.int32)).to(dev)
                arrays["val"] = torch.from_numpy(np.ascontiguousarray(cv, np.float64)).to(dev)
                rp_p, ci_p, cv_p = (arrays[k].data_ptr() for k in ("row_ptr", "col_idx", "val"))
        if cost_diag is not None:
            arrays["diag"] = torch.from_numpy(np.ascontiguousarray(cost_diag, np.float64)).to(dev)
            dg_p = arrays["diag"].data_ptr()
        kw = dict(n=n, nnz=nnz, row_ptr=rp_p, col_idx=ci_p, val=cv_p, ell_width=0, diag=dg_p, j_coef=float(j_coef),
                  cons_kind=_lib.CONS_TRACE_EDGES, m=E + 1, b=t_b.data_ptr(), trace_coef=float(trace_coef),
                  n_edges=E, edge_i=t_ei.data_ptr(), edge_j=t_ej.data_ptr(), precision=_lib.PRECISIONS[precision],
                  r_max=r_max, lanczos_kmax=lanczos_kmax, validate=int(validate),
                  rank_block_max=int(rank_block_max), lbfgs_memory_max=0, hub_min_degree=-1)
        return cls(kw, arrays, precision, dev)

    @classmethod
    def lovasz(cls, n, ei, ej, **kw):
        """Lovasz theta: min <-J, X>, tr X = 1, X_ij = 0 on edges; theta = -<C, X*>."""
        b = np.zeros(len(ei) + 1)
        b[0] = 1.0
        return cls.edges(n, ei, ej, b, 1.0, j_coef=1.0, **kw)

    @classmethod
    def matrix_completion(cls, n1, n2, rows, cols, vals, **kw):
        """Matrix completion (Sec. 6): min tr(X)/2 over X = [[W1, Y], [Y^T, W2]] PSD
        with Y_ij = M_ij on the observed entries (rows, cols sorted by (row, col),
        unique).  The factor is (n1 + n2) x r, U above V; entry (i, j) of Y is the
        entry constraint X_{i, n1 + j}; no trace row (its coefficient is 0)."""
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        b = np.concatenate([[0.0], np.asarray(vals, dtype=np.float64)])
        n = int(n1) + int(n2)
        return cls.edges(n, rows, int(n1) + cols, b, 0.0, j_coef=0.0, cost_diag=np.full(n, 0.5), **kw)

    # ------------------------------------------------------------ lifetime

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.alm_bm_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ helpers

    def factor(self, R):
        """Device copy of a host/torch factor in the handle's storage precision."""
        t = torch.as_tensor(R)
        return t.to(device=self.device, dtype=self.dtype).contiguous()

    def _check_R(self, R):
        if R.device != self.device or R.dtype != self.dtype or not R.is_contiguous() or R.dim() != 2:
            raise ValueError(f"R must be a contiguous {self.dtype} n x r tensor on {self.device}")
        if R.shape[0] != self.n:
            raise ValueError("R must have n rows")

    def _check_y(self, y):
        if y.device != self.device or y.dtype != torch.float64 or y.numel() != self.m or not y.is_contiguous():
            raise ValueError(f"y must be a contiguous float64 vector of length m={self.m} on {self.device}")

    # ------------------------------------------------------------ entry points

    def objective_grad(self, R, y, sigma, want_G=True, want_Av=True, stream=None):
        """(f, G, Av): eq. (AL-BM) objective, gradient 2 (C - A*(w)) R and A(RR^T)."""
        self._check_R(R)
        self._check_y(y)
        f = torch.empty(1, dtype=torch.float64, device=self.device)
        G = torch.empty_like(R) if want_G else None
        Av = torch.empty(self.m, dtype=torch.float64, device=self.device) if want_Av else None
        check(lib.alm_bm_objective_grad(self._h, R.shape[1], _ptr(R), _ptr(y), float(sigma), _ptr(f), _ptr(G),
                                        _ptr(Av), _stream(stream)), "objective_grad")
        return f, G, Av

    def cost_apply(self, X, P=None, want_xpx=False, stream=None):
        """P = C X (arithmetic precision: float64 for f64, float32 otherwise) and,
        if asked, <X, C X> as a device scalar."""
        self._check_R(X)
        if P is None:
            pdt = torch.float64 if self.precision == "f64" else torch.float32
            P = torch.empty(X.shape, dtype=pdt, device=self.device)
        xpx = torch.empty(1, dtype=torch.float64, device=self.device) if want_xpx else None
        check(lib.alm_bm_cost_apply(self._h, X.shape[1], _ptr(X), _ptr(P), _ptr(xpx), _stream(stream)),
              "cost_apply")
        return (P, xpx) if want_xpx else P

    def line_search(self, R, G, y, sigma, stream=None):
        """(coeffs[5], t*) of phi(t) = Lbar(R - tG)."""
        self._check_R(R)
        self._check_R(G)
        self._check_y(y)
        k = torch.empty(5, dtype=torch.float64, device=self.device)
        t = torch.empty(1, dtype=torch.float64, device=self.device)
        check(lib.alm_bm_line_search(self._h, R.shape[1], _ptr(R), _ptr(G), _ptr(y), float(sigma), _ptr(k), _ptr(t),
                                     _stream(stream)), "line_search")
        return k, t

    def gd_step(self, R, y, sigma, f=None, t=None, G=None, stream=None):
        """One gradient step with exact line search, R updated in place.
        f, t: optional device float64 scalars receiving the objective and step."""
        self._check_R(R)
        self._check_y(y)
        check(lib.alm_bm_gd_step(self._h, R.shape[1], _ptr(R), _ptr(y), float(sigma), _ptr(f), _ptr(t), _ptr(G),
                                 _stream(stream)), "gd_step")

    def dual_update(self, Av, sigma, y, stream=None):
        """y <- y + sigma (b - Av) in place; returns pinf (device scalar)."""
        self._check_y(y)
        pinf = torch.empty(1, dtype=torch.float64, device=self.device)
        check(lib.alm_bm_dual_update(self._h, _ptr(Av), float(sigma), _ptr(y), _ptr(pinf), _stream(stream)),
              "dual_update")
        return pinf

    def lanczos_min_eig(self, y, max_iter=100, tol=1e-8, seed=1, want_vector=True, stream=None):
        """(theta, v, resid, iters) for lambda_min(C - A*(y)) (host floats/ints, v on device)."""
        self._check_y(y)
        th = torch.empty(1, dtype=torch.float64, device=self.device)
        rs = torch.empty(1, dtype=torch.float64, device=self.device)
        it = torch.empty(1, dtype=torch.int32, device=self.device)
        v = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_vector else None
        check(lib.alm_bm_lanczos_min_eig(self._h, _ptr(y), int(max_iter), float(tol), int(seed), _ptr(th), _ptr(v),
                                         _ptr(rs), _ptr(it), _stream(stream)), "lanczos_min_eig")
        return float(th.item()), v, float(rs.item()), int(it.item())

    def ladder_factor(self, r, stream=None):
        """Float factor (n x r, device) of the last solve on this BF16 handle that
        switched to float storage: the point its status and KKT values refer to."""
        R = torch.empty((self.n, int(r)), dtype=torch.float32, device=self.device)
        check(lib.alm_bm_ladder_factor(self._h, int(r), _ptr(R), _stream(stream)), "ladder_factor")
        return R

    def lanczos_block(self, y, q, max_iter=60, seed=1, stream=None):
        """(theta[q] host, V n x q device column-major, resid[q] host, basis size)
        for the q smallest eigenpairs of C - A*(y) by block Lanczos."""
        self._check_y(y)
        th = np.zeros(int(q), dtype=np.float64)
        rs = np.zeros(int(q), dtype=np.float64)
        V = torch.empty((int(q), self.n), dtype=torch.float64, device=self.device)  # row k = column k of n x q
        m = C.c_int32(0)
        check(lib.alm_bm_lanczos_block(self._h, _ptr(y), int(q), int(max_iter), int(seed), th.ctypes.data, _ptr(V),
                                       rs.ctypes.data, C.byref(m), _stream(stream)), "lanczos_block")
        return th, V.t(), rs, m.value

    def set_tiles(self, variant=0, row_blocks=0):
        check(lib.alm_bm_set_tiles(self._h, int(variant), int(row_blocks)), "set_tiles")

    def set_hub_threshold(self, min_degree=0):
        """Rows with more than min_degree entries become hub rows (0: the
        default threshold, < 0: none); returns the number of hub rows."""
        h = C.c_int32(0)
        check(lib.alm_bm_set_hub_threshold(self._h, int(min_degree), C.byref(h)), "set_hub_threshold")
        return h.value

    def autotune(self, r, reps=5, stream=None):
        """Pick the fastest (tile variant, row-kernel grid) for rank r; returns it."""
        v = C.c_int32(0)
        nb = C.c_int32(0)
        check(lib.alm_bm_autotune(self._h, int(r), int(reps), C.byref(v), C.byref(nb), _stream(stream)), "autotune")
        return v.value, nb.value

    def block_moments(self, V, edge_weight=1.0, stream=None):
        """M4 of the block rank step for orthonormal directions V (n x q,
        float64, on the device): host numpy np x np, np = q(q+1)/2."""
        V = torch.as_tensor(V).to(device=self.device, dtype=torch.float64)
        q = int(V.shape[1])
        Vc = V.t().contiguous()  # column-major n x q
        npair = q * (q + 1) // 2
        M4 = np.empty((npair, npair), dtype=np.float64)
        check(lib.alm_bm_block_moments(self._h, q, _ptr(Vc), float(edge_weight), M4.ctypes.data, _stream(stream)),
              "block_moments")
        return M4

    def kkt(self, R, y, lam_min, stream=None):
        self._check_R(R)
        self._check_y(y)
        out = (C.c_double * 6)()
        check(lib.alm_bm_kkt(self._h, R.shape[1], _ptr(R), _ptr(y), float(lam_min), out, _stream(stream)), "kkt")
        return dict(zip(["pinf", "dinf", "gap", "kkt", "pobj", "dobj"], list(out)))

    def inner_solve(self, R, y, tol, max_steps, stream=None, **opts):
        """Inner gradient loop at fixed y, R (device, handle precision) in place.
        Returns (steps_done, stop_flag, f_last)."""
        self._check_R(R)
        self._check_y(y)
        o = default_options()
        for k, v in opts.items():
            if not hasattr(o, k):
                raise KeyError(f"unknown option {k!r}")
            setattr(o, k, v)
        sd, fl, fv = C.c_int32(0), C.c_int32(0), C.c_double(0.0)
        check(lib.alm_bm_inner_solve(self._h, C.byref(o), R.shape[1], _ptr(R), _ptr(y), float(tol), int(max_steps),
                                     C.byref(sd), C.byref(fl), C.byref(fv), _stream(stream)), "inner_solve")
        return sd.value, fl.value, fv.value

    def solve(self, R0, y0=None, stream=None, **opts):
        """Full ALM-BM solve.  R0: n x r0 factor (any device/dtype), y0: m vector or
        None (zero).  Options are the fields of alm_bm_options.  Returns
        (status, result dict, R n x r final, y)."""
        o = default_options()
        for k, v in opts.items():
            if not hasattr(o, k):
                raise KeyError(f"unknown solve option {k!r}")
            setattr(o, k, v)
        R0 = torch.as_tensor(R0)
        r0 = int(R0.shape[1])
        if r0 > self.r_max:
            raise ValueError("initial rank exceeds r_max")
        buf = torch.zeros(self.n * self.r_max, dtype=self.dtype, device=self.device)
        buf[: self.n * r0] = R0.to(device=self.device, dtype=self.dtype).reshape(-1)
        y = (torch.zeros(self.m, dtype=torch.float64, device=self.device) if y0 is None
             else torch.as_tensor(y0).to(device=self.device, dtype=torch.float64).clone().contiguous())
        r = C.c_int32(r0)
        res = _lib.Result()
        st = check(lib.alm_bm_solve(self._h, C.byref(o), _ptr(buf), C.byref(r), _ptr(y), C.byref(res),
                                    _stream(stream)), "solve")
        R = buf[: self.n * r.value].view(self.n, r.value)
        return st, res.as_dict(), R, y


class Batch:
    """Many MaxCut-type instances solved together (alm_bm_batch_*): one launch
    per step of the method covers every instance.  `problems` are Problem
    objects (DIAG family, one precision); their arrays are copied at creation."""

    def __init__(self, problems, rank_stride, stream=None):
        if not problems:
            raise ValueError("empty batch")
        self.precision = problems[0].precision
        self.dtype = problems[0].dtype
        self.device = problems[0].device
        self.count = len(problems)
        self.rank_stride = int(rank_stride)
        descs = (_lib.Desc * self.count)(*[p.desc for p in problems])
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib.alm_bm_batch_create(self.count, descs, self.rank_stride, _stream(stream), C.byref(h)),
                  "batch_create")
        self._h = h
        offs = np.zeros(self.count + 1, dtype=np.int64)
        check(lib.alm_bm_batch_offsets(self._h, offs.ctypes.data), "batch_offsets")
        self.offsets = offs
        self.n_total = int(offs[-1])

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.alm_bm_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, factors):
        """Device (sum n) x rank_stride factor from per-instance n_q x r_q arrays."""
        R = torch.zeros((self.n_total, self.rank_stride), dtype=self.dtype, device=self.device)
        for q, F in enumerate(factors):
            F = torch.as_tensor(F)
            R[self.offsets[q]:self.offsets[q + 1], : F.shape[1]] = F.to(device=self.device, dtype=self.dtype)
        return R

    def solve(self, factors, y0=None, stream=None, **opts):
        """Returns (status, per-instance status list, results list, R, ranks, y)."""
        o = default_options()
        for k, v in opts.items():
            if not hasattr(o, k):
                raise KeyError(f"unknown solve option {k!r}")
            setattr(o, k, v)
        R = self.pack(factors)
        r = np.array([int(torch.as_tensor(F).shape[1]) for F in factors], dtype=np.int32)
        y = (torch.zeros(self.n_total, dtype=torch.float64, device=self.device) if y0 is None
             else torch.as_tensor(y0).to(device=self.device, dtype=torch.float64).clone().contiguous())
        res = (_lib.Result * self.count)()
        sts = np.zeros(self.count, dtype=np.int32)
        st = check(lib.alm_bm_batch_solve(self._h, C.byref(o), _ptr(R), r.ctypes.data, _ptr(y), res,
                                          sts.ctypes.data, _stream(stream)), "batch_solve")
        return st, sts.tolist(), [x.as_dict() for x in res], R, r.tolist(), y

    def autotune(self, reps=3, stream=None):
        """Time the tile variants for every width a solve can use
        (alm_bm_batch_autotune); returns {width: variant}."""
        cap = 16  # ALM_BM_BATCH_TUNE_MAX
        ws = np.zeros(cap, dtype=np.int32)
        vs = np.zeros(cap, dtype=np.int32)
        n = C.c_int32(0)
        check(lib.alm_bm_batch_autotune(self._h, int(reps), ws.ctypes.data, vs.ctypes.data, C.byref(n),
                                        _stream(stream)), "batch_autotune")
        return {int(ws[i]): int(vs[i]) for i in range(n.value)}

    def instance(self, q, R, y, r):
        """Instance q's factor (n_q x r_q view) and dual."""
        a, b = self.offsets[q], self.offsets[q + 1]
        return R[a:b, :r], y[a:b]
