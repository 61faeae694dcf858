"""FP64 CPU oracle for the ALM-BM hot path (TEST INFRASTRUCTURE ONLY).

This package is a plain, slow, obviously-correct NumPy/SciPy statement of what
the ALM-BM method computes (arxiv 2505.15775: the SDP (P) and its augmented
Lagrangian in Sec. 1.2, eq. (AL-BM), the dual update of eq. (ALM), gradient
descent eq. (GD) in Sec. 4.2, Alg. 1 (ALORA) in Sec. 5 and the relative KKT
measure of Sec. 6).

It is the checker for the HIP library, not part of it: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It imports nothing from the HIP package, and the HIP package
imports nothing from here.

Pinned functions and their pins are listed in each module's docstring; a
function without an independent pin says "parity unpinned".
"""

from .sdp import (  # noqa: F401
    SDP,
    maxcut_sdp,
    lovasz_sdp,
    edges_sdp,
    completion_sdp,
    generic_sdp,
    cost_apply,
    cost_fro_norm,
    min_eigs,
    amap,
    amap_uv,
    adjoint_apply,
    objective,
    objective_grad,
    dual_update,
    slack_dense,
    slack_matvec,
    min_eig,
    kkt,
    rank_one_norm2,
    maxcut_objective_grad_rows,
)
from .alm import (  # noqa: F401
    SolveOptions,
    line_search_coeffs,
    quartic_argmin,
    inner_gd,
    inner_lbfgs,
    solve,
    curvature_step,
    penalty_moments,
)
from .dense_alm import dense_alm  # noqa: F401
from . import warmstart  # noqa: F401
