"""Preconditioned conjugate gradients (FP64 reference).

Test infrastructure only (see the package docstring).

The paper pairs its multigrid with a Krylov method (section 2.5) without
naming it; the pinned pressure matrix is symmetric positive definite and the
V-cycle preconditioner is symmetric, so conjugate gradients applies.  The
stopping rule is ||b - A x||_2 <= rtol ||b||_2; when the recurred residual
meets it the true residual is recomputed, and if that one does not, the
iteration restarts from it: r = b - A x, and the next direction is M r alone
(beta = 0).  Carrying the old direction across the replaced residual loses
conjugacy, and near the attainable accuracy (a tolerance the rounding of A x
cannot reach) repeated replacements then drive the iterate away instead of
leaving it where it stagnates.  ``flexible`` selects the flexible form
for preconditioners that are only approximately fixed (a lower-precision
V-cycle): alpha = (r.p) / (p.Ap), the exact line search along p, and
beta = -(z_new.Ap) / (p.Ap), which makes the new direction A-orthogonal to
the previous one whatever the preconditioner did (flexible CG with one
stored direction, Notay 2000).  For a fixed SPD preconditioner both forms
equal the standard ones in exact arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, -4


@dataclass
class PcgResult:
    x: np.ndarray
    iterations: int
    status: int
    rel_residual: float
    history: List[float] = field(default_factory=list)


def pcg(A, b, M: Optional[Callable] = None, x0=None, rtol=1e-10, max_iter=500,
        flexible=False) -> PcgResult:
    b = np.asarray(b, dtype=np.float64)
    M = M if M is not None else (lambda r: r.copy())
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    if bnorm == 0.0:
        return PcgResult(np.zeros_like(b), 0, OK, 0.0)
    r = b - A @ x
    rn = float(np.linalg.norm(r))
    hist = [rn / bnorm]
    if rn <= rtol * bnorm:
        return PcgResult(x, 0, OK, rn / bnorm, hist)
    z = M(r)
    p = z.copy()
    rz = float(r @ z)
    if not rz > 0.0:
        return PcgResult(x, 0, BREAKDOWN, rn / bnorm, hist)
    restart = False
    for k in range(1, max_iter + 1):
        q = A @ p
        pq = float(p @ q)
        if not pq > 0.0:
            return PcgResult(x, k - 1, BREAKDOWN, hist[-1], hist)
        alpha = float(r @ p) / pq if flexible else rz / pq
        x = x + alpha * p
        r = r - alpha * q
        rn = float(np.linalg.norm(r))
        hist.append(rn / bnorm)
        if rn <= rtol * bnorm:
            rt = b - A @ x
            rtn = float(np.linalg.norm(rt))
            if rtn <= rtol * bnorm:
                hist[-1] = rtn / bnorm
                return PcgResult(x, k, OK, rtn / bnorm, hist)
            r = rt
            restart = True
        z = M(r)
        rz_new = float(r @ z)
        if not rz_new > 0.0:
            return PcgResult(x, k, BREAKDOWN, hist[-1], hist)
        if restart:
            beta, restart = 0.0, False
        else:
            beta = -float(z @ q) / pq if flexible else rz_new / rz
        p = z + beta * p
        rz = rz_new
    rt = b - A @ x
    return PcgResult(x, max_iter, NOT_CONVERGED, float(np.linalg.norm(rt)) / bnorm, hist)
