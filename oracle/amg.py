"""Smoothed-aggregation algebraic multigrid (FP64 reference).

Test infrastructure only (see the package docstring).

The paper (section 2.5) solves the pressure system with algebraic multigrid,
which builds its coarse levels from the matrix alone by heuristic coarsening
and couples them through prolongation and relaxation; it names no variant or
parameter.  This project's reading is smoothed aggregation:

  strength   j is a strong neighbour of i (i != j) iff
             a_ij^2 >= theta_l^2 * (a_ii * a_jj), with the threshold halved on
             each coarser level: theta_l = 0.08 * 0.5^l on level l (the
             finest is level 0), the level-halved threshold of Vanek, Mandel
             and Brezina's smoothed aggregation (1996).  Galerkin operators spread their couplings over
             more, weaker entries than the finest operator does; a fixed
             0.08 cut many of them, which left small aggregates, dense coarse
             levels and three times the PCG iterations on the plate and the
             128^3 cube;
  MIS-2      a distance-2 maximal independent set of the strength graph,
             found in synchronous rounds: node keys are (state, priority,
             -index) compared lexicographically, state IN > UNDECIDED > OUT,
             priority = fmix32(index xor salt(level)); each round takes the
             maximum key over the distance-2 neighbourhood; an undecided node
             whose own key is that maximum joins the set, one whose maximum
             belongs to a set node leaves.  Nodes with no strong neighbour are
             OUT from the start and never aggregated;
  aggregates each set node is a root; its strong neighbours join it; every
             node still left joins the aggregate of its strong neighbour
             (already placed in the first pass) with the largest |a_ij|,
             ties to the lowest index; aggregate ids follow root order;
  P_tent     near-null vector B (all ones on the finest level); column J
             holds B restricted to aggregate J divided by its 2-norm, and
             the coarse near-null vector is those norms;
  rho        upper estimate of the spectral radius of D^-1 A: on the finest
             level the Gershgorin bound max_i sum_j |a_ij| / a_ii (sharp for
             that M-matrix); on coarse levels, where Gershgorin overshoots by
             about 2x, 1.1 times a 15-step power-iteration estimate started
             from x_i = 1/2 + fmix32(i xor salt(level)) / 2^32;
  P          P_tent - omega D^-1 A P_tent, omega = 4 / (3 rho);
  A_c        Galerkin product P^T A P; R = P^T;
  smoother   Chebyshev polynomial of degree k (default 2) in D^-1 A on
             [rho / 7, rho] (the ratio measured best among 5, 7, 10, 15 and
             30); or (smoother = "l1jacobi") k sweeps of
             l1-Jacobi relaxation x <- x + D_l1^-1 (b - A x), D_l1 the
             diagonal of row l1 norms sum_j |a_ij|, convergent for every SPD
             A because D_l1 - A is diagonally dominant;
  cycle      V-cycle with the same smoother before and after the coarse
             correction (so the preconditioner is symmetric); the coarsest
             level (at most coarse_max rows, default 512) is solved with a
             dense inverse;
  reuse      (optional) after a mask change, keep the coarse levels of an
             earlier hierarchy and rebuild only the finest one, its
             prolongator's rows re-indexed to the new active cells
             (reuse_coarse_levels).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .hash import priority

OUT, UND, IN = 0, 1, 2


def strength(A: sp.csr_matrix, theta: float) -> sp.csr_matrix:
    """Strong off-diagonal entries of A, keeping their values a_ij."""
    A = A.tocsr()
    n = A.shape[0]
    d = A.diagonal()
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    v = A.data
    theta2 = theta * theta
    strong = (rows != cols) & (v != 0.0) & (v * v >= theta2 * (d[rows] * d[cols]))
    S = sp.csr_matrix((v[strong], (rows[strong], cols[strong])), shape=A.shape)
    S.sort_indices()
    return S


def _neighbour_max(S: sp.csr_matrix, key: np.ndarray) -> np.ndarray:
    """out_i = max(key_i, max over strong neighbours j of key_j)."""
    out = key.copy()
    deg = np.diff(S.indptr)
    nz = np.nonzero(deg > 0)[0]
    if nz.size:
        seg = np.maximum.reduceat(key[S.indices], S.indptr[nz])
        out[nz] = np.maximum(out[nz], seg)
    return out


def mis2(S: sp.csr_matrix, level: int):
    """Final node states (IN / OUT) and the number of rounds taken."""
    n = S.shape[0]
    if n >= 2**30:
        raise ValueError("level too large for 30-bit index keys")
    deg = np.diff(S.indptr)
    state = np.where(deg > 0, UND, OUT).astype(np.uint64)
    h = priority(n, level)
    low = np.uint64(2**30 - 1) - np.arange(n, dtype=np.uint64)
    rounds = 0
    while np.any(state == UND):
        key = (state << np.uint64(62)) | (h << np.uint64(30)) | low
        m2 = _neighbour_max(S, _neighbour_max(S, key))
        und = state == UND
        win = und & (m2 == key)
        lose = und & ~win & ((m2 >> np.uint64(62)) == IN)
        state = state.copy()
        state[win] = IN
        state[lose] = OUT
        rounds += 1
    return state.astype(np.int64), rounds


def aggregate(S: sp.csr_matrix, state: np.ndarray):
    """Aggregate id per node (-1 if not aggregated) and the aggregate count."""
    n = S.shape[0]
    rows = np.repeat(np.arange(n), np.diff(S.indptr))
    cols = S.indices
    absv = np.abs(S.data)
    roots = state == IN
    n_agg = int(roots.sum())
    agg = np.full(n, -1, dtype=np.int64)
    agg[roots] = np.arange(n_agg)
    # first pass: strong neighbours of a root join it (the root is unique
    # because roots are at least three edges apart)
    m = ~roots[rows] & roots[cols]
    first = agg.copy()
    first[rows[m]] = agg[cols[m]]
    # second pass: leftover nodes join the first-pass node they are most
    # strongly coupled to (largest |a_ij|, ties to the lowest j)
    deg = np.diff(S.indptr)
    left = (first < 0) & (deg > 0)
    cand = left[rows] & (first[cols] >= 0)
    r, c, v = rows[cand], cols[cand], absv[cand]
    out = first.copy()
    if r.size:
        order = np.lexsort((c, -v, r))
        r, c = r[order], c[order]
        head = np.ones(r.shape[0], dtype=bool)
        head[1:] = r[1:] != r[:-1]
        out[r[head]] = first[c[head]]
    if np.any((out < 0) & (deg > 0)):
        raise AssertionError("MIS-2 left a node with strong neighbours unaggregated")
    return out, n_agg


def tentative(agg: np.ndarray, n_agg: int, B: np.ndarray):
    """P_tent (n x n_agg) and the coarse near-null vector."""
    n = agg.shape[0]
    rows = np.nonzero(agg >= 0)[0]
    J = agg[rows]
    norm = np.sqrt(np.bincount(J, weights=B[rows] * B[rows], minlength=n_agg))
    P = sp.csr_matrix((B[rows] / norm[J], (rows, J)), shape=(n, n_agg))
    P.sort_indices()
    return P, norm


def gershgorin(A: sp.csr_matrix) -> float:
    """max_i sum_j |a_ij| / a_ii (an upper bound on the spectrum of D^-1 A)."""
    rs = np.asarray(abs(A).sum(axis=1)).ravel()
    return float(np.max(rs / A.diagonal())) if A.shape[0] else 1.0


POWER_ITERS = 15
POWER_SAFETY = 1.1


def power_estimate(A: sp.csr_matrix, level: int, iters: int = POWER_ITERS) -> float:
    """Power iteration for the largest eigenvalue of D^-1 A: y = D^-1 A x,
    lambda = ||y|| / ||x||, x <- y / ||y||, from the hashed start vector."""
    n = A.shape[0]
    if n == 0:
        return 1.0
    d = A.diagonal()
    x = 0.5 + priority(n, level).astype(np.float64) / 2.0**32
    lam = 0.0
    for _ in range(iters):
        y = (A @ x) / d
        ny = np.linalg.norm(y)
        lam = ny / np.linalg.norm(x)
        if ny == 0.0:
            break
        x = y / ny
    return float(lam)


def spectral_bound(A: sp.csr_matrix, level: int) -> float:
    """rho used by the prolongator smoothing and the Chebyshev smoother."""
    if level == 0:
        return gershgorin(A)
    return POWER_SAFETY * power_estimate(A, level)


def smooth_prolongator(A: sp.csr_matrix, P_tent: sp.csr_matrix, rho: float):
    omega = 4.0 / (3.0 * rho)
    Dinv = sp.diags(1.0 / A.diagonal(), format="csr")
    P = (P_tent - omega * (Dinv @ (A @ P_tent))).tocsr()
    P.sort_indices()
    return P


def galerkin(A: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    Ac = (P.T @ (A @ P)).tocsr()
    Ac.sort_indices()
    return Ac


def chebyshev_coefficients(lmax: float, lmin: float, degree: int):
    """Coefficients of the Chebyshev semi-iteration on [lmin, lmax]:
    step 1 is d = r / theta; step j > 1 is d = c1_j d + c2_j r.  Returns
    (1/theta, [(c1_j, c2_j) for j = 2..degree])."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho_prev = 1.0 / sigma
    steps = []
    for _ in range(2, degree + 1):
        rho_j = 1.0 / (2.0 * sigma - rho_prev)
        steps.append((rho_j * rho_prev, 2.0 * rho_j / delta))
        rho_prev = rho_j
    return 1.0 / theta, steps


def chebyshev(A, diag, b, x, lmax, lmin, degree):
    """Chebyshev smoothing of A x = b, preconditioned by the diagonal.
    ``x is None`` means a zero initial guess."""
    inv_theta, steps = chebyshev_coefficients(lmax, lmin, degree)
    if x is None:
        x = np.zeros_like(b)
        r = b / diag
    else:
        r = (b - A @ x) / diag
    d = inv_theta * r
    x = x + d
    for c1, c2 in steps:
        r = (b - A @ x) / diag
        d = c1 * d + c2 * r
        x = x + d
    return x


def l1_diagonal(A: sp.csr_matrix) -> np.ndarray:
    """Row l1 norms sum_j |a_ij| (the diagonal included)."""
    return np.asarray(abs(A).sum(axis=1)).ravel()


def l1_jacobi(A, dl1, b, x, sweeps):
    """`sweeps` l1-Jacobi sweeps x <- x + (b - A x) / dl1; ``x is None``
    means a zero initial guess."""
    if x is None:
        x = b / dl1
        sweeps -= 1
    for _ in range(sweeps):
        x = x + (b - A @ x) / dl1
    return x


@dataclass
class Level:
    A: sp.csr_matrix
    diag: np.ndarray
    rho: float
    B: np.ndarray
    dl1: Optional[np.ndarray] = None
    agg: Optional[np.ndarray] = None
    n_agg: int = 0
    mis_rounds: int = 0
    P_tent: Optional[sp.csr_matrix] = None
    P: Optional[sp.csr_matrix] = None
    R: Optional[sp.csr_matrix] = None
    Ainv: Optional[np.ndarray] = None


@dataclass
class Hierarchy:
    levels: List[Level] = field(default_factory=list)
    degree: int = 2
    ratio: float = 7.0
    smoother: str = "chebyshev"

    @property
    def operator_complexity(self) -> float:
        nnz0 = self.levels[0].A.nnz
        return sum(l.A.nnz for l in self.levels) / nnz0 if nnz0 else 1.0


def build_hierarchy(A0: sp.csr_matrix, theta=0.08, coarse_max=512, max_levels=10,
                    degree=2, ratio=7.0, dense_max=4096, smoother="chebyshev",
                    theta_decay=0.5) -> Hierarchy:
    """Levels until coarse_max rows; level l's strength threshold is
    theta * theta_decay^l (theta_decay = 1: the same threshold everywhere)."""
    if smoother not in ("chebyshev", "l1jacobi"):
        raise ValueError(f"unknown smoother {smoother!r}")
    H = Hierarchy(degree=degree, ratio=ratio, smoother=smoother)
    A = A0.tocsr()
    B = np.ones(A.shape[0])
    for lvl in range(max_levels):
        lev = Level(A=A, diag=A.diagonal().copy(), rho=spectral_bound(A, lvl), B=B,
                    dl1=l1_diagonal(A))
        H.levels.append(lev)
        if A.shape[0] <= coarse_max or lvl == max_levels - 1:
            break
        S = strength(A, theta * theta_decay ** lvl)
        state, rounds = mis2(S, lvl)
        agg, n_agg = aggregate(S, state)
        if n_agg == 0:
            break
        lev.agg, lev.n_agg, lev.mis_rounds = agg, n_agg, rounds
        lev.P_tent, Bc = tentative(agg, n_agg, B)
        lev.P = smooth_prolongator(A, lev.P_tent, lev.rho)
        lev.R = lev.P.T.tocsr()
        A = galerkin(A, lev.P)
        B = Bc
    last = H.levels[-1]
    if 0 < last.A.shape[0] <= dense_max:
        c = sla.cho_factor(last.A.toarray(), lower=True)
        last.Ainv = sla.cho_solve(c, np.eye(last.A.shape[0]))
    return H


def reuse_coarse_levels(H: Hierarchy, A_new: sp.csr_matrix, base_row, pinned) -> Hierarchy:
    """A hierarchy for a new masked operator that keeps the coarse levels of H.

    Level 0 becomes A_new, with its own diagonal, Gershgorin bound and row l1
    norms.  Its prolongator takes, for every row i of A_new, row base_row[i]
    of H's finest prolongator (the same cell in H's numbering); rows of pinned
    cells and of cells H did not have (base_row < 0) are empty.  R = P^T.
    Every coarser level is H's own.  The V-cycle stays symmetric with SPD
    coarse operators, so it is still an SPD preconditioner of A_new, and
    nothing of the aggregation or the Galerkin products is recomputed."""
    A_new = A_new.tocsr()
    base_row = np.asarray(base_row)
    pinned = np.asarray(pinned, dtype=bool)
    P0 = H.levels[0].P.tocsr()
    keep = (base_row >= 0) & ~pinned
    rows = np.nonzero(keep)[0]
    lengths = np.zeros(A_new.shape[0], dtype=np.int64)
    lengths[rows] = np.diff(P0.indptr)[base_row[rows]]
    indptr = np.concatenate([[0], np.cumsum(lengths)])
    cols = np.concatenate([P0.indices[P0.indptr[o]:P0.indptr[o + 1]] for o in base_row[rows]]) \
        if rows.size else np.zeros(0, dtype=np.int64)
    vals = np.concatenate([P0.data[P0.indptr[o]:P0.indptr[o + 1]] for o in base_row[rows]]) \
        if rows.size else np.zeros(0)
    P = sp.csr_matrix((vals, cols, indptr), shape=(A_new.shape[0], P0.shape[1]))
    lev0 = Level(A=A_new, diag=A_new.diagonal().copy(), rho=spectral_bound(A_new, 0),
                 B=np.ones(A_new.shape[0]), dl1=l1_diagonal(A_new))
    lev0.P, lev0.R = P, P.T.tocsr()
    lev0.agg, lev0.n_agg = None, P0.shape[1]
    G = Hierarchy(degree=H.degree, ratio=H.ratio, smoother=H.smoother)
    G.levels = [lev0] + list(H.levels[1:])
    return G


def _smooth(H: Hierarchy, lev: Level, b, x):
    if H.smoother == "l1jacobi":
        return l1_jacobi(lev.A, lev.dl1, b, x, H.degree)
    return chebyshev(lev.A, lev.diag, b, x, lev.rho, lev.rho / H.ratio, H.degree)


def vcycle(H: Hierarchy, b, level=0):
    """One V-cycle applied to b with a zero initial guess."""
    lev = H.levels[level]
    if level == len(H.levels) - 1:
        if lev.Ainv is not None:
            return lev.Ainv @ b
        return _smooth(H, lev, b, _smooth(H, lev, b, None))
    x = _smooth(H, lev, b, None)
    r = b - lev.A @ x
    xc = vcycle(H, lev.R @ r, level + 1)
    x = x + lev.P @ xc
    return _smooth(H, lev, b, x)
