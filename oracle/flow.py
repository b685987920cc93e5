"""One time step of the fractional-step solidification solver (section 2.2,
steps 1-4): the oracle of the time-step driver.  Test infrastructure only:
the tests, the smoke check and the benchmark's CPU leg use it; the product
path never does.

What one step computes, and where the paper defines it:

* Solid fraction (Eq. 21): the Gulliver-Scheil relation of Eq. 5 with its
  jump at the solidus replaced by a straight line over [T_sol - T_eps,
  T_sol + T_eps]; its derivative in closed form on each branch.  Branch
  boundaries: T > T_liq is liquid, T < T_sol - T_eps solid, the closed band
  |T - T_sol| <= T_eps linear, Scheil in between.
* Darcy drag (Eq. 3, Blake-Kozeny): mu/K = 180 mu f_s^2 / (lam^2 (1-f_s)^3),
  0 for f_s = 0, and capped at 1e12 rho/dt (reading: beyond it u* is below
  1e-12 of its value without drag, and the cap keeps the coefficient finite
  in every precision).  Only cells with f_s < 1 are solved.
* Diffusion of a cell field phi with coefficient Gamma (Eq. 10-12):
      D_i = Gamma sum_{interior f of i} s_if [c'_f (phi_C2 - phi_C1) + t'_f.grad(phi)_f]
          + Gamma sum_{wall f of i} w_f (phi_wall - phi_i),
  s_if = +1 for the owner and -1 for the neighbour, c'_f = |S_f|^2/(S_f.d_f)
  the direct coefficient, t'_f = S_f - c'_f d_f the cross vector, grad_f the
  Eq. 12 gradient over all cells sharing a vertex with the face, and
  w_f = |S_f|^2/(S_f.(x_f - x_C1)) a wall held at phi_wall at its centre.
  Reading: the direct part is Crank-Nicolson (half at each level), the cross
  part is deferred to the old level.
* Convection (Eq. 2, 4): C_i = rho_eff sum_{interior f of i} s_if F_f
  (phi_C1 + phi_C2)/2 with the corrected volume fluxes F (section 2.4.3);
  Adams-Bashforth 3/2 C^n - 1/2 C^(n-1) (Euler on the first step).
* Momentum predictor (Eq. 6) on the cells with f_s < 1, each component k:
      (rho V/dt + V mu/K) u*_i - 1/2 D^dir_i(u*) =
          rho V/dt u^n_i - AB(C(u)) + 1/2 D^dir_i(u^n) + D^cross_i(u^n)
          - V g_k rho beta (T^n_i - T_ref).
  Solid cells hold u = 0: their rows and columns are deleted and a fluid
  cell's diagonal keeps the coefficient of a face towards one (section
  2.4.2, momentum).  Walls are no-slip.
* Pressure, face flux and velocity correction (Eq. 7-9, 11-17): the
  masked projection of `projection.project` with f_l = 1 - f_s^n and the
  pressure coefficient c'_f / rho.
* Energy (Eq. 4 with Eq. 18-20) on every cell, Picard iteration m from
  T^0 = T^n, f_s^0 = f_s^n:
      (rho c_p V/dt - S_p) T^(m+1)_i - 1/2 D^dir_i(T^(m+1)) =
          rho c_p V/dt T^n_i - AB(C^T) + 1/2 D^dir_i(T^n) + D^cross_i(T^n) + S_c,
      S_p = (rho L_f V/dt) f_s'(T^m),
      S_c = (rho L_f V/dt) (f_s^m - f_s^n - f_s'(T^m) T^m)
  (reading: Eq. 18 is the latent term integrated over the cell and the
  step; divided by the step it carries rho/dt, as Eq. 4 does), with
  C^T = rho c_p sum s_if F^(n+1)_f (T^n_C1 + T^n_C2)/2.  The solved
  temperature T* becomes T^(m+1) except where it lies beyond a kink of
  Eq. 21 seen from T^m: there the cell stops at the first kink it crosses
  (reading: Eq. 19-20 are Newton's linearisation of a piecewise-smooth
  relation, which cycles when a cell jumps across a kink in one pass; the
  limit changes the path only, since at convergence no cell crosses a kink).
  Then f_s^(m+1) = (1 - lambda) f_s^m + lambda f_s(T^(m+1)) (lambda = 1 by
  default, as the paper finds for its aluminium alloy), until
  max|T* - T^m| <= tol max|T^(m+1)| and max|f_s^(m+1) - f_s^m| <= tol.
  Walls are held at T_wall, or insulated (T_wall None).
* Mask evolution: cells with f_s^(n+1) = 1 get u = 0, faces no longer open
  under the new mask get F = 0 (reading: they are blocked from now on).

Every linear system is solved exactly (sparse LU); nothing is blocked or
reordered beyond these definitions.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import projection as pj

DARCY_CAP = 1e12   # times rho/dt


@dataclass(frozen=True)
class Props:
    rho: float
    cp: float
    k: float
    mu: float
    beta: float
    lam: float
    Lf: float
    T_f: float
    T_liq: float
    T_sol: float
    T_eps: float
    k_p: float
    T_ref: float
    g: tuple
    T_wall: float | None

    @staticmethod
    def of(d) -> "Props":
        return d if isinstance(d, Props) else Props(**d)


@dataclass
class State:
    u: np.ndarray            # [n, 3] cell velocities (0 on solid cells)
    T: np.ndarray            # [n] temperature
    fs: np.ndarray           # [n] solid fraction
    F: np.ndarray            # [n_faces] corrected volume fluxes (0 on blocked and wall faces)
    p: np.ndarray            # [n] pressure of the last step
    conv_u: np.ndarray | None = None   # [n, 3] C(u) of the last step (Adams-Bashforth)
    conv_T: np.ndarray | None = None   # [n] C^T of the last step


# ---------------------------------------------------------------- Eq. 21, 3
def _scheil(T, a: Props):
    x = (T - a.T_f) / (a.T_liq - a.T_f)
    e = 1.0 / (a.k_p - 1.0)
    return 1.0 - x ** e, -e * x ** (e - 1.0) / (a.T_liq - a.T_f)


def _branches(T, a: Props):
    T = np.asarray(T, dtype=np.float64)
    liquid = T > a.T_liq
    solid = T < a.T_sol - a.T_eps
    band = ~liquid & ~solid & (np.abs(T - a.T_sol) <= a.T_eps)
    scheil = ~liquid & ~solid & ~band
    return T, liquid, solid, band, scheil


def solid_fraction(T, a):
    """f_s(T) of Eq. 21."""
    a = Props.of(a)
    T, liquid, solid, band, scheil = _branches(T, a)
    fhat = _scheil(np.float64(a.T_sol + a.T_eps), a)[0]
    fs = np.zeros_like(T)
    fs[solid] = 1.0
    fs[band] = fhat - (T[band] - a.T_sol - a.T_eps) * ((1.0 - fhat) / (2.0 * a.T_eps))
    fs[scheil] = _scheil(T[scheil], a)[0]
    return fs


def solid_fraction_slope(T, a):
    """df_s/dT of Eq. 21 (0 on the liquid and solid branches)."""
    a = Props.of(a)
    T, liquid, solid, band, scheil = _branches(T, a)
    fhat = _scheil(np.float64(a.T_sol + a.T_eps), a)[0]
    d = np.zeros_like(T)
    d[band] = -(1.0 - fhat) / (2.0 * a.T_eps)
    d[scheil] = _scheil(T[scheil], a)[1]
    return d


def darcy(fs, a, dt):
    """mu/K of Eq. 3 for f_s < 1, capped at DARCY_CAP rho/dt."""
    a = Props.of(a)
    fs = np.asarray(fs, dtype=np.float64)
    out = np.zeros_like(fs)
    m = (fs > 0) & (fs < 1)
    out[m] = 180.0 * a.mu * fs[m] ** 2 / (a.lam ** 2 * (1.0 - fs[m]) ** 3)
    return np.minimum(out, DARCY_CAP * a.rho / dt)


# ------------------------------------------------------- geometry (Eq. 10-12)
def direct_coeff(mesh):
    """c'_f = |S_f|^2 / (S_f.d_f) on interior faces, 0 on walls."""
    c = np.zeros(mesh.n_faces)
    f = np.nonzero(mesh.neigh >= 0)[0]
    S = mesh.face_area[f]
    d = mesh.cell_centre[mesh.neigh[f]] - mesh.cell_centre[mesh.owner[f]]
    c[f] = np.einsum("fd,fd->f", S, S) / np.einsum("fd,fd->f", S, d)
    return c


def wall_coeff(mesh):
    """w_f = |S_f|^2 / (S_f.(x_f - x_C1)) on wall faces, 0 elsewhere."""
    w = np.zeros(mesh.n_faces)
    f = np.nonzero(mesh.neigh < 0)[0]
    S = mesh.face_area[f]
    d = mesh.face_centre[f] - mesh.cell_centre[mesh.owner[f]]
    w[f] = np.einsum("fd,fd->f", S, S) / np.einsum("fd,fd->f", S, d)
    return w


class Geometry:
    """Per-mesh quantities of the step: coefficients, the cross operator and
    the interior incidence."""

    def __init__(self, mesh):
        self.mesh = mesh
        n, nf = mesh.n_cells, mesh.n_faces
        self.V = np.asarray(mesh.cell_volume, dtype=np.float64)
        self.c = direct_coeff(mesh)
        self.w = wall_coeff(mesh)
        inner = mesh.neigh >= 0
        self.inner = inner
        f = np.nonzero(inner)[0]
        self.f_in = f
        d = mesh.cell_centre[mesh.neigh[f]] - mesh.cell_centre[mesh.owner[f]]
        t = np.zeros((nf, 3))
        t[f] = mesh.face_area[f] - self.c[f, None] * d
        self.t = t
        Gm = pj.gradient_matrices(pj.face_stencils(mesh), n)
        # x_f(phi) = t'_f . grad(phi)_f
        self.X = sum(sp.diags(t[:, k]) @ Gm[k] for k in range(3)).tocsr()
        # E: +1 at (f, owner), -1 at (f, neighbour) on interior faces
        rows = np.concatenate([f, f])
        cols = np.concatenate([mesh.owner[f], mesh.neigh[f]]).astype(np.int64)
        vals = np.concatenate([np.ones(len(f)), -np.ones(len(f))])
        self.E = sp.csr_matrix((vals, (rows, cols)), shape=(nf, n))
        # wall coefficient summed per cell
        wf = np.nonzero(~inner)[0]
        self.W = np.bincount(mesh.owner[wf], weights=self.w[wf], minlength=n)


def laplacian(geo: Geometry, coef, faces):
    """L with L_ii = sum coef_f, L_ij = -coef_f over the given interior faces
    (boolean mask): (L phi)_i = sum_f coef_f (phi_i - phi_other)."""
    m = geo.mesh
    f = np.nonzero(faces)[0]
    o, nb = m.owner[f].astype(np.int64), m.neigh[f].astype(np.int64)
    cf = np.asarray(coef)[f]
    rows = np.concatenate([o, nb, o, nb])
    cols = np.concatenate([o, nb, nb, o])
    vals = np.concatenate([cf, cf, -cf, -cf])
    return sp.csr_matrix((vals, (rows, cols)), shape=(m.n_cells, m.n_cells))


def diffusion_direct(geo: Geometry, phi, gamma, phi_wall):
    """Gamma [sum_f s_if c'_f (phi_C2 - phi_C1) + sum_wall w_f (phi_wall - phi_i)]
    over every interior face (phi_wall None: insulated walls)."""
    m = geo.mesh
    L = laplacian(geo, geo.c, geo.inner)
    out = -(L @ phi)
    if phi_wall is not None:
        out = out + geo.W * (phi_wall - phi)
    return gamma * out


def diffusion_cross(geo: Geometry, phi, gamma):
    """Gamma sum_f s_if t'_f . grad(phi)_f over every interior face."""
    return gamma * (geo.E.T @ (geo.X @ phi))


def convection(geo: Geometry, F, phi, rho_eff):
    """rho_eff sum_f s_if F_f (phi_C1 + phi_C2) / 2 (net outflow of phi)."""
    m = geo.mesh
    f = geo.f_in
    flux = np.zeros(m.n_faces)
    flux[f] = F[f] * 0.5 * (phi[m.owner[f]] + phi[m.neigh[f]])
    return rho_eff * (geo.E.T @ flux)


def _ab(cur, prev):
    return cur if prev is None else 1.5 * cur - 0.5 * prev


# ----------------------------------------------------------- step 1 (Eq. 6)
def momentum_predictor(geo: Geometry, a, st: State, dt):
    """u* and C(u^n) (for the next step's Adams-Bashforth term)."""
    a = Props.of(a)
    m = geo.mesh
    n = m.n_cells
    act = st.fs < 1.0
    idx = np.nonzero(act)[0]
    opn = geo.inner.copy()
    opn[geo.inner] = act[m.owner[geo.inner]] & act[m.neigh[geo.inner]]
    # interior faces from a fluid cell to a solid one: coefficient on the diagonal
    blk = geo.inner & ~opn
    diag_blk = (np.bincount(m.owner[blk], weights=geo.c[blk], minlength=n)
                + np.bincount(m.neigh[blk], weights=geo.c[blk], minlength=n))
    shift = (a.rho * geo.V / dt + darcy(st.fs, a, dt) * geo.V
             + 0.5 * a.mu * (geo.W + diag_blk))
    M = (sp.diags(shift) + 0.5 * a.mu * laplacian(geo, geo.c, opn)).tocsr()
    Ma = M[idx][:, idx].tocsc()
    conv = np.stack([convection(geo, st.F, st.u[:, k], a.rho) for k in range(3)], axis=1)
    ab = _ab(conv, st.conv_u)
    ustar = np.zeros((n, 3))
    for k in range(3):
        rhs = (a.rho * geo.V / dt * st.u[:, k] - ab[:, k]
               + 0.5 * diffusion_direct(geo, st.u[:, k], a.mu, 0.0)
               + diffusion_cross(geo, st.u[:, k], a.mu)
               - geo.V * a.g[k] * a.rho * a.beta * (st.T - a.T_ref))
        if len(idx):
            ustar[idx, k] = spla.spsolve(Ma, rhs[idx])
    return ustar, conv


# ------------------------------------------------ step 4 (Eq. 4, 18-21)
def branch_limited(T_prev, T_solved, a):
    """The next Picard iterate: T_solved, except that a cell whose solved
    temperature lies beyond a kink of Eq. 21 (T_liq, T_sol + T_eps,
    T_sol - T_eps) as seen from T_prev stops at the first kink it crosses.
    A cell already on a kink moves freely; the kink belongs to the branch
    below it (Eq. 21's liquid branch is T > T_liq, its band is closed), so
    the next pass linearises with the slope of the branch the cell entered.
    At convergence no cell crosses a kink, so the fixed point is the plain
    iteration's."""
    a = Props.of(a)
    out = np.array(T_solved, dtype=np.float64, copy=True)
    lo = np.minimum(T_prev, T_solved)
    hi = np.maximum(T_prev, T_solved)
    down = T_solved < T_prev
    done = np.zeros(out.shape, dtype=bool)
    kinks = (a.T_liq, a.T_sol + a.T_eps, a.T_sol - a.T_eps)
    # cooling cells stop at the highest kink strictly between, heating ones at the lowest
    for K in kinks:
        hit = down & ~done & (lo < K) & (K < hi)
        out[hit] = K
        done |= hit
    done[:] = False
    for K in reversed(kinks):
        hit = ~down & ~done & (lo < K) & (K < hi)
        out[hit] = K
        done |= hit
    return out


def energy(geo: Geometry, a, st: State, F_new, dt, tol=1e-10, max_picard=50, relax=1.0):
    """T^(n+1), f_s^(n+1), C^T (for the next step) and the Picard count
    (negative when max_picard passes did not converge).  relax is the
    under-relaxation lambda of the f_s update (0 < lambda <= 1).  Each
    pass's new iterate is branch_limited: Newton's linearisation of Eq. 19
    is kept, and a cell does not jump over a kink of Eq. 21 in one pass."""
    a = Props.of(a)
    rcv = a.rho * a.cp * geo.V / dt
    rlv = a.rho * a.Lf * geo.V / dt
    conv = convection(geo, F_new, st.T, a.rho * a.cp)
    base = (rcv * st.T - _ab(conv, st.conv_T)
            + 0.5 * diffusion_direct(geo, st.T, a.k, a.T_wall)
            + diffusion_cross(geo, st.T, a.k))
    Wk = 0.0 * geo.W if a.T_wall is None else geo.W
    if a.T_wall is not None:
        base = base + 0.5 * a.k * geo.W * a.T_wall
    L = 0.5 * a.k * laplacian(geo, geo.c, geo.inner)
    Tm, fm = st.T.copy(), st.fs.copy()
    for it in range(1, max_picard + 1):
        slope = solid_fraction_slope(Tm, a)
        Sp = rlv * slope
        Sc = rlv * (fm - st.fs - slope * Tm)
        A = (sp.diags(rcv - Sp + 0.5 * a.k * Wk) + L).tocsc()
        Ts = spla.spsolve(A, base + Sc)
        Tn = branch_limited(Tm, Ts, a)
        fn = (1.0 - relax) * fm + relax * solid_fraction(Tn, a)
        dT = np.abs(Ts - Tm).max()
        df = np.abs(fn - fm).max()
        Tm, fm = Tn, fn
        if dT <= tol * np.abs(Tn).max() and df <= tol:
            return Tm, fm, conv, it
    return Tm, fm, conv, -max_picard


# ----------------------------------------------------------------- the step
@dataclass
class StepInfo:
    ustar: np.ndarray
    picard: int            # Picard iterations (negative: not converged)
    projection: object     # projection.Projection


def step(geo: Geometry, a, st: State, dt, picard_tol=1e-10, max_picard=50, relax=1.0):
    """Advance (u, T, f_s, F, p) by one step: steps 1-4 of section 2.2."""
    a = Props.of(a)
    m = geo.mesh
    ustar, conv_u = momentum_predictor(geo, a, st, dt)
    fl = 1.0 - st.fs
    pr = pj.project(m, geo.c / a.rho, fl, ustar, a.rho, dt)
    T, fs, conv_T, picard = energy(geo, a, State(pr.u, st.T, st.fs, pr.flux, pr.p, st.conv_u,
                                                 st.conv_T), pr.flux, dt, picard_tol, max_picard,
                                   relax)
    u = pr.u.copy()
    F = pr.flux.copy()
    solid = fs >= 1.0
    u[solid] = 0.0
    f = geo.f_in
    closed = solid[m.owner[f]] | solid[m.neigh[f]]
    F[f[closed]] = 0.0
    return State(u, T, fs, F, pr.p, conv_u, conv_T), StepInfo(ustar, picard, pr)


def initial_state(mesh, a, T0=None, u0=None):
    """Fluid at rest at T0 (default T_ref), f_s from Eq. 21."""
    a = Props.of(a)
    n = mesh.n_cells
    T = np.full(n, a.T_ref) if T0 is None else np.asarray(T0, dtype=np.float64).copy()
    fs = solid_fraction(T, a)
    u = np.zeros((n, 3)) if u0 is None else np.asarray(u0, dtype=np.float64).copy()
    u[fs >= 1.0] = 0.0
    return State(u, T, fs, np.zeros(mesh.n_faces), np.zeros(n))


def enthalpy(geo: Geometry, a, T, fs):
    """sum_i V_i (rho c_p T_i - rho L_f f_s,i): conserved by the energy step
    with insulated walls (the diffusive and convective fluxes telescope)."""
    a = Props.of(a)
    return float(np.sum(geo.V * (a.rho * a.cp * T - a.rho * a.Lf * fs)))
