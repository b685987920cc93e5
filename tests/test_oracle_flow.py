"""Pins of the time-step oracle (section 2.2 steps 1-4) against facts the
paper and the mathematics fix:

- Eq. 21: the smeared solid fraction is continuous, 0 at the liquidus, 1
  below the band, non-increasing, and its closed-form slope matches a
  central difference on every branch.
- Crank-Nicolson (Eq. 6 and the energy equation): on a uniform box with
  walls held at their face centres, the cell-centred TPFA operator has the
  discrete sine modes sin(k pi (i + 1/2) / N) as eigenvectors with
  eigenvalue sum_d (2 - 2 cos(k_d pi / N_d)) / h_d^2; one step multiplies
  such a mode by (a/dt - G lam / 2) / (a/dt + D + G lam / 2) exactly.
- Latent heat (Eq. 18-20 with the Picard loop): a uniform, insulated,
  resting melt that starts with too little solid releases latent heat until
  c_p (T - T^n) = L_f (f_s(T) - f_s^n), the root of a scalar equation found
  here by bracketing.
- Enthalpy sum V (rho c_p T - rho L_f f_s) is conserved by a whole step with
  insulated walls (fluxes telescope), to the Picard tolerance.
- A uniform body force (buoyancy of a uniform temperature) in a closed
  inviscid box is balanced by the hydrostatic pressure: no face flux.
- Direct + cross diffusion of a quadratic field on a sheared uniform mesh
  is exact: tr(H) V_i per interior cell (the direct part alone is not).
- Convection telescopes (its cell sum is zero), vanishes for a constant
  field carried by a divergence-free flux, and carries a linear field out
  of a cell at the rate rho (U.G) V for a uniform flow U.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import flow
from oracle import projection as pj
from synth import al_si_alloy, box_mesh, t_wall_layer

DT = 1e-3
SHEAR = np.array([[1.0, 0.3, 0.1], [0.0, 1.0, 0.25], [0.0, 0.0, 1.0]])


def _props(**kw):
    a = al_si_alloy()
    a.update(kw)
    return flow.Props.of(a)


def test_solid_fraction_branches_and_slope():
    a = _props()
    fs = lambda T: flow.solid_fraction(np.atleast_1d(np.float64(T)), a)[0]
    assert fs(a.T_liq) == pytest.approx(0.0, abs=1e-15)
    assert fs(a.T_liq + 1.0) == 0.0
    assert fs(a.T_sol - a.T_eps - 1e-9) == 1.0
    # continuity at both ends of the band
    for Tk in (a.T_sol + a.T_eps, a.T_sol - a.T_eps):
        assert abs(fs(Tk + 1e-9) - fs(Tk - 1e-9)) < 1e-9
    T = np.linspace(a.T_sol - 10, a.T_liq + 10, 4001)
    f = flow.solid_fraction(T, a)
    assert np.all(np.diff(f) <= 1e-15)
    assert f.min() == 0.0 and f.max() == 1.0
    # slope against a central difference away from the kinks
    kinks = np.array([a.T_sol - a.T_eps, a.T_sol + a.T_eps, a.T_liq])
    Tm = T[np.abs(T[:, None] - kinks[None, :]).min(axis=1) > 1e-3]
    h = 1e-5
    fd = (flow.solid_fraction(Tm + h, a) - flow.solid_fraction(Tm - h, a)) / (2 * h)
    sl = flow.solid_fraction_slope(Tm, a)
    assert np.abs(fd - sl).max() <= 1e-6 * np.abs(sl).max()
    assert np.any(sl < 0)


def test_darcy_drag():
    a = _props()
    d = flow.darcy(np.array([0.0, 0.5, 1.0 - 1e-12, 1.0]), a, DT)
    assert d[0] == 0.0 and d[3] == 0.0
    assert d[1] > 0
    assert d[2] == flow.DARCY_CAP * a.rho / DT   # capped


def _uniform_box(shape=(6, 5, 4), lengths=(1e-2, 8e-3, 6e-3)):
    return box_mesh(shape, lengths=lengths, jitter=0.0, mode=None)


def _mode(m, ks):
    N = np.array(m.shape)
    h = np.array(m.spacing)
    ijk = m.grid_index
    phi = np.ones(m.n_cells)
    lam = 0.0
    for d in range(3):
        th = ks[d] * np.pi / N[d]
        phi *= np.sin(th * (ijk[:, d] + 0.5))
        lam += (2.0 - 2.0 * np.cos(th)) / h[d] ** 2
    return phi, lam


@pytest.mark.parametrize("fs0", [0.0, 0.3])
def test_momentum_crank_nicolson_decay_of_a_sine_mode(fs0):
    a = _props()
    m = _uniform_box()
    geo = flow.Geometry(m)
    phi, lam = _mode(m, (1, 2, 1))
    st = flow.initial_state(m, a)           # T = T_ref: no buoyancy, liquid
    st.fs[:] = fs0                          # uniform mushy drag (the mask stays open)
    st.u = np.stack([0.01 * phi, -0.02 * phi, 0.005 * phi], axis=1)
    us, _ = flow.momentum_predictor(geo, a, st, DT)
    D = flow.darcy(np.array([fs0]), a, DT)[0]
    g = (a.rho / DT - 0.5 * a.mu * lam) / (a.rho / DT + D + 0.5 * a.mu * lam)
    assert np.abs(us - g * st.u).max() <= 1e-12 * np.abs(st.u).max()
    if fs0:
        assert g < 0.5   # the drag really acts


def test_momentum_solid_neighbours_hold_zero_velocity():
    # the last x-layer is solid: its cells are removed and a fluid cell next to
    # one sees u = 0 at its centre, a full spacing away (the diagonal keeps
    # that face's coefficient).  In x the modes become sin(th (i + 1/2)) with
    # sin(th (N + 1/2)) = 0, i.e. th = k pi / (N + 1/2) over the N fluid layers.
    a = _props()
    m = _uniform_box((7, 5, 4), lengths=(7e-3, 5e-3, 4e-3))
    geo = flow.Geometry(m)
    N = m.shape[0] - 1
    h = np.array(m.spacing)
    ijk = m.grid_index
    th = np.array([2 * np.pi / (N + 0.5), 1 * np.pi / m.shape[1], 2 * np.pi / m.shape[2]])
    phi = np.sin(th[0] * (ijk[:, 0] + 0.5)) * np.sin(th[1] * (ijk[:, 1] + 0.5)) \
        * np.sin(th[2] * (ijk[:, 2] + 0.5))
    lam = float(np.sum((2.0 - 2.0 * np.cos(th)) / h ** 2))
    st = flow.initial_state(m, a)
    solid = ijk[:, 0] == N
    st.fs[solid] = 1.0
    phi[solid] = 0.0
    st.u = np.stack([0.01 * phi, 0.02 * phi, -0.01 * phi], axis=1)
    us, _ = flow.momentum_predictor(geo, a, st, DT)
    g = (a.rho / DT - 0.5 * a.mu * lam) / (a.rho / DT + 0.5 * a.mu * lam)
    assert np.all(us[solid] == 0)
    assert np.abs(us - g * st.u).max() <= 1e-12 * np.abs(st.u).max()


def test_energy_crank_nicolson_decay_of_a_sine_mode():
    a = _props(T_wall=950.0)                # liquid throughout: no latent term
    m = _uniform_box()
    geo = flow.Geometry(m)
    phi, lam = _mode(m, (2, 1, 3))
    dt = 0.05                               # alpha lam dt / 2 of order one
    T = a.T_wall + 20.0 * phi
    st = flow.initial_state(m, a, T0=T)
    Tn, fsn, _, it = flow.energy(geo, a, st, np.zeros(m.n_faces), dt)
    g = (a.rho * a.cp / dt - 0.5 * a.k * lam) / (a.rho * a.cp / dt + 0.5 * a.k * lam)
    assert 0 < it <= 3
    assert np.all(fsn == 0)
    assert np.abs((Tn - a.T_wall) - g * (T - a.T_wall)).max() <= 1e-11 * 20.0
    assert abs(g) < 0.9


@pytest.mark.parametrize("T0,fs0", [(860.0, 0.0), (849.0, 0.4)])
def test_uniform_latent_heat_release(T0, fs0):
    a = _props(T_wall=None)
    m = box_mesh((4, 4, 3), lengths=(1e-2, 1e-2, 8e-3), jitter=0.1, seed=3)
    geo = flow.Geometry(m)
    st = flow.initial_state(m, a, T0=np.full(m.n_cells, T0))
    st.fs[:] = fs0                          # less solid than f_s(T0): heat is released
    T, fs, _, it = flow.energy(geo, a, st, np.zeros(m.n_faces), DT)
    root = brentq(lambda t: a.cp * (t - T0) - a.Lf * (flow.solid_fraction(np.array([t]), a)[0] - fs0),
                  T0, a.T_liq + 1.0, xtol=1e-13, rtol=1e-15)
    assert 0 < it <= 30
    assert np.abs(T - root).max() <= 1e-8 * root
    assert np.abs(fs - flow.solid_fraction(np.array([root]), a)[0]).max() <= 1e-8


def test_enthalpy_is_conserved_with_insulated_walls():
    a = _props(T_wall=None)
    m = box_mesh((6, 5, 5), lengths=(1e-2, 8e-3, 8e-3), jitter=0.1, seed=5)
    geo = flow.Geometry(m)
    x = m.cell_centre
    T0 = 858.0 + 1500.0 * (x[:, 0] - 5e-3) + 4.0 * np.sin(600 * x[:, 2])
    rng = np.random.default_rng(1)
    u0 = 1e-3 * rng.normal(size=(m.n_cells, 3))
    st = flow.initial_state(m, a, T0=T0, u0=u0)
    assert np.any(st.fs == 1) and np.any(st.fs == 0) and np.any((st.fs > 0) & (st.fs < 1))
    H0 = flow.enthalpy(geo, a, st.T, st.fs)
    scale = float(np.sum(geo.V * a.rho * a.cp * np.abs(st.T)))
    for _ in range(3):
        st, info = flow.step(geo, a, st, 5e-3)
        assert info.picard > 0
        assert abs(flow.enthalpy(geo, a, st.T, st.fs) - H0) <= 1e-11 * scale
    assert np.abs(st.F).max() > 0       # the flow really carries heat


def test_uniform_body_force_is_balanced_by_hydrostatic_pressure():
    a = _props(mu=0.0, T_wall=None)
    m = box_mesh((6, 5, 4), lengths=(1e-2, 8e-3, 6e-3), jitter=0.15, seed=2, mode="plane")
    geo = flow.Geometry(m)
    st = flow.initial_state(m, a, T0=np.full(m.n_cells, a.T_ref + 10.0))
    new, info = flow.step(geo, a, st, DT)
    f = -np.array(a.g) * a.rho * a.beta * 10.0                  # body force per volume
    assert np.allclose(info.ustar, DT * f / a.rho, rtol=1e-13, atol=0)
    Fstar = np.abs(pj.star_flux(m, info.ustar, m.neigh >= 0)).max()
    assert np.abs(new.F).max() <= 1e-11 * Fstar
    p_ref = (m.cell_centre - m.cell_centre[0]) @ f
    assert np.abs(new.p - p_ref).max() <= 1e-10 * np.abs(p_ref).max()
    assert np.allclose(new.T, st.T, rtol=1e-14)


def test_diffusion_of_a_quadratic_field_on_a_sheared_mesh():
    # On an affine image of a uniform mesh the Eq. 12 gradient of a quadratic
    # phi = x.H x / 2 is exact at the face centres of faces whose vertices all
    # have eight cells (the vertex means shift every vertex value by the same
    # constant), so the face fluxes are exact and a cell's net diffusion is
    # the volume integral of div grad phi = tr(H): exactly tr(H) V_i.
    m = box_mesh((6, 5, 5), jitter=0.0, mode=None, affine=SHEAR)
    geo = flow.Geometry(m)
    H = np.array([[1.0, 0.2, -0.3], [0.2, 2.0, 0.5], [-0.3, 0.5, -0.7]])
    x = m.cell_centre
    phi = 0.5 * np.einsum("ci,ij,cj->c", x, H, x)
    vc = pj.vertex_cells(m.nodes.shape[0], m.extra["cell_nodes"])
    fn = m.extra["face_nodes"]
    exact = np.array([m.neigh[f] >= 0 and all(len(vc[v]) == 8 for v in fn[f])
                      for f in range(m.n_faces)])
    inner_cells = np.ones(m.n_cells, dtype=bool)
    bad = np.nonzero(~exact)[0]
    inner_cells[m.owner[bad]] = False
    inner_cells[m.neigh[bad][m.neigh[bad] >= 0]] = False
    assert inner_cells.sum() >= 10
    ref = np.trace(H) * geo.V
    D = flow.diffusion_direct(geo, phi, 1.0, None) + flow.diffusion_cross(geo, phi, 1.0)
    assert np.abs(D - ref)[inner_cells].max() <= 1e-12 * np.abs(ref).max()
    # the direct part alone misses the shear
    Dd = flow.diffusion_direct(geo, phi, 1.0, None)
    assert np.abs(Dd - ref)[inner_cells].max() > 1e-2 * np.abs(ref).max()


def test_convection_telescopes_and_carries_constants():
    a = _props()
    m = box_mesh((5, 5, 4), jitter=0.1, seed=7)
    geo = flow.Geometry(m)
    rng = np.random.default_rng(4)
    us = rng.normal(size=(m.n_cells, 3))
    pr = pj.project(m, geo.c / a.rho, np.ones(m.n_cells), us, a.rho, DT)
    phi = rng.normal(size=m.n_cells)
    C = flow.convection(geo, pr.flux, phi, 2.0)
    assert abs(C.sum()) <= 1e-12 * np.abs(C).sum()
    C1 = flow.convection(geo, pr.flux, np.full(m.n_cells, 3.0), 2.0)
    assert np.abs(C1).max() <= 1e-10 * 6.0 * np.abs(pr.flux).max()


def test_cooling_step_solidifies_and_masks():
    # the paper's die-casting set-up (melt at 1000 K, walls at 500 K) after a
    # boundary layer has formed, so that the front moves from the first step
    a = _props()
    m = box_mesh((8, 8, 8), lengths=(1e-2, 1e-2, 1e-2), jitter=0.1, seed=1)
    geo = flow.Geometry(m)
    st = flow.initial_state(m, a, T0=t_wall_layer(m, a.T_wall, 1000.0, 2.6e-3))
    n_solid0 = int((st.fs >= 1).sum())
    rng = np.random.default_rng(2)
    st.u = 1e-3 * rng.normal(size=(m.n_cells, 3))
    st.u[st.fs >= 1] = 0.0
    for _ in range(4):
        new, info = flow.step(geo, a, st, 2e-3)
        assert 0 < info.picard <= 10
        solid_before = st.fs >= 1
        assert np.all(info.ustar[solid_before] == 0)
        solid = new.fs >= 1
        assert np.all(new.u[solid] == 0)
        inner = np.nonzero(m.neigh >= 0)[0]
        closed = solid[m.owner[inner]] | solid[m.neigh[inner]]
        assert np.all(new.F[inner[closed]] == 0)
        assert np.all(new.F[m.neigh < 0] == 0)
        st = new
    assert int((st.fs >= 1).sum()) > n_solid0 > 0
    assert np.any((st.fs > 0) & (st.fs < 1))


def test_convection_of_a_linear_field_by_a_uniform_flow():
    # midpoint face values are exact on a uniform mesh, so a cell without wall
    # faces carries rho_eff (U.G) V_i out: the divergence of phi U
    m = _uniform_box((5, 4, 4))
    geo = flow.Geometry(m)
    U = np.array([0.3, -0.2, 0.5])
    G = np.array([1.5, 0.7, -2.0])
    F = m.face_area @ U
    F[m.neigh < 0] = 0.0
    C = flow.convection(geo, F, m.cell_centre @ G, 2.5)
    interior = np.all((m.grid_index > 0) & (m.grid_index < np.array(m.shape) - 1), axis=1)
    assert interior.sum() >= 4
    ref = 2.5 * (U @ G) * geo.V
    assert np.abs(C - ref)[interior].max() <= 1e-12 * np.abs(ref).max()


def test_branch_limited_iterate():
    """Eq. 21's kinks seen from the previous iterate: a cooling cell stops
    at the highest kink it would cross, a heating one at the lowest; with no
    kink strictly between (a start on a kink included) the solved value
    stays."""
    a = flow.Props.of(_props())
    k1, k2, k3 = a.T_liq, a.T_sol + a.T_eps, a.T_sol - a.T_eps
    prev = np.array([k1 + 5, k1 + 5, k2 + 1, k1 - 1, k3 - 5, k3 - 5, k2 + 1, k1, k3, 700.0])
    solv = np.array([k1 - 1, 700.0, k3 - 3, k1 - 3, 1000.0, k3 + 1, k2 + 2, k1 - 9, k3 + 9, 650.0])
    # (from k3 heating past k2 the next kink still stops the cell)
    want = np.array([k1, k1, k2, k1 - 3, k3, k3, k2 + 2, k1 - 9, k2, 650.0])
    assert np.array_equal(flow.branch_limited(prev, solv, a), want)


@pytest.mark.parametrize("T0,fs0", [(840.0, 0.3), (700.0, 0.0), (845.0, 0.9)])
def test_latent_release_across_kinks_converges(T0, fs0):
    """A solid block holding far less solid than Eq. 21 gives it releases
    enough heat to cross one or more kinks upward in one step: the plain
    Newton passes jump between the solid and liquid branches and never
    settle, the branch-limited ones reach the bracketed root of the cell's
    energy balance c_p (T - T0) = L_f (f_s(T) - f_s0)."""
    a = _props(T_wall=None)
    m = box_mesh((3, 3, 2), lengths=(1e-2, 1e-2, 8e-3), jitter=0.1, seed=3)
    geo = flow.Geometry(m)
    st = flow.initial_state(m, a, T0=np.full(m.n_cells, T0))
    st.fs[:] = fs0
    T, fs, _, it = flow.energy(geo, a, st, np.zeros(m.n_faces), DT, max_picard=40)
    root = brentq(lambda t: a.cp * (t - T0) - a.Lf * (flow.solid_fraction(np.array([t]), a)[0] - fs0),
                  T0, 2000.0, xtol=1e-13, rtol=1e-15)
    assert 0 < it <= 40, it
    assert np.abs(T - root).max() <= 1e-8 * root
    assert np.abs(fs - flow.solid_fraction(np.array([root]), a)[0]).max() <= 1e-8
