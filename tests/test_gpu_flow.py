"""GPU parity of the fractional-step driver (section 2.2 steps 1-4) and of
the shifted assembly it solves with, against the oracle:

- shifted systems diag(s) + L (masked and unmasked) solve to the exact
  (sparse LU) solution within 1e-10 relative L2 at rtol 1e-12, with zeros on
  removed cells and no pins;
- whole steps (momentum predictor, masked projection, energy with the
  Picard loop, mask evolution) match the oracle field by field over several
  steps in which cells solidify: same solid set, same Picard count,
  temperature within 1e-9 relative, solid fraction within 1e-7, pressure,
  velocities and fluxes within 1e-8 relative (the pressure error of the
  projection's 1e-10 residual bar, carried into u and F by dt/rho), and the
  stored convection terms within 1e-8 of the size of the face terms they
  sum (they nearly cancel, so their own size is no scale);
- at 64^3 with insulated walls (beyond the oracle's reach) the properties
  that hold at any size: enthalpy conserved, fluxes divergence-free on
  fluid cells, zero on closed faces, u = 0 on solid cells.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import flow
from oracle import projection as pj
from synth import al_alloy, al_si_alloy, box_mesh, face_coeff, fl_planar_front, t_wall_layer
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu
SHEAR = np.array([[1.0, 0.3, 0.1], [0.0, 1.0, 0.25], [0.0, 0.0, 1.0]])


def _lap(m, c, act):
    inner = m.neigh >= 0
    f = np.nonzero(inner)[0]
    f = f[act[m.owner[f]] & act[m.neigh[f]]]
    o, nb = m.owner[f].astype(np.int64), m.neigh[f].astype(np.int64)
    rows = np.concatenate([o, nb, o, nb])
    cols = np.concatenate([o, nb, nb, o])
    vals = np.concatenate([c[f], c[f], -c[f], -c[f]])
    return sp.csr_matrix((vals, (rows, cols)), shape=(m.n_cells, m.n_cells))


@pytest.mark.parametrize("masked", [True, False])
def test_shifted_assembly_matches_direct(masked):
    import torch

    import paper_1810_08572_amd as ppe

    m = box_mesh((14, 12, 10), jitter=0.1, seed=3)
    c = face_coeff(m, 2400.0)
    fl = fl_planar_front(m.cell_centre, seed=2) if masked else np.ones(m.n_cells)
    act = fl > 0
    rng = np.random.default_rng(5)
    shift = (0.5 + rng.random(m.n_cells)) * 4.0 * c.max()
    b = rng.normal(size=m.n_cells)
    A = (sp.diags(shift) + _lap(m, c, act)).tocsr()
    idx = np.nonzero(act)[0]
    ref = np.zeros(m.n_cells)
    ref[idx] = spla.spsolve(A[idx][:, idx].tocsc(), b[idx])
    s = ppe.Solver(rtol=1e-12)
    s.set_mesh(m.n_cells, to_dev(m.owner, torch.int32), to_dev(m.neigh, torch.int32))
    s.assemble_shifted(to_dev(c, torch.float64), to_dev(shift, torch.float64),
                       to_dev(fl, torch.float64) if masked else None)
    r = s.solve(to_dev(b, torch.float64))
    x = r.p.cpu().numpy()
    assert r.stats["n_components"] == 0
    assert r.stats["n_active"] == act.sum()
    assert np.all(x[~act] == 0)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    res = np.linalg.norm(A[idx][:, idx] @ x[idx] - b[idx]) / np.linalg.norm(b[idx])
    assert res <= 1e-12
    # a shifted system has no pins: the pressure-only calls refuse it
    with pytest.raises(ppe.PpeError):
        s.project(to_dev(c, torch.float64), to_dev(np.zeros((m.n_cells, 3)), torch.float64),
                  2400.0, 1e-3)


def _flow(m, krylov="deferred"):
    import torch

    import paper_1810_08572_amd as ppe

    fw = ppe.Flow(krylov=krylov)
    fw.set_mesh(to_dev(m.owner, torch.int32), to_dev(m.neigh, torch.int32),
                to_dev(m.nodes, torch.float64), to_dev(m.extra["face_nodes"], torch.int32),
                to_dev(m.extra["cell_nodes"], torch.int32), to_dev(m.cell_centre, torch.float64),
                to_dev(m.face_area, torch.float64), to_dev(m.face_centre, torch.float64),
                to_dev(m.cell_volume, torch.float64))
    return fw


def _cases():
    # a melt in the solidus band against walls just below it: the wall layers
    # release their latent heat and solidify step by step (0 -> 37 -> 86 ->
    # 167 of 720 cells), so the mask changes between the steps
    m = box_mesh((10, 9, 8), lengths=(1e-2, 9e-3, 8e-3), jitter=0.1, seed=1)
    T0 = 849.0 + 0.3 * np.sin(500.0 * m.cell_centre[:, 1])
    yield "solidifying_band", m, al_si_alloy(T_wall=840.0), T0, 0.02, 4
    # sheared cells (cross terms everywhere), insulated walls, a ramp from
    # solid through the band into the Scheil range: solid cells re-melt
    m = box_mesh((9, 8, 8), lengths=(1e-2, 1e-2, 1e-2), jitter=0.0, mode=None, affine=SHEAR)
    T0 = 853.0 + 1500.0 * (m.cell_centre[:, 0] - 5e-3)
    yield "sheared_remelting", m, al_si_alloy(T_wall=None), T0, 2e-3, 3
    # the paper's die casting (melt 1000 K, walls 500 K) after a boundary
    # layer has formed, on several reduction tiles with a ragged tail
    m = box_mesh((23, 19, 13), lengths=(2e-2, 1.6e-2, 1.1e-2), jitter=0.12, seed=8)
    yield "die_casting_5681", m, al_si_alloy(), t_wall_layer(m, 500.0, 1000.0, 4e-3), 1e-3, 2
    # a uniform melt at 950 K against walls at 600 K at the 64^3 cavity's
    # spacing (10 mm / 64) and time step (1e-3 s): alpha dt / h^2 = 2.8, so
    # the wall cells cross the whole mushy range in one step and the Picard
    # passes must not jump over the kinks of Eq. 21
    h = 1e-2 / 64
    m = box_mesh((10, 9, 8), lengths=(10 * h, 9 * h, 8 * h), jitter=0.1, seed=2)
    yield "cavity_dt_1e-3", m, al_alloy(), np.full(m.n_cells, 950.0), 1e-3, 3


CASES = list(_cases())


@pytest.mark.parametrize("krylov", ["deferred", "bicgstab"])
@pytest.mark.parametrize("name,m,props,T0,dt,steps", CASES, ids=[c[0] for c in CASES])
def test_steps_match_oracle(name, m, props, T0, dt, steps, krylov):
    import torch

    geo = flow.Geometry(m)
    a = flow.Props.of(props)
    rng = np.random.default_rng(3)
    st = flow.initial_state(m, a, T0=T0, u0=2e-3 * rng.normal(size=(m.n_cells, 3)))
    fw = _flow(m, krylov)
    gs = fw.new_state(to_dev(st.T, torch.float64), to_dev(st.fs, torch.float64),
                      to_dev(st.u, torch.float64))
    for k in range(steps):
        print(f"{name}: step {k}", flush=True)
        st, info = flow.step(geo, a, st, dt)
        status, stats = fw.step(props, gs, dt)
        assert info.picard > 0
        assert stats["picard"] == info.picard, (stats["picard"], info.picard)
        T, fs = gs.T.cpu().numpy(), gs.fs.cpu().numpy()
        u, p = gs.u.cpu().numpy(), gs.p.cpu().numpy()
        F = gs.flux.cpu().numpy()[: m.n_faces]
        cu, cT = gs.conv_u.cpu().numpy(), gs.conv_T.cpu().numpy()
        # the convection terms are sums of +-F_f phi_f over a cell's (at most
        # six) faces that nearly cancel: their error scale is that of the terms
        Fm = np.abs(st.F).max()
        err = {
            "T": np.abs(T - st.T).max() / np.abs(st.T).max(),
            "fs": np.abs(fs - st.fs).max(),
            "p": np.linalg.norm(p - st.p) / np.linalg.norm(st.p),
            "u": np.abs(u - st.u).max() / np.abs(st.u).max(),
            "F": np.abs(F - st.F).max() / Fm,
            "conv_u": np.abs(cu - st.conv_u).max() / (6 * a.rho * Fm * np.abs(st.u).max()),
            "conv_T": np.abs(cT - st.conv_T).max() / (6 * a.rho * a.cp * Fm * np.abs(st.T).max()),
        }
        print(f"  picard {stats['picard']} solid {stats['n_solid']} "
              + " ".join(f"{k} {v:.1e}" for k, v in err.items()), flush=True)
        assert np.array_equal(fs >= 1, st.fs >= 1), k
        assert stats["n_solid"] == int((st.fs >= 1).sum())
        assert err["T"] <= 1e-9 and err["fs"] <= 1e-7
        assert err["p"] <= 1e-8 and err["u"] <= 1e-8 and err["F"] <= 1e-8
        assert err["conv_u"] <= 1e-8 and err["conv_T"] <= 1e-8


def test_invariants_at_64cube_insulated():
    import torch

    props = al_si_alloy(T_wall=None)
    a = flow.Props.of(props)
    m = box_mesh((64, 64, 64), lengths=(1e-2, 1e-2, 1e-2), jitter=0.1, seed=0)
    T0 = 858.0 + 3000.0 * (m.cell_centre[:, 0] - 5e-3) + 5.0 * np.sin(900.0 * m.cell_centre[:, 2])
    fs0 = flow.solid_fraction(T0, a)
    rng = np.random.default_rng(0)
    u0 = 1e-3 * rng.normal(size=(m.n_cells, 3))
    u0[fs0 >= 1] = 0.0
    fw = _flow(m)
    gs = fw.new_state(to_dev(T0, torch.float64), to_dev(fs0, torch.float64),
                      to_dev(u0, torch.float64))
    V = m.cell_volume
    H = lambda T, fs: float(np.sum(V * (a.rho * a.cp * T - a.rho * a.Lf * fs)))
    H0 = H(T0, fs0)
    scale = float(np.sum(V * a.rho * a.cp * np.abs(T0)))
    inner = np.nonzero(m.neigh >= 0)[0]
    solid_prev = fs0 >= 1
    for k in range(3):
        print(f"64^3 insulated: step {k}", flush=True)
        status, stats = fw.step(props, gs, 5e-6)
        T, fs = gs.T.cpu().numpy(), gs.fs.cpu().numpy()
        u, F = gs.u.cpu().numpy(), gs.flux.cpu().numpy()[: m.n_faces]
        assert 0 < stats["picard"] <= 10
        # the energy solve's residual (1e-12 of its right-hand side) bounds the drift
        assert abs(H(T, fs) - H0) <= 1e-10 * scale, (H(T, fs) - H0) / scale
        solid = fs >= 1
        assert np.all(u[solid] == 0)
        closed = solid[m.owner[inner]] | solid[m.neigh[inner]]
        assert np.all(F[inner[closed]] == 0) and np.all(F[m.neigh < 0] == 0)
        # balanced on fluid cells, except next to cells that solidified in
        # this step (their faces were closed after the projection)
        div = pj.divergence(m, F, m.neigh >= 0)
        new = solid & ~solid_prev
        near = np.zeros(m.n_cells, dtype=bool)
        fn = inner[new[m.owner[inner]] | new[m.neigh[inner]]]
        near[m.owner[fn]] = True
        near[m.neigh[fn]] = True
        ok = ~solid & ~near
        assert ok.sum() > m.n_cells // 4
        assert np.abs(div[ok]).max() <= 1e-8 * np.abs(F).max()
        solid_prev = solid
        print(f"  picard {stats['picard']} fluid {stats['n_fluid']} ms {stats['ms']:.1f}", flush=True)


def test_solid_fraction_matches_oracle():
    import torch

    props = al_si_alloy()
    a = flow.Props.of(props)
    fw = _flow(box_mesh((3, 3, 2), jitter=0.0, mode=None))
    kinks = [a.T_liq, a.T_sol - a.T_eps, a.T_sol + a.T_eps, a.T_sol]
    T = np.concatenate([np.linspace(800.0, 900.0, 4099), kinks,
                        np.nextafter(kinks, np.inf), np.nextafter(kinks, -np.inf)])
    fs = fw.solid_fraction(props, to_dev(T, torch.float64)).cpu().numpy()
    ref = flow.solid_fraction(T, a)
    assert np.array_equal(fs == 1.0, ref == 1.0) and np.array_equal(fs == 0.0, ref == 0.0)
    assert np.abs(fs - ref).max() <= 4e-16


def test_refresh_shift_solves_the_new_system():
    import torch

    import paper_1810_08572_amd as ppe

    m = box_mesh((24, 20, 16), jitter=0.1, seed=4)
    c = face_coeff(m, 2400.0)
    rng = np.random.default_rng(8)
    # weak shifts: a multi-level hierarchy, kept by the refresh
    s1 = (0.5 + rng.random(m.n_cells)) * 0.05 * c.max()
    s2 = s1 * (1.0 + 3.0 * rng.random(m.n_cells))
    b = rng.normal(size=m.n_cells)
    A2 = (sp.diags(s2) + _lap(m, c, np.ones(m.n_cells, dtype=bool))).tocsc()
    ref = spla.spsolve(A2, b)
    s = ppe.Solver(rtol=1e-12)
    s.set_mesh(m.n_cells, to_dev(m.owner, torch.int32), to_dev(m.neigh, torch.int32))
    s.assemble_shifted(to_dev(c, torch.float64), to_dev(s1, torch.float64))
    levels = s.stats()["levels"]
    assert levels >= 2
    s.refresh_shift(to_dev(c, torch.float64), to_dev(s2, torch.float64))
    r = s.solve(to_dev(b, torch.float64))
    x = r.p.cpu().numpy()
    assert s.stats()["levels"] == levels
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    fresh = ppe.Solver(rtol=1e-12)
    fresh.set_mesh(m.n_cells, to_dev(m.owner, torch.int32), to_dev(m.neigh, torch.int32))
    fresh.assemble_shifted(to_dev(c, torch.float64), to_dev(s2, torch.float64))
    rf = fresh.solve(to_dev(b, torch.float64))
    print(f"refresh: {r.stats['iterations']} iterations, fresh: {rf.stats['iterations']}")
    assert r.stats["iterations"] <= 2 * rf.stats["iterations"] + 2
    # errors: a bad shift, and a pressure system
    bad = s2.copy()
    bad[5] = -1.0
    with pytest.raises(ppe.PpeError) as e:
        s.refresh_shift(to_dev(c, torch.float64), to_dev(bad, torch.float64))
    assert e.value.status == ppe.PPE_ERR_ARG
    with pytest.raises(ppe.PpeError) as e:
        s.solve(to_dev(b, torch.float64))
    assert e.value.status == ppe.PPE_ERR_STATE
    s.assemble(to_dev(c, torch.float64), to_dev(np.ones(m.n_cells), torch.float64))
    with pytest.raises(ppe.PpeError) as e:
        s.refresh_shift(to_dev(c, torch.float64), to_dev(s2, torch.float64))
    assert e.value.status == ppe.PPE_ERR_STATE


def test_flow_edge_cases_and_errors():
    """All cells solid: nothing moves, p = 0, fluxes 0, the energy step still
    conducts (walls at 500 K cool the block).  A uniform melt at T_ref at
    rest with insulated walls is a fixed point.  Argument and state errors
    are reported without touching the state."""
    import torch

    import paper_1810_08572_amd as ppe

    m = box_mesh((6, 5, 4), lengths=(6e-3, 5e-3, 4e-3), jitter=0.1, seed=2)
    props = al_si_alloy()
    a = flow.Props.of(props)
    fw = ppe.Flow()
    # a step before the mesh
    gs = ppe.FlowState(*(to_dev(np.zeros(sh), torch.float64) for sh in
                         ((m.n_cells, 3), m.n_cells, m.n_cells, m.n_faces, m.n_cells,
                          (m.n_cells, 3), m.n_cells)))
    fw.n_cells, fw.n_faces = m.n_cells, m.n_faces
    with pytest.raises(ppe.PpeError) as e:
        fw.step(props, gs, 1e-3)
    assert e.value.status == ppe.PPE_ERR_STATE
    fw = _flow(m)
    # all solid
    T0 = np.full(m.n_cells, 700.0)
    gs = fw.new_state(to_dev(T0, torch.float64), props=props)
    assert float(gs.fs.min()) == 1.0
    geo = flow.Geometry(m)
    st = flow.initial_state(m, a, T0=T0)
    for _ in range(2):
        status, stats = fw.step(props, gs, 1e-3)
        st, info = flow.step(geo, a, st, 1e-3)
        assert stats["n_fluid"] == 0 and stats["n_solid"] == m.n_cells
        assert float(gs.u.abs().max()) == 0 and float(gs.p.abs().max()) == 0
        assert float(gs.flux.abs().max()) == 0
        T = gs.T.cpu().numpy()
        assert np.abs(T - st.T).max() <= 1e-9 * np.abs(st.T).max()
    assert T.max() < 700.0
    # a uniform melt at T_ref, at rest, insulated: nothing changes
    ins = al_si_alloy(T_wall=None)
    gs = fw.new_state(to_dev(np.full(m.n_cells, ins["T_ref"]), torch.float64), props=ins)
    status, stats = fw.step(ins, gs, 1e-3)
    assert float(gs.u.abs().max()) == 0 and float(gs.flux.abs().max()) == 0
    assert np.all(gs.T.cpu().numpy() == ins["T_ref"]) and float(gs.fs.abs().max()) == 0
    assert stats["picard"] == 1
    # bad arguments leave the state alone
    before = gs.T.clone()
    for bad in (dict(mu=0.0), dict(k=-1.0), dict(k_p=1.0), dict(T_eps=0.0)):
        with pytest.raises(ppe.PpeError) as e:
            fw.step(dict(ins, **bad), gs, 1e-3)
        assert e.value.status == ppe.PPE_ERR_ARG
    for kw in (dict(relax=0.0), dict(relax=1.5), dict(max_picard=0)):
        with pytest.raises(ppe.PpeError) as e:
            fw.step(ins, gs, 1e-3, **kw)
        assert e.value.status == ppe.PPE_ERR_ARG
    with pytest.raises(ppe.PpeError) as e:
        fw.step(ins, gs, 0.0)
    assert e.value.status == ppe.PPE_ERR_ARG
    assert torch.equal(gs.T, before)


def test_uncertainty_over_steps_matches_oracle():
    """The die-casting uncertainty study on a small block: 27 tensor samples
    of (C0, T_init, T_wall), two steps each; the per-sample outputs (mean
    temperature, solid volume fraction, peak speed) and the degree-2
    expansion fitted to them match the oracle's (flow.step + uq.fit)."""
    import torch

    import paper_1810_08572_amd as ppe
    from oracle import uq

    m = box_mesh((6, 5, 5), lengths=(6e-3, 5e-3, 5e-3), jitter=0.1, seed=6)
    geo = flow.Geometry(m)
    kinds = ["normal"] * 3
    q = ppe.PolynomialChaos(kinds, 2)
    X, _ = q.nodes("tensor", 3)
    fw = _flow(m)
    V = m.cell_volume
    Yg = torch.empty((X.shape[0], 3), dtype=torch.float64, device="cuda")
    Yr = np.empty((X.shape[0], 3))
    for k, x in enumerate(X):
        props = al_si_alloy(si_wt=10.0 + 0.2 * x[0], T_wall=500.0 + 5.0 * x[2])
        T0 = t_wall_layer(m, props["T_wall"], 1000.0 + 10.0 * x[1], 1.5e-3)
        a = flow.Props.of(props)
        st = flow.initial_state(m, a, T0=T0)
        gs = fw.new_state(to_dev(T0, torch.float64), props=props)
        for _ in range(2):
            st, _ = flow.step(geo, a, st, 2e-4)
        fw.run(props, gs, 2e-4, 2)
        Yr[k] = [np.sum(V * st.T) / V.sum(), np.sum(V * st.fs) / V.sum(),
                 np.linalg.norm(st.u, axis=1).max()]
        Vd = to_dev(V, torch.float64)
        Yg[k, 0] = (Vd * gs.T).sum() / Vd.sum()
        Yg[k, 1] = (Vd * gs.fs).sum() / Vd.sum()
        Yg[k, 2] = gs.u.norm(dim=1).max()
    y = Yg.cpu().numpy()
    assert np.abs(y[:, 0] - Yr[:, 0]).max() <= 1e-9 * np.abs(Yr[:, 0]).max()
    assert np.abs(y[:, 1] - Yr[:, 1]).max() <= 1e-8
    assert np.abs(y[:, 2] - Yr[:, 2]).max() <= 1e-8 * np.abs(Yr[:, 2]).max()
    W = q.fit(X, Yg).cpu().numpy()
    Wr = uq.fit(uq.vandermonde(kinds, uq.total_degree_indices(3, 2), X), Yr)
    for j in range(3):
        assert np.abs(W[:, j] - Wr[:, j]).max() <= 1e-7 * np.abs(Wr[:, j]).max(), j
    # the inputs matter: the melt temperature drives the mean temperature
    mean, var, first, total = (v.cpu().numpy() for v in q.stats(Yg.new_tensor(W)))
    assert first[1, 0] > 0.5
