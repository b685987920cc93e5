"""Pins of the oracle's smoothed-aggregation hierarchy and PCG.

Nothing in the paper fixes these numbers (it names no AMG variant or
parameter), so every pin is a property of the mathematics: published hash
test vectors, brute-force greedy MIS-2 on small graphs, structural rules of
aggregation, orthonormality and near-null-space identities of the
prolongators, closed-form Chebyshev error polynomials, symmetry of the
V-cycle, and agreement of PCG with dense direct solves."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

from oracle import amg, assembly, direct, hash as ohash, pcg
from synth import box_mesh, face_coeff, fl_linear_x, fl_planar_front, rhs_uniform


def _murmur3_32(data: bytes, seed: int) -> int:
    """Full MurmurHash3_x86_32 around the oracle's finaliser."""
    rotl = lambda x, r: ((x << r) | (x >> (32 - r))) & 0xFFFFFFFF
    c1, c2 = 0xCC9E2D51, 0x1B873593
    h = seed & 0xFFFFFFFF
    n = len(data)
    for i in range(0, n - n % 4, 4):
        k = int.from_bytes(data[i:i + 4], "little")
        k = rotl((k * c1) & 0xFFFFFFFF, 15) * c2 & 0xFFFFFFFF
        h = (rotl(h ^ k, 13) * 5 + 0xE6546B64) & 0xFFFFFFFF
    tail = data[n - n % 4:]
    if tail:
        k = int.from_bytes(tail, "little")
        h ^= rotl((k * c1) & 0xFFFFFFFF, 15) * c2 & 0xFFFFFFFF
    return int(ohash.fmix32(h ^ n))


@pytest.mark.parametrize("data,seed,expect", [
    (b"", 0, 0), (b"", 1, 0x514E28B7), (b"", 0xFFFFFFFF, 0x81F16F39),
    (b"\0\0\0\0", 0, 0x2362F9DE), (b"aaaa", 0x9747B28C, 0x5A97808A),
    (b"Hello, world!", 1234, 0xFAF6CDB3),
    (b"The quick brown fox jumps over the lazy dog", 0, 0x2E4FF723),
])
def test_fmix32_published_vectors(data, seed, expect):
    assert _murmur3_32(data, seed) == expect


def _c1_system(jitter=0.1):
    m = box_mesh((16, 16, 16), jitter=jitter, seed=0)
    fl = fl_linear_x(m.cell_centre)
    c = face_coeff(m, 2400.0)
    return m, fl, c, assembly.masked_system(m.n_cells, m.owner, m.neigh, c, fl)


def _greedy_mis2(S, level):
    """Sequential greedy distance-2 MIS in descending (priority, -index)
    order, by breadth-first distances."""
    n = S.shape[0]
    D = shortest_path(S != 0, unweighted=True, directed=False)
    deg = np.diff(S.indptr)
    h = ohash.priority(n, level).astype(np.int64)
    order = sorted(range(n), key=lambda i: (-h[i], i))
    taken = []
    for i in order:
        if deg[i] == 0:
            continue
        if all(D[i, j] > 2 for j in taken):
            taken.append(i)
    out = np.zeros(n, dtype=np.int64)
    out[taken] = amg.IN
    return out


@pytest.mark.parametrize("seed", range(8))
def test_mis2_equals_greedy_on_random_graphs(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    M = sp.random(n, n, density=0.12, random_state=seed, format="csr")
    M = ((M + M.T) > 0).astype(float)
    M.setdiag(0)
    M.eliminate_zeros()
    S = (-M).tocsr()
    state, _ = amg.mis2(S, level=seed % 3)
    assert np.array_equal(state == amg.IN, _greedy_mis2(S, seed % 3) == amg.IN)


def test_aggregation_rules_on_c1():
    _, _, _, sy = _c1_system()
    A = sy.A
    S = amg.strength(A, 0.08)
    assert S.nnz == A.nnz - A.shape[0] - 0  # every fine coupling is strong at theta = 0.08
    state, _ = amg.mis2(S, 0)
    agg, n_agg = amg.aggregate(S, state)
    roots = np.nonzero(state == amg.IN)[0]
    D = shortest_path(S != 0, unweighted=True, directed=False, indices=roots)
    Dr = D[:, roots]
    np.fill_diagonal(Dr, np.inf)
    assert Dr.min() >= 3                                  # distance-2 independent
    deg = np.diff(S.indptr)
    assert np.all(D.min(axis=0)[deg > 0] <= 2)            # maximal
    assert np.all(agg[deg == 0] == -1) and np.all(agg[deg > 0] >= 0)
    assert np.array_equal(agg[roots], np.arange(n_agg))
    for J in range(n_agg):                               # connected aggregates
        members = np.nonzero(agg == J)[0]
        sub = S[members][:, members]
        assert sp.csgraph.connected_components(sub, directed=False)[0] == 1
        # every strong neighbour of the root belongs to it
        r = roots[J]
        assert np.all(agg[S[r].indices] == J)
    assert np.all(agg[sy.cid[sy.pins]] == -1)             # pins are isolated


def test_tentative_orthonormal_and_near_null():
    """P_tent has orthonormal columns; on the unpinned operator the coarse
    near-null vector s = sqrt(|agg|) satisfies A_c s = 0, since
    P s = (I - omega D^-1 L) 1 = 1 and L 1 = 0."""
    _, _, _, sy = _c1_system()
    L = sy.L
    S = amg.strength(L, 0.08)
    state, _ = amg.mis2(S, 0)
    agg, n_agg = amg.aggregate(S, state)
    Pt, Bc = amg.tentative(agg, n_agg, np.ones(L.shape[0]))
    G = (Pt.T @ Pt).toarray()
    assert np.abs(G - np.eye(n_agg)).max() <= 1e-14
    assert np.allclose(Bc, np.sqrt(np.bincount(agg, minlength=n_agg)), rtol=1e-15)
    P = amg.smooth_prolongator(L, Pt, amg.gershgorin(L))
    assert np.abs(P @ Bc - 1.0).max() <= 1e-13
    Ac = amg.galerkin(L, P)
    scale = np.abs(Ac).max()
    assert np.abs(Ac @ Bc).max() <= 1e-12 * scale * Bc.max()
    assert abs(Ac - Ac.T).max() <= 1e-14 * scale


def test_power_estimate_against_eigenvalues():
    _, _, _, sy = _c1_system()
    H = amg.build_hierarchy(sy.A)
    for lvl, lev in enumerate(H.levels):
        d = lev.diag
        ev = np.linalg.eigvalsh(lev.A.toarray() / np.sqrt(np.outer(d, d)))
        if lvl == 0:
            assert ev.max() <= lev.rho * (1 + 1e-12)            # Gershgorin is a bound
        est = amg.power_estimate(lev.A, lvl)
        assert 0.8 * ev.max() <= est <= ev.max() * (1 + 1e-12)  # Rayleigh-type lower estimate


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_chebyshev_error_polynomial(degree):
    """For b = 0 the smoother maps an error e to E e with
    E = T_k((theta - D^-1 A) / delta) / T_k(theta / delta)."""
    rng = np.random.default_rng(degree)
    n = 30
    Q = rng.normal(size=(n, n))
    A = Q @ Q.T + n * np.eye(n)
    d = np.diag(A).copy()
    Ah = A / np.sqrt(np.outer(d, d))
    lam, V = np.linalg.eigh(Ah)
    lmax, lmin = lam.max() * 1.05, lam.max() / 30.0
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    T = np.polynomial.chebyshev.Chebyshev.basis(degree)
    g = T((theta - lam) / delta) / T(theta / delta)
    E = np.diag(1 / np.sqrt(d)) @ V @ np.diag(g) @ V.T @ np.diag(np.sqrt(d))
    e = rng.normal(size=n)
    out = amg.chebyshev(sp.csr_matrix(A), d, np.zeros(n), e, lmax, lmin, degree)
    assert np.allclose(out, E @ e, rtol=1e-12, atol=1e-12 * np.abs(e).max())


def test_vcycle_symmetric_positive():
    _, _, _, sy = _c1_system()
    H = amg.build_hierarchy(sy.A, coarse_max=128)  # three levels: a recursive V-cycle
    assert len(H.levels) >= 3
    rng = np.random.default_rng(0)
    r1, r2 = rng.normal(size=(2, sy.n_active))
    a = amg.vcycle(H, r1) @ r2
    b = r1 @ amg.vcycle(H, r2)
    assert abs(a - b) <= 1e-12 * abs(a)
    assert amg.vcycle(H, r1) @ r1 > 0


@pytest.mark.parametrize("x0kind", ["zero", "random", "exact"])
def test_pcg_matches_dense(x0kind):
    m, fl, c, sy = _c1_system()
    b = rhs_uniform(m.n_cells, seed=1, center_mask=fl > 0)
    p_ref = direct.solve_dense(sy, b)
    bp = assembly.pinned_rhs(sy, b)
    H = amg.build_hierarchy(sy.A)
    x0 = {"zero": None, "random": np.random.default_rng(4).normal(size=sy.n_active) * 1e3,
          "exact": p_ref[sy.perm]}[x0kind]
    res = pcg.pcg(sy.A, bp, M=lambda r: amg.vcycle(H, r), x0=x0, rtol=1e-10)
    assert res.status == pcg.OK
    if x0kind == "exact":
        assert res.iterations == 0
    p = assembly.scatter(sy, res.x)
    assert assembly.relative_residual(sy, b, p) <= 1e-10
    assert np.linalg.norm(p - p_ref) <= 1e-9 * np.linalg.norm(p_ref)


def test_pcg_energy_error_monotone():
    m, fl, c, sy = _c1_system()
    b = rhs_uniform(m.n_cells, seed=1, center_mask=fl > 0)
    bp = assembly.pinned_rhs(sy, b)
    xs = direct.solve_dense(sy, b)[sy.perm]
    H = amg.build_hierarchy(sy.A)
    errs = []
    for k in range(1, 12):
        x = pcg.pcg(sy.A, bp, M=lambda r: amg.vcycle(H, r), rtol=0.0, max_iter=k).x
        e = x - xs
        errs.append(e @ (sy.A @ e))
    assert all(b2 <= b1 * (1 + 1e-9) for b1, b2 in zip(errs, errs[1:]))


def test_pcg_zero_rhs_and_flexible():
    m, fl, c, sy = _c1_system()
    res = pcg.pcg(sy.A, np.zeros(sy.n_active))
    assert res.iterations == 0 and not res.x.any()
    b = rhs_uniform(m.n_cells, seed=1, center_mask=fl > 0)
    bp = assembly.pinned_rhs(sy, b)
    H = amg.build_hierarchy(sy.A)
    r1 = pcg.pcg(sy.A, bp, M=lambda r: amg.vcycle(H, r), rtol=1e-10)
    r2 = pcg.pcg(sy.A, bp, M=lambda r: amg.vcycle(H, r), rtol=1e-10, flexible=True)
    assert abs(r1.iterations - r2.iterations) <= 1
    assert np.linalg.norm(r1.x - r2.x) <= 1e-9 * np.linalg.norm(r1.x)


def test_pockets_never_mix_in_hierarchy():
    """Two liquid pockets separated by a solid slab: no aggregate spans both
    and every coarse operator stays block diagonal (section 2.5: pockets
    decouple numerically; here no coarse diagonal can vanish)."""
    m = box_mesh((12, 12, 12), jitter=0.1, seed=2)
    x = m.cell_centre[:, 0]
    fl = np.where(np.abs(x - 0.5) < 0.1, 0.0, 1.0)
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, face_coeff(m, 2400.0), fl)
    assert len(sy.pins) == 2
    H = amg.build_hierarchy(sy.A, coarse_max=16)
    side = (x[sy.perm] > 0.5).astype(int)
    for lev in H.levels[:-1]:
        ok = lev.agg >= 0
        assert np.all(np.bincount(lev.agg[ok], weights=side[ok]) % np.bincount(lev.agg[ok]) == 0)
        A = lev.P.T @ sp.diags(side.astype(float)) @ lev.P
        side = (np.asarray(A.sum(axis=1)).ravel() > 0).astype(int)
        assert np.all(lev.A.diagonal() > 0)
    assert np.all(H.levels[-1].A.diagonal() > 0)


@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_l1_jacobi_on_a_ring(sweeps):
    """On the periodic chain tridiag(-1, 2, -1) every row's l1 norm is 4, so
    a sweep multiplies the Fourier mode cos(k theta j) of the error by
    1 - (2 - 2 cos theta) / 4 = (1 + cos theta) / 2 (textbook damped Jacobi
    with weight 1/2)."""
    n = 24
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="lil")
    A[0, n - 1] = A[n - 1, 0] = -1.0
    A = A.tocsr()
    dl1 = amg.l1_diagonal(A)
    assert np.array_equal(dl1, 4 * np.ones(n))
    j = np.arange(n)
    for k in (1, 5, 12):
        th = 2 * np.pi * k / n
        e = np.cos(th * j)
        out = amg.l1_jacobi(A, dl1, np.zeros(n), e, sweeps)   # b = 0: out is the new error
        assert np.allclose(out, ((1 + np.cos(th)) / 2) ** sweeps * e, rtol=0, atol=1e-13)


def test_l1_jacobi_contracts_the_energy_norm():
    """For SPD A, D_l1 - A is diagonally dominant, so l1-Jacobi reduces the
    A-norm of the error of every start (here the C1 system)."""
    _, _, _, sy = _c1_system()
    A = sy.A.tocsr()
    dl1 = amg.l1_diagonal(A)
    assert np.all(dl1 >= A.diagonal())
    rng = np.random.default_rng(3)
    for _ in range(5):
        e = rng.normal(size=A.shape[0])
        e1 = amg.l1_jacobi(A, dl1, np.zeros_like(e), e, 1)
        assert e1 @ (A @ e1) < e @ (A @ e)


def test_l1_jacobi_vcycle_symmetric_and_pcg_matches_dense():
    _, _, _, sy = _c1_system()
    H = amg.build_hierarchy(sy.A, smoother="l1jacobi")
    rng = np.random.default_rng(0)
    r1, r2 = rng.normal(size=(2, sy.n_active))
    a, b = amg.vcycle(H, r1) @ r2, r1 @ amg.vcycle(H, r2)
    assert abs(a - b) <= 1e-12 * abs(a)
    assert amg.vcycle(H, r1) @ r1 > 0
    b0 = rhs_uniform(sy.A.shape[0], seed=1)
    res = pcg.pcg(sy.A, b0, M=lambda r: amg.vcycle(H, r), rtol=1e-12)
    ref = np.linalg.solve(sy.A.toarray(), b0)
    assert res.status == pcg.OK
    assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref)


def _front_system(x0):
    m = box_mesh((14, 12, 10), jitter=0.1, seed=5)
    fl = np.clip((m.cell_centre[:, 0] - x0) / 0.1, 0.0, 1.0)
    c = face_coeff(m, 2400.0)
    return m, assembly.masked_system(m.n_cells, m.owner, m.neigh, c, fl)


def test_reused_coarse_levels_give_an_spd_preconditioner():
    """The front moves one layer and leaves dangling mushy cells: the reused
    hierarchy's V-cycle is symmetric and positive on the new system, its
    finest prolongator holds exactly the base rows of the kept cells (empty
    for pins), and PCG with it reaches the dense solution."""
    m, sy0 = _front_system(0.18)
    H0 = amg.build_hierarchy(sy0.A)
    _, sy = _front_system(0.26)
    assert sy.n_active < sy0.n_active
    base_of_cell = np.full(m.n_cells, -1)
    base_of_cell[sy0.perm] = np.arange(sy0.n_active)
    base_row = base_of_cell[sy.perm]
    pinned = np.zeros(sy.n_active, dtype=bool)
    pinned[sy.pinned] = True
    G = amg.reuse_coarse_levels(H0, sy.A, base_row, pinned)
    assert G.levels[1] is H0.levels[1]
    P, P0 = G.levels[0].P, H0.levels[0].P.tocsr()
    for i in range(sy.n_active):
        row = P.getrow(i)
        if pinned[i]:
            assert row.nnz == 0
        else:
            ref = P0.getrow(base_row[i])
            assert np.array_equal(row.indices, ref.indices) and np.array_equal(row.data, ref.data)
    assert (G.levels[0].R != P.T).nnz == 0
    rng = np.random.default_rng(4)
    r1, r2 = rng.normal(size=(2, sy.n_active))
    a, b = amg.vcycle(G, r1) @ r2, r1 @ amg.vcycle(G, r2)
    assert abs(a - b) <= 1e-12 * abs(a)
    assert amg.vcycle(G, r1) @ r1 > 0
    b0 = assembly.pinned_rhs(sy, rhs_uniform(m.n_cells, seed=2, center_mask=None))
    res = pcg.pcg(sy.A, b0, M=lambda r: amg.vcycle(G, r), rtol=1e-12)
    ref = np.linalg.solve(sy.A.toarray(), b0)
    assert res.status == pcg.OK
    assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref)
