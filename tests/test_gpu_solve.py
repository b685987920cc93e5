"""End-to-end GPU parity of the pressure solve: relative residual <= 1e-10
(recomputed in FP64 by the oracle from the GPU's pressure) and relative L2
error <= 1e-9 against an exact reference (dense Cholesky / SuperLU)."""
import numpy as np
import pytest

from oracle import amg, assembly, direct, pcg
from synth import box_mesh, face_coeff
from tests.gpu_util import case, gpu_solver, to_dev

pytestmark = pytest.mark.gpu


def _solve(m, f, c, b, x0=None, **opts):
    import torch

    s = gpu_solver(m, f, c, **opts)
    res = s.solve(to_dev(b, torch.float64),
                  x0=None if x0 is None else to_dev(x0, torch.float64))
    return s, res


@pytest.mark.parametrize("x0kind", ["zero", "random", "exact"])
def test_c1_against_dense(x0kind):
    m, f, c, b = case()
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    pref = direct.solve_dense(sy, b)
    x0 = {"zero": None, "random": np.random.default_rng(5).normal(size=m.n_cells) * 1e3,
          "exact": pref}[x0kind]
    s, res = _solve(m, f, c, b, x0)
    p = res.p.cpu().numpy()
    assert res.status == 0
    assert assembly.relative_residual(sy, b, p) <= 1e-10
    assert abs(res.stats["rel_residual"] - assembly.relative_residual(sy, b, p)) <= 1e-11
    assert np.linalg.norm(p - pref) <= 1e-9 * np.linalg.norm(pref)
    assert np.all(p[~sy.active] == 0) and np.all(p[sy.pins] == 0)
    if x0kind == "zero":
        H = amg.build_hierarchy(sy.A)
        ref = pcg.pcg(sy.A, assembly.pinned_rhs(sy, b), M=lambda r: amg.vcycle(H, r), rtol=1e-10)
        assert abs(res.stats["iterations"] - ref.iterations) <= 1


@pytest.mark.parametrize("shape,fl,seed", [((32, 32, 32), "front", 2), ((29, 17, 23), "front", 9),
                                           ((24, 24, 24), "ones", 0)])
def test_ragged_against_superlu(shape, fl, seed):
    m, f, c, b = case(shape=shape, fl=fl, fl_seed=seed, seed=seed)
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    pref = direct.solve_sparse(sy, b)
    s, res = _solve(m, f, c, b)
    p = res.p.cpu().numpy()
    assert assembly.relative_residual(sy, b, p) <= 1e-10
    assert np.linalg.norm(p - pref) <= 1e-9 * np.linalg.norm(pref)


def test_pockets_and_uncentred_rhs():
    """Several pockets, b not balanced: each pin absorbs its pocket's
    imbalance; the result is still the unique pinned solution."""
    m = box_mesh((18, 14, 10), jitter=0.1, seed=1)
    x = m.cell_centre
    f = np.where((np.abs(x[:, 0] - 0.5) < 0.08) | (np.abs(x[:, 1] - 0.4) < 0.06), 0.0, 0.7)
    c = face_coeff(m, 2400.0)
    b = np.random.default_rng(2).uniform(-1, 1, m.n_cells)
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    assert len(sy.pins) == 4
    pref = direct.solve_sparse(sy, b)
    s, res = _solve(m, f, c, b)
    p = res.p.cpu().numpy()
    assert assembly.relative_residual(sy, b, p) <= 1e-10
    assert np.linalg.norm(p - pref) <= 1e-9 * np.linalg.norm(pref)


def test_not_converged_and_determinism():
    import torch

    import paper_1810_08572_amd as ppe

    m, f, c, b = case(shape=(20, 20, 20), fl="front")
    s = gpu_solver(m, f, c, max_iter=2)
    with pytest.raises(ppe.PpeError) as e:
        s.solve(to_dev(b, torch.float64))
    assert e.value.status == ppe.PPE_NOT_CONVERGED
    r = s.solve(to_dev(b, torch.float64), allow_not_converged=True)
    assert r.status == ppe.PPE_NOT_CONVERGED and r.stats["iterations"] == 2
    s2 = gpu_solver(m, f, c)
    p1 = s2.solve(to_dev(b, torch.float64)).p.cpu().numpy()
    p2 = s2.solve(to_dev(b, torch.float64)).p.cpu().numpy()
    assert np.array_equal(p1, p2)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotuned_solver_meets_bars(precision):
    """With the autotuner choosing lanes per row and fused or split first
    smoothing steps, the pressure still meets both bars; a re-assembly of the
    same system reuses the cached choices and repeats the result bitwise."""
    import torch

    m, f, c, b = case(shape=(32, 32, 32), fl="front", fl_seed=2, seed=2)
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    pref = direct.solve_sparse(sy, b)
    s = gpu_solver(m, f, c, precision=precision, autotune=True)
    res = s.solve(to_dev(b, torch.float64))
    p = res.p.cpu().numpy()
    assert assembly.relative_residual(sy, b, p) <= 1e-10
    assert np.linalg.norm(p - pref) <= 1e-9 * np.linalg.norm(pref)
    s.assemble(to_dev(c, torch.float64), to_dev(f, torch.float64))
    again = s.solve(to_dev(b, torch.float64)).p.cpu().numpy()
    assert np.array_equal(p, again)


def test_every_launch_choice_meets_bars_and_repeats_after_reassembly():
    """Each lane count of each level's smoother, restriction and prolongation
    (fused with the first post-smoothing step and separate), and the split
    first smoothing step, set by hand one at a time: the pressure meets the
    bars, and a re-assembly with the same choice repeats it bitwise (the
    hierarchy never depends on the choices).  Choices outside the allowed
    sets are refused."""
    import torch

    import paper_1810_08572_amd as ppe

    m, f, c, b = case(shape=(24, 24, 24), fl="front", fl_seed=2, seed=2)
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    pref = direct.solve_sparse(sy, b)
    s = gpu_solver(m, f, c)
    bd, cd, fd = to_dev(b, torch.float64), to_dev(c, torch.float64), to_dev(f, torch.float64)
    nlev = s.n_levels()
    variants = []
    for lvl in range(nlev - 1):
        for k in range(3):
            # the smoother takes 4..64 lanes, the transfers 1..64 (a fused
            # prolongation runs 1 and 2 as 4)
            for lpr in (4, 8, 16, 32, 64) if k == 0 else (1, 2, 4, 8, 16, 32, 64):
                if k == 0 and lvl == 0:
                    continue  # the finest level is ELL: no lanes per row
                for fuse_p in ((0, 1) if k == 2 else (1,)):
                    ch = [0, 0, 0, 1, fuse_p]
                    ch[k] = lpr
                    variants.append((lvl, tuple(ch)))
        variants.append((lvl, (0, 0, 0, 0, 1)))
        variants.append((lvl, (0, 0, 0, 0, 0)))
    for bad in ((2, 0, 0, 1, 1), (0, 3, 0, 1, 1), (0, 0, 128, 1, 1), (0, 0, 0, 2, 1),
                (0, 0, 0, 1, 2)):
        with pytest.raises(ppe.PpeError):
            s.set_level_launch(0, bad)
    for lvl, ch in variants:
        outs = []
        for _ in range(2):
            s.assemble(cd, fd)
            s.set_level_launch(lvl, ch)
            assert s.level_launch(lvl) == ch
            outs.append(s.solve(bd).p.cpu().numpy())
        assert assembly.relative_residual(sy, b, outs[0]) <= 1e-10, (lvl, ch)
        assert np.linalg.norm(outs[0] - pref) <= 1e-9 * np.linalg.norm(pref), (lvl, ch)
        assert np.array_equal(outs[0], outs[1]), (lvl, ch)


def test_reuse_of_an_unchanged_system():
    """reuse_unchanged: an assembly whose coefficients and mask equal the
    last one's keeps the system (liquid-fraction values may change); any
    change of the mask or of a coefficient rebuilds.  Every result equals a
    fresh solver's bitwise."""
    import torch

    import paper_1810_08572_amd as ppe

    m, f, c, b = case(shape=(20, 18, 16), fl="front", fl_seed=3, seed=1)
    bd = to_dev(b, torch.float64)

    def fresh(cc, ff):
        return gpu_solver(m, ff, cc).solve(bd).p.cpu().numpy()

    s = gpu_solver(m, f, c, reuse_unchanged=True)
    p0 = s.solve(bd).p.cpu().numpy()
    assert s.stats()["reused_setup"] == 0
    f2 = np.where(f > 0, 0.5 * f + 0.25, 0.0)  # same mask, other values
    s.assemble(to_dev(c, torch.float64), to_dev(f2, torch.float64))
    assert s.stats()["reused_setup"] == 1
    assert np.array_equal(s.solve(bd).p.cpu().numpy(), p0)
    assert np.array_equal(p0, fresh(c, f))
    f3 = f.copy()
    f3[np.nonzero(f > 0)[0][7]] = 0.0  # one more cell removed
    s.assemble(to_dev(c, torch.float64), to_dev(f3, torch.float64))
    assert s.stats()["reused_setup"] == 1
    assert np.array_equal(s.solve(bd).p.cpu().numpy(), fresh(c, f3))
    c4 = c.copy()
    c4[np.nonzero(m.neigh >= 0)[0][11]] *= 1.5
    s.assemble(to_dev(c4, torch.float64), to_dev(f3, torch.float64))
    assert s.stats()["reused_setup"] == 1
    assert np.array_equal(s.solve(bd).p.cpu().numpy(), fresh(c4, f3))
    s.assemble(to_dev(c4, torch.float64), to_dev(f3, torch.float64))
    assert s.stats()["reused_setup"] == 2
    bad = f3.copy()
    bad[0] = 2.0
    with pytest.raises(ppe.PpeError) as e:
        s.assemble(to_dev(c4, torch.float64), to_dev(bad, torch.float64))
    assert e.value.status == ppe.PPE_ERR_ARG


def test_profile_times_every_solve_kernel():
    """With profiling on, each V-cycle and PCG dispatch is timed and booked
    under its kernel instantiation with its algorithmic bytes.  The finest
    level's first post-smoothing step (the ELL step from x = x1 + P e, with
    no previous update to read) runs once per V-cycle and moves the stored
    off-diagonal entries (8-byte value + 4-byte column), the diagonal and
    four vectors (iterate in and out, right-hand side, step update); the
    outer q = A p moves the same entries, the diagonal, p and q; the x, r
    update six vectors and the p update three."""
    import torch

    m, f, c, b = case(shape=(24, 24, 24), fl="front", fl_seed=2, seed=2)
    s = gpu_solver(m, f, c)
    i0 = s.level_info(0)
    n, off = i0["n"], i0["nnz"] - i0["n"]
    s.profile(True)
    res = s.solve(to_dev(b, torch.float64))
    prof = s.profile_read()
    s.profile(False)
    assert res.status == 0
    it = res.stats["iterations"]
    cheb = prof["k_ell<2, double, 6>"]
    assert cheb["launches"] >= it >= 1 and cheb["kernel_ms"] > 0.0
    assert cheb["bytes"] == (12.0 * off + 8.0 * n + 4 * 8.0 * n) * cheb["launches"]
    spmv = prof["k_ell_dot_t<6>"]
    assert spmv["launches"] >= it
    assert spmv["bytes"] == (12.0 * off + 8.0 * n + 2 * 8.0 * n) * spmv["launches"]
    assert prof["k_update_xr_t"]["bytes"] == 48.0 * n * prof["k_update_xr_t"]["launches"]
    assert prof["k_update_p_t"]["bytes"] == 24.0 * n * prof["k_update_p_t"]["launches"]
    assert any(k.startswith("k_csr<") for k in prof)          # coarse levels
    assert "k_dense_gemv" in prof                              # coarsest level
    assert all(v["kernel_ms"] > 0 and v["bytes"] > 0 for v in prof.values())
    # profiling off: the table stays as it was
    s.solve(to_dev(b, torch.float64))
    assert s.profile_read() == prof
