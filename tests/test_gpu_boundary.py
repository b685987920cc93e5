"""The boundary's options beyond the default solve:

- smoother = l1-Jacobi (section 2.5's relaxation, the alternative to the
  Chebyshev smoother): one V-cycle agrees with the oracle's l1-Jacobi
  V-cycle on the same hierarchy to rounding (FP64), and with the oracle's
  V-cycle on the FP32-rounded values (mixed); the solve meets the FP64 bars
  (1e-10 residual recomputed by the oracle, 1e-9 relative L2 against sparse
  LU) with the oracle's iteration count, in both precisions;
- the caller's allocator: a solver whose device memory comes from PyTorch's
  caching allocator gives bitwise the pressure of one that uses hipMalloc,
  hands every block back when it is destroyed, and an allocator that refuses
  a request makes the call fail with PPE_ERR_OOM, after which the solver
  still works once memory is available again."""
import numpy as np
import pytest

from oracle import amg, assembly, direct, pcg
from tests.gpu_util import case, gpu_solver, to_dev

pytestmark = pytest.mark.gpu


def _rounded(H):
    import copy

    G = copy.deepcopy(H)
    q = lambda a: a.astype(np.float32).astype(np.float64)
    for lev in G.levels:
        lev.A, lev.diag, lev.dl1 = q(lev.A), q(lev.diag), q(lev.dl1)
        if lev.P is not None:
            lev.P, lev.R = q(lev.P), q(lev.R)
    return G


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape,fl", [((16, 16, 16), "linear"), ((23, 19, 17), "front")])
def test_l1_jacobi_vcycle_matches_oracle(precision, shape, fl):
    import torch

    m, f, c, _ = case(shape=shape, fl=fl, seed=4)
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    H = amg.build_hierarchy(sy.A, smoother="l1jacobi")
    s = gpu_solver(m, f, c, precision=precision, smoother="l1jacobi")
    assert s.n_levels() == len(H.levels)
    r = np.random.default_rng(5).normal(size=sy.n_active)
    z = s.apply_vcycle(to_dev(r, torch.float64)).cpu().numpy()
    zr = amg.vcycle(H if precision == "fp64" else _rounded(H), r)
    assert np.linalg.norm(z - zr) <= 1e-12 * np.linalg.norm(zr)
    # and it is not the Chebyshev V-cycle
    zc = amg.vcycle(amg.build_hierarchy(sy.A), r)
    assert np.linalg.norm(z - zc) > 1e-3 * np.linalg.norm(zc)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", [(32, 32, 32), (29, 17, 23)])
def test_l1_jacobi_solve_meets_bars(precision, shape):
    import torch

    m, f, c, b = case(shape=shape, fl="front", seed=2)
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    pref = direct.solve_sparse(sy, b)
    H = amg.build_hierarchy(sy.A, smoother="l1jacobi")
    ref = pcg.pcg(sy.A, assembly.pinned_rhs(sy, b), M=lambda r: amg.vcycle(H, r), rtol=1e-10)
    s = gpu_solver(m, f, c, precision=precision, smoother="l1jacobi")
    res = s.solve(to_dev(b, torch.float64))
    p = res.p.cpu().numpy()
    rr = assembly.relative_residual(sy, b, p)
    err = np.linalg.norm(p - pref) / np.linalg.norm(pref)
    print(f"l1-Jacobi {precision} {shape}: iterations {res.stats['iterations']} "
          f"(oracle {ref.iterations}), residual {rr:.2e}, L2 {err:.2e}", flush=True)
    assert res.status == 0
    assert rr <= 1e-10
    assert err <= 1e-9
    assert abs(res.stats["iterations"] - ref.iterations) <= 1


def test_torch_allocator_gives_the_same_pressure_and_returns_every_block():
    import torch

    import paper_1810_08572_amd as ppe

    m, f, c, b = case(shape=(24, 20, 18), fl="front", seed=6)
    bd = to_dev(b, torch.float64)
    before = torch.cuda.memory_allocated()
    s_t = gpu_solver(m, f, c, allocator="torch")
    p_t = s_t.solve(bd).p.clone()
    alloc = s_t.allocator
    assert isinstance(alloc, ppe.TorchAllocator)
    assert alloc.allocations > 0 and alloc.live > 0
    # the library's hierarchy and workspace now count as PyTorch memory
    assert torch.cuda.memory_allocated() > before
    s_h = gpu_solver(m, f, c, allocator="hip")
    p_h = s_h.solve(bd).p
    assert s_h.allocator is None
    assert torch.equal(p_t, p_h)
    s_t.close()
    assert alloc.live == 0


def test_a_refusing_allocator_fails_the_call_cleanly():
    import torch

    import paper_1810_08572_amd as ppe

    m, f, c, b = case(shape=(20, 20, 20), fl="front", seed=1)

    class Capped(ppe.TorchAllocator):
        """Refuses blocks beyond `cap` bytes while cap is set."""

        def __init__(self, device):
            super().__init__(device)
            self.cap = 4096
            inner = self._alloc

            def _alloc(nbytes, stream, ctx):
                if self.cap is not None and nbytes > self.cap:
                    return None
                return inner(nbytes, stream, ctx)

            self._alloc = ppe.ALLOC_FN(_alloc)

    cap = Capped(torch.device("cuda", 0))
    cap.cap = None
    s = ppe.Solver(allocator=cap)
    s.set_mesh(m.n_cells, to_dev(m.owner, torch.int32), to_dev(m.neigh, torch.int32))
    cap.cap = 4096   # the assembly's first larger block is refused
    with pytest.raises(ppe.PpeError) as e:
        s.assemble(to_dev(c, torch.float64), to_dev(f, torch.float64))
    assert e.value.status == ppe.PPE_ERR_OOM
    assert "allocator returned NULL" in str(e.value)
    cap.cap = None
    s.assemble(to_dev(c, torch.float64), to_dev(f, torch.float64))
    res = s.solve(to_dev(b, torch.float64))
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    assert res.status == 0
    assert assembly.relative_residual(sy, b, res.p.cpu().numpy()) <= 1e-10
    s.close()
    assert cap.live == 0
