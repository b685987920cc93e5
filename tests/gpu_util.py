"""Helpers shared by the GPU parity tests: seeded cases and tensor moves."""
import numpy as np
import scipy.sparse as sp

from synth import box_mesh, face_coeff, fl_linear_x, fl_planar_front, rhs_uniform


def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch.device("cuda", 0)


def to_dev(a, dtype):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=torch_dev())


def case(shape=(16, 16, 16), jitter=0.1, seed=0, fl="linear", rho=2400.0, fl_seed=2,
         rhs_seed=1, center=True, mesh=None):
    m = mesh if mesh is not None else box_mesh(shape, jitter=jitter, seed=seed,
                                                mode="node" if jitter else None)
    if isinstance(fl, np.ndarray):
        f = fl
    elif fl == "linear":
        f = fl_linear_x(m.cell_centre)
    elif fl == "front":
        f = fl_planar_front(m.cell_centre, seed=fl_seed)
    elif fl == "ones":
        f = np.ones(m.n_cells)
    else:
        raise ValueError(fl)
    c = face_coeff(m, rho)
    b = rhs_uniform(m.n_cells, seed=rhs_seed, center_mask=(f > 0) if center else None)
    return m, f, c, b


def gpu_solver(m, f, c, **opts):
    import torch

    import paper_1810_08572_amd as ppe

    torch_dev()
    s = ppe.Solver(**opts)
    s.set_mesh(m.n_cells, to_dev(m.owner, torch.int32), to_dev(m.neigh, torch.int32))
    s.assemble(to_dev(c, torch.float64), to_dev(f, torch.float64))
    return s


def csr(rp, ci, v, shape):
    return sp.csr_matrix((v.cpu().numpy(), ci.cpu().numpy(), rp.cpu().numpy()), shape=shape)


def _absmax(M):
    """max |entry| without densifying a sparse operand (0 for an empty one)."""
    if sp.issparse(M):
        M = sp.csr_matrix(M)
        return float(np.abs(M.data).max()) if M.nnz else 0.0
    M = np.asarray(M)
    return float(np.abs(M).max()) if M.size else 0.0


def rel_max(A, B):
    """max |A - B| / max |B| for sparse or dense operands."""
    D = _absmax(A - B)
    s = _absmax(B)
    return D / s if s else D
