"""Python binding of libppe: the masked pressure-correction Poisson solve
(smoothed-aggregation AMG-preconditioned conjugate gradients) on MI355X.

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch supplies device memory (tensors) and the stream.  The functions
mirror the C ABI of include/ppe.h one to one (``ppe_create``,
``ppe_set_mesh``, ``ppe_assemble``, ``ppe_solve``, ...); ``Solver`` wraps
them with tensor checks.  If the library is not built this module raises on
first use - there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppe.so")

PPE_OK = 0
PPE_NOT_CONVERGED = 1
PPE_ERR_ARG = -1
PPE_ERR_HIP = -2
PPE_ERR_OOM = -3
PPE_ERR_BREAKDOWN = -4
PPE_ERR_STATE = -5
PPE_ERR_INTERNAL = -6
PPE_FP64 = 0
PPE_MIXED = 1
PPE_SMOOTH_CHEBYSHEV = 0
PPE_SMOOTH_L1JACOBI = 1


class ppe_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("rtol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("cheb_degree", ctypes.c_int),
        ("cheb_ratio", ctypes.c_double),
        ("coarse_max", ctypes.c_int),
        ("max_levels", ctypes.c_int),
        ("theta", ctypes.c_double),
        ("check_every", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("use_graph", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("reuse_unchanged", ctypes.c_int),
        ("project_krylov", ctypes.c_int),
        ("smoother", ctypes.c_int),
        ("alloc", ctypes.c_void_p),
        ("free", ctypes.c_void_p),
        ("alloc_ctx", ctypes.c_void_p),
        ("coarse_reuse", ctypes.c_int),
        ("theta_decay", ctypes.c_double),
    ]


class ppe_stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("rel_residual", ctypes.c_double),
        ("setup_ms", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
        ("n_active", ctypes.c_int),
        ("n_components", ctypes.c_int),
        ("levels", ctypes.c_int),
        ("op_complexity", ctypes.c_double),
        ("bytes_per_iter", ctypes.c_double),
        ("reused_setup", ctypes.c_int),
        ("coarse_reused", ctypes.c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ppe_project_stats(ctypes.Structure):
    _fields_ = [
        ("outer", ctypes.c_int),
        ("pcg_iterations", ctypes.c_int),
        ("rel_residual", ctypes.c_double),
        ("ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ppe_alloy(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("rho", "cp", "k", "mu", "beta", "lam", "Lf",
                                               "T_f", "T_liq", "T_sol", "T_eps", "k_p", "T_ref")] + [
        ("g", ctypes.c_double * 3),
        ("fixed_wall_T", ctypes.c_int),
        ("T_wall", ctypes.c_double),
    ]


class ppe_step_params(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double),
        ("picard_tol", ctypes.c_double),
        ("max_picard", ctypes.c_int),
        ("relax", ctypes.c_double),
        ("have_history", ctypes.c_int),
    ]


class ppe_flow_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("picard", "momentum_iterations", "pressure_outer",
                                            "pressure_iterations", "energy_iterations", "n_fluid",
                                            "n_solid")] + [
        (n, ctypes.c_double) for n in ("momentum_ms", "pressure_ms", "energy_ms", "ms")]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# symbol -> (restype, argtypes); the exported C ABI
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_SIGS = {
    "ppe_default_options": (None, [ctypes.POINTER(ppe_options)]),
    "ppe_create": (ctypes.c_int, [ctypes.POINTER(ppe_options), ctypes.POINTER(_P)]),
    "ppe_destroy": (None, [_P]),
    "ppe_set_mesh": (ctypes.c_int, [_P, _I32, _I32, _P, _P]),
    "ppe_assemble": (ctypes.c_int, [_P, _P, _P]),
    "ppe_assemble_shifted": (ctypes.c_int, [_P, _P, _P, _P]),
    "ppe_refresh_shift": (ctypes.c_int, [_P, _P, _P]),
    "ppe_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.POINTER(ppe_stats)]),
    "ppe_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(ppe_stats)]),
    "ppe_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ppe_last_error": (ctypes.c_char_p, [_P]),
    "ppe_level_info": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(_I32),
                                      ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_I32),
                                      ctypes.POINTER(ctypes.c_double)]),
    "ppe_copy_level_matrix": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P]),
    "ppe_copy_prolongator": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P]),
    "ppe_copy_aggregates": (ctypes.c_int, [_P, ctypes.c_int, _P]),
    "ppe_copy_mask": (ctypes.c_int, [_P, _P, _P]),
    "ppe_apply_matrix": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "ppe_apply_vcycle": (ctypes.c_int, [_P, _P, _P]),
    "ppe_set_segments": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_I32)]),
    "ppe_get_level_launch": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(_I32)]),
    "ppe_set_level_launch": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(_I32)]),
    "ppe_get_segment_stats": (ctypes.c_int, [_P, ctypes.POINTER(_I32),
                                             ctypes.POINTER(ctypes.c_double)]),
    "ppe_mlp_create": (ctypes.c_int, [_I32, _I32, _I32, _P, ctypes.POINTER(_P)]),
    "ppe_mlp_destroy": (None, [_P]),
    "ppe_mlp_num_params": (ctypes.c_int64, [_P]),
    "ppe_mlp_last_error": (ctypes.c_char_p, [_P]),
    "ppe_mlp_set_params": (ctypes.c_int, [_P, _P]),
    "ppe_mlp_get_params": (ctypes.c_int, [_P, _P]),
    "ppe_mlp_forward": (ctypes.c_int, [_P, _I32, _P, _P, ctypes.c_int]),
    "ppe_mlp_loss_grad": (ctypes.c_int, [_P, _I32, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "ppe_mlp_train_step": (ctypes.c_int, [_P, _I32, _P, _P, ctypes.c_float,
                                          ctypes.POINTER(ctypes.c_double)]),
    "ppe_warm_start_features": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P,
                                               ctypes.POINTER(ctypes.c_double)]),
    "ppe_warm_start_features_noalloc": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P,
                                                       ctypes.POINTER(ctypes.c_double)]),
    "ppe_warm_start_apply": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, _P]),
    "ppe_warm_start_targets": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, _P]),
    "ppe_set_geometry": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _P]),
    "ppe_project": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_double, _P, _P, _P,
                                   ctypes.POINTER(ppe_project_stats)]),
    "ppe_project_warm": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_double, _P, _P,
                                        _P, ctypes.POINTER(ppe_project_stats)]),
    "ppe_face_gradient": (ctypes.c_int, [_P, _P, ctypes.c_double, _P, _P, _P]),
    "ppe_pce_create": (ctypes.c_int, [_I32, ctypes.POINTER(_I32), _I32, _P, ctypes.POINTER(_P)]),
    "ppe_pce_destroy": (None, [_P]),
    "ppe_pce_num_terms": (_I32, [_P]),
    "ppe_pce_last_error": (ctypes.c_char_p, [_P]),
    "ppe_pce_terms": (ctypes.c_int, [_P, ctypes.POINTER(_I32)]),
    "ppe_pce_nodes": (ctypes.c_int, [_P, _I32, _I32, ctypes.POINTER(_I32), _P, _P]),
    "ppe_pce_fit": (ctypes.c_int, [_P, _I32, _P, ctypes.c_int64, _P, _P]),
    "ppe_pce_eval": (ctypes.c_int, [_P, _I32, _P, ctypes.c_int64, _P, _P]),
    "ppe_pce_stats": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, _P, _P, _P]),
    "ppe_flow_create": (ctypes.c_int, [ctypes.POINTER(ppe_options), ctypes.c_double,
                                       ctypes.POINTER(_P)]),
    "ppe_flow_destroy": (None, [_P]),
    "ppe_flow_set_mesh": (ctypes.c_int, [_P, _I32, _I32, _P, _P, _I32, _P, _P, _P, _P, _P, _P,
                                         _P]),
    "ppe_flow_step": (ctypes.c_int, [_P, ctypes.POINTER(ppe_alloy),
                                     ctypes.POINTER(ppe_step_params), _P, _P, _P, _P, _P, _P, _P,
                                     ctypes.POINTER(ppe_flow_stats)]),
    "ppe_flow_last_error": (ctypes.c_char_p, [_P]),
    "ppe_flow_solid_fraction": (ctypes.c_int, [_P, ctypes.POINTER(ppe_alloy), ctypes.c_int64, _P,
                                               _P]),
    "ppe_profile_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "ppe_profile_count": (ctypes.c_int, [_P, ctypes.POINTER(_I32)]),
    "ppe_profile_entry": (ctypes.c_int, [_P, _I32, ctypes.c_char_p, _I32,
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
}
SYMBOLS = tuple(_SIGS)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libppe.so (built in-tree by ``build()``); raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libppe.so not built at {path}; run paper_1810_08572_amd.build.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PpeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _check(status, handle=None, allow=(PPE_OK,)):
    if status in allow:
        return status
    lib = load_library()
    detail = lib.ppe_last_error(handle).decode() if handle is not None else ""
    name = lib.ppe_status_string(status).decode()
    raise PpeError(status, f"{name}: {detail}")


# ---- one-to-one wrappers of the C ABI ---------------------------------------
# Caller allocator hooks of ppe_options (ppe_alloc_fn, ppe_free_fn).
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """The library's device memory from PyTorch's caching allocator: alloc
    takes a block on the device the object was made on, in stream order on
    the library's stream; free hands it back (the library has drained its
    streams first).  A failed allocation returns NULL, which the library
    reports as PPE_ERR_OOM.  Keep the object alive as long as the solver."""

    def __init__(self, device):
        import torch

        self.device = torch.device(device).index
        self.live = 0           # blocks handed out and not yet returned
        self.allocations = 0    # alloc calls that succeeded

        def _alloc(nbytes, stream, ctx):
            try:
                import torch as _t

                p = _t.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
                self.live += 1
                self.allocations += 1
                return p
            except Exception:  # noqa: BLE001 - out of memory or a torch error: NULL
                return None

        def _free(ptr, ctx):
            try:
                import torch as _t

                _t.cuda.caching_allocator_delete(int(ptr))
                self.live -= 1
            except Exception:  # noqa: BLE001 - torch already torn down at exit
                pass

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)

    def install(self, o):
        o.alloc = ctypes.cast(self._alloc, ctypes.c_void_p)
        o.free = ctypes.cast(self._free, ctypes.c_void_p)
        o.alloc_ctx = None


def _allocator_for(allocator, device):
    """allocator: "torch" (PyTorch's caching allocator), "hip" (the
    library's own hipMalloc) or a TorchAllocator-like object."""
    if allocator == "torch":
        return TorchAllocator(device)
    if allocator == "hip" or allocator is None:
        return None
    return allocator


def ppe_default_options():
    o = ppe_options()
    load_library().ppe_default_options(ctypes.byref(o))
    return o


def ppe_create(options: ppe_options):
    h = ctypes.c_void_p()
    _check(load_library().ppe_create(ctypes.byref(options), ctypes.byref(h)))
    return h


def ppe_destroy(handle):
    load_library().ppe_destroy(handle)


def ppe_set_mesh(handle, n_cells, n_faces, owner_ptr, neigh_ptr):
    return load_library().ppe_set_mesh(handle, n_cells, n_faces, owner_ptr, neigh_ptr)


def ppe_assemble(handle, coeff_ptr, fl_ptr):
    return load_library().ppe_assemble(handle, coeff_ptr, fl_ptr)


def ppe_solve(handle, rhs_ptr, p_ptr, use_x0, stats: ppe_stats):
    return load_library().ppe_solve(handle, rhs_ptr, p_ptr, int(use_x0), ctypes.byref(stats))


def ppe_status_string(status):
    return load_library().ppe_status_string(status).decode()


def ppe_last_error(handle=None):
    return load_library().ppe_last_error(handle).decode()


# ---- tensor-level wrapper ----------------------------------------------------
def _dev_ptr(t, dtype, n, name):
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class SolveResult:
    p: "object"
    status: int
    stats: dict


class Solver:
    """Pressure solver bound to the current device and torch stream."""

    def __init__(self, precision="fp64", rtol=1e-10, max_iter=500, cheb_degree=2,
                 cheb_ratio=7.0, coarse_max=512, max_levels=10, theta=0.08, stream=None,
                 use_graph=True, check_every=2, autotune=False, reuse_unchanged=False,
                 krylov="bicgstab", smoother="chebyshev", allocator="torch", coarse_reuse=0,
                 theta_decay=0.5):
        import torch

        lib = load_library()
        o = ppe_default_options()
        o.project_krylov = {"deferred": 0, "bicgstab": 1}[krylov]
        o.smoother = {"chebyshev": PPE_SMOOTH_CHEBYSHEV, "l1jacobi": PPE_SMOOTH_L1JACOBI}[smoother]
        o.precision = {"fp64": PPE_FP64, "mixed": PPE_MIXED}[precision]
        o.rtol, o.max_iter, o.cheb_degree, o.cheb_ratio = rtol, max_iter, cheb_degree, cheb_ratio
        o.coarse_max, o.max_levels, o.theta = coarse_max, max_levels, theta
        o.theta_decay = theta_decay
        o.use_graph, o.check_every = int(bool(use_graph)), int(check_every)
        o.autotune = int(bool(autotune))
        o.reuse_unchanged = int(bool(reuse_unchanged))
        o.coarse_reuse = int(coarse_reuse)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        o.stream = ctypes.c_void_p(stream.cuda_stream)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.allocator = _allocator_for(allocator, self.device)
        if self.allocator is not None:
            self.allocator.install(o)
        self._lib = lib
        self._h = ppe_create(o)
        self.n_cells = 0
        self.n_faces = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ppe_destroy(self._h)
            self._h = None

    __del__ = close

    def _chk(self, st, allow=(PPE_OK,)):
        return _check(st, self._h, allow)

    def set_mesh(self, n_cells, owner, neigh):
        import torch

        nf = owner.numel()
        self.n_cells, self.n_faces = 0, 0
        self._chk(self._lib.ppe_set_mesh(self._h, int(n_cells), int(nf),
                                         _dev_ptr(owner, torch.int32, nf, "owner"),
                                         _dev_ptr(neigh, torch.int32, nf, "neigh")))
        self.n_cells, self.n_faces = int(n_cells), int(nf)
        self.n_seg = 1

    def set_segments(self, cell_offsets):
        """Declare independent samples: cells [off[k], off[k+1]) form sample k."""
        off = [int(v) for v in cell_offsets]
        arr = (_I32 * len(off))(*off)
        self._chk(self._lib.ppe_set_segments(self._h, len(off) - 1, arr))
        self.n_seg = len(off) - 1

    def segment_stats(self):
        n = getattr(self, "n_seg", 1)
        it = (_I32 * n)()
        rr = (ctypes.c_double * n)()
        self._chk(self._lib.ppe_get_segment_stats(self._h, it, rr))
        return list(it), list(rr)

    def assemble(self, face_coeff, liquid_fraction):
        import torch

        # before set_mesh the sizes are unknown: the library reports the state error
        nf = self.n_faces if self.n_cells else None
        nc = self.n_cells if self.n_cells else None
        self._chk(self._lib.ppe_assemble(
            self._h, _dev_ptr(face_coeff, torch.float64, nf, "face_coeff"),
            _dev_ptr(liquid_fraction, torch.float64, nc, "liquid_fraction")))

    def assemble_shifted(self, face_coeff, diag_shift, liquid_fraction=None):
        """diag(diag_shift) + L over the open faces, no pins
        (liquid_fraction None: every cell kept)."""
        import torch

        nf = self.n_faces if self.n_cells else None
        nc = self.n_cells if self.n_cells else None
        fl = (ctypes.c_void_p(None) if liquid_fraction is None
              else _dev_ptr(liquid_fraction, torch.float64, nc, "liquid_fraction"))
        self._chk(self._lib.ppe_assemble_shifted(
            self._h, _dev_ptr(face_coeff, torch.float64, nf, "face_coeff"), fl,
            _dev_ptr(diag_shift, torch.float64, nc, "diag_shift")))

    def refresh_shift(self, face_coeff, diag_shift):
        """New diagonal shift, same coefficients and mask: finest level only."""
        import torch

        self._chk(self._lib.ppe_refresh_shift(
            self._h, _dev_ptr(face_coeff, torch.float64, self.n_faces, "face_coeff"),
            _dev_ptr(diag_shift, torch.float64, self.n_cells, "diag_shift")))

    def solve(self, rhs, x0=None, out=None, allow_not_converged=False):
        import torch

        if out is None:
            out = torch.empty(self.n_cells, dtype=torch.float64, device=rhs.device)
        use_x0 = x0 is not None
        if use_x0 and x0.data_ptr() != out.data_ptr():
            out.copy_(x0)
        st = ppe_stats()
        allow = (PPE_OK, PPE_NOT_CONVERGED) if allow_not_converged else (PPE_OK,)
        status = self._lib.ppe_solve(self._h, _dev_ptr(rhs, torch.float64, self.n_cells, "rhs"),
                                     _dev_ptr(out, torch.float64, self.n_cells, "p"),
                                     int(use_x0), ctypes.byref(st))
        self._chk(status, allow)
        return SolveResult(out, status, st.as_dict())

    def stats(self):
        st = ppe_stats()
        self._chk(self._lib.ppe_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    # ---- pressure-correction step with cross diffusion ----
    def set_geometry(self, nodes, face_nodes, cell_nodes, cell_centre, face_area):
        """nodes [n_nodes, 3] f64, face_nodes [n_faces, 4] i32 (V1..V4),
        cell_nodes [n_cells, 8] i32, cell_centre [n_cells, 3] f64,
        face_area [n_faces, 3] f64 (owner -> neighbour); device tensors."""
        import torch

        nn = nodes.numel() // 3
        self._chk(self._lib.ppe_set_geometry(
            self._h, int(nn), _dev_ptr(nodes, torch.float64, 3 * nn, "nodes"),
            _dev_ptr(face_nodes, torch.int32, 4 * self.n_faces, "face_nodes"),
            _dev_ptr(cell_nodes, torch.int32, 8 * self.n_cells, "cell_nodes"),
            _dev_ptr(cell_centre, torch.float64, 3 * self.n_cells, "cell_centre"),
            _dev_ptr(face_area, torch.float64, 3 * self.n_faces, "face_area")))

    def project(self, face_coeff, ustar, rho, dt, allow_not_converged=False, p0=None):
        """One pressure-correction step; returns (p, flux, u, stats).  p0: a
        starting pressure (ppe_project_warm), else zero."""
        import torch

        dev = ustar.device
        if p0 is not None:
            _dev_ptr(p0, torch.float64, self.n_cells, "p0")  # type, device and size checks
            p = p0.clone()
        else:
            p = torch.empty(self.n_cells, dtype=torch.float64, device=dev)
        flux = torch.empty(max(self.n_faces, 1), dtype=torch.float64, device=dev)
        u = torch.empty((self.n_cells, 3), dtype=torch.float64, device=dev)
        st = ppe_project_stats()
        allow = (PPE_OK, PPE_NOT_CONVERGED) if allow_not_converged else (PPE_OK,)
        fn = self._lib.ppe_project if p0 is None else self._lib.ppe_project_warm
        status = fn(
            self._h, _dev_ptr(face_coeff, torch.float64, self.n_faces, "face_coeff"),
            _dev_ptr(ustar, torch.float64, 3 * self.n_cells, "ustar"), float(rho), float(dt),
            ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(flux.data_ptr()),
            ctypes.c_void_p(u.data_ptr()), ctypes.byref(st))
        self._chk(status, allow)
        return p, flux[: self.n_faces], u, st.as_dict()

    def face_gradient(self, face_coeff, rho, p):
        """Masked face gradients [n_faces, 3] of p and the cross fluxes t_f.grad_f."""
        import torch

        g = torch.empty((max(self.n_faces, 1), 3), dtype=torch.float64, device=p.device)
        x = torch.empty(max(self.n_faces, 1), dtype=torch.float64, device=p.device)
        self._chk(self._lib.ppe_face_gradient(
            self._h, _dev_ptr(face_coeff, torch.float64, self.n_faces, "face_coeff"), float(rho),
            _dev_ptr(p, torch.float64, self.n_cells, "p"), ctypes.c_void_p(g.data_ptr()),
            ctypes.c_void_p(x.data_ptr())))
        return g[: self.n_faces], x[: self.n_faces]

    # ---- dominant-kernel measurement ----
    def profile(self, enable=True):
        self._chk(self._lib.ppe_profile_enable(self._h, int(enable)))

    def profile_read(self):
        """{kernel name: dict(launches, kernel_ms, bytes)} recorded since
        profiling was enabled."""
        cnt = _I32()
        self._chk(self._lib.ppe_profile_count(self._h, ctypes.byref(cnt)))
        out = {}
        for k in range(cnt.value):
            name = ctypes.create_string_buffer(256)
            n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
            self._chk(self._lib.ppe_profile_entry(self._h, k, name, 256, ctypes.byref(n),
                                                  ctypes.byref(ms), ctypes.byref(by)))
            out[name.value.decode()] = dict(launches=n.value, kernel_ms=ms.value, bytes=by.value)
        return out

    # ---- inspection (parity tests) ----
    def n_levels(self):
        return self.stats()["levels"]

    def level_info(self, level):
        n = ctypes.c_int32()
        nnz = ctypes.c_int64()
        nnzp = ctypes.c_int64()
        na = ctypes.c_int32()
        rho = ctypes.c_double()
        self._chk(self._lib.ppe_level_info(self._h, level, ctypes.byref(n), ctypes.byref(nnz),
                                           ctypes.byref(nnzp), ctypes.byref(na),
                                           ctypes.byref(rho)))
        return dict(n=n.value, nnz=nnz.value, nnz_p=nnzp.value, n_agg=na.value, rho=rho.value)

    def _csr(self, fn, level, rows, nnz):
        import torch

        rp = torch.empty(rows + 1, dtype=torch.int32, device=self.device)
        ci = torch.empty(max(nnz, 1), dtype=torch.int32, device=self.device)
        v = torch.empty(max(nnz, 1), dtype=torch.float64, device=self.device)
        self._chk(fn(self._h, level, ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(ci.data_ptr()),
                     ctypes.c_void_p(v.data_ptr())))
        return rp, ci[:nnz], v[:nnz]

    def level_matrix(self, level):
        info = self.level_info(level)
        return self._csr(self._lib.ppe_copy_level_matrix, level, info["n"], info["nnz"])

    def prolongator(self, level):
        info = self.level_info(level)
        return self._csr(self._lib.ppe_copy_prolongator, level, info["n"], info["nnz_p"])

    def aggregates(self, level):
        import torch

        info = self.level_info(level)
        a = torch.empty(max(info["n"], 1), dtype=torch.int32, device=self.device)
        self._chk(self._lib.ppe_copy_aggregates(self._h, level, ctypes.c_void_p(a.data_ptr())))
        return a[:info["n"]]

    def mask(self):
        import torch

        cid = torch.empty(self.n_cells, dtype=torch.int32, device=self.device)
        comp = torch.empty(self.n_cells, dtype=torch.int32, device=self.device)
        self._chk(self._lib.ppe_copy_mask(self._h, ctypes.c_void_p(cid.data_ptr()),
                                          ctypes.c_void_p(comp.data_ptr())))
        return cid, comp

    def apply_matrix(self, level, x):
        import torch

        n = self.level_info(level)["n"]
        y = torch.empty(n, dtype=torch.float64, device=self.device)
        self._chk(self._lib.ppe_apply_matrix(self._h, level, _dev_ptr(x, torch.float64, n, "x"),
                                             ctypes.c_void_p(y.data_ptr())))
        return y

    def level_launch(self, level):
        """(lanes smoother, lanes restriction, lanes prolongation, fused first
        steps, fused prolongation)."""
        c = (_I32 * 5)()
        self._chk(self._lib.ppe_get_level_launch(self._h, level, c))
        return tuple(c)

    def set_level_launch(self, level, choice):
        if len(choice) != 5:
            raise ValueError("a launch choice has five entries")
        c = (_I32 * 5)(*[int(v) for v in choice])
        self._chk(self._lib.ppe_set_level_launch(self._h, level, c))

    def apply_vcycle(self, r):
        import torch

        n = self.level_info(0)["n"]
        z = torch.empty(n, dtype=torch.float64, device=self.device)
        self._chk(self._lib.ppe_apply_vcycle(self._h, _dev_ptr(r, torch.float64, n, "r"),
                                             ctypes.c_void_p(z.data_ptr())))
        return z


class WarmStartNet:
    """The warm-start network (FP32 parameters on the device)."""

    def __init__(self, n_in=10, width=128, n_hidden=3, stream=None):
        import torch

        self._lib = load_library()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        st = self._lib.ppe_mlp_create(n_in, width, n_hidden, ctypes.c_void_p(stream.cuda_stream),
                                      ctypes.byref(h))
        _check(st)
        self._h = h
        self.n_in, self.width, self.n_hidden = n_in, width, n_hidden
        self.n_params = int(self._lib.ppe_mlp_num_params(h))
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ppe_mlp_destroy(self._h)
            self._h = None

    __del__ = close

    def _chk(self, st):
        if st != PPE_OK:
            raise PpeError(st, f"{ppe_status_string(st)}: "
                               f"{self._lib.ppe_mlp_last_error(self._h).decode()}")

    def set_params(self, theta):
        import torch

        self._chk(self._lib.ppe_mlp_set_params(
            self._h, _dev_ptr(theta, torch.float32, self.n_params, "params")))

    def get_params(self):
        import torch

        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        self._chk(self._lib.ppe_mlp_get_params(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def forward(self, x, bf16=False):
        import torch

        n = x.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=self.device)
        self._chk(self._lib.ppe_mlp_forward(self._h, n, _dev_ptr(x, torch.float32, n * self.n_in, "x"),
                                            ctypes.c_void_p(y.data_ptr()), int(bool(bf16))))
        return y

    def loss_grad(self, x, t):
        import torch

        n = x.shape[0]
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        self._chk(self._lib.ppe_mlp_loss_grad(self._h, n, _dev_ptr(x, torch.float32, n * self.n_in, "x"),
                                              _dev_ptr(t, torch.float32, n, "t"),
                                              ctypes.c_void_p(g.data_ptr()), ctypes.byref(loss)))
        return loss.value, g

    def train_step(self, x, t, lr):
        import torch

        n = x.shape[0]
        loss = ctypes.c_double()
        self._chk(self._lib.ppe_mlp_train_step(
            self._h, n, _dev_ptr(x, torch.float32, n * self.n_in, "x"),
            _dev_ptr(t, torch.float32, n, "t"), ctypes.c_float(lr), ctypes.byref(loss)))
        return loss.value


PPE_INPUT_NORMAL, PPE_INPUT_UNIFORM = 0, 1
PPE_GRID_TENSOR, PPE_GRID_SMOLYAK = 0, 1


def _alloy(props):
    """ppe_alloy from a property mapping (rho, cp, k, mu, beta, lam, Lf, T_f,
    T_liq, T_sol, T_eps, k_p, T_ref, g, T_wall; T_wall None = insulated)."""
    a = ppe_alloy()
    for n in ("rho", "cp", "k", "mu", "beta", "lam", "Lf", "T_f", "T_liq", "T_sol", "T_eps",
              "k_p", "T_ref"):
        setattr(a, n, float(props[n]))
    for i, v in enumerate(props["g"]):
        a.g[i] = float(v)
    a.fixed_wall_T = 0 if props["T_wall"] is None else 1
    a.T_wall = 0.0 if props["T_wall"] is None else float(props["T_wall"])
    return a


@dataclass
class FlowState:
    """Device state of the time-step driver (float64 tensors)."""
    u: "object"        # [n, 3]
    T: "object"        # [n]
    fs: "object"       # [n]
    flux: "object"     # [n_faces]
    p: "object"        # [n]
    conv_u: "object"   # [n, 3]
    conv_T: "object"   # [n]
    have_history: bool = False
    step: int = 0      # steps taken since the state was created
    time: float = 0.0  # simulated time

    _FIELDS = ("u", "T", "fs", "flux", "p", "conv_u", "conv_T")

    def save(self, path):
        """Snapshot to an .npz file (host copies; a restart needs all of it,
        the convection history included)."""
        import numpy as np

        arrays = {k: getattr(self, k).detach().cpu().numpy() for k in self._FIELDS}
        np.savez(path, have_history=np.array(bool(self.have_history)),
                 step=np.array(int(self.step)), time=np.array(float(self.time)), **arrays)

    @classmethod
    def load(cls, path, device):
        """State saved by save(), on `device`."""
        import numpy as np
        import torch

        with np.load(path, allow_pickle=False) as z:
            t = {k: torch.as_tensor(z[k], dtype=torch.float64, device=device).contiguous()
                 for k in cls._FIELDS}
            return cls(**t, have_history=bool(z["have_history"]), step=int(z["step"]),
                       time=float(z["time"]))


class Flow:
    """One fractional step per call (section 2.2): momentum predictor,
    masked projection, energy with the latent-heat Picard loop.  The
    pressure solver takes the Solver options; momentum and energy solve in
    FP64 to transport_rtol."""

    def __init__(self, precision="fp64", rtol=1e-10, transport_rtol=1e-12, stream=None,
                 use_graph=True, autotune=False, krylov="bicgstab", reuse_unchanged=True,
                 allocator="torch"):
        import torch

        self._lib = load_library()
        o = ppe_default_options()
        o.project_krylov = {"deferred": 0, "bicgstab": 1}[krylov]
        o.reuse_unchanged = int(bool(reuse_unchanged))
        o.precision = {"fp64": PPE_FP64, "mixed": PPE_MIXED}[precision]
        o.rtol = rtol
        o.use_graph = int(bool(use_graph))
        o.autotune = int(bool(autotune))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        o.stream = ctypes.c_void_p(stream.cuda_stream)
        self.allocator = _allocator_for(allocator, torch.device("cuda", torch.cuda.current_device()))
        if self.allocator is not None:
            self.allocator.install(o)
        h = _P()
        _check(self._lib.ppe_flow_create(ctypes.byref(o), float(transport_rtol), ctypes.byref(h)))
        self._h = h
        self.n_cells = self.n_faces = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ppe_flow_destroy(self._h)
            self._h = None

    __del__ = close

    def _chk(self, st, allow=(PPE_OK,)):
        if st in allow:
            return st
        detail = self._lib.ppe_flow_last_error(self._h).decode()
        raise PpeError(st, f"{self._lib.ppe_status_string(st).decode()}: {detail}")

    def set_mesh(self, owner, neigh, nodes, face_nodes, cell_nodes, cell_centre, face_area,
                 face_centre, cell_volume):
        import torch

        nc = cell_volume.numel()
        nf = owner.numel()
        nn = nodes.numel() // 3
        self._chk(self._lib.ppe_flow_set_mesh(
            self._h, int(nc), int(nf), _dev_ptr(owner, torch.int32, nf, "owner"),
            _dev_ptr(neigh, torch.int32, nf, "neigh"), int(nn),
            _dev_ptr(nodes, torch.float64, 3 * nn, "nodes"),
            _dev_ptr(face_nodes, torch.int32, 4 * nf, "face_nodes"),
            _dev_ptr(cell_nodes, torch.int32, 8 * nc, "cell_nodes"),
            _dev_ptr(cell_centre, torch.float64, 3 * nc, "cell_centre"),
            _dev_ptr(face_area, torch.float64, 3 * nf, "face_area"),
            _dev_ptr(face_centre, torch.float64, 3 * nf, "face_centre"),
            _dev_ptr(cell_volume, torch.float64, nc, "cell_volume")))
        self.n_cells, self.n_faces = int(nc), int(nf)

    def solid_fraction(self, props, T):
        """f_s(T) of Eq. 21 on the device."""
        import torch

        fs = torch.empty_like(T)
        a = _alloy(props)
        self._chk(self._lib.ppe_flow_solid_fraction(
            self._h, ctypes.byref(a), int(T.numel()), _dev_ptr(T, torch.float64, None, "T"),
            ctypes.c_void_p(fs.data_ptr())))
        return fs

    def new_state(self, T, fs=None, u=None, props=None):
        """State at rest (or with velocity u), no convection history; fs None:
        f_s(T) of Eq. 21 for the given props."""
        import torch

        dev = T.device
        if fs is None:
            fs = self.solid_fraction(props, T)
        n, nf = self.n_cells, self.n_faces
        z = lambda *shape: torch.zeros(*shape, dtype=torch.float64, device=dev)
        u = z(n, 3) if u is None else u.clone()
        return FlowState(u.contiguous(), T.clone().contiguous(), fs.clone().contiguous(),
                         z(max(nf, 1)), z(n), z(n, 3), z(n))

    def step(self, props, state: FlowState, dt, picard_tol=1e-10, max_picard=50, relax=1.0,
             allow_not_converged=False):
        """Advance `state` in place by one step; returns (status, stats)."""
        import torch

        a = _alloy(props)
        prm = ppe_step_params(float(dt), float(picard_tol), int(max_picard), float(relax),
                              int(bool(state.have_history)))
        st = ppe_flow_stats()
        n, nf = self.n_cells, self.n_faces
        allow = (PPE_OK, PPE_NOT_CONVERGED) if allow_not_converged else (PPE_OK,)
        status = self._lib.ppe_flow_step(
            self._h, ctypes.byref(a), ctypes.byref(prm),
            _dev_ptr(state.u, torch.float64, 3 * n, "u"), _dev_ptr(state.T, torch.float64, n, "T"),
            _dev_ptr(state.fs, torch.float64, n, "fs"),
            _dev_ptr(state.flux, torch.float64, max(nf, 1), "flux"),
            _dev_ptr(state.p, torch.float64, n, "p"),
            _dev_ptr(state.conv_u, torch.float64, 3 * n, "conv_u"),
            _dev_ptr(state.conv_T, torch.float64, n, "conv_T"), ctypes.byref(st))
        self._chk(status, allow)
        state.have_history = True
        state.step += 1
        state.time += float(dt)
        return status, st.as_dict()

    def run(self, props, state: FlowState, dt, n_steps, snapshot_every=0, snapshot=None,
            **step_kw):
        """n_steps steps; every snapshot_every steps (0: never) calls
        snapshot(state) (e.g. lambda st: st.save(f"snap_{st.step:06d}.npz")).
        Returns the per-step statistics."""
        out = []
        for _ in range(int(n_steps)):
            out.append(self.step(props, state, dt, **step_kw)[1])
            if snapshot_every and snapshot is not None and state.step % snapshot_every == 0:
                snapshot(state)
        return out


class PolynomialChaos:
    """Polynomial chaos by stochastic collocation (section 3): inputs
    "normal" (standard normal) or "uniform" (on [-1, 1]), total degree."""

    def __init__(self, kinds, degree, stream=None):
        import numpy as np

        self._lib = load_library()
        k = [PPE_INPUT_NORMAL if x == "normal" else PPE_INPUT_UNIFORM for x in kinds]
        arr = (_I32 * len(k))(*k)
        h = _P()
        st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(self._lib.ppe_pce_create(len(k), arr, int(degree), st, ctypes.byref(h)))
        self._h = h
        self.d = len(k)
        self.n_terms = int(self._lib.ppe_pce_num_terms(h))
        a = np.zeros(self.n_terms * self.d, dtype=np.int32)
        self._chk(self._lib.ppe_pce_terms(h, a.ctypes.data_as(ctypes.POINTER(_I32))))
        self.terms = a.reshape(self.n_terms, self.d)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ppe_pce_destroy(self._h)
            self._h = None

    __del__ = close

    def _chk(self, st):
        if st != PPE_OK:
            raise PpeError(st, f"{self._lib.ppe_status_string(st).decode()}: "
                               f"{self._lib.ppe_pce_last_error(self._h).decode()}")

    def nodes(self, grid, level):
        """(nodes [n, d], probability weights [n]) as numpy arrays; grid
        "tensor" or "smolyak"."""
        import numpy as np

        g = PPE_GRID_TENSOR if grid == "tensor" else PPE_GRID_SMOLYAK
        n = _I32(0)
        self._chk(self._lib.ppe_pce_nodes(self._h, g, int(level), ctypes.byref(n), None, None))
        X = np.zeros((n.value, self.d))
        w = np.zeros(n.value)
        self._chk(self._lib.ppe_pce_nodes(self._h, g, int(level), ctypes.byref(n),
                                          X.ctypes.data_as(_P), w.ctypes.data_as(_P)))
        return X, w

    def fit(self, xi, Y):
        """W [n_terms, n_out] from outputs Y [M, n_out] (device) at points xi [M, d] (host)."""
        import numpy as np
        import torch

        xi = np.ascontiguousarray(xi, dtype=np.float64)
        M, n_out = Y.shape
        W = torch.empty((self.n_terms, n_out), dtype=torch.float64, device=Y.device)
        self._chk(self._lib.ppe_pce_fit(self._h, M, xi.ctypes.data_as(_P), n_out,
                                        _dev_ptr(Y, torch.float64, M * n_out, "Y"),
                                        ctypes.c_void_p(W.data_ptr())))
        return W

    def eval(self, xi, W):
        import numpy as np
        import torch

        xi = np.ascontiguousarray(xi, dtype=np.float64)
        T = xi.shape[0]
        n_out = W.shape[1]
        Y = torch.empty((T, n_out), dtype=torch.float64, device=W.device)
        self._chk(self._lib.ppe_pce_eval(self._h, T, xi.ctypes.data_as(_P), n_out,
                                         _dev_ptr(W, torch.float64, self.n_terms * n_out, "W"),
                                         ctypes.c_void_p(Y.data_ptr())))
        return Y

    def stats(self, W):
        """(mean, variance, first-order Sobol [d, n_out], total Sobol [d, n_out])."""
        import torch

        n_out = W.shape[1]
        dev = W.device
        mean = torch.empty(n_out, dtype=torch.float64, device=dev)
        var = torch.empty(n_out, dtype=torch.float64, device=dev)
        first = torch.empty((self.d, n_out), dtype=torch.float64, device=dev)
        total = torch.empty((self.d, n_out), dtype=torch.float64, device=dev)
        self._chk(self._lib.ppe_pce_stats(self._h, n_out,
                                          _dev_ptr(W, torch.float64, self.n_terms * n_out, "W"),
                                          ctypes.c_void_p(mean.data_ptr()), ctypes.c_void_p(var.data_ptr()),
                                          ctypes.c_void_p(first.data_ptr()),
                                          ctypes.c_void_p(total.data_ptr())))
        return mean, var, first, total


def warm_start_features(solver, dp_prev, rhs, face_coeff, fl, cell_volume, mu, sigma):
    """Features [n_active, 10] (FP32) and the increment scale of the
    assembled solver."""
    import torch

    na = solver.stats()["n_active"]
    feats = torch.empty((max(na, 1), 10), dtype=torch.float32, device=solver.device)
    scale = ctypes.c_double()
    nc, nf = solver.n_cells, solver.n_faces
    solver._chk(load_library().ppe_warm_start_features(
        solver._h, _dev_ptr(dp_prev, torch.float64, nc, "dp_prev"),
        _dev_ptr(rhs, torch.float64, nc, "rhs"), _dev_ptr(face_coeff, torch.float64, nf, "coeff"),
        _dev_ptr(fl, torch.float64, nc, "fl"), _dev_ptr(cell_volume, torch.float64, nc, "volume"),
        _dev_ptr(mu, torch.float32, 10, "mu"), _dev_ptr(sigma, torch.float32, 10, "sigma"),
        ctypes.c_void_p(feats.data_ptr()), ctypes.byref(scale)))
    return feats[:na], scale.value


def warm_start_features_noalloc(solver, dp_prev, rhs, face_coeff, fl, cell_volume, mu, sigma,
                                out):
    """ppe_warm_start_features_noalloc: the features written into the
    caller's out [>= n_active, 10] (FP32, device) with the library's static
    workspace; returns the increment scale.  Allocates nothing."""
    import torch

    na = solver.stats()["n_active"]
    if out.dtype != torch.float32 or out.device != solver.device or not out.is_contiguous() \
            or out.dim() != 2 or out.shape[1] != 10 or out.shape[0] < na:
        raise ValueError("out must be a contiguous float32 [>= n_active, 10] tensor on the "
                         "solver's device")
    scale = ctypes.c_double()
    nc, nf = solver.n_cells, solver.n_faces
    solver._chk(load_library().ppe_warm_start_features_noalloc(
        solver._h, _dev_ptr(dp_prev, torch.float64, nc, "dp_prev"),
        _dev_ptr(rhs, torch.float64, nc, "rhs"), _dev_ptr(face_coeff, torch.float64, nf, "coeff"),
        _dev_ptr(fl, torch.float64, nc, "fl"), _dev_ptr(cell_volume, torch.float64, nc, "volume"),
        _dev_ptr(mu, torch.float32, 10, "mu"), _dev_ptr(sigma, torch.float32, 10, "sigma"),
        ctypes.c_void_p(out.data_ptr()), ctypes.byref(scale)))
    return scale.value


def warm_start_apply(solver, p_prev, y, scale):
    import torch

    x0 = torch.empty(solver.n_cells, dtype=torch.float64, device=solver.device)
    solver._chk(load_library().ppe_warm_start_apply(
        solver._h, _dev_ptr(p_prev, torch.float64, solver.n_cells, "p_prev"),
        ctypes.c_void_p(y.data_ptr()), ctypes.c_double(scale), ctypes.c_void_p(x0.data_ptr())))
    return x0


def warm_start_targets(solver, p_new, p_prev, scale):
    import torch

    na = solver.stats()["n_active"]
    t = torch.empty(max(na, 1), dtype=torch.float32, device=solver.device)
    solver._chk(load_library().ppe_warm_start_targets(
        solver._h, _dev_ptr(p_new, torch.float64, solver.n_cells, "p_new"),
        _dev_ptr(p_prev, torch.float64, solver.n_cells, "p_prev"), ctypes.c_double(scale),
        ctypes.c_void_p(t.data_ptr())))
    return t[:na]
