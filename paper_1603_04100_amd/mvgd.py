"""ctypes binding of the MVGD C ABI (include/mvgd.h).

Argument marshalling only: torch tensors provide device memory and the current stream; every
step of assembly and apply runs in the HIP kernels of ``libmvgd.so``. There is no CPU fallback:
importing this module fails loudly when the library has not been built.

    L = mvgd_assemble(points, k=32, precision="fp32")   # points: [N, n] cuda tensor
    y = mvgd_apply(L, x)                                 # x: [N] or [N, R]
    row_ptr, col, val = mvgd_csr(L)
    mvgd_free(L)
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmvgd.so")

MVGD_OK, MVGD_EINVAL, MVGD_ENOMEM, MVGD_EDEVICE, MVGD_EUNSUPPORTED = 0, -1, -2, -3, -4
MVGD_FP64, MVGD_FP32_MIXED = 0, 1
MVGD_FLAG_LS, MVGD_FLAG_H_OVERRIDE, MVGD_FLAG_KEEP_DIAG, MVGD_FLAG_TIME = 1, 2, 4, 8
MVGD_FLAG_MLS, MVGD_FLAG_DIVERGENCE = 16, 32

EXPORTS = ("mvgd_assemble", "mvgd_apply", "mvgd_free", "mvgd_csr", "mvgd_row_diag", "mvgd_info",
           "mvgd_timing", "mvgd_row_stats", "mvgd_solve", "mvgd_assemble_neumann", "mvgd_eigs",
           "mvgd_dense_eigvals",
           "mvgd_pool_trim", "mvgd_status_str",
           "mvgd_last_error", "mvgd_version")


class MvgdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class mvgd_params(ctypes.Structure):
    _fields_ = [("n_ambient", ctypes.c_int32), ("d_manifold", ctypes.c_int32),
                ("k", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("h_override", ctypes.c_double),
                ("cell_alpha", ctypes.c_float), ("radius_mu", ctypes.c_float),
                ("cells_per_point", ctypes.c_float), ("launch", ctypes.c_int32),
                ("search", ctypes.c_int32)]


MVGD_LAUNCH_DEFAULT, MVGD_LAUNCH_GRID, MVGD_LAUNCH_PERSISTENT = 0, 1, 2
MVGD_SEARCH_DEFAULT, MVGD_SEARCH_GROUP, MVGD_SEARCH_LANE, MVGD_SEARCH_TILE = 0, 1, 2, 3


class mvgd_info_t(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_clouds", ctypes.c_int32), ("k", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("n_ambient", ctypes.c_int32), ("n_degenerate", ctypes.c_int64),
                ("n_slow_knn", ctypes.c_int64), ("device_bytes", ctypes.c_size_t),
                ("n_subgroups", ctypes.c_int64), ("n_streamed", ctypes.c_int64),
                ("n_growths", ctypes.c_int64)]


class mvgd_timing_t(ctypes.Structure):
    _fields_ = [("bin_ms", ctypes.c_float), ("assemble_ms", ctypes.c_float),
                ("apply_ms", ctypes.c_float), ("have_apply", ctypes.c_int32),
                ("search_ms", ctypes.c_float), ("fit_ms", ctypes.c_float)]


class mvgd_row_stats_t(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_diag_negative", ctypes.c_int64),
                ("n_m_rows", ctypes.c_int64), ("n_offdiag_negative", ctypes.c_int64),
                ("n_zero_diagonal", ctypes.c_int64), ("mean_ratio", ctypes.c_double),
                ("max_ratio", ctypes.c_double)]


MVGD_SOLVE_BICGSTAB, MVGD_SOLVE_JACOBI = 0, 1


class mvgd_solve_params(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("sigma", ctypes.c_double),
                ("omega", ctypes.c_double), ("pin_first", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("fixed", ctypes.c_void_p)]


class mvgd_eigs_params(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int32), ("block", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("fixed", ctypes.c_void_p),
                ("seed", ctypes.c_uint64)]


class mvgd_eigs_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("block", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("spectrum_bound", ctypes.c_double), ("max_change", ctypes.c_double)]


class mvgd_neumann_info(ctypes.Structure):
    _fields_ = [("n_interior", ctypes.c_int64), ("n_ghost", ctypes.c_int64)]


class mvgd_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_residual", ctypes.c_double)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"MVGD HIP library not built: {path} is missing "
                          "(run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.mvgd_assemble.argtypes = [vp, i64, vp, i32, ctypes.POINTER(mvgd_params), vp,
                                  ctypes.POINTER(vp)]
    lib.mvgd_assemble.restype = i32
    lib.mvgd_apply.argtypes = [vp, vp, vp, i32, vp]
    lib.mvgd_apply.restype = i32
    lib.mvgd_free.argtypes = [vp]
    lib.mvgd_free.restype = None
    lib.mvgd_csr.argtypes = [vp, vp, vp, vp, vp]
    lib.mvgd_csr.restype = i32
    lib.mvgd_row_diag.argtypes = [vp, vp, vp, vp]
    lib.mvgd_row_diag.restype = i32
    lib.mvgd_timing.argtypes = [vp, ctypes.POINTER(mvgd_timing_t)]
    lib.mvgd_timing.restype = i32
    lib.mvgd_info.argtypes = [vp, ctypes.POINTER(mvgd_info_t)]
    lib.mvgd_info.restype = i32
    lib.mvgd_row_stats.argtypes = [vp, vp, ctypes.POINTER(mvgd_row_stats_t), vp]
    lib.mvgd_row_stats.restype = i32
    lib.mvgd_solve.argtypes = [vp, vp, vp, ctypes.POINTER(mvgd_solve_params),
                               ctypes.POINTER(mvgd_solve_info), vp]
    lib.mvgd_solve.restype = i32
    lib.mvgd_assemble_neumann.argtypes = [vp, i64, vp, i32, ctypes.POINTER(mvgd_params), vp,
                                          ctypes.POINTER(vp), vp, vp,
                                          ctypes.POINTER(mvgd_neumann_info)]
    lib.mvgd_assemble_neumann.restype = i32
    lib.mvgd_eigs.argtypes = [vp, ctypes.POINTER(mvgd_eigs_params), vp, vp,
                              ctypes.POINTER(mvgd_eigs_info), vp]
    lib.mvgd_eigs.restype = i32
    lib.mvgd_dense_eigvals.argtypes = [i32, vp, vp, vp]
    lib.mvgd_dense_eigvals.restype = i32
    lib.mvgd_pool_trim.argtypes = [ctypes.c_size_t]
    lib.mvgd_pool_trim.restype = i32
    lib.mvgd_status_str.argtypes = [i32]
    lib.mvgd_status_str.restype = ctypes.c_char_p
    lib.mvgd_last_error.argtypes = []
    lib.mvgd_last_error.restype = ctypes.c_char_p
    lib.mvgd_version.argtypes = []
    lib.mvgd_version.restype = i32
    return lib


_lib = load_library()


def _check(status: int):
    if status != MVGD_OK:
        raise MvgdError(status, f"{_lib.mvgd_status_str(status).decode()}: "
                                f"{_lib.mvgd_last_error().decode()}")


def _stream(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class Matrix:
    """Handle of an assembled MVGD matrix (owns its device memory until ``free``)."""

    def __init__(self, handle: int, n_rows: int, k: int, dtype: torch.dtype, device):
        self._h = ctypes.c_void_p(handle)
        self.n_rows, self.k, self.dtype, self.device = n_rows, k, dtype, device

    @property
    def handle(self):
        if not self._h:
            raise ValueError("matrix already freed")
        return self._h

    def free(self):
        if self._h:
            _lib.mvgd_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _params(points, k, precision, flags, h_override, d_manifold, tuning, n_per_cloud):
    if not isinstance(points, torch.Tensor) or points.dim() != 2:
        raise ValueError("points must be a 2-D torch tensor")
    if precision is None:
        precision = "fp64" if points.dtype == torch.float64 else "fp32"
    prec = {"fp64": MVGD_FP64, "fp32": MVGD_FP32_MIXED}[precision]
    want = torch.float64 if prec == MVGD_FP64 else torch.float32
    if points.dtype != want:
        raise ValueError(f"points dtype {points.dtype} does not match precision {precision}")
    if not points.is_contiguous():
        raise ValueError("points must be contiguous")
    if h_override is not None:
        flags |= MVGD_FLAG_H_OVERRIDE
    if tuning is None:
        from . import autotune
        tuning = autotune.lookup(points.shape[1], k, precision, n_per_cloud, d_manifold)
    t = tuning or {}
    p = mvgd_params(points.shape[1], d_manifold, k, prec, flags, float(h_override or 0.0),
                    float(t.get("cell_alpha", 0.0)), float(t.get("radius_mu", 0.0)),
                    float(t.get("cells_per_point", 0.0)), int(t.get("launch", 0)),
                    int(t.get("search", 0)))
    return p, want


def mvgd_assemble(points: torch.Tensor, k: int, *, cloud_offsets=None, precision=None,
                  flags: int = 0, h_override: float | None = None, d_manifold: int = 2,
                  tuning: dict | None = None, stream=None) -> Matrix:
    """Assemble L from device points [N, n] (float32 -> FP32-mixed, float64 -> FP64).

    tuning: neighbour-search tunables {cell_alpha, radius_mu, cells_per_point, launch}; by
    default the autotuner's table (tuning.json) is consulted for this shape.
    """
    n_per = (points.shape[0] if cloud_offsets is None
             else points.shape[0] // max(1, len(cloud_offsets) - 1))
    p, want = _params(points, k, precision, flags, h_override, d_manifold, tuning, n_per)
    offs_ptr, n_clouds = None, 1
    if cloud_offsets is not None:
        offs = (ctypes.c_int64 * len(cloud_offsets))(*[int(v) for v in cloud_offsets])
        offs_ptr, n_clouds = ctypes.cast(offs, ctypes.c_void_p), len(cloud_offsets) - 1
    out = ctypes.c_void_p()
    _check(_lib.mvgd_assemble(ctypes.c_void_p(points.data_ptr()), points.shape[0], offs_ptr,
                              n_clouds, ctypes.byref(p), ctypes.c_void_p(_stream(stream)),
                              ctypes.byref(out)))
    return Matrix(out.value, points.shape[0], k, want, points.device)


def mvgd_assemble_neumann(points: torch.Tensor, boundary: torch.Tensor, k: int,
                          k_boundary: int = 8, *, precision=None, flags: int = 0,
                          h_override: float | None = None, tuning: dict | None = None,
                          stream=None):
    """L on an open surface in R^3 with the homogeneous Neumann condition by reflection.

    points [N, 3] (device), boundary [N] (device bool or uint8, nonzero = boundary point).
    Returns (L, n_interior, ghost_xyz [n_ghost, 3] float64, ghost_src [n_ghost] int32): rows
    [0, n_interior) of L are the interior points in ascending index order, the rest are the
    ghosts' zero rows.
    """
    p, want = _params(points, k, precision, flags, h_override, 2, tuning, points.shape[0])
    if boundary.shape != (points.shape[0],):
        raise ValueError("boundary must have one entry per point")
    b = boundary.to(torch.uint8).contiguous()
    n = points.shape[0]
    gx = torch.empty((n, 3), dtype=torch.float64, device=points.device)
    gs = torch.empty((n,), dtype=torch.int32, device=points.device)
    out, info = ctypes.c_void_p(), mvgd_neumann_info()
    _check(_lib.mvgd_assemble_neumann(ctypes.c_void_p(points.data_ptr()), n,
                                      ctypes.c_void_p(b.data_ptr()), int(k_boundary),
                                      ctypes.byref(p), ctypes.c_void_p(_stream(stream)),
                                      ctypes.byref(out), ctypes.c_void_p(gx.data_ptr()),
                                      ctypes.c_void_p(gs.data_ptr()), ctypes.byref(info)))
    ni, ng = int(info.n_interior), int(info.n_ghost)
    L = Matrix(out.value, ni + ng, k, want, points.device)
    return L, ni, gx[:ng], gs[:ng]


def mvgd_apply(L: Matrix, x: torch.Tensor, y: torch.Tensor | None = None, stream=None):
    """y = L x for x [N] or [N, R] (matrix dtype, contiguous, on the matrix's device)."""
    squeeze = x.dim() == 1
    x2 = x.reshape(x.shape[0], -1)
    if x2.dtype != L.dtype or not x2.is_contiguous() or x2.shape[0] != L.n_rows:
        raise ValueError("x must be a contiguous tensor of the matrix dtype with n_rows rows")
    if y is None:
        y = torch.empty_like(x2)
    _check(_lib.mvgd_apply(L.handle, ctypes.c_void_p(x2.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                           x2.shape[1], ctypes.c_void_p(_stream(stream))))
    return y.reshape(-1) if squeeze else y


def mvgd_free(L: Matrix):
    L.free()


def mvgd_csr(L: Matrix, stream=None):
    """CSR in the caller's point order: (row_ptr int64 [N+1], col int32 [nnz], val [nnz])."""
    nnz = L.n_rows * (L.k + 1)
    row_ptr = torch.empty(L.n_rows + 1, dtype=torch.int64, device=L.device)
    col = torch.empty(nnz, dtype=torch.int32, device=L.device)
    val = torch.empty(nnz, dtype=L.dtype, device=L.device)
    _check(_lib.mvgd_csr(L.handle, ctypes.c_void_p(row_ptr.data_ptr()),
                         ctypes.c_void_p(col.data_ptr()), ctypes.c_void_p(val.data_ptr()),
                         ctypes.c_void_p(_stream(stream))))
    return row_ptr, col, val


def mvgd_row_diag(L: Matrix, stream=None):
    """Per-row spacing h (float64) and status bits (uint8); needs MVGD_FLAG_KEEP_DIAG."""
    h = torch.empty(L.n_rows, dtype=torch.float64, device=L.device)
    st = torch.empty(L.n_rows, dtype=torch.uint8, device=L.device)
    _check(_lib.mvgd_row_diag(L.handle, ctypes.c_void_p(h.data_ptr()),
                              ctypes.c_void_p(st.data_ptr()), ctypes.c_void_p(_stream(stream))))
    return h, st


def mvgd_info(L: Matrix) -> dict:
    info = mvgd_info_t()
    _check(_lib.mvgd_info(L.handle, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in mvgd_info_t._fields_}


def mvgd_timing(L: Matrix) -> dict:
    """Device durations (ms) of the last assembly / apply; needs MVGD_FLAG_TIME."""
    t = mvgd_timing_t()
    _check(_lib.mvgd_timing(L.handle, ctypes.byref(t)))
    return {name: getattr(t, name) for name, _ in mvgd_timing_t._fields_}


def mvgd_row_stats(L: Matrix, ratio: bool = False, stream=None):
    """Row sign statistics (dict); with ratio=True also the per-row negative off-diagonal mass
    over |diagonal| (float64 tensor in the caller's order, NaN on zero diagonals)."""
    r = torch.empty(L.n_rows, dtype=torch.float64, device=L.device) if ratio else None
    st = mvgd_row_stats_t()
    _check(_lib.mvgd_row_stats(L.handle, ctypes.c_void_p(r.data_ptr() if ratio else 0),
                               ctypes.byref(st), ctypes.c_void_p(_stream(stream))))
    out = {name: getattr(st, name) for name, _ in mvgd_row_stats_t._fields_}
    return (out, r) if ratio else out


def mvgd_solve(L: Matrix, b: torch.Tensor, x: torch.Tensor | None = None, *,
               method: str = "bicgstab", max_iter: int = 1000, rtol: float = 1e-10,
               sigma: float = 0.0, omega: float = 0.0, pin_first: bool = False,
               check_every: int = 0, fixed: torch.Tensor | None = None, stream=None):
    """Solve (sigma I - L) x = b on the device; x (if given) is the initial guess and is
    overwritten. fixed: optional uint8/bool device mask of identity rows (Dirichlet points,
    x = b there). Returns (x, info dict with iterations, converged, rel_residual)."""
    if b.dtype != L.dtype or not b.is_contiguous() or b.numel() != L.n_rows:
        raise ValueError("b must be a contiguous vector of the matrix dtype with n_rows entries")
    if x is None:
        x = torch.zeros_like(b)
    elif x.dtype != L.dtype or not x.is_contiguous() or x.numel() != L.n_rows:
        raise ValueError("x must be a contiguous vector of the matrix dtype with n_rows entries")
    m = {"bicgstab": MVGD_SOLVE_BICGSTAB, "jacobi": MVGD_SOLVE_JACOBI}[method]
    if fixed is not None:
        fixed = fixed.to(torch.uint8).contiguous()
        if fixed.numel() != L.n_rows or fixed.device != b.device:
            raise ValueError("fixed must have n_rows entries on the matrix's device")
    prm = mvgd_solve_params(m, int(max_iter), float(rtol), float(sigma), float(omega),
                            1 if pin_first else 0, int(check_every),
                            fixed.data_ptr() if fixed is not None else None)
    info = mvgd_solve_info()
    _check(_lib.mvgd_solve(L.handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                           ctypes.byref(prm), ctypes.byref(info), ctypes.c_void_p(_stream(stream))))
    return x, {"iterations": info.iterations, "converged": info.converged,
               "rel_residual": info.rel_residual}


def mvgd_eigs(L: Matrix, nev: int, *, block: int = 0, degree: int = 0, max_iter: int = 0,
              tol: float = 0.0, fixed: torch.Tensor | None = None, seed: int = 1, stream=None):
    """The nev eigenvalues of -L with the smallest real parts (complex numpy array, sorted by
    real part) and the iteration info; `fixed` (device bool/uint8 [n_rows]) removes rows."""
    import numpy as np
    if fixed is not None:
        if fixed.shape != (L.n_rows,):
            raise ValueError("fixed must have one entry per row")
        fixed = fixed.to(torch.uint8).contiguous()
    prm = mvgd_eigs_params(int(nev), int(block), int(degree), int(max_iter), float(tol),
                           fixed.data_ptr() if fixed is not None else None, int(seed))
    re = (ctypes.c_double * int(nev))()
    im = (ctypes.c_double * int(nev))()
    info = mvgd_eigs_info()
    _check(_lib.mvgd_eigs(L.handle, ctypes.byref(prm), ctypes.cast(re, ctypes.c_void_p),
                          ctypes.cast(im, ctypes.c_void_p), ctypes.byref(info),
                          ctypes.c_void_p(_stream(stream))))
    lam = np.array(re[:]) + 1j * np.array(im[:])
    return lam, {f: getattr(info, f) for f, _ in mvgd_eigs_info._fields_}


def mvgd_dense_eigvals(a):
    """Eigenvalues of a real square matrix (host numpy array) by the library's dense routine."""
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("a must be square")
    m = a.shape[0]
    re, im = np.empty(m), np.empty(m)
    _check(_lib.mvgd_dense_eigvals(m, a.ctypes.data, re.ctypes.data, im.ctypes.data))
    return re + 1j * im


def mvgd_pool_trim(keep_bytes: int = 0):
    """Return the unused device memory of the library's pool (current device) to the system."""
    _check(_lib.mvgd_pool_trim(int(keep_bytes)))


def version() -> int:
    return int(_lib.mvgd_version())
