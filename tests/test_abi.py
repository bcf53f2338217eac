"""The C-ABI library loads, exports every symbol include/mvgd.h declares, and rejects invalid
arguments on the host before touching a device (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mvgd.h")
LIB = os.path.join(ROOT, "paper_1603_04100_amd", "libmvgd.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mvgd_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def mv():
    from paper_1603_04100_amd import mvgd
    return mvgd


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("mvgd_assemble", "mvgd_apply", "mvgd_free", "mvgd_csr", "mvgd_info"):
        assert n in names


def test_library_exports_every_declared_symbol(mv):
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mvgd_\w+)", out))
    assert set(_declared()) <= exported
    assert set(mv.EXPORTS) == set(_declared())


def test_status_strings_and_version(mv):
    lib = mv._lib
    assert lib.mvgd_status_str(0) == b"MVGD_OK"
    assert lib.mvgd_status_str(-1) == b"MVGD_EINVAL"
    assert lib.mvgd_status_str(-4) == b"MVGD_EUNSUPPORTED"
    assert lib.mvgd_version() >= 100


def _call(mv, params, n_total=1000, offsets=None, n_clouds=1, points=0x1000, out=True):
    lib = mv._lib
    o = ctypes.c_void_p()
    offs = None
    if offsets is not None:
        arr = (ctypes.c_int64 * len(offsets))(*offsets)
        offs = ctypes.cast(arr, ctypes.c_void_p)
    st = lib.mvgd_assemble(ctypes.c_void_p(points), n_total, offs, n_clouds,
                           ctypes.byref(params) if params is not None else None, None,
                           ctypes.byref(o) if out else None)
    return st, o.value


@pytest.mark.parametrize("field,value,status", [
    ("k", 4, -1), ("k", 64, -1), ("n_ambient", 2, -1), ("n_ambient", 5, -1),
    ("d_manifold", 3, -1), ("d_manifold", 0, -1), ("precision", 7, -1), ("flags", 1 << 9, -1),
    ("launch", 3, -1), ("search", 4, -1),
])
def test_invalid_parameters_rejected_on_host(mv, field, value, status):
    p = mv.mvgd_params(3, 2, 20, mv.MVGD_FP64, 0, 0.0)
    setattr(p, field, value)
    st, h = _call(mv, p)
    assert st == status and h is None
    assert mv._lib.mvgd_last_error()


@pytest.mark.parametrize("n_amb,d,k,flags", [
    (4, 1, 6, 0),      # curves live in R^2 or R^3
    (3, 1, 1, 0),      # K >= 2 for the three monomials of a curve
    (3, 2, 20, 32),    # the divergence form is for curves
    (2, 1, 6, 32 | 1), # and excludes the LS variant
])
def test_curve_parameters_rejected_on_host(mv, n_amb, d, k, flags):
    p = mv.mvgd_params(n_amb, d, k, mv.MVGD_FP64, flags, 0.0)
    st, h = _call(mv, p)
    assert st == -1 and h is None


def test_invalid_shapes_rejected_on_host(mv):
    p = mv.mvgd_params(3, 2, 20, mv.MVGD_FP32_MIXED, 0, 0.0)
    assert _call(mv, None)[0] == -1
    assert _call(mv, p, points=0)[0] == -1
    assert _call(mv, p, out=False)[0] == -1
    assert _call(mv, p, n_total=0)[0] == -1
    assert _call(mv, p, n_total=20)[0] == -1                      # needs more than k points
    assert _call(mv, p, offsets=[0, 500, 900], n_clouds=2)[0] == -1  # does not end at n_total
    assert _call(mv, p, offsets=[0, 990, 1000], n_clouds=2)[0] == -1  # second cloud too small
    assert _call(mv, p, offsets=[1, 500, 1000], n_clouds=2)[0] == -1
    q = mv.mvgd_params(3, 2, 20, mv.MVGD_FP64, mv.MVGD_FLAG_H_OVERRIDE, -1.0)
    assert _call(mv, q)[0] == -1


def test_apply_and_free_accept_null_safely(mv):
    lib = mv._lib
    assert lib.mvgd_apply(None, None, None, 1, None) == -1
    assert lib.mvgd_csr(None, None, None, None, None) == -1
    st = mv.mvgd_row_stats_t()
    assert lib.mvgd_row_stats(None, None, ctypes.byref(st), None) == -1
    assert lib.mvgd_pool_trim(0) in (0, -3)  # -3 (no device) on a host without a GPU
    prm, info = mv.mvgd_solve_params(0, 10, 1e-8, 0.0, 0.0, 0, 0, None), mv.mvgd_solve_info()
    assert lib.mvgd_solve(None, None, None, ctypes.byref(prm), ctypes.byref(info), None) == -1
    lib.mvgd_free(None)


def test_neumann_arguments_rejected_on_host(mv):
    lib = mv._lib
    fake = ctypes.c_void_p(0x2000)

    def call(p, kb=8, boundary=fake, src=fake, info=True):
        o, inf = ctypes.c_void_p(), mv.mvgd_neumann_info()
        st = lib.mvgd_assemble_neumann(ctypes.c_void_p(0x1000), 1000, boundary, kb,
                                       ctypes.byref(p), None, ctypes.byref(o), None, src,
                                       ctypes.byref(inf) if info else None)
        assert o.value is None
        return st

    p3 = mv.mvgd_params(3, 2, 20, mv.MVGD_FP64, 0, 0.0)
    assert call(p3, boundary=None) == mv.MVGD_EINVAL
    assert call(p3, src=None) == mv.MVGD_EINVAL
    assert call(p3, info=False) == mv.MVGD_EINVAL
    assert call(p3, kb=2) == mv.MVGD_EINVAL
    assert call(p3, kb=17) == mv.MVGD_EINVAL
    assert call(mv.mvgd_params(4, 2, 20, mv.MVGD_FP64, 0, 0.0)) == mv.MVGD_EUNSUPPORTED
    assert call(mv.mvgd_params(3, 1, 6, mv.MVGD_FP64, 0, 0.0)) == mv.MVGD_EUNSUPPORTED
    assert call(mv.mvgd_params(3, 2, 4, mv.MVGD_FP64, 0, 0.0)) == mv.MVGD_EINVAL  # k too small


def test_dense_eigvals_against_lapack_and_closed_forms(mv):
    """The host step of mvgd_eigs (Hessenberg reduction + double-shift QR) against LAPACK's
    eigenvalues on random, symmetric, Hessenberg and nearly defective matrices, and against closed
    forms: a rotation block (e^{+-i t}) and a companion matrix with known roots."""
    from scipy.optimize import linear_sum_assignment
    rng = __import__("numpy").random.default_rng(0)
    np = __import__("numpy")
    for m in (1, 2, 3, 5, 8, 16, 33, 64):
        for kind in range(4):
            A = rng.standard_normal((m, m))
            if kind == 1:
                A = A + A.T
            elif kind == 2:
                A = np.triu(A, -1)
            elif kind == 3:
                A = np.diag(np.repeat(rng.standard_normal(m // 2 + 1), 2)[:m]) + \
                    1e-3 * rng.standard_normal((m, m))
            ev, ref = mv.mvgd_dense_eigvals(A), np.linalg.eigvals(A)
            C = np.abs(ev[:, None] - ref[None, :])
            r, c = linear_sum_assignment(C)
            assert C[r, c].max() <= 1e-10 * max(1.0, np.abs(ref).max()), (m, kind)
    t = 0.7
    ev = mv.mvgd_dense_eigvals(np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]]))
    assert np.allclose(np.sort_complex(ev), np.sort_complex(np.exp([-1j * t, 1j * t])), atol=1e-15)
    roots = np.array([1.0, -2.0, 3.0, 0.5, -0.25])
    coef = np.poly(roots)
    comp = np.zeros((5, 5))
    comp[0] = -coef[1:] / coef[0]
    comp[1:, :-1] = np.eye(4)
    ev = mv.mvgd_dense_eigvals(comp)
    assert np.allclose(np.sort(ev.real), np.sort(roots), atol=1e-12) and np.abs(ev.imag).max() < 1e-12


def test_eigs_arguments_rejected_on_host(mv):
    lib = mv._lib
    info = mv.mvgd_eigs_info()
    re = (ctypes.c_double * 4)()
    im = (ctypes.c_double * 4)()
    prm = mv.mvgd_eigs_params(4, 0, 0, 0, 0.0, None, 1)
    assert lib.mvgd_eigs(None, ctypes.byref(prm), re, im, ctypes.byref(info), None) == -1
    assert lib.mvgd_dense_eigvals(0, None, None, None) == -1
