"""FP64 CPU oracle for the MVGD Laplace-Beltrami discretisation (arXiv:1603.04100).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
CPU-baseline leg of ``bench.py``. The GPU library never imports or links it, and it shares no
code with the GPU path. The arithmetic lives in ``mvgd_oracle.c`` (plain C, double, no FMA);
this module only marshals numpy arrays through ctypes.

Functions follow the paper's steps (see the header of ``mvgd_oracle.c``):

* ``knn``     O1, brute force, ascending (key, index).
* ``rows``    O1-O11 for a list of rows: MVGD (Sec. 3.1) or the plain least-squares variant
              (Sec. 2), with optional per-row diagnostics.
* ``assemble``  ``rows`` for every point, returned as CSR (row_ptr, cols, vals).
* ``apply``   O12, y = L x.
* ``lb_coefficients``  O8 alone: (G, q) of Eq. eqn3 from fitted graph coefficients.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mvgd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
ODIAG = 64

# column layout of the per-row diagnostics returned by ``rows(..., diag=True)``
DIAG_FIELDS = {
    "h": 0, "degenerate": 1, "lam": slice(2, 6), "frame": slice(6, 22), "a": slice(22, 40),
    "G": slice(40, 44), "q": slice(44, 46), "ell": slice(46, 52), "rdiag": slice(52, 58),
    "tau": 58, "rcond": 59, "kth_key": 60,
}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (FP64, -ffp-contract=off, OpenMP over rows)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.oracle_knn.argtypes = [P, i64, i32, i32, P, i64, P, P, i32]
    lib.oracle_knn.restype = i32
    lib.oracle_rows.argtypes = [P, i64, i32, i32, i32, i32, i32, f64, f64, P, i64, P, P, P, i32]
    lib.oracle_rows.restype = i32
    lib.oracle_apply.argtypes = [i64, P, P, P, i32, P, P]
    lib.oracle_apply.restype = i32
    lib.oracle_lb_coefficients.argtypes = [i32, i32, P, P, P]
    lib.oracle_lb_coefficients.restype = i32
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = i32
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def threads() -> int:
    return int(_load().oracle_threads())


def _points(points):
    p = np.ascontiguousarray(points, dtype=np.float64)
    if p.ndim != 2:
        raise ValueError("points must be [N, n]")
    return p


def _rows_arg(rows, n):
    if rows is None:
        return None, n
    r = np.ascontiguousarray(rows, dtype=np.int64)
    return r, r.shape[0]


def knn(points, k: int, rows=None, nthreads: int = 0):
    """K nearest neighbours (indices [R, K], keys [R, K]) ascending by (key, index)."""
    p = _points(points)
    r, nr = _rows_arg(rows, p.shape[0])
    idx = np.empty((nr, k), dtype=np.int64)
    key = np.empty((nr, k), dtype=np.float64)
    rc = _load().oracle_knn(_ptr(p), p.shape[0], p.shape[1], k, _ptr(r), nr, _ptr(idx), _ptr(key),
                            nthreads)
    if rc != 0:
        raise ValueError(f"oracle_knn failed ({rc})")
    return idx, key


def rows(points, k: int, rows=None, d: int = 2, variant: str = "mvgd", h_override=None,
         diag: bool = False, nthreads: int = 0, weight_nbr: float = 1.0):
    """MVGD rows (or the plain LS variant) for the given rows.

    variant: "mvgd" (Eq. center and its 2-D form), "ls" (derivatives of the fit, no centre
    term) or, for curves only, "div" (the divergence form, Eq. divergence).
    weight_nbr: least-squares weight of every neighbour (p_i has weight 1); 1 is the unweighted
    fit, 1/k the moving-least-squares weights of the paper's comparison (Sec. 4).
    Returns (cols [R, K+1] int64 ascending, vals [R, K+1] float64[, diag [R, 64]]).
    """
    p = _points(points)
    r, nr = _rows_arg(rows, p.shape[0])
    cols = np.empty((nr, k + 1), dtype=np.int64)
    vals = np.empty((nr, k + 1), dtype=np.float64)
    dg = np.empty((nr, ODIAG), dtype=np.float64) if diag else None
    var = {"mvgd": 0, "ls": 1, "div": 2}[variant]
    use_h = 0 if h_override is None else 1
    rc = _load().oracle_rows(_ptr(p), p.shape[0], p.shape[1], d, k, var, use_h,
                             float(h_override or 0.0), float(weight_nbr), _ptr(r), nr,
                             _ptr(cols), _ptr(vals), _ptr(dg), nthreads)
    if rc == -2:
        raise ValueError("oracle_rows: non-finite coordinates")
    if rc != 0:
        raise ValueError(f"oracle_rows: invalid arguments ({rc})")
    return (cols, vals, dg) if diag else (cols, vals)


def assemble(points, k: int, d: int = 2, variant: str = "mvgd", h_override=None,
             nthreads: int = 0, weight_nbr: float = 1.0):
    """The whole matrix as CSR: (row_ptr int64 [N+1], cols int64 [nnz], vals float64 [nnz])."""
    cols, vals = rows(points, k, None, d=d, variant=variant, h_override=h_override,
                      nthreads=nthreads, weight_nbr=weight_nbr)
    n = cols.shape[0]
    row_ptr = np.arange(n + 1, dtype=np.int64) * (k + 1)
    return row_ptr, cols.reshape(-1), vals.reshape(-1)


def apply(row_ptr, cols, vals, x):
    """y = L x (x: [N] or [N, R])."""
    x = np.asarray(x, dtype=np.float64)
    squeeze = x.ndim == 1
    x2 = np.ascontiguousarray(x.reshape(x.shape[0], -1))
    n = row_ptr.shape[0] - 1
    y = np.empty((n, x2.shape[1]), dtype=np.float64)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    _load().oracle_apply(n, _ptr(rp), _ptr(c), _ptr(v), x2.shape[1], _ptr(x2), _ptr(y))
    return y[:, 0] if squeeze else y


def lb_coefficients(a, d: int = 2):
    """O8 alone: inverse metric G (d x d) and drift q (d) from the unscaled fit coefficients.

    a: [n_codim, 6] (d = 2: a00, a10, a01, a20, a11, a02) or [n_codim, 3] (d = 1).
    """
    a = np.ascontiguousarray(np.atleast_2d(a), dtype=np.float64)
    G = np.empty(d * d)
    q = np.empty(d)
    rc = _load().oracle_lb_coefficients(d, a.shape[0], _ptr(a), _ptr(G), _ptr(q))
    if rc != 0:
        raise ValueError("degenerate metric")
    return G.reshape(d, d), q


def row_stats(row_ids, cols, vals):
    """Sign statistics of matrix rows (the property Sec. 3.2 argues for: the centre modification
    pushes the off-diagonal entries to the sign opposite to the negative diagonal, towards
    an M-matrix -L, where plain least-squares rows have off-diagonal entries of mixed sign).

    row_ids [R]: the row index of each row; cols/vals [R, K+1]: the row's columns (ascending,
    containing row_ids[r] once) and values. Per row, with d the diagonal value and o_j the
    off-diagonal values in column order:
      neg_mass = sum_j max(0, -o_j), one float64 addition per entry in column order;
      ratio    = neg_mass / |d| (NaN where d == 0; rows that sum to zero are diagonally
                 dominant exactly when ratio == 0);
      m_row    = d < 0 and every o_j >= 0.
    Returns (per-row dict of arrays, totals dict).
    """
    row_ids = np.asarray(row_ids, dtype=np.int64)
    cols = np.asarray(cols)
    vals = np.asarray(vals, dtype=np.float64)
    R = vals.shape[0]
    ratio = np.empty(R)
    m_row = np.zeros(R, dtype=bool)
    diag_neg = np.zeros(R, dtype=bool)
    n_off_neg = 0
    for r in range(R):
        on = cols[r] == row_ids[r]
        d = float(vals[r][on][0])
        off = vals[r][~on]
        neg = 0.0
        for v in off:
            neg += max(0.0, -float(v))
        ratio[r] = neg / abs(d) if d != 0.0 else np.nan
        diag_neg[r] = d < 0.0
        m_row[r] = d < 0.0 and bool((off >= 0.0).all())
        n_off_neg += int((off < 0.0).sum())
    ok = ~np.isnan(ratio)
    totals = {"n_rows": R, "n_diag_negative": int(diag_neg.sum()), "n_m_rows": int(m_row.sum()),
              "n_offdiag_negative": n_off_neg,
              "max_ratio": float(ratio[ok].max()) if ok.any() else 0.0,
              "mean_ratio": float(ratio[ok].mean()) if ok.any() else 0.0}
    return {"ratio": ratio, "m_row": m_row, "diag_negative": diag_neg}, totals


def solve(row_ptr, cols, vals, b, sigma: float = 0.0, pinned=()):
    """Exact solution of A x = b with A = sigma I - L (L the CSR matrix), where every row listed
    in `pinned` is replaced by the identity row (x_p = b_p): the systems of Sec. 4 (-Delta U = f
    with sigma = 0 and one pinned value on a closed manifold). Sparse LU (SuperLU via scipy) as
    the one library step; returns float64 [N]."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    n = len(row_ptr) - 1
    L = sp.csr_matrix((np.asarray(vals, dtype=np.float64), np.asarray(cols),
                       np.asarray(row_ptr)), shape=(n, n))
    A = (sigma * sp.identity(n, format="csr") - L).tocsr()
    keep = np.ones(n)
    keep[list(pinned)] = 0.0
    A = sp.diags(keep) @ A + sp.diags(1.0 - keep)
    return spla.spsolve(A.tocsc(), np.asarray(b, dtype=np.float64))


def eigenvalues(row_ptr, cols, vals, nev: int, keep=None):
    """The nev eigenvalues of -L with the smallest real parts (Sec. 4: -Delta nu = lambda nu),
    sorted by real part, with L the CSR matrix restricted to the rows and columns in `keep` (all by
    default; removing boundary points gives the Dirichlet problem, removing ghost rows the
    Neumann one). Dense eigenvalues of the nonsymmetric matrix (LAPACK via numpy) as the one
    library step."""
    import scipy.sparse as sp
    n = len(row_ptr) - 1
    A = -sp.csr_matrix((np.asarray(vals, dtype=np.float64), np.asarray(cols),
                        np.asarray(row_ptr)), shape=(n, n)).toarray()
    if keep is not None:
        keep = np.asarray(keep)
        A = A[np.ix_(keep, keep)]
    ev = np.linalg.eigvals(A)
    order = np.lexsort((ev.imag, ev.real))
    return ev[order][:nev]


def neumann_ghosts(points, boundary, k: int, k_boundary: int):
    """Ghost points of the reflection method for the Neumann condition on an open surface in R^3
    (Sec. 3.1), step by step:

    * interior points P^I (boundary == False), boundary points P^B;
    * an interior point gets a ghost if one of its K nearest neighbours in the whole cloud is a
      boundary point (O1 kNN);
    * p^B_j = its closest boundary point (FP64 squared distance, ties to the smaller index);
    * at p^B_j: the boundary curve through its k_boundary nearest boundary points (p^B_j
      included) as (xi, eta(xi), zeta(xi)) in their PCA frame, quadratic least squares; its
      tangent at p^B_j is e1 = (1, eta'(xi_j), zeta'(xi_j)) back in ambient coordinates,
      normalised; e2 = the surface normal, the smallest-eigenvalue eigenvector of the covariance
      of the K nearest neighbours of p^B_j in the whole cloud; e3 = e1 x e2 (normalised);
    * the ghost is the mirror image p^R = p^I - 2 ((p^I - p^B_j) . e3) e3.

    Returns (interior indices [NI], ghost points [NG, 3], ghost source = index into the interior
    list [NG], ghost boundary point index [NG]); ghosts are listed in the order of their source.
    """
    P = _points(points)
    B = np.asarray(boundary, dtype=bool)
    n = P.shape[0]
    interior = np.nonzero(~B)[0]
    bidx = np.nonzero(B)[0]
    nbr, _ = knn(P, k)
    has_b = B[nbr].any(axis=1)
    src_i = [r for r, i in enumerate(interior) if has_b[i]]
    PB = P[bidx]
    # the frames at the boundary points that are used
    frames = {}

    def frame(j):
        if j in frames:
            return frames[j]
        d2 = ((PB - PB[j]) ** 2).sum(1)
        order = np.lexsort((np.arange(len(PB)), d2))[:k_boundary]
        Q = PB[order]
        c = Q.mean(0)
        w, V = np.linalg.eigh((Q - c).T @ (Q - c))
        t, n1, n2 = V[:, 2], V[:, 1], V[:, 0]
        xi = (Q - PB[j]) @ t
        A = np.stack([np.ones_like(xi), xi, xi * xi], 1)
        ce = np.linalg.lstsq(A, (Q - PB[j]) @ n1, rcond=None)[0]
        cz = np.linalg.lstsq(A, (Q - PB[j]) @ n2, rcond=None)[0]
        e1 = t + ce[1] * n1 + cz[1] * n2  # derivative of the fitted curve at xi = 0 (p^B_j)
        e1 /= np.linalg.norm(e1)
        nb = nbr[bidx[j]]
        D = P[nb] - P[nb].mean(0)
        e2 = np.linalg.eigh(D.T @ D)[1][:, 0]
        e3 = np.cross(e1, e2)
        e3 /= np.linalg.norm(e3)
        frames[j] = e3
        return e3

    ghosts, bsrc = [], []
    for r in src_i:
        p = P[interior[r]]
        d2 = ((PB - p) ** 2).sum(1)
        j = int(np.lexsort((np.arange(len(PB)), d2))[0])
        e3 = frame(j)
        ghosts.append(p - 2.0 * np.dot(p - PB[j], e3) * e3)
        bsrc.append(bidx[j])
    return (interior, np.array(ghosts).reshape(-1, 3), np.array(src_i, dtype=np.int64),
            np.array(bsrc, dtype=np.int64))


def neumann_rows(points, boundary, k: int, k_boundary: int, ghosts=None, nthreads: int = 0):
    """MVGD rows of the interior points with the homogeneous Neumann condition (Sec. 3.1): the
    rows of the augmented cloud P^I u P^R, every ghost column folded into its source interior
    point (U(p^R) = U(p^I) when the normal derivative is zero). `ghosts` (the output of
    neumann_ghosts) may be given to assemble on exactly those ghost points.
    Returns (row_ptr, cols, vals) over the NI interior points, columns = interior list indices
    (a folded ghost shares its source's column; duplicates are merged), plus the ghost tuple."""
    P = _points(points)
    g = neumann_ghosts(P, boundary, k, k_boundary) if ghosts is None else ghosts
    interior, G, src = g[0], g[1], g[2]
    ni = len(interior)
    A = np.concatenate([P[interior], G]) if len(G) else P[interior]
    cols, vals = rows(A, k, rows=np.arange(ni), nthreads=nthreads)
    fold = np.concatenate([np.arange(ni), src])
    rp, cc, vv = [0], [], []
    for r in range(ni):
        merged = {}
        for c, v in zip(fold[cols[r]], vals[r]):
            merged[int(c)] = merged.get(int(c), 0.0) + v
        keys = sorted(merged)
        cc.extend(keys)
        vv.extend(merged[c] for c in keys)
        rp.append(len(cc))
    return np.array(rp, dtype=np.int64), np.array(cc, dtype=np.int64), np.array(vv), g
