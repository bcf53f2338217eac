"""GPU path (HIP, through the C ABI) against the FP64 oracle, element by element.

Bars (the targets of the build):
* kNN sets and CSR sparsity: bit-exact (columns identical).
* FP64 mode: row-relative error max_j |L_gpu - L_oracle| / max_j |L_oracle| <= 1e-12.
  Exception derived from the arithmetic: the in-plane PCA axes fix h, and rounding of the
  covariance (~1e-16 relative) rotates them by ~1e-16/gap, gap = (lam1 - lam2)/lam1; so rows
  get tol = max(1e-12, 4e-15 / gap). Rows with gap < 4e-3 are the only ones it widens.
  Likewise both sides are backward-stable solvers of the same least-squares problem and agree
  to O(kappa(V) u): the bound adds 64 u kappa, kappa = the 2-norm condition number of the
  oracle's design V (rebuilt from its frame and h); it matters only for kappa > ~140, i.e.
  nearly square designs (K = 5).
* FP32-mixed mode: the oracle runs on the same FP32-rounded coordinates; rows <= 1e-4.
* Apply: y = L x against the exported CSR times x in FP64 (accumulation in double on the GPU).
Every case prints its L.f error against the FP64 oracle.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1603_04100_amd import clouds

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def mv():
    from paper_1603_04100_amd import mvgd
    return mvgd


def _gpu_csr(mv, pts, k, precision, offsets=None, **kw):
    dt = torch.float64 if precision == "fp64" else torch.float32
    P = torch.tensor(pts, dtype=dt, device=DEV)
    L = mv.mvgd_assemble(P, k, precision=precision, cloud_offsets=offsets, **kw)
    rp, col, val = mv.mvgd_csr(L)
    info = mv.mvgd_info(L)
    torch.cuda.synchronize()
    return L, P, rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy().astype(np.float64), info


def _oracle_points(pts, precision):
    return pts.astype(np.float32).astype(np.float64) if precision == "fp32" else pts


def _kappa(pts, rows, cols, dg, w_nbr=1.0, d=2):
    """2-norm condition number of each row's (weighted) design W^1/2 V (centre row, then N(i)),
    from the oracle's frame and spacing."""
    n = pts.shape[1]
    i = np.asarray(rows)
    nb = cols[cols != i[:, None]].reshape(len(i), -1)
    F = dg[:, 6:22].reshape(-1, 4, 4)[:, :d, :n]
    u = np.einsum("rkn,rtn->rkt", pts[nb] - pts[i][:, None, :], F) / dg[:, 0][:, None, None]
    if d == 2:
        x, y = u[..., 0], u[..., 1]
        V = np.stack([np.ones_like(x), x, y, x * x, x * y, y * y], -1) * np.sqrt(w_nbr)
    else:
        x = u[..., 0]
        V = np.stack([np.ones_like(x), x, x * x], -1) * np.sqrt(w_nbr)
    m = V.shape[-1]
    V = np.concatenate([np.eye(m)[None, :1, :].repeat(len(i), 0), V], 1)
    s = np.linalg.svd(V, compute_uv=False)
    return s[:, 0] / s[:, -1]


def _row_tol(precision, dg, kappa):
    """Per-row bound from the oracle's diagnostics (in-plane gap) and kappa(V)."""
    gap = (dg[:, 2] - dg[:, 3]) / dg[:, 2]
    if precision == "fp32":
        return np.maximum(1e-4, 64 * 2.0 ** -24 * kappa)
    return np.maximum(1e-12, 4e-15 / np.maximum(gap, 1e-300) + 64 * 2.0 ** -53 * kappa)


def _compare_rows(g_cols, g_vals, o_cols, o_vals, tol):
    assert (g_cols == o_cols).all(), "kNN / sparsity differ"
    scale = np.abs(o_vals).max(1)
    err = np.abs(g_vals - o_vals).max(1)
    zero = scale == 0
    assert (err[zero] == 0).all(), "degenerate rows must be zero on both sides"
    rel = np.where(zero, 0.0, err / np.where(zero, 1.0, scale))
    bad = np.nonzero(rel > tol)[0]
    assert bad.size == 0, f"{bad.size} rows over tolerance, worst {rel.max():.3e} at {bad[:5]}"
    return rel


def _lf_error(mv, L, P, f, o_rp, o_cols, o_vals, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    y = mv.mvgd_apply(L, torch.tensor(f, dtype=dt, device=DEV)).cpu().numpy().astype(np.float64)
    ref = oracle.apply(o_rp, o_cols, o_vals, f)
    return np.abs(y - ref).max() / np.abs(ref).max(), y


def _full_case(mv, cl, precision, **kw):
    pts = cl.points
    k = cl.k
    n = pts.shape[0]
    L, P, rp, col, val, info = _gpu_csr(mv, pts, k, precision, **kw)
    opts = _oracle_points(pts, precision)
    flags = kw.get("flags", 0)
    d = kw.get("d_manifold", 2)
    w_nbr = 1.0 / k if flags & mv.MVGD_FLAG_MLS else 1.0
    variant = ("ls" if flags & mv.MVGD_FLAG_LS else
               "div" if flags & mv.MVGD_FLAG_DIVERGENCE else "mvgd")
    o_cols, o_vals, dg = oracle.rows(opts, k, diag=True, weight_nbr=w_nbr, variant=variant, d=d)
    kap = _kappa(opts, np.arange(n), o_cols, dg, w_nbr, d)
    rel = _compare_rows(col.reshape(n, k + 1), val.reshape(n, k + 1), o_cols, o_vals,
                        _row_tol(precision, dg, kap))
    assert (rp == np.arange(n + 1) * (k + 1)).all()
    o_rp = np.arange(n + 1, dtype=np.int64) * (k + 1)
    lf, y = _lf_error(mv, L, P, cl.f[:, 0], o_rp, o_cols.reshape(-1), o_vals.reshape(-1), precision)
    print(f"\n[{cl.name} N={n} K={k} {precision}] max row rel err {rel.max():.2e} "
          f"(max kappa(V) {kap.max():.1f}, min gap {((dg[:, 2] - dg[:, 3]) / dg[:, 2]).min():.1e}), "
          f"L.f rel err vs FP64 oracle {lf:.2e}, max|Lf - Delta f| {np.abs(y - cl.lap_f[:, 0]).max():.3e}, "
          f"degenerate {info['n_degenerate']}, slow-knn {info['n_slow_knn']}")
    return L, P, col, val, rel, lf, info


# ----------------------------------------------------------------------------------------------
# whole matrices at sizes the oracle finishes in seconds (several tiles and a ragged tail)
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sphere_2k(mv, precision):
    cl = clouds.sphere(2000, 1, 20)
    L, P, col, val, rel, lf, info = _full_case(mv, cl, precision)
    v = val.reshape(2000, 21)
    assert np.all(np.abs(v.sum(1)) <= (1e-12 if precision == "fp64" else 1e-5) * np.abs(v).sum(1))
    assert info["n_degenerate"] == 0
    L.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_torus_nonuniform(mv, precision):
    cl = clouds.torus(20_037, 2, 24)
    L, *_ = _full_case(mv, cl, precision)
    L.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_flat_torus_r4(mv, precision):
    cl = clouds.flat_torus4(30_001, 4, 32)
    L, *_ = _full_case(mv, cl, precision)
    L.free()


@pytest.mark.parametrize("k", [5, 12, 63])
def test_k_range_and_tiny_clouds(mv, k):
    cl = clouds.sphere(k + 1 + 70, 9, k)
    L, *_ = _full_case(mv, cl, "fp64")
    L.free()
    cl = clouds.sphere(k + 1, 10, k)  # minimal cloud: every other point is a neighbour
    L, *_ = _full_case(mv, cl, "fp64")
    L.free()


def test_ls_variant_and_h_override(mv):
    cl = clouds.sphere(3000, 17, 20)
    L, *_ = _full_case(mv, cl, "fp64", flags=mv.MVGD_FLAG_LS)
    L.free()
    pts = cl.points
    P = torch.tensor(pts, device=DEV)
    L = mv.mvgd_assemble(P, 20, h_override=0.05)
    rp, col, val = mv.mvgd_csr(L)
    oc, ov, dg = oracle.rows(pts, 20, h_override=0.05, diag=True)
    _compare_rows(col.cpu().numpy().reshape(-1, 21), val.cpu().numpy().reshape(-1, 21), oc, ov,
                  _row_tol("fp64", dg, _kappa(pts, np.arange(3000), oc, dg)))
    L.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", ["mvgd", "ls"])
def test_mls_weights(mv, precision, variant):
    """Weighted fits (1 at p_i, 1/K at the neighbours), with and without the centre term."""
    cl = clouds.torus(5000, 23, 24) if variant == "mvgd" else clouds.sphere(3000, 24, 20)
    flags = mv.MVGD_FLAG_MLS | (mv.MVGD_FLAG_LS if variant == "ls" else 0)
    L, *_ = _full_case(mv, cl, precision, flags=flags)
    L.free()


def _stats_of_export(mv, L, n, k, offs=None):
    """The row statistics' definition applied to the library's own exported rows (columns are
    local to each cloud)."""
    rp, col, val = mv.mvgd_csr(L)
    col = col.cpu().numpy().reshape(n, k + 1)
    val = val.cpu().numpy().astype(np.float64).reshape(n, k + 1)
    offs = [0, n] if offs is None else offs
    local = np.concatenate([np.arange(b - a) for a, b in zip(offs[:-1], offs[1:])])
    return oracle.row_stats(local, col, val)


@pytest.mark.parametrize("case", ["sphere-mvgd", "sphere-ls", "torus-mls", "batch-fp32",
                                  "degenerate"])
def test_row_stats_match_definition(mv, case):
    """GPU statistics equal the definition evaluated on the same matrix: counts and per-row
    ratios bit-identical (same order of additions), mean within rounding of the reduction."""
    offs = None
    if case.startswith("sphere"):
        cl = clouds.sphere(3000, 31, 20)
        P = torch.tensor(cl.points, device=DEV)
        flags = mv.MVGD_FLAG_LS if case.endswith("ls") else 0
    elif case == "torus-mls":
        cl = clouds.torus(6000, 32, 24)
        P = torch.tensor(cl.points, device=DEV)
        flags = mv.MVGD_FLAG_MLS
    elif case == "batch-fp32":
        cl = clouds.ellipsoid_batch(n_clouds=4, seed=33, k=20, n_min=500, n_max=5000)
        P = torch.tensor(cl.points.astype(np.float32), device=DEV)
        offs = [int(v) for v in cl.offsets]
        flags = mv.MVGD_FLAG_MLS
    else:
        rng = np.random.default_rng(34)
        base = clouds.sphere(1000, 35, 16).points
        pts = np.concatenate([base, np.repeat(base[:3], 20, 0)])  # clusters of duplicates
        cl = clouds.Cloud("dups", pts, np.array([0, len(pts)]), 16, None, None, {})
        P = torch.tensor(pts[rng.permutation(len(pts))], device=DEV)
        flags = 0
    n, k = P.shape[0], cl.k
    L = mv.mvgd_assemble(P, k, flags=flags, cloud_offsets=offs)
    got, ratio = mv.mvgd_row_stats(L, ratio=True)
    per, tot = _stats_of_export(mv, L, n, k, offs)
    for key in ("n_rows", "n_diag_negative", "n_m_rows", "n_offdiag_negative"):
        assert got[key] == tot[key], key
    r = ratio.cpu().numpy()
    assert np.array_equal(np.isnan(r), np.isnan(per["ratio"]))
    ok = ~np.isnan(r)
    assert (r[ok] == per["ratio"][ok]).all()
    assert got["n_zero_diagonal"] == int((~ok).sum())
    assert got["max_ratio"] == tot["max_ratio"]
    assert got["mean_ratio"] == pytest.approx(tot["mean_ratio"], rel=1e-12, abs=1e-300)
    if case == "degenerate":
        assert got["n_zero_diagonal"] > 0
    L.free()


def test_row_stats_paper_claim_on_the_gpu(mv):
    """The centre modification cuts the negative off-diagonal mass (FP32-mixed, torus), and with
    the MLS weights most MVGD rows are M-rows while almost no LS rows are; per-row M decisions
    agree with the FP64 oracle's wherever the smallest off-diagonal is clear of zero."""
    cl = clouds.torus(8000, 36, 24)
    P = torch.tensor(cl.points.astype(np.float32), device=DEV)
    res = {}
    for name, flags in (("mvgd", 0), ("ls", mv.MVGD_FLAG_LS), ("mvgd-mls", mv.MVGD_FLAG_MLS),
                        ("ls-mls", mv.MVGD_FLAG_LS | mv.MVGD_FLAG_MLS)):
        L = mv.mvgd_assemble(P, 24, flags=flags)
        res[name] = mv.mvgd_row_stats(L)
        if name == "mvgd-mls":
            rp, col, val = mv.mvgd_csr(L)
            gv = val.cpu().numpy().astype(np.float64).reshape(-1, 25)
            opts = cl.points.astype(np.float32).astype(np.float64)
            oc, ov = oracle.rows(opts, 24, weight_nbr=1.0 / 24)
            ids = np.arange(cl.n_points)
            g_m = oracle.row_stats(ids, col.cpu().numpy().reshape(-1, 25), gv)[0]["m_row"]
            o_m = oracle.row_stats(ids, oc, ov)[0]["m_row"]
            off = np.where(oc == ids[:, None], np.inf, np.abs(ov))
            clear = off.min(1) > 1e-3 * np.abs(ov).max(1)
            assert (g_m[clear] == o_m[clear]).all()
            assert clear.mean() > 0.8
        L.free()
    n = cl.n_points
    assert res["mvgd"]["mean_ratio"] < 0.1 * res["ls"]["mean_ratio"]
    assert res["mvgd-mls"]["n_m_rows"] > 0.3 * n and res["ls-mls"]["n_m_rows"] < 0.01 * n
    print(f"\n[row stats torus 8k fp32] " + ", ".join(
        f"{k}: M-rows {v['n_m_rows']}/{n}, mean ratio {v['mean_ratio']:.4f}" for k, v in res.items()))


# ----------------------------------------------------------------------------------------------
# curves (d = 1): centred and divergence forms, plain LS, MLS weights
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["circle-mvgd", "circle-div", "helix-mvgd", "helix-div",
                                  "helix-ls-mls", "circle-uniform-mvgd"])
def test_curves(mv, precision, case):
    if case.startswith("circle"):
        cl = clouds.circle(4000, 61, 6, sampling="uniform" if "uniform" in case else "random")
    else:
        cl = clouds.helix(5000, 62, 8)
    flags = {"mvgd": 0, "div": mv.MVGD_FLAG_DIVERGENCE,
             "mls": mv.MVGD_FLAG_LS | mv.MVGD_FLAG_MLS}[case.split("-")[-1]]
    L, *_ = _full_case(mv, cl, precision, flags=flags, d_manifold=1)
    L.free()


def test_curve_worked_example_on_the_gpu(mv):
    """The paper's 5-point example (K = 4): rows (4, 19, -46, 19, 4)/35k^2 (MVGD, and the
    divergence form on a straight line) and (2, -1, -2, -1, 2)/7k^2 (LS), in any direction."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example_1d.json")))
    for n_amb, k in ((2, 0.5), (3, 0.1)):
        p = clouds.line_example(k, n_amb, direction=np.arange(1, n_amb + 1, dtype=float))
        P = torch.tensor(p, device=DEV)
        for flags, key, den in ((0, "mvgd_row_at_h_eq_k_times_35k2", 35.0),
                                (mv.MVGD_FLAG_DIVERGENCE, "mvgd_row_at_h_eq_k_times_35k2", 35.0),
                                (mv.MVGD_FLAG_LS, "ls_row_times_7k2", 7.0)):
            L = mv.mvgd_assemble(P, 4, d_manifold=1, flags=flags)
            rp, col, val = mv.mvgd_csr(L)
            row = val.cpu().numpy().reshape(5, 5)[2]
            want = np.array(g[key]) / (den * k * k)
            assert list(col.cpu().numpy().reshape(5, 5)[2]) == [0, 1, 2, 3, 4]
            np.testing.assert_allclose(row, want, rtol=0, atol=1e-12 * np.abs(want).max())
            L.free()


def test_curve_converges_on_the_gpu(mv):
    """Unit circle, random sampling, FP64: the rms of Lf - Delta f falls with the sampling
    density in both forms (the oracle's convergence pin, same inputs). FP64 because random
    sampling puts near-coincident points on the curve: h and the row weights (~1/h^2) then span
    many orders of magnitude, and float storage of the weights costs ~2^-24 sum_j |w_j f_j|."""
    for flags in (0, mv.MVGD_FLAG_DIVERGENCE):
        errs = []
        for n in (500, 2000, 8000):
            t = np.random.default_rng(n).uniform(0, 2 * np.pi, n)
            P = torch.tensor(np.stack([np.cos(t), np.sin(t)], 1), device=DEV)
            L = mv.mvgd_assemble(P, 6, d_manifold=1, flags=flags)
            y = mv.mvgd_apply(L, torch.tensor(np.sin(2 * t), device=DEV))
            e = y.cpu().numpy() + 4 * np.sin(2 * t)
            errs.append(np.sqrt((e ** 2).mean()))
            L.free()
        assert errs[0] / errs[2] > 4.0, errs


# ----------------------------------------------------------------------------------------------
# iterative solves on the device against the exact (sparse LU) solution of the same system
# ----------------------------------------------------------------------------------------------
def _export_csr(mv, L, n, k):
    rp, col, val = mv.mvgd_csr(L)
    return (rp.cpu().numpy(), col.cpu().numpy().astype(np.int64),
            val.cpu().numpy().astype(np.float64))


def _cond_bound(rp, c, v, sigma, pinned):
    """2-norm condition number of A = sigma I - L with pinned identity rows (dense SVD)."""
    import scipy.sparse as sp
    n = len(rp) - 1
    A = (sigma * sp.identity(n) - sp.csr_matrix((v, c, rp), shape=(n, n))).toarray()
    A[pinned] = 0.0
    A[pinned, pinned] = 1.0
    sv = np.linalg.svd(A, compute_uv=False)
    return sv[0] / sv[-1]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bicgstab_sphere_poisson(mv, precision):
    """-Delta U = 2x on the unit sphere (Sec. 4.2), one pinned value: BiCGSTAB on the device
    agrees with the exact solution of the same (exported) matrix to kappa(A) times the residual,
    and the solution approaches x."""
    cl = clouds.sphere(2000, 5, 20)
    dt = torch.float64 if precision == "fp64" else torch.float32
    P = torch.tensor(cl.points, dtype=dt, device=DEV)
    L = mv.mvgd_assemble(P, 20)
    pts = _oracle_points(cl.points, precision)
    b = 2.0 * pts[:, 0]
    b[0] = pts[0, 0]
    rtol = 1e-12 if precision == "fp64" else 1e-6
    x, info = mv.mvgd_solve(L, torch.tensor(b, dtype=dt, device=DEV), rtol=rtol, max_iter=3000,
                            pin_first=True)
    assert info["converged"] == 1, info
    assert info["rel_residual"] <= rtol  # convergence is judged by the true residual
    rp, c, v = _export_csr(mv, L, 2000, 20)
    ref = oracle.solve(rp, c, v, b, sigma=0.0, pinned=[0])  # b is exact in either dtype
    kappa = _cond_bound(rp, c, v, 0.0, [0])
    got = x.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    store = 0.0 if precision == "fp64" else 2.0 ** -24  # the returned x is rounded to float
    assert rel <= 10 * kappa * info["rel_residual"] + 4 * store, (rel, kappa, info)
    assert np.abs(got - cl.points[:, 0]).max() < 5e-3
    print(f"\n[bicgstab sphere 2k {precision}] {info}, kappa(A) {kappa:.3e}, |x - x_LU|/|x_LU| "
          f"{rel:.2e}, max|x - x_exact| {np.abs(got - cl.points[:, 0]).max():.2e}")
    # reproducible: the same solve twice gives the same bits
    x2, info2 = mv.mvgd_solve(L, torch.tensor(b, dtype=dt, device=DEV), rtol=rtol, max_iter=3000,
                              pin_first=True)
    assert torch.equal(x, x2) and info == info2
    L.free()


def test_bicgstab_converges_by_the_true_residual(mv):
    """A long BiCGSTAB run (100k points, tight tolerance): the returned iterate's recomputed
    residual meets the tolerance whenever convergence is reported (restarts absorb the drift of
    the recursive residual), and the solution approaches x."""
    cl = clouds.sphere(100_000, 5, 20)
    L = mv.mvgd_assemble(torch.tensor(cl.points, device=DEV), 20)
    b = 2.0 * cl.points[:, 0]
    b[0] = cl.points[0, 0]
    rtol = 1e-11
    x, info = mv.mvgd_solve(L, torch.tensor(b, device=DEV), rtol=rtol, max_iter=30000,
                            pin_first=True, check_every=50)
    assert info["converged"] == 1 and info["rel_residual"] <= rtol, info
    assert np.abs(x.cpu().numpy() - cl.points[:, 0]).max() < 2e-4
    print(f"\n[bicgstab sphere 100k fp64 rtol {rtol}] {info}")
    L.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bicgstab_hemisphere_dirichlet(mv, precision):
    """Dirichlet points (identity rows at the sampled boundary circle) on the upper hemisphere:
    -Delta U = 2z, U = 0 on the boundary; the device solution matches the sparse-LU solution of
    the same matrix and approaches U = z."""
    cl = clouds.hemisphere(4000, 8, 20)
    dt = torch.float64 if precision == "fp64" else torch.float32
    pts = _oracle_points(cl.points, precision)
    m = cl.meta["boundary"]
    P = torch.tensor(cl.points, dtype=dt, device=DEV)
    L = mv.mvgd_assemble(P, 20)
    b = 2.0 * pts[:, 2]
    b[m] = 0.0
    rtol = 1e-12 if precision == "fp64" else 1e-6
    x, info = mv.mvgd_solve(L, torch.tensor(b, dtype=dt, device=DEV), rtol=rtol, max_iter=4000,
                            fixed=torch.tensor(m, device=DEV))
    assert info["converged"] == 1, info
    rp, c, v = _export_csr(mv, L, cl.n_points, 20)
    ref = oracle.solve(rp, c, v, b, pinned=np.nonzero(m)[0])
    got = x.cpu().numpy().astype(np.float64)
    assert np.abs(got[m]).max() <= 1e-12
    kappa = _cond_bound(rp, c, v, 0.0, np.nonzero(m)[0])
    store = 0.0 if precision == "fp64" else 2.0 ** -24
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= 10 * kappa * info["rel_residual"] + 4 * store, (rel, kappa, info)
    assert np.abs(got - cl.points[:, 2]).max() < 5e-4
    print(f"\n[dirichlet hemisphere 4k {precision}] {info}, kappa {kappa:.2e}, rel err {rel:.2e}, "
          f"max|x - z| {np.abs(got - cl.points[:, 2]).max():.2e}")
    L.free()


def test_jacobi_screened_and_batched(mv):
    """Damped Jacobi on (sigma I - L) x = b, sigma = 1000, two clouds in one handle (a pinned
    first point in each): agrees with the exact block solution."""
    cl = clouds.ellipsoid_batch(n_clouds=2, seed=41, k=20, n_min=1500, n_max=3000)
    offs = [int(v) for v in cl.offsets]
    n = cl.n_points
    P = torch.tensor(cl.points, device=DEV)
    L = mv.mvgd_assemble(P, 20, cloud_offsets=offs)
    b = np.sin(3 * cl.points[:, 0]) + cl.points[:, 1]
    x, info = mv.mvgd_solve(L, torch.tensor(b, device=DEV), method="jacobi", sigma=1000.0,
                            rtol=1e-11, max_iter=20000, pin_first=True, check_every=200)
    assert info["converged"] == 1, info
    rp, c, v = _export_csr(mv, L, n, 20)
    # columns of the export are local to each cloud: solve block by block
    ref = np.empty(n)
    for a, e in zip(offs[:-1], offs[1:]):
        ref[a:e] = oracle.solve(rp[a:e + 1] - rp[a], c[rp[a]:rp[e]], v[rp[a]:rp[e]], b[a:e],
                                sigma=1000.0, pinned=[0])
    got = x.cpu().numpy()
    assert got[offs[0]] == b[offs[0]] and got[offs[1]] == b[offs[1]]
    kappa = max(_cond_bound(rp[a:e + 1] - rp[a], c[rp[a]:rp[e]], v[rp[a]:rp[e]], 1000.0, [0])
                for a, e in zip(offs[:-1], offs[1:]))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= 10 * kappa * info["rel_residual"], (rel, kappa, info)
    print(f"\n[jacobi sigma=1000, 2 clouds] {info}, kappa {kappa:.2e}, rel err {rel:.2e}")
    L.free()


def test_solver_on_ls_rows_reports_failure(mv):
    """Plain least-squares rows (Sec. 4.1: not solvable by common iterative methods): Jacobi
    diverges and is reported as not converged (breakdown or max_iter), without an error."""
    cl = clouds.sphere(2000, 5, 20)
    P = torch.tensor(cl.points, device=DEV)
    L = mv.mvgd_assemble(P, 20, flags=mv.MVGD_FLAG_LS)
    b = torch.tensor(2.0 * cl.points[:, 0], device=DEV)
    x, info = mv.mvgd_solve(L, b, method="jacobi", max_iter=2000, rtol=1e-8, pin_first=True)
    assert info["converged"] != 1, info
    L.free()
    L = mv.mvgd_assemble(P, 20)  # the MVGD rows with the same smoother: residual decreases
    x, info2 = mv.mvgd_solve(L, b, method="jacobi", max_iter=2000, rtol=1e-8, pin_first=True)
    assert info2["converged"] != -1 and info2["rel_residual"] < 1.0, info2
    with pytest.raises(mv.MvgdError):
        mv.mvgd_solve(L, b, method="jacobi", omega=2.5)  # damping outside (0, 2)
    L.free()


def test_exact_ties_on_a_lattice(mv):
    """Planar lattice: many equal distances; the tie-break (smaller index) must match."""
    g = np.stack(np.meshgrid(np.arange(40), np.arange(30), indexing="ij"), -1).reshape(-1, 2)
    pts = np.concatenate([g * 0.5, np.zeros((g.shape[0], 1))], 1).astype(np.float64)
    pts = pts @ np.linalg.qr(np.random.default_rng(1).standard_normal((3, 3)))[0].T
    perm = np.random.default_rng(2).permutation(pts.shape[0])
    pts = np.ascontiguousarray(pts[perm])
    for precision in ("fp64", "fp32"):
        L, P, rp, col, val, info = _gpu_csr(mv, pts, 12, precision)
        oc, ov = oracle.rows(_oracle_points(pts, precision), 12)
        assert (col.reshape(-1, 13) == oc).all()
        L.free()


def test_duplicates_and_degenerate(mv):
    rng = np.random.default_rng(3)
    base = clouds.sphere(1500, 5, 16).points
    pts = np.concatenate([base, base[:200]])  # exact duplicates
    pts = np.ascontiguousarray(pts[rng.permutation(pts.shape[0])])
    L, *_ = _full_case(mv, clouds.Cloud("dups", pts, np.array([0, pts.shape[0]]), 16,
                                        pts[:, :1].copy(), np.full((pts.shape[0], 1), np.nan)),
                       "fp64")
    L.free()
    t = np.linspace(0, 1, 300)
    line = np.ascontiguousarray(np.stack([t, 2 * t, -t], 1))
    L, P, rp, col, val, info = _gpu_csr(mv, line, 8, "fp64")
    oc, ov = oracle.rows(line, 8)
    assert (col.reshape(-1, 9) == oc).all()
    assert (val == 0).all() and info["n_degenerate"] == 300
    L.free()


# ----------------------------------------------------------------------------------------------
# batched clouds: per-cloud parity, and batched == alone (bit-identical)
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_clouds(mv, precision):
    cl = clouds.ellipsoid_batch(n_clouds=6, seed=3, k=20, n_min=400, n_max=6000)
    pts, offs = cl.points, cl.offsets
    L, P, rp, col, val, info = _gpu_csr(mv, pts, 20, precision, offsets=list(offs))
    opts = _oracle_points(pts, precision)
    for c in range(len(offs) - 1):
        a, b = offs[c], offs[c + 1]
        oc, ov, dg = oracle.rows(opts[a:b], 20, diag=True)
        kap = _kappa(opts[a:b], np.arange(b - a), oc, dg)
        _compare_rows(col[a * 21:b * 21].reshape(-1, 21), val[a * 21:b * 21].reshape(-1, 21), oc,
                      ov, _row_tol(precision, dg, kap))
        L1, P1, rp1, col1, val1, _ = _gpu_csr(mv, np.ascontiguousarray(pts[a:b]), 20, precision)
        assert (col1 == col[a * 21:b * 21]).all()
        assert (val1 == val[a * 21:b * 21]).all()
        L1.free()
    # apply with 4 right-hand sides
    dt = torch.float64 if precision == "fp64" else torch.float32
    x = torch.tensor(cl.f, dtype=dt, device=DEV)
    y = mv.mvgd_apply(L, x).cpu().numpy().astype(np.float64)
    ref = np.stack([oracle.apply(rp, col.astype(np.int64) + np.repeat(offs[:-1], np.diff(offs) * 21),
                                 val, cl.f[:, r].astype(np.float32 if precision == "fp32" else np.float64))
                    for r in range(4)], 1)
    tol = 1e-13 if precision == "fp64" else 1e-6
    assert np.abs(y - ref).max() <= tol * np.abs(ref).max()
    L.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_tiny_clouds(mv, precision):
    """Many clouds smaller than a thread block of the binning (several clouds per wave and per
    block): the batch equals each cloud assembled alone, bit for bit, and a sample of rows
    matches the oracle."""
    cl = clouds.ellipsoid_batch(n_clouds=40, seed=11, k=10, n_min=24, n_max=300)
    pts, offs = cl.points, cl.offsets
    assert (np.diff(offs) < 256).sum() >= 20
    L, P, rp, col, val, info = _gpu_csr(mv, pts, 10, precision, offsets=list(offs))
    opts = _oracle_points(pts, precision)
    for c in range(len(offs) - 1):
        a, b = offs[c], offs[c + 1]
        L1, P1, rp1, col1, val1, _ = _gpu_csr(mv, np.ascontiguousarray(pts[a:b]), 10, precision)
        assert (col1 == col[a * 11:b * 11]).all()
        assert (val1 == val[a * 11:b * 11]).all()
        L1.free()
        if c % 8 == 0:
            oc, ov, dg = oracle.rows(opts[a:b], 10, diag=True)
            kap = _kappa(opts[a:b], np.arange(b - a), oc, dg)
            _compare_rows(col[a * 11:b * 11].reshape(-1, 11), val[a * 11:b * 11].reshape(-1, 11), oc,
                          ov, _row_tol(precision, dg, kap))
    L.free()


# ----------------------------------------------------------------------------------------------
# apply against the exported CSR, several right-hand-side counts
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nrhs", [1, 3, 8])
def test_apply_matches_exported_csr(mv, precision, nrhs):
    cl = clouds.torus(9_999, 21, 24)
    L, P, rp, col, val, info = _gpu_csr(mv, cl.points, 24, precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    x = torch.randn(cl.points.shape[0], nrhs, dtype=dt, device=DEV)
    y = mv.mvgd_apply(L, x).cpu().numpy().astype(np.float64)
    ref = oracle.apply(rp, col.astype(np.int64), val, x.cpu().numpy().astype(np.float64))
    tol = 1e-13 if precision == "fp64" else 2e-7
    assert np.abs(y - ref).max() <= tol * np.abs(ref).max() * 10
    L.free()


def test_determinism(mv):
    cl = clouds.flat_torus4(20_000, 8, 32)
    a = _gpu_csr(mv, cl.points, 32, "fp32")
    b = _gpu_csr(mv, cl.points, 32, "fp32")
    assert (a[3] == b[3]).all() and (a[4] == b[4]).all()
    a[0].free()
    b[0].free()


# ----------------------------------------------------------------------------------------------
# full-size workloads, in the launch configuration the benchmark times: sampled rows
# ----------------------------------------------------------------------------------------------
def _sampled(mv, cl, precision, n_rows=600):
    pts, k = cl.points, cl.k
    n = pts.shape[0]
    L, P, rp, col, val, info = _gpu_csr(mv, pts, k, precision)
    rows = np.random.default_rng(0).choice(n, n_rows, replace=False)
    opts = _oracle_points(pts, precision)
    oc, ov, dg = oracle.rows(opts, k, rows=rows, diag=True)
    rel = _compare_rows(col.reshape(n, k + 1)[rows], val.reshape(n, k + 1)[rows], oc, ov,
                        _row_tol(precision, dg, _kappa(opts, rows, oc, dg)))
    v = val.reshape(n, k + 1)
    rs = np.abs(v.sum(1)) / np.abs(v).sum(1)
    y = mv.mvgd_apply(L, torch.tensor(cl.f[:, 0], dtype=P.dtype, device=DEV)).cpu().numpy()
    ref = (ov * cl.f[oc, 0]).sum(1)  # oracle rows applied to f, FP64
    lf = np.abs(ref - y[rows]).max() / np.abs(ref).max()
    print(f"\n[{cl.name} N={n} {precision} sampled {n_rows}] max row rel err {rel.max():.2e}, "
          f"L.f rel err (sampled rows) {lf:.2e}, max row-sum/|row| {rs.max():.1e}, "
          f"max|Lf - Delta f| {np.abs(y - cl.lap_f[:, 0]).max():.3e}, slow-knn {info['n_slow_knn']}")
    assert info["n_degenerate"] == 0
    L.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_torus_200k_sampled(mv, precision):
    _sampled(mv, clouds.torus(200_000, 2, 24), precision)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_flat_torus_1m_sampled(mv, precision):
    _sampled(mv, clouds.flat_torus4(1_000_000, 4, 32), precision, n_rows=400)


@pytest.mark.parametrize("name", ["flat_torus4_1m", "torus_200k", "ellipsoids_256",
                                  "flat_torus4_1m-fp64"])
def test_tile_search_full_size_equals_group(mv, name):
    """At the benchmark sizes the tile search gives the group search's matrix bit for bit (the
    group search is compared with the oracle above)."""
    name, _, prec = name.partition("-")
    cl = clouds.config(name)
    P = torch.tensor(cl.points.astype(np.float64 if prec == "fp64" else np.float32), device=DEV)
    offs = [int(v) for v in cl.offsets] if cl.offsets.shape[0] > 2 else None
    res = []
    for search in (mv.MVGD_SEARCH_GROUP, mv.MVGD_SEARCH_TILE):
        L = mv.mvgd_assemble(P, cl.k, cloud_offsets=offs, tuning={"search": search, "launch": 2})
        rp, col, val = mv.mvgd_csr(L)
        res.append((col, val, mv.mvgd_info(L)))
        L.free()
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])
    print(f"\n[{name} tile == group] slow-knn group {res[0][2]['n_slow_knn']}, "
          f"tile {res[1][2]['n_slow_knn']}")


# ----------------------------------------------------------------------------------------------
# error paths on the device
# ----------------------------------------------------------------------------------------------
def test_nonfinite_points_rejected(mv):
    pts = clouds.sphere(500, 1, 10).points.copy()
    pts[17, 2] = np.nan
    with pytest.raises(mv.MvgdError) as e:
        mv.mvgd_assemble(torch.tensor(pts, device=DEV), 10)
    assert e.value.status == mv.MVGD_EINVAL


def test_host_pointer_rejected(mv):
    P = torch.tensor(clouds.sphere(500, 1, 10).points)  # CPU tensor
    with pytest.raises(mv.MvgdError) as e:
        mv.mvgd_assemble(P, 10)
    assert e.value.status == mv.MVGD_EINVAL


def test_allocation_failure_cleans_up(mv):
    """Every allocation of assemble/apply can fail: the call returns ENOMEM, leaks nothing that
    breaks later calls, and a clean call afterwards gives the same matrix."""
    pts = torch.tensor(clouds.sphere(3000, 1, 20).points, device=DEV)
    ref = mv.mvgd_assemble(pts, 20)
    rc, cc, vc = mv.mvgd_csr(ref)
    seen = []
    for at in range(1, 24):
        os.environ["MVGD_FAIL_ALLOC_AT"] = f"{at}#{at}"
        try:
            L = mv.mvgd_assemble(pts, 20)
            y = mv.mvgd_apply(L, pts[:, 0].contiguous())
            seen.append(0)
            L.free()
        except mv.MvgdError as e:
            assert e.status == mv.MVGD_ENOMEM, e
            seen.append(e.status)
        finally:
            del os.environ["MVGD_FAIL_ALLOC_AT"]
    assert mv.MVGD_ENOMEM in seen and seen[-1] == 0
    L = mv.mvgd_assemble(pts, 20)
    r2, c2, v2 = mv.mvgd_csr(L)
    assert torch.equal(c2, cc) and torch.equal(v2, vc)
    L.free()
    ref.free()


def test_pool_trim_keeps_live_handles(mv):
    pts = torch.tensor(clouds.sphere(3000, 1, 20).points, device=DEV)
    A = mv.mvgd_assemble(pts, 20)
    rp, col, val = mv.mvgd_csr(A)
    B = mv.mvgd_assemble(pts, 20)
    B.free()
    mv.mvgd_pool_trim(0)
    r2, c2, v2 = mv.mvgd_csr(A)
    assert torch.equal(c2, col) and torch.equal(v2, val)
    C = mv.mvgd_assemble(pts, 20)
    r3, c3, v3 = mv.mvgd_csr(C)
    assert torch.equal(c3, col) and torch.equal(v3, val)
    A.free()
    C.free()


# ----------------------------------------------------------------------------------------------
# launch modes and tuning change only performance: results are bit-identical
# ----------------------------------------------------------------------------------------------
def test_launch_modes_and_tuning_do_not_change_results(mv):
    cl = clouds.ellipsoid_batch(n_clouds=5, seed=13, k=20, n_min=300, n_max=20000)
    P = torch.tensor(cl.points.astype(np.float32), device=DEV)
    offs = [int(v) for v in cl.offsets]
    ref = None
    for tuning in ({"launch": 1}, {"launch": 2},
                   {"launch": 2, "cell_alpha": 1.0, "radius_mu": 1.4, "cells_per_point": 4.0},
                   {"launch": 1, "cell_alpha": 0.45, "radius_mu": 2.0, "cells_per_point": 16.0}):
        L = mv.mvgd_assemble(P, 20, cloud_offsets=offs, tuning=tuning)
        rp, col, val = mv.mvgd_csr(L)
        y = mv.mvgd_apply(L, torch.tensor(cl.f.astype(np.float32), device=DEV))
        out = (col.cpu().numpy(), val.cpu().numpy(), y.cpu().numpy())
        L.free()
        if ref is None:
            ref = out
        else:
            for a, b in zip(ref, out):
                assert (a == b).all(), tuning


def _lattice_with_ties():
    g = np.stack(np.meshgrid(np.arange(40), np.arange(30), indexing="ij"), -1).reshape(-1, 2)
    pts = np.concatenate([g * 0.5, np.zeros((g.shape[0], 1))], 1).astype(np.float64)
    pts = pts @ np.linalg.qr(np.random.default_rng(1).standard_normal((3, 3)))[0].T
    return np.ascontiguousarray(pts[np.random.default_rng(2).permutation(pts.shape[0])])


@pytest.mark.parametrize("case", ["flat4-fp32", "flat4-fp64", "torus-fp32", "lattice-fp64",
                                  "lattice-fp32", "dups-fp32", "helix-fp64", "helix-fp32",
                                  "batch-fp32", "sphere2d-fp32"])
def test_search_modes_agree(mv, case):
    """The per-lane search (every query walks its own cell box), the group search (64 queries
    stream their common box) and the tile search (the group search with the query-candidate
    distances from the matrix cores) select the same neighbours and give bit-identical matrices,
    in both precisions, on clouds with exact ties, duplicates, curves, planar clouds and batches;
    and the oracle agrees on the sets."""
    name, precision = case.split("-")
    d, offs, k = 2, None, 20
    if name == "flat4":
        cl = clouds.flat_torus4(30000, 71, 32)
        pts, k = cl.points, 32
    elif name == "torus":
        pts, k = clouds.torus(20000, 72, 24).points, 24
    elif name == "lattice":
        pts, k = _lattice_with_ties(), 12
    elif name == "dups":
        base = clouds.sphere(1500, 5, 16).points
        pts = np.concatenate([base, base[:200], base[:50]])
        pts, k = np.ascontiguousarray(pts[np.random.default_rng(3).permutation(len(pts))]), 16
    elif name == "helix":
        pts, k, d = clouds.helix(5000, 73, 8).points, 8, 1
    elif name == "sphere2d":
        pts, k, d = clouds.circle(6000, 75, 6).points, 6, 1
    else:
        cl = clouds.ellipsoid_batch(n_clouds=5, seed=74, k=20, n_min=300, n_max=8000)
        pts, offs = cl.points, [int(v) for v in cl.offsets]
    dt = torch.float64 if precision == "fp64" else torch.float32
    P = torch.tensor(pts, dtype=dt, device=DEV)
    out = []
    modes = (mv.MVGD_SEARCH_GROUP, mv.MVGD_SEARCH_LANE, mv.MVGD_SEARCH_TILE)
    for search in modes:
        for launch in (1, 2):
            L = mv.mvgd_assemble(P, k, cloud_offsets=offs, d_manifold=d,
                                 tuning={"search": search, "launch": launch})
            rp, col, val = mv.mvgd_csr(L)
            out.append((col.cpu().numpy(), val.cpu().numpy()))
            L.free()
    for c, v in out[1:]:
        assert (c == out[0][0]).all() and (v == out[0][1]).all()
    if offs is None:
        oc, _ = oracle.rows(_oracle_points(pts, precision), k, d=d)
        assert (out[0][0].reshape(-1, k + 1) == oc).all()


# ----------------------------------------------------------------------------------------------
# serving: results are the same alone and in the mix; admission under a tiny HBM budget
# ----------------------------------------------------------------------------------------------
def test_serving_alone_equals_mixed():
    from paper_1603_04100_amd import serve
    reqs = serve.make_requests(duration_s=0.1, rate_hz=300, seed=11, k=24, n_min=2000,
                               n_max=20000, n_apply=8, max_requests=24)
    assert len(reqs) >= 10
    mixed = serve.Server(precision="fp32", n_streams=3, max_batch=8).run(reqs, batching=True)
    got = {r.id: r.result.copy() for r in reqs}
    assert mixed.summary()["requests"] == len(reqs) and max(mixed.batch_sizes) > 1
    alone = serve.Server(precision="fp32", n_streams=1, max_batch=1).run(reqs, batching=False)
    for r in reqs:
        assert (r.result == got[r.id]).all(), r.id
    # each result is L f of its own cloud: compare with the oracle on the first few requests
    for r in reqs[:3]:
        pts = r.points.astype(np.float32).astype(np.float64)
        oc, ov = oracle.rows(pts, r.k)
        ref = np.stack([(ov * r.rhs.astype(np.float32).astype(np.float64)[oc, j]).sum(1)
                        for j in range(r.rhs.shape[1])], 1)
        assert np.abs(r.result - ref).max() <= 1e-3 * np.abs(ref).max()
    print(f"\n[serving] mixed {mixed.summary()}\n[serving] alone {alone.summary()}")


def test_serving_admission_with_tiny_budget():
    from paper_1603_04100_amd import serve
    reqs = serve.make_requests(duration_s=0.05, rate_hz=400, seed=12, k=24, n_min=3000,
                               n_max=6000, max_requests=8)
    budget = serve.footprint_bytes(6000, 3, 24, 8, 4) + 1
    st = serve.Server(precision="fp32", n_streams=4, max_batch=8, hbm_budget_bytes=budget).run(reqs)
    assert st.summary()["requests"] == len(reqs)
    assert st.admission_waits > 0 and max(st.batch_sizes) == 1


# ----------------------------------------------------------------------------------------------
# Neumann condition by reflection (Sec. 3.1)
# ----------------------------------------------------------------------------------------------
def _neumann_case(mv, n, precision, k=20, kb=6, seed=8):
    cl = clouds.hemisphere(n, seed, k)
    m = cl.meta["boundary"]
    dt = torch.float64 if precision == "fp64" else torch.float32
    P = torch.tensor(cl.points, dtype=dt, device=DEV)
    L, ni, gx, gs = mv.mvgd_assemble_neumann(P, torch.tensor(m, device=DEV), k, kb)
    torch.cuda.synchronize()
    pts = _oracle_points(cl.points, precision)
    interior, G, src, _ = oracle.neumann_ghosts(pts, m, k, kb)
    gxyz, gsrc = gx.cpu().numpy(), gs.cpu().numpy().astype(np.int64)
    return cl, m, pts, L, ni, gxyz, gsrc, interior, G, src


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [4000, 20000])
def test_neumann_ghosts_and_rows(mv, precision, n):
    """Ghost set (which interior points get one, and their order) exactly as the oracle's; ghost
    coordinates (FP64 on both sides, from the same coordinates) to 1e-10; the folded interior rows
    against the oracle's rows on the GPU's ghosts to the row bar (twice the per-row tolerance: a
    folded entry is the sum of two), ghost rows zero, no ghost column left."""
    k, kb = 20, 6
    cl, m, pts, L, ni, gxyz, gsrc, interior, G, src = _neumann_case(mv, n, precision, k, kb)
    assert ni == len(interior)
    assert gsrc.shape == src.shape and (gsrc == src).all()
    gerr = np.abs(gxyz - G).max()
    assert gerr <= 1e-10, gerr
    ng = len(gsrc)
    # the oracle on the ghosts the GPU assembled on (rounded to the matrix dtype, as in its cloud)
    Gg = gxyz if precision == "fp64" else gxyz.astype(np.float32).astype(np.float64)
    A = np.concatenate([pts[interior], Gg])
    o_cols, o_vals, dg = oracle.rows(A, k, rows=np.arange(ni), diag=True)
    tol = 2.0 * _row_tol(precision, dg, _kappa(A, np.arange(ni), o_cols, dg))
    orp, oc, ov, _ = oracle.neumann_rows(pts, m, k, kb, ghosts=(interior, Gg, gsrc, None))
    rp, c, v = _export_csr(mv, L, ni + ng, k)
    assert (np.abs(v[rp[ni]:]) == 0).all(), "ghost rows must be zero"
    live = v[:rp[ni]] != 0
    assert (c[:rp[ni]][live] < ni).all(), "an interior row still references a ghost"
    import scipy.sparse as sp
    Ag = sp.csr_matrix((v[:rp[ni]], c[:rp[ni]], rp[:ni + 1]), shape=(ni, ni + ng))[:, :ni]
    Ao = sp.csr_matrix((ov, oc, orp), shape=(ni, ni))
    D = (Ag - Ao).tocsr()
    err = np.zeros(ni)
    np.maximum.at(err, np.repeat(np.arange(ni), np.diff(D.indptr)), np.abs(D.data))
    rel = err / np.abs(o_vals).max(1)
    bad = np.nonzero(rel > tol)[0]
    assert bad.size == 0, f"{bad.size} rows over tolerance, worst {rel.max():.3e} at {bad[:5]}"
    # every distinct column once: no duplicate nonzero (row, column) pair in the export
    rows = np.repeat(np.arange(ni), np.diff(rp[:ni + 1]))
    key = rows[live] * (ni + ng) + c[:rp[ni]][live]
    assert len(np.unique(key)) == len(key)
    # rows sum to zero: constants are in the kernel of the Neumann Laplacian
    rs = np.asarray(Ag.sum(1)).ravel()
    assert np.abs(rs).max() <= (1e-10 if precision == "fp64" else 1e-3) * np.abs(o_vals).max()
    print(f"\n[neumann hemisphere N={cl.n_points} {precision}] interior {ni}, ghosts {ng}, "
          f"max ghost err {gerr:.2e}, max row rel err {rel.max():.2e}")
    L.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_neumann_hemisphere_solve(mv, precision):
    """(sigma - Delta) U = (sigma + 6) z^2 - 2 on the upper hemisphere with dU/dn = 0 on the
    equator (solution U = z^2), sigma = 1: BiCGSTAB on the Neumann handle (ghost rows zero, so
    their unknowns solve sigma x = 0) matches the sparse-LU solution of the exported matrix and
    approaches z^2."""
    cl = clouds.hemisphere(4000, 8, 20)
    m = cl.meta["boundary"]
    dt = torch.float64 if precision == "fp64" else torch.float32
    P = torch.tensor(cl.points, dtype=dt, device=DEV)
    L, ni, gx, gs = mv.mvgd_assemble_neumann(P, torch.tensor(m, device=DEV), 20, 6)
    ng = gs.shape[0]
    pts = _oracle_points(cl.points, precision)
    z = pts[~m, 2]
    b = np.concatenate([7.0 * z ** 2 - 2.0, np.zeros(ng)])
    rtol = 1e-12 if precision == "fp64" else 1e-6
    x, info = mv.mvgd_solve(L, torch.tensor(b, dtype=dt, device=DEV), sigma=1.0, rtol=rtol,
                            max_iter=4000)
    assert info["converged"] == 1, info
    got = x.cpu().numpy().astype(np.float64)
    assert (got[ni:] == 0).all()
    rp, c, v = _export_csr(mv, L, ni + ng, 20)
    ref = oracle.solve(rp, c, v, b, sigma=1.0)
    kappa = _cond_bound(rp, c, v, 1.0, [])
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    store = 0.0 if precision == "fp64" else 2.0 ** -24
    assert rel <= 10 * kappa * info["rel_residual"] + 4 * store, (rel, kappa, info)
    err = np.abs(got[:ni] - cl.points[~m, 2] ** 2).max()
    assert err < 2e-3, err
    print(f"\n[neumann hemisphere solve 4k {precision}] {info}, kappa {kappa:.2e}, rel err vs LU {rel:.2e}, "
          f"max|x - z^2| {err:.2e}")
    L.free()


# ----------------------------------------------------------------------------------------------
# eigenvalues (Sec. 4: -Delta nu = lambda nu)
# ----------------------------------------------------------------------------------------------
def _match(got, ref):
    """Largest distance between the two eigenvalue lists after an optimal pairing."""
    from scipy.optimize import linear_sum_assignment
    C = np.abs(got[:, None] - ref[None, :])
    r, c = linear_sum_assignment(C)
    return C[r, c].max()


# The device's Ritz values converge to the eigenvalues of its own matrix; that matrix differs from
# the oracle's by the row bars (1e-12 FP64, ~4e-7 FP32-mixed relative), which moves eigenvalues of
# these nearly normal matrices by about that much times ||L|| (~5e3).
_EIG_TOL = {"fp64": 1e-8, "fp32": 5e-3}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_eigs_sphere(mv, precision):
    """The 16 eigenvalues of -L with the smallest real parts on a 2,000-point sphere against the
    oracle's (LAPACK on the oracle's matrix of the same points), and near l (l + 1)."""
    cl = clouds.sphere(2000, 1, 20)
    dt = torch.float64 if precision == "fp64" else torch.float32
    L = mv.mvgd_assemble(torch.tensor(cl.points, dtype=dt, device=DEV), 20)
    lam, info = mv.mvgd_eigs(L, 16, tol=1e-11)
    assert info["converged"] == 1, info
    ref = oracle.eigenvalues(*oracle.assemble(_oracle_points(cl.points, precision), 20), 16)
    err = _match(lam, ref)
    assert err <= _EIG_TOL[precision] * max(1.0, np.abs(ref).max()), (err, lam, ref)
    exact = np.concatenate([np.full(2 * l + 1, l * (l + 1.0)) for l in range(4)])
    rel = np.abs(np.sort(lam.real) - exact)[1:] / exact[1:]
    assert abs(lam.real[0]) < 1e-6 and rel.max() < 0.02, (lam, rel)
    print(f"\n[eigs sphere 2k {precision}] {info}, |GPU - oracle| {err:.2e}, "
          f"max rel err vs l(l+1) {rel.max():.2e}, max |imag| {np.abs(lam.imag).max():.1e}")
    L.free()


def test_eigs_parameters(mv):
    """Explicit block, fixed degree and a looser tolerance find the same bottom of the spectrum;
    out-of-range parameters are argument errors."""
    cl = clouds.sphere(2000, 1, 20)
    L = mv.mvgd_assemble(torch.tensor(cl.points, device=DEV), 20)
    lam, info = mv.mvgd_eigs(L, 4, block=12, degree=16, tol=1e-9)
    assert info["converged"] == 1 and info["block"] == 12 and info["degree"] == 16, info
    ref = oracle.eigenvalues(*oracle.assemble(cl.points, 20), 4)
    assert _match(lam, ref) <= 1e-6 * np.abs(ref).max(), (lam, ref)
    for kw in ({"nev": 0}, {"nev": 65}, {"nev": 8, "block": 4}, {"nev": 4, "degree": -1}):
        nev = kw.pop("nev")
        with pytest.raises(mv.MvgdError) as e:
            mv.mvgd_eigs(L, nev, **kw)
        assert e.value.status == mv.MVGD_EINVAL
    L.free()


def test_eigs_hemisphere_dirichlet_and_neumann(mv):
    """Open upper hemisphere (FP64): with the boundary points removed (Dirichlet) and on the
    Neumann handle with its ghost rows removed, against the oracle's eigenvalues of the same
    problems (its own ghosts for Neumann)."""
    cl = clouds.hemisphere(2000, 8, 20)
    m = cl.meta["boundary"]
    P = torch.tensor(cl.points, device=DEV)
    L = mv.mvgd_assemble(P, 20)
    lam, info = mv.mvgd_eigs(L, 10, tol=1e-11, fixed=torch.tensor(m, device=DEV))
    assert info["converged"] == 1, info
    ref = oracle.eigenvalues(*oracle.assemble(cl.points, 20), 10, keep=np.nonzero(~m)[0])
    err = _match(lam, ref)
    assert err <= _EIG_TOL["fp64"] * np.abs(ref).max(), (err, lam, ref)
    print(f"\n[eigs hemisphere Dirichlet] {info}, |GPU - oracle| {err:.2e}")
    L.free()
    L, ni, gx, gs = mv.mvgd_assemble_neumann(P, torch.tensor(m, device=DEV), 20, 6)
    ghost = torch.zeros(ni + gs.shape[0], dtype=torch.uint8, device=DEV)
    ghost[ni:] = 1
    lam, info = mv.mvgd_eigs(L, 10, tol=1e-11, fixed=ghost)
    assert info["converged"] == 1, info
    rp, c, v, _ = oracle.neumann_rows(cl.points, m, 20, 6)
    ref = oracle.eigenvalues(rp, c, v, 10)
    err = _match(lam, ref)
    assert err <= _EIG_TOL["fp64"] * max(1.0, np.abs(ref).max()), (err, lam, ref)
    print(f"\n[eigs hemisphere Neumann] {info}, |GPU - oracle| {err:.2e}")
    L.free()


def test_neumann_rejects_too_few_boundary_points(mv):
    """k_boundary larger than the number of boundary points is an argument error, and leaves no
    handle."""
    cl = clouds.hemisphere(2000, 8, 20, n_boundary=5)
    P = torch.tensor(cl.points, device=DEV)
    with pytest.raises(mv.MvgdError) as e:
        mv.mvgd_assemble_neumann(P, torch.tensor(cl.meta["boundary"], device=DEV), 20, 6)
    assert e.value.status == mv.MVGD_EINVAL
