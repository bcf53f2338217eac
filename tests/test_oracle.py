"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check is against a value the paper
prints, a closed form, a library routine (LAPACK through numpy, scipy's k-d tree), an
independent definition (the divergence form of the Laplace-Beltrami operator), brute force
on tiny inputs, or an invariance that a plausible mistake would break.
"""
import json
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1603_04100_amd import clouds

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _dense_row(cols, vals, i):
    return {int(c): float(v) for c, v in zip(cols, vals)}


# ----------------------------------------------------------------------------------------
# The paper's 1-D worked example (Sec. 3.2, Fig. Analysis, Eq. condition)
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1.0, 0.1, 3.7])
@pytest.mark.parametrize("n_ambient", [2, 3])
def test_worked_example_rows(oracle_mod, k, n_ambient):
    g = _golden("worked_example_1d.json")
    rng = np.random.default_rng(int(k * 10) + n_ambient)
    p = clouds.line_example(k, n_ambient, direction=rng.standard_normal(n_ambient),
                            offset=rng.standard_normal(n_ambient))
    cols, vals, dg = oracle_mod.rows(p, 4, rows=[2], d=1, diag=True)
    assert list(cols[0]) == [0, 1, 2, 3, 4]
    # the spacing rule gives h = k (Eq. DefH)
    assert dg[0, 0] == pytest.approx(g["h_rule_value_over_k"] * k, rel=1e-13)
    want = np.array(g["mvgd_row_at_h_eq_k_times_35k2"]) / (35.0 * k * k)
    np.testing.assert_allclose(vals[0], want, rtol=0, atol=1e-12 * np.abs(want).max())
    cols_ls, vals_ls = oracle_mod.rows(p, 4, rows=[2], d=1, variant="ls")
    want_ls = np.array(g["ls_row_times_7k2"]) / (7.0 * k * k)
    np.testing.assert_allclose(vals_ls[0], want_ls, rtol=0, atol=1e-12 * np.abs(want_ls).max())
    # MVGD - LS = (2/h^2)(a0 - T0): recovers the printed a0 row of the LS coefficient matrix
    a0 = (vals[0] - vals_ls[0]) * k * k / 2.0 + np.array([0, 0, 1, 0, 0])
    want_a0 = np.array(g["ls_coefficients_times_70k2"]["a0_over_k2"]) / 70.0
    np.testing.assert_allclose(a0, want_a0, rtol=0, atol=1e-12)
    # and LS row = 2 a2
    want_a2 = np.array(g["ls_coefficients_times_70k2"]["a2"]) / (70.0 * k * k)
    np.testing.assert_allclose(vals_ls[0] / 2.0, want_a2, rtol=0, atol=1e-12 * np.abs(want_a2).max())


@pytest.mark.parametrize("r", [0.5, 0.6, 1.0, 2.0, 4.8, 5.0])
def test_worked_example_m_matrix_window(oracle_mod, r):
    """Off-diagonals are >= 0 (opposite to the negative centre) iff 3/5 <= (h/k)^2 <= 24/5."""
    g = _golden("worked_example_1d.json")
    k = 0.5
    h = k * np.sqrt(r)
    p = clouds.line_example(k, 2)
    _, vals = oracle_mod.rows(p, 4, rows=[2], d=1, h_override=h)
    want = 2.0 / (70.0 * h * h) * np.array([-6 + 10 * r, 24 - 5 * r, -36 - 10 * r, 24 - 5 * r,
                                           -6 + 10 * r])
    np.testing.assert_allclose(vals[0], want, rtol=0, atol=1e-12 * np.abs(want).max())
    lo, hi = g["m_matrix_window_r"]
    off = np.delete(vals[0], 2)
    tol = 1e-12 * np.abs(vals[0]).max()
    inside = lo <= r <= hi
    assert vals[0][2] < 0
    assert (off >= -tol).all() == inside
    assert abs(vals[0].sum()) <= tol * 10


# ----------------------------------------------------------------------------------------
# Exactness on planes: b00 = U_i for quadratics, central differences exact on quadratics
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("n_ambient,k,seed", [(3, 12, 0), (3, 24, 1), (4, 20, 2), (4, 32, 3)])
def test_plane_exactness(oracle_mod, n_ambient, k, seed):
    p, basis, _ = clouds.random_plane(600, n_ambient, seed)
    rng = np.random.default_rng(100 + seed)
    A = rng.standard_normal((n_ambient, n_ambient))
    A = A + A.T
    b = rng.standard_normal(n_ambient)
    f = np.einsum("ni,ij,nj->n", p, A, p) + p @ b + 0.3
    lap = 2.0 * np.trace(basis @ A @ basis.T)
    rp, cols, vals = oracle_mod.assemble(p, k)
    y = oracle_mod.apply(rp, cols, vals, f)
    scale = np.abs(vals).reshape(-1, k + 1).sum(1) * np.abs(f).max()
    assert np.all(np.abs(y - lap) <= 1e-11 * scale + 1e-9)


def test_plane_linear_functions_vanish_on_second_derivative(oracle_mod):
    p, basis, _ = clouds.random_plane(400, 3, 7)
    rp, cols, vals = oracle_mod.assemble(p, 16)
    for c in range(3):
        y = oracle_mod.apply(rp, cols, vals, p[:, c])
        assert np.abs(y).max() <= 1e-9 * np.abs(vals).max()


# ----------------------------------------------------------------------------------------
# Consistency: rows sum to zero (Sec. 3.2)
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("cloud", ["sphere", "torus", "flat4"])
def test_row_sums_zero(oracle_mod, cloud):
    cl = {"sphere": lambda: clouds.sphere(1500, 11, 20),
          "torus": lambda: clouds.torus(3000, 12, 24),
          "flat4": lambda: clouds.flat_torus4(3000, 13, 32)}[cloud]()
    rp, cols, vals = oracle_mod.assemble(cl.points, cl.k)
    v = vals.reshape(-1, cl.k + 1)
    assert np.all(np.abs(v.sum(1)) <= 1e-12 * np.abs(v).sum(1))
    # negative diagonal (L approximates +Delta)
    c = cols.reshape(-1, cl.k + 1)
    diag = v[c == np.arange(v.shape[0])[:, None]]
    assert (diag < 0).all()


# ----------------------------------------------------------------------------------------
# kNN: scipy's k-d tree, brute force with exact ties
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("n_ambient,k", [(3, 20), (4, 32), (2, 8)])
def test_knn_matches_kdtree(oracle_mod, n_ambient, k):
    rng = np.random.default_rng(n_ambient * 7 + k)
    p = rng.standard_normal((3000, n_ambient))
    idx, key = oracle_mod.knn(p, k)
    dist, ref = cKDTree(p).query(p, k + 1)
    for i in range(p.shape[0]):
        r = [j for j in ref[i] if j != i][:k]
        assert set(idx[i]) == set(r)
    np.testing.assert_allclose(np.sqrt(key), dist[:, 1:], rtol=1e-12)


def test_knn_ties_brute_force(oracle_mod):
    g = np.stack(np.meshgrid(np.arange(4), np.arange(4), np.arange(4), indexing="ij"), -1)
    p = g.reshape(-1, 3).astype(np.float64)
    perm = np.random.default_rng(0).permutation(p.shape[0])
    p = p[perm]
    for k in (6, 7, 18, 26, 40):
        idx, _ = oracle_mod.knn(p, k)
        for i in range(p.shape[0]):
            keys = sorted(((float(((p[j] - p[i]) ** 2).sum()), j) for j in range(p.shape[0])
                           if j != i))
            assert list(idx[i]) == [j for _, j in keys[:k]]


# ----------------------------------------------------------------------------------------
# Frame, spacing and fits against LAPACK
# ----------------------------------------------------------------------------------------
def _local(cl, oracle_mod, rows):
    cols, vals, dg = oracle_mod.rows(cl.points, cl.k, rows=rows, diag=True)
    return cols, vals, dg


@pytest.mark.parametrize("which", ["sphere", "flat4"])
def test_frame_h_and_fits_against_lapack(oracle_mod, which):
    cl = clouds.sphere(3000, 21, 20) if which == "sphere" else clouds.flat_torus4(6000, 22, 32)
    P, K, n = cl.points, cl.k, cl.n_ambient
    rows = np.arange(0, P.shape[0], 97)
    cols, vals, dg = _local(cl, oracle_mod, rows)
    for r, i in enumerate(rows):
        nb = cols[r][cols[r] != i]
        # covariance over N(i) about its barycentre (Sec. 2), p_i excluded
        c = P[nb].mean(0)
        C = (P[nb] - c).T @ (P[nb] - c)
        lam, E = np.linalg.eigh(C)
        lam, E = lam[::-1], E[:, ::-1].T
        np.testing.assert_allclose(dg[r, 2:2 + n], lam, rtol=1e-10, atol=1e-14 * lam[0])
        F = dg[r, 6:22].reshape(4, 4)[:n, :n]
        # tangent subspace agreement
        s = np.linalg.svd(F[:2] @ E[:2].T, compute_uv=False)
        np.testing.assert_allclose(s, 1.0, atol=1e-10)
        # h rule
        u = (P[nb] - P[i]) @ F[:2].T
        h = 0.25 * min(np.ptp(u[:, 0]), np.ptp(u[:, 1]))
        assert dg[r, 0] == pytest.approx(h, rel=1e-13)
        # quadratic LS fit of the normal coordinates (Eq. poly), over p_i and N(i)
        z = (P[nb] - P[i]) @ F[2:].T
        x, y = u[:, 0], u[:, 1]
        V = np.vstack([[1, 0, 0, 0, 0, 0], np.stack([np.ones(K), x, y, x * x, x * y, y * y], 1)])
        Z = np.vstack([np.zeros((1, n - 2)), z])
        a_ref = np.linalg.lstsq(V, Z, rcond=None)[0].T
        a = dg[r, 22:22 + 6 * (n - 2)].reshape(n - 2, 6)
        np.testing.assert_allclose(a, a_ref, rtol=1e-8, atol=1e-9 * np.abs(a_ref).max())


# ----------------------------------------------------------------------------------------
# O8 against the divergence-form definition of the LB operator (Eq. SurLapEqn / Eq. LB1)
# ----------------------------------------------------------------------------------------
def _lb_divergence_2d(a, b, s):
    """(1/sqrt g) d_alpha (sqrt g g^{alpha beta} d_beta U) at 0 for the graph (x, y, z_c)."""
    def flux(x, y):
        zx = np.array([ac[1] + 2 * ac[3] * x + ac[4] * y for ac in a])
        zy = np.array([ac[2] + 2 * ac[5] * y + ac[4] * x for ac in a])
        g = np.array([[1 + zx @ zx, zx @ zy], [zx @ zy, 1 + zy @ zy]])
        Ux = b[1] + 2 * b[3] * x + b[4] * y
        Uy = b[2] + 2 * b[5] * y + b[4] * x
        return np.sqrt(np.linalg.det(g)) * np.linalg.solve(g, [Ux, Uy]), np.linalg.det(g)

    d1 = (flux(s, 0)[0][0] - flux(-s, 0)[0][0]) / (2 * s)
    d2 = (flux(0, s)[0][1] - flux(0, -s)[0][1]) / (2 * s)
    return (d1 + d2) / np.sqrt(flux(0, 0)[1])


@pytest.mark.parametrize("n_codim", [1, 2, 3])
def test_lb_coefficients_match_divergence_form(oracle_mod, n_codim):
    rng = np.random.default_rng(n_codim)
    for _ in range(20):
        a = rng.standard_normal((n_codim, 6)) * 0.7
        b = rng.standard_normal(6)
        G, q = oracle_mod.lb_coefficients(a, 2)
        ours = G[0, 0] * 2 * b[3] + 2 * G[0, 1] * b[4] + G[1, 1] * 2 * b[5] - q @ b[1:3]
        s = 1e-3
        ref = (4 * _lb_divergence_2d(a, b, s / 2) - _lb_divergence_2d(a, b, s)) / 3
        assert ours == pytest.approx(ref, rel=1e-8, abs=1e-9)


def test_lb_coefficients_reduce_to_eq_lb1(oracle_mod):
    """d = 1, one normal coordinate: G = 1/(1 + y_x^2), q = y_x y_xx/(1 + y_x^2)^2 (Eq. LB1)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        a = rng.standard_normal(3)
        G, q = oracle_mod.lb_coefficients(a[None, :], 1)
        yx, yxx = a[1], 2 * a[2]
        assert G[0, 0] == pytest.approx(1 / (1 + yx * yx), rel=1e-14)
        assert q[0] == pytest.approx(yx * yxx / (1 + yx * yx) ** 2, rel=1e-13)
        # and the divergence form (1/sqrt g) d/dx (U'/sqrt g) of the same curve
        b = rng.standard_normal(3)

        def flux(x):
            gx = 1 + (a[1] + 2 * a[2] * x) ** 2
            return (b[1] + 2 * b[2] * x) / np.sqrt(gx)

        s = 1e-4
        ref = (flux(s) - flux(-s)) / (2 * s) / np.sqrt(1 + a[1] ** 2)
        ours = G[0, 0] * 2 * b[2] - q[0] * b[1]
        assert ours == pytest.approx(ref, rel=1e-6, abs=1e-8)


# ----------------------------------------------------------------------------------------
# MVGD - LS identity (generalises Eq. accuracy): L_mvgd U - L_ls U = tau (b00 - U_i)
# ----------------------------------------------------------------------------------------
def test_mvgd_minus_ls_identity(oracle_mod):
    cl = clouds.sphere(2500, 31, 20, degrees=(3,))
    P, K = cl.points, cl.k
    rows = np.arange(0, P.shape[0], 53)
    cols, vals, dg = oracle_mod.rows(P, K, rows=rows, diag=True)
    cols_ls, vals_ls = oracle_mod.rows(P, K, rows=rows, variant="ls")
    assert (cols == cols_ls).all()
    f = cl.f[:, 0]
    for r, i in enumerate(rows):
        nb = cols[r][cols[r] != i]
        F = dg[r, 6:18].reshape(3, 4)[:3, :3]
        u = (P[nb] - P[i]) @ F[:2].T
        V = np.vstack([[1, 0, 0, 0, 0, 0],
                       np.stack([np.ones(K), u[:, 0], u[:, 1], u[:, 0] ** 2, u[:, 0] * u[:, 1],
                                 u[:, 1] ** 2], 1)])
        b = np.linalg.lstsq(V, np.concatenate([[f[i]], f[nb]]), rcond=None)[0]
        lhs = vals[r] @ f[cols[r]] - vals_ls[r] @ f[cols_ls[r]]
        rhs = dg[r, 58] * (b[0] - f[i])
        assert lhs == pytest.approx(rhs, rel=1e-7, abs=1e-9 * np.abs(vals[r]).sum())


# ----------------------------------------------------------------------------------------
# Closed-form Laplacians: error falls as the sampling refines (Sec. 3.2 accuracy, Sec. 4)
# ----------------------------------------------------------------------------------------
def test_sphere_position_converges_second_order(oracle_mod):
    """-Delta x = 2x on the unit sphere (Eq. lapsphere); max error ~ h^2 for f = x."""
    errs = []
    for n in (2000, 8000, 32000):
        cl = clouds.sphere(n, 1, 20)
        rp, c, v = oracle_mod.assemble(cl.points, 20)
        errs.append(np.abs(oracle_mod.apply(rp, c, v, cl.f[:, 0]) - cl.lap_f[:, 0]).max())
    assert errs[0] < 0.05
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 2.0  # h halves each step


def test_sphere_harmonics_rms_decreases(oracle_mod):
    """Delta Re((x+iy)^l) = -l(l+1) Re((x+iy)^l), l = 1..4."""
    rms = []
    for n in (2000, 8000, 32000):
        cl = clouds.sphere(n, 2, 20, degrees=(1, 2, 3, 4))
        rp, c, v = oracle_mod.assemble(cl.points, 20)
        e = oracle_mod.apply(rp, c, v, cl.f) - cl.lap_f
        rms.append(np.sqrt((e ** 2).mean(0)))
    rms = np.array(rms)
    assert (rms[0] / rms[2] > 2.0).all(), rms


def test_torus_closed_form_rms_decreases(oracle_mod):
    rms = []
    for n in (5000, 20000):
        cl = clouds.torus(n, 2, 24)
        rp, c, v = oracle_mod.assemble(cl.points, 24)
        e = oracle_mod.apply(rp, c, v, cl.f[:, 0]) - cl.lap_f[:, 0]
        rms.append(np.sqrt((e ** 2).mean()))
    assert rms[0] / rms[1] > 1.5, rms


def test_flat_torus_r4_closed_form(oracle_mod):
    """Flat torus in R^4 (codimension 2): Delta cos(2t)cos(3p) = -13 cos(2t)cos(3p)."""
    rms = []
    for n in (5000, 20000):
        cl = clouds.flat_torus4(n, 4, 32, noise=0.0)
        rp, c, v = oracle_mod.assemble(cl.points, 32)
        e = oracle_mod.apply(rp, c, v, cl.f[:, 0]) - cl.lap_f[:, 0]
        rms.append(np.sqrt((e ** 2).mean()))
    assert rms[1] < 0.1 * 13 and rms[0] / rms[1] > 1.5, rms


# ----------------------------------------------------------------------------------------
# Invariances
# ----------------------------------------------------------------------------------------
def _matrix(oracle_mod, p, k):
    rp, c, v = oracle_mod.assemble(p, k)
    return c.reshape(-1, k + 1), v.reshape(-1, k + 1)


def test_rigid_motion_invariance(oracle_mod):
    cl = clouds.torus(3000, 41, 16)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    c0, v0 = _matrix(oracle_mod, cl.points, 16)
    c1, v1 = _matrix(oracle_mod, cl.points @ Q.T + rng.standard_normal(3), 16)
    assert (c0 == c1).all()
    assert np.all(np.abs(v0 - v1) <= 1e-8 * np.abs(v0).max(1, keepdims=True))


def test_scaling_law(oracle_mod):
    cl = clouds.sphere(2000, 42, 20)
    c0, v0 = _matrix(oracle_mod, cl.points, 20)
    c1, v1 = _matrix(oracle_mod, 3.0 * cl.points, 20)
    assert (c0 == c1).all()
    np.testing.assert_allclose(v1 * 9.0, v0, rtol=0, atol=1e-10 * np.abs(v0).max())


def test_relabelling_equivariance(oracle_mod):
    cl = clouds.sphere(1500, 43, 20)
    perm = np.random.default_rng(0).permutation(1500)
    c0, v0 = _matrix(oracle_mod, cl.points, 20)
    c1, v1 = _matrix(oracle_mod, cl.points[perm], 20)
    inv = np.argsort(perm)
    for i in range(0, 1500, 7):
        r1 = dict(zip(perm[c1[inv[i]]], v1[inv[i]]))
        r0 = dict(zip(c0[i], v0[i]))
        assert set(r0) == set(r1)
        for j in r0:
            assert r1[j] == pytest.approx(r0[j], rel=1e-9, abs=1e-9 * np.abs(v0[i]).max())


# ----------------------------------------------------------------------------------------
# Degenerate neighbourhoods and argument errors
# ----------------------------------------------------------------------------------------
def test_degenerate_rows_are_flagged(oracle_mod):
    # collinear points in R^3 with d = 2: h = 0
    t = np.linspace(0, 1, 40)
    line = np.stack([t, 2 * t, -t], 1)
    cols, vals, dg = oracle_mod.rows(line, 8, diag=True)
    assert (dg[:, 1] == 1).all() and (vals == 0).all()
    assert all(len(set(r)) == 9 for r in cols)
    # a ladder: two parallel lines, so eta takes two values and V loses rank
    x = np.arange(30, dtype=np.float64)
    ladder = np.concatenate([np.stack([x, np.ones(30), 0 * x], 1),
                             np.stack([x, -np.ones(30), 0 * x], 1)])
    cols, vals, dg = oracle_mod.rows(ladder, 10, diag=True)
    assert (dg[:, 1] == 1).all() and (vals == 0).all()


def test_argument_errors(oracle_mod):
    p = clouds.sphere(100, 0, 10).points
    with pytest.raises(ValueError):
        oracle_mod.rows(p, 100)
    q = p.copy()
    q[5, 1] = np.nan
    with pytest.raises(ValueError):
        oracle_mod.rows(q, 10)
    with pytest.raises(ValueError):
        oracle_mod.rows(p[:, :2], 10, d=2)


# ----------------------------------------------------------------------------------------
# Whole rows against the literal virtual-grid differences (Eq. centered1, Eq. center and the
# higher-dimensional rule of Sec. 3.1): fit U by LAPACK least squares in the oracle's frame,
# evaluate the fitted quadratic at the virtual grid nodes (+-h), put U_i at the centre node,
# and combine the differences with the coefficients of Eq. eqn3 (pinned above).
# ----------------------------------------------------------------------------------------
def _virtual_grid_value(P, i, nb, frame, h, d, U, oracle_mod, variant="mvgd", w_nbr=1.0):
    """Weighted variants: LAPACK least squares on rows scaled by sqrt(weight) (weight 1 at p_i,
    w_nbr at the neighbours). The LS variant puts the fitted value, not U_i, at the centre."""
    n = P.shape[1]
    D = P[nb] - P[i]
    u = D @ frame[:d].T
    z = D @ frame[d:n].T
    if d == 2:
        mono = lambda x, y: np.stack([np.ones_like(x), x, y, x * x, x * y, y * y], -1)
        V = np.vstack([mono(np.zeros(1), np.zeros(1)), mono(u[:, 0], u[:, 1])])
    else:
        mono = lambda x: np.stack([np.ones_like(x), x, x * x], -1)
        V = np.vstack([mono(np.zeros(1)), mono(u[:, 0])])
    sw = np.sqrt(np.concatenate([[1.0], np.full(len(nb), w_nbr)]))
    Z = np.vstack([np.zeros((1, n - d)), z])
    a = np.linalg.lstsq(V * sw[:, None], Z * sw[:, None], rcond=None)[0].T
    G, q = oracle_mod.lb_coefficients(a, d)
    b = np.linalg.lstsq(V * sw[:, None], U * sw, rcond=None)[0]
    Ui = U[0] if variant == "mvgd" else b[0]
    if d == 2:
        Uh = lambda x, y: (mono(np.array([x]), np.array([y])) @ b)[0]
        Dx = (Uh(h, 0) - Uh(-h, 0)) / (2 * h)
        Dy = (Uh(0, h) - Uh(0, -h)) / (2 * h)
        Dxx = (Uh(h, 0) - 2 * Ui + Uh(-h, 0)) / h ** 2
        Dyy = (Uh(0, h) - 2 * Ui + Uh(0, -h)) / h ** 2
        Dxy = (Uh(h, h) - Uh(h, -h) - Uh(-h, h) + Uh(-h, -h)) / (4 * h * h)
        return G[0, 0] * Dxx + 2 * G[0, 1] * Dxy + G[1, 1] * Dyy - q[0] * Dx - q[1] * Dy
    Uh = lambda x: (mono(np.array([x])) @ b)[0]
    if variant == "div":  # Eq. divergence with the fitted curve's slope at 0 and +-h/2
        s = lambda x: np.sqrt(1.0 + sum((ac[1] + 2 * ac[2] * x) ** 2 for ac in a))
        return (Uh(h) / s(h / 2) - (1 / s(h / 2) + 1 / s(-h / 2)) * U[0]
                + Uh(-h) / s(-h / 2)) / (h * h * s(0))
    Dx = (Uh(h) - Uh(-h)) / (2 * h)
    Dxx = (Uh(h) - 2 * Ui + Uh(-h)) / h ** 2
    return G[0, 0] * Dxx - q[0] * Dx


@pytest.mark.parametrize("which,variant,weighted", [
    ("sphere", "mvgd", False), ("torus", "mvgd", False), ("flat4", "mvgd", False),
    ("circle", "mvgd", False), ("helix", "mvgd", False),
    ("sphere", "ls", False), ("flat4", "ls", True), ("torus", "mvgd", True),
    ("helix", "ls", True), ("circle", "mvgd", True),
    ("circle", "div", False), ("helix", "div", False), ("helix", "div", True)])
def test_rows_equal_virtual_grid_definition(oracle_mod, which, variant, weighted):
    rng = np.random.default_rng(7)
    if which == "sphere":
        P, K, d = clouds.sphere(2000, 51, 20).points, 20, 2
    elif which == "torus":
        P, K, d = clouds.torus(4000, 52, 24, r=0.5).points, 24, 2
    elif which == "flat4":
        P, K, d = clouds.flat_torus4(4000, 53, 32, noise=0.0).points, 32, 2
    elif which == "circle":
        t = rng.uniform(0, 2 * np.pi, 500)
        P, K, d = np.stack([np.cos(t), np.sin(t)], 1), 6, 1
    else:
        t = rng.uniform(0, 4 * np.pi, 800)
        P, K, d = np.stack([np.cos(t), np.sin(t), 0.3 * t], 1), 8, 1
    rows = np.arange(0, P.shape[0], 41)
    w_nbr = 1.0 / K if weighted else 1.0
    cols, vals, dg = oracle_mod.rows(P, K, rows=rows, d=d, diag=True, variant=variant,
                                     weight_nbr=w_nbr)
    n = P.shape[1]
    for r, i in enumerate(rows):
        nb = cols[r][cols[r] != i]
        frame = dg[r, 6:22].reshape(4, 4)[:n, :n]
        h = dg[r, 0]
        for _ in range(3):
            U = rng.standard_normal(K + 1)  # U[0] at p_i, then N(i) ascending
            ref = _virtual_grid_value(P, i, nb, frame, h, d, U, oracle_mod, variant, w_nbr)
            Ucol = dict(zip(np.concatenate([[i], nb]), U))
            ours = sum(v * Ucol[c] for c, v in zip(cols[r], vals[r]))
            assert ours == pytest.approx(ref, rel=1e-9, abs=1e-11 * np.abs(vals[r]).sum())


@pytest.mark.parametrize("variant", ["mvgd", "div"])
def test_circle_converges(oracle_mod, variant):
    """Unit circle, Delta sin(2t) = -4 sin(2t) (Sec. 4.2): both curve forms converge."""
    errs = []
    for n in (500, 2000, 8000):
        t = np.random.default_rng(n).uniform(0, 2 * np.pi, n)
        P = np.stack([np.cos(t), np.sin(t)], 1)
        rp, c, v = oracle_mod.assemble(P, 6, d=1, variant=variant)
        e = oracle_mod.apply(rp, c, v, np.sin(2 * t)) + 4 * np.sin(2 * t)
        errs.append(np.sqrt((e ** 2).mean()))
        rs = v.reshape(n, 7).sum(1)
        assert np.abs(rs).max() <= 1e-12 * np.abs(v).reshape(n, 7).sum(1).max()
    assert errs[0] / errs[2] > 4.0, errs


def test_divergence_form_on_straight_lines(oracle_mod):
    """On a straight line the fitted slope is constant, s(x) = s(0), and the divergence form is
    the centred form: identical rows (the printed 1-D row at h = k included)."""
    g = _golden("worked_example_1d.json")
    p = clouds.line_example(0.3, 3, direction=[1.0, 2.0, -0.5], offset=[0.1, 0.2, 0.3])
    _, v_div = oracle_mod.rows(p, 4, rows=[2], d=1, variant="div")
    want = np.array(g["mvgd_row_at_h_eq_k_times_35k2"]) / (35.0 * 0.09)
    np.testing.assert_allclose(v_div[0], want, rtol=0, atol=1e-12 * np.abs(want).max())
    t = np.sort(np.random.default_rng(3).uniform(-5, 5, 300))
    P = t[:, None] * np.array([[0.6, -0.8]]) + np.array([[2.0, 1.0]])
    _, v1 = oracle_mod.rows(P, 8, d=1, variant="mvgd")
    _, v2 = oracle_mod.rows(P, 8, d=1, variant="div")
    np.testing.assert_allclose(v2, v1, rtol=0, atol=1e-10 * np.abs(v1).max())
    with pytest.raises(ValueError):
        oracle_mod.rows(clouds.sphere(200, 0, 10).points, 10, variant="div")


# ----------------------------------------------------------------------------------------
# Weighted (moving) least squares (Sec. 4: weight 1 at p_i and 1/K at the neighbours)
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("variant", ["mvgd", "ls"])
def test_weighted_fits_keep_plane_exactness(oracle_mod, variant):
    """A weighted fit still reproduces quadratics, so on a plane L f = Delta f exactly and
    rows sum to zero."""
    p, basis, _ = clouds.random_plane(500, 3, 4)
    rng = np.random.default_rng(40)
    A = rng.standard_normal((3, 3))
    A = A + A.T
    f = np.einsum("ni,ij,nj->n", p, A, p) + p @ rng.standard_normal(3)
    lap = 2.0 * np.trace(basis @ A @ basis.T)
    rp, cols, vals = oracle_mod.assemble(p, 16, variant=variant, weight_nbr=1.0 / 16)
    y = oracle_mod.apply(rp, cols, vals, f)
    v = vals.reshape(-1, 17)
    assert np.all(np.abs(y - lap) <= 1e-11 * np.abs(v).sum(1) * np.abs(f).max() + 1e-9)
    assert np.all(np.abs(v.sum(1)) <= 1e-12 * np.abs(v).sum(1))


def test_weights_change_the_rows_off_planes(oracle_mod):
    """On a curved surface the weighted rows differ from the unweighted ones (the weight reaches
    both fits), and the centre weight 1 dominates as w_nbr -> 0."""
    cl = clouds.sphere(1500, 31, 20)
    rows = np.arange(0, 1500, 50)
    _, v1 = oracle_mod.rows(cl.points, 20, rows=rows)
    _, vw = oracle_mod.rows(cl.points, 20, rows=rows, weight_nbr=1.0 / 20)
    assert np.abs(vw - v1).max() > 1e-3 * np.abs(v1).max()
    with pytest.raises(ValueError):
        oracle_mod.rows(cl.points, 20, rows=rows, weight_nbr=0.0)


# ----------------------------------------------------------------------------------------
# Row sign statistics (Sec. 3.2: the M-matrix property of the modified difference)
# ----------------------------------------------------------------------------------------
def test_row_stats_on_the_printed_rows(oracle_mod):
    """The paper's two 1-D rows: MVGD (4, 19, -46, 19, 4) is an M-row, LS (2, -1, -2, -1, 2)
    is not; the negative off-diagonal mass of the LS row is 2/2 of its diagonal."""
    g = _golden("worked_example_1d.json")
    cols = np.array([[0, 1, 2, 3, 4], [0, 1, 2, 3, 4]])
    vals = np.array([g["mvgd_row_at_h_eq_k_times_35k2"], g["ls_row_times_7k2"]], dtype=float)
    per, tot = oracle_mod.row_stats([2, 2], cols, vals)
    assert list(per["m_row"]) == [True, False]
    assert per["ratio"][0] == 0.0 and per["ratio"][1] == 1.0
    assert tot["n_offdiag_negative"] == 2 and tot["n_diag_negative"] == 2
    # a zero diagonal gives NaN and is left out of the means
    per, tot = oracle_mod.row_stats([0], [[0, 1]], [[0.0, -1.0]])
    assert np.isnan(per["ratio"][0]) and tot["mean_ratio"] == 0.0 and not per["m_row"][0]


@pytest.mark.parametrize("r,inside", [(0.5, False), (0.7, True), (2.0, True), (4.7, True),
                                      (5.0, False)])
def test_row_stats_follow_the_m_matrix_window(oracle_mod, r, inside):
    k = 0.5
    p = clouds.line_example(k, 2)
    cols, vals = oracle_mod.rows(p, 4, rows=[2], d=1, h_override=k * np.sqrt(r))
    per, _ = oracle_mod.row_stats([2], cols, vals)
    assert bool(per["m_row"][0]) == inside
    assert (per["ratio"][0] == 0.0) == inside


@pytest.mark.parametrize("cloud", ["sphere", "torus"])
def test_centre_modification_reduces_negative_mass(oracle_mod, cloud):
    """On curved surfaces the MVGD rows carry far less negative off-diagonal mass than the
    plain least-squares rows, and with the paper's MLS weights most MVGD rows are M-rows while
    almost no LS rows are."""
    cl = clouds.sphere(2000, 1, 20) if cloud == "sphere" else clouds.torus(6000, 2, 24)
    ids = np.arange(cl.n_points)
    tot = {}
    for var in ("mvgd", "ls"):
        for w in (1.0, 1.0 / cl.k):
            c, v = oracle_mod.rows(cl.points, cl.k, variant=var, weight_nbr=w)
            tot[var, w] = oracle_mod.row_stats(ids, c, v)[1]
    w = 1.0 / cl.k
    assert tot["mvgd", 1.0]["mean_ratio"] < 0.1 * tot["ls", 1.0]["mean_ratio"]
    assert tot["mvgd", w]["n_m_rows"] > 0.3 * cl.n_points
    assert tot["ls", w]["n_m_rows"] < 0.01 * cl.n_points


# ----------------------------------------------------------------------------------------
# Linear solves with the assembled matrix (Sec. 4.2: -Delta U = 2x on the unit sphere)
# ----------------------------------------------------------------------------------------
def test_solve_sphere_position_converges(oracle_mod):
    """-Delta U = 2x on the unit sphere has the solution U = x (up to a constant, fixed by one
    pinned value): the discrete solution approaches x at about second order, as Sec. 4.2 reports."""
    errs = []
    for n in (1000, 4000):
        cl = clouds.sphere(n, 5, 20)
        P = cl.points
        rp, c, v = oracle_mod.assemble(P, 20)
        b = 2.0 * P[:, 0]
        b[0] = P[0, 0]
        x = oracle_mod.solve(rp, c, v, b, sigma=0.0, pinned=[0])
        assert x[0] == pytest.approx(P[0, 0], abs=1e-12)
        # the residual of the unpinned rows: (-L x)_i = b_i
        r = -oracle_mod.apply(rp, c, v, x)[1:] - b[1:]
        assert np.abs(r).max() <= 1e-8 * np.abs(v).max()
        errs.append(np.abs(x - P[:, 0]).max())
    assert errs[0] < 3e-3 and errs[0] / errs[1] > 2.5, errs


def test_solve_screened_circle(oracle_mod):
    """(sigma - Delta) U = f on an equispaced circle with U = sin 2t, f = (sigma + 4) sin 2t: the
    solve reproduces U to the discretisation error, and a wrong sign of sigma would not."""
    cl = clouds.circle(1000, 3, 6, sampling="uniform")
    t = np.arctan2(cl.points[:, 1], cl.points[:, 0])
    rp, c, v = oracle_mod.assemble(cl.points, 6, d=1)
    for sigma in (1.0, 10.0):
        x = oracle_mod.solve(rp, c, v, (sigma + 4.0) * np.sin(2 * t), sigma=sigma)
        assert np.abs(x - np.sin(2 * t)).max() < 1e-6


def test_solve_hemisphere_dirichlet(oracle_mod):
    """Open surface with the Dirichlet condition enforced at the boundary points and MVGD rows at
    the interior points (Sec. 3.1): on the upper hemisphere -Delta U = 2z with U = 0 on the
    boundary circle has the solution U = z; the discrete solution approaches it."""
    errs = []
    for n in (1000, 4000):
        cl = clouds.hemisphere(n, 8, 20)
        P, m = cl.points, cl.meta["boundary"]
        rp, c, v = oracle_mod.assemble(P, 20)
        b = 2.0 * P[:, 2]
        b[m] = 0.0
        x = oracle_mod.solve(rp, c, v, b, pinned=np.nonzero(m)[0])
        assert np.abs(x[m]).max() <= 1e-10
        errs.append(np.abs(x - P[:, 2]).max())
    assert errs[0] < 1.5e-3 and errs[0] / errs[1] > 3.0, errs


# ----------------------------------------------------------------------------------------
# Neumann condition by reflection (Sec. 3.1)
# ----------------------------------------------------------------------------------------
def _half_square(n=1500, seed=9, nb=60):
    """Points of the square [0, 1]^2 (plane z = 0, rotated into R^3) with the edge x = 0 sampled
    as the boundary (listed last)."""
    rng = np.random.default_rng(seed)
    q = rng.uniform(0.0, 1.0, (n, 2))
    q[:, 0] = 0.02 + 0.98 * q[:, 0]
    b = np.stack([np.zeros(nb), (np.arange(nb) + 0.5) / nb], 1)
    pts = np.concatenate([q, b])
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    P = np.concatenate([pts, np.zeros((len(pts), 1))], 1) @ R.T + rng.standard_normal(3)
    mask = np.zeros(len(pts), dtype=bool)
    mask[n:] = True
    return P, mask, pts, R


def test_neumann_ghosts_mirror_a_straight_boundary(oracle_mod):
    """With a straight boundary line in a plane the boundary frame is exact, and every ghost is
    the mirror image of its source across the line: (x, y) -> (-x, y)."""
    P, mask, pts, R = _half_square()
    interior, G, src, bsrc = oracle_mod.neumann_ghosts(P, mask, 16, 6)
    assert len(G) > 0
    # back to the plane's coordinates
    off = P[0] - np.concatenate([pts[0], [0.0]]) @ R.T
    g2 = (G - off) @ R
    s2 = pts[interior[src]]
    np.testing.assert_allclose(g2[:, 0], -s2[:, 0], atol=1e-12)
    np.testing.assert_allclose(g2[:, 1], s2[:, 1], atol=1e-12)
    np.testing.assert_allclose(g2[:, 2], 0.0, atol=1e-12)
    # every ghost's source had a boundary point among its K nearest neighbours
    nbr, _ = oracle_mod.knn(P, 16)
    assert mask[nbr[interior[src]]].any(1).all()


def test_neumann_rows_sum_to_zero_and_converge(oracle_mod):
    """Folded rows still sum to zero (constants are in the kernel of the Neumann Laplacian), and
    on the upper hemisphere (sigma - Delta) U = (sigma + 6) z^2 - 2 with dU/dn = 0 at the equator
    has the solution U = z^2: the discrete solution approaches it."""
    errs = []
    for n in (2000, 8000):
        cl = clouds.hemisphere(n, 8, 20)
        P, m = cl.points, cl.meta["boundary"]
        rp, c, v, g = oracle_mod.neumann_rows(P, m, 20, 6)
        rs = np.add.reduceat(v, rp[:-1])
        assert np.abs(rs).max() <= 1e-12 * np.abs(v).max() * 20
        z = P[g[0], 2]
        x = oracle_mod.solve(rp, c, v, 7.0 * z ** 2 - 2.0, sigma=1.0)
        errs.append(np.abs(x - z ** 2).max())
    assert errs[0] < 5e-3 and errs[0] / errs[1] > 3.0, errs


# ----------------------------------------------------------------------------------------------
# eigenvalues (Sec. 4: -Delta nu = lambda nu)
# ----------------------------------------------------------------------------------------------
def test_eigenvalues_match_the_closed_form_spectra(oracle_mod):
    """Unit sphere: l (l + 1) with multiplicity 2 l + 1; upper hemisphere with the boundary points
    removed (Dirichlet): n (n + 1) with multiplicity n; with the reflection ghosts folded
    (Neumann): n (n - 1) with multiplicity n. At 2,000 points the smallest eigenvalues of the
    oracle's matrices lie within 2-3% of them, and the error falls when the sampling refines."""
    def spectrum(levels, mult):
        return np.concatenate([np.full(mult(l), lam) for l, lam in levels])

    errs = []
    for n in (1000, 2000):
        P = clouds.sphere(n, 1, 20).points
        rp, c, v = oracle_mod.assemble(P, 20)
        lam = oracle_mod.eigenvalues(rp, c, v, 16)
        exact = spectrum([(0, 0.0), (1, 2.0), (2, 6.0), (3, 12.0)], lambda l: 2 * l + 1)
        assert abs(lam[0]) < 1e-8
        errs.append((np.abs(np.sort(lam.real) - exact)[1:] / exact[1:]).max())
    assert errs[1] < 0.02 and errs[1] < errs[0], errs
    cl = clouds.hemisphere(2000, 8, 20)
    m = cl.meta["boundary"]
    rp, c, v = oracle_mod.assemble(cl.points, 20)
    lam = oracle_mod.eigenvalues(rp, c, v, 10, keep=np.nonzero(~m)[0])
    exact = spectrum([(1, 2.0), (2, 6.0), (3, 12.0), (4, 20.0)], lambda l: l)
    assert (np.abs(np.sort(lam.real) - exact) / exact).max() < 0.03
    rp, c, v, g = oracle_mod.neumann_rows(cl.points, m, 20, 6)
    lam = oracle_mod.eigenvalues(rp, c, v, 10)
    exact = spectrum([(1, 0.0), (2, 2.0), (3, 6.0), (4, 12.0)], lambda l: l)
    assert abs(lam[0]) < 1e-8
    assert (np.abs(np.sort(lam.real) - exact)[1:] / exact[1:]).max() < 0.03
