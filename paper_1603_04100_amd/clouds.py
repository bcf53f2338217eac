"""Seeded synthetic point clouds and test functions with closed-form Laplace-Beltrami values.

This module holds no part of the MVGD discretisation itself. It produces the inputs that
both the GPU path and the FP64 oracle consume, plus the exact surface Laplacians used to
report discretisation error. Everything is numpy, seeded with ``numpy.random.default_rng``
(PCG64), so every workload is reproducible from its seed.

Workloads (the paper's experiments sample a unit sphere at random, Sec. 4.2 and 4.3; the
remaining surfaces are synthetic stand-ins of the same kind, since the paper's public clouds
are not available):

* ``sphere``           unit sphere in R^3, normalised standard Gaussian (uniform density).
* ``hemisphere``       upper unit hemisphere with its boundary circle sampled (open surface).
* ``circle``, ``helix`` curves (d = 1): the unit circle of Sec. 4.2 and an open helix in R^3.
* ``torus``            torus in R^3 with tube-angle density proportional to 1 + 0.5 cos(theta).
* ``ellipsoid_batch``  many ellipsoids of log-uniform size (batched assembly).
* ``flat_torus4``      flat torus (cos t, sin t, cos p, sin p) in R^4 plus Gaussian noise.
* ``serving_stream``   Poisson arrivals of random spheres / ellipsoids / tori.

Closed forms used for the exact Laplacians:

* sphere: Re((x+iy)^l) is a degree-l spherical harmonic, so Delta f = -l(l+1) f; on any surface
  Delta of the position vector is -2H n, so on the unit sphere Delta x = -2x (Sec. 4.2).
* torus (R, r): Delta f = f_tt / r^2 - sin(t) f_t / (r rho) + f_pp / rho^2, rho = R + r cos t.
* flat torus: Delta = d_tt + d_pp.
* implicit surface phi = 0 with unit normal n = grad phi / |grad phi|:
  Delta_S f = Delta f - n^T (Hess f) n - (div n)(n . grad f).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Cloud", "sphere", "hemisphere", "circle", "helix", "torus", "ellipsoid_batch", "flat_torus4", "serving_stream",
    "random_plane", "line_example", "sphere_harmonic", "implicit_laplacian",
    "ellipsoid_functions", "config", "CONFIGS",
]


@dataclass
class Cloud:
    """A point cloud (or a batch of clouds) with test functions.

    points:  float64 array [N, n] (row-major). For FP32-mixed runs callers round it with
             ``points.astype(np.float32)`` and hand the same rounded values to the oracle.
    offsets: int64 array [n_clouds + 1] of row offsets (a single cloud has [0, N]).
    f:       float64 array [N, R] of test function samples (R right-hand sides).
    lap_f:   float64 array [N, R] of the exact surface Laplacian of ``f`` (NaN if unknown).
    """
    name: str
    points: np.ndarray
    offsets: np.ndarray
    k: int
    f: np.ndarray
    lap_f: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_points(self) -> int:
        return int(self.points.shape[0])

    @property
    def n_ambient(self) -> int:
        return int(self.points.shape[1])


def _single(name, pts, k, f, lap, **meta):
    f = np.asarray(f, dtype=np.float64)
    lap = np.asarray(lap, dtype=np.float64)
    if f.ndim == 1:
        f = f[:, None]
        lap = lap[:, None]
    return Cloud(name, np.ascontiguousarray(pts, dtype=np.float64),
                 np.array([0, pts.shape[0]], dtype=np.int64), k, f, lap, dict(meta))


# ----------------------------------------------------------------------------------------
# sphere
# ----------------------------------------------------------------------------------------
def sphere_points(n: int, rng: np.random.Generator) -> np.ndarray:
    x = rng.standard_normal((n, 3))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x


def sphere_harmonic(points: np.ndarray, l: int) -> np.ndarray:
    """Re((x + i y)^l): a degree-l harmonic polynomial; on the unit sphere Delta f = -l(l+1) f."""
    z = (points[:, 0] + 1j * points[:, 1]) ** l
    return np.real(z)


def sphere(n: int = 2000, seed: int = 1, k: int = 20, degrees=(1,)) -> Cloud:
    """Unit sphere, uniform density. Default f = x (degree 1), Delta f = -2 f."""
    rng = np.random.default_rng(seed)
    p = sphere_points(n, rng)
    f = np.stack([sphere_harmonic(p, l) for l in degrees], axis=1)
    lap = np.stack([-l * (l + 1) * sphere_harmonic(p, l) for l in degrees], axis=1)
    return _single("sphere", p, k, f, lap, seed=seed, degrees=list(degrees))


def hemisphere(n: int = 4000, seed: int = 8, k: int = 20, n_boundary: int | None = None) -> Cloud:
    """Upper unit hemisphere (Sec. 4.3's open surface): n random points with z > 0 plus
    n_boundary (default ~ sqrt(pi n)) equispaced points on the boundary circle z = 0, listed last;
    meta["boundary"] is the boundary mask. f = z: Delta f = -2 f and f = 0 on the boundary, so U = z
    solves -Delta U = 2z with the Dirichlet condition U = 0."""
    rng = np.random.default_rng(seed)
    p = sphere_points(n, rng)
    p[:, 2] = np.abs(p[:, 2])
    nb = int(round(math.sqrt(math.pi * n))) if n_boundary is None else n_boundary
    t = rng.uniform(0.0, 2.0 * np.pi) + 2.0 * np.pi * np.arange(nb) / nb
    q = np.stack([np.cos(t), np.sin(t), np.zeros(nb)], axis=1)
    pts = np.concatenate([p, q])
    mask = np.zeros(len(pts), dtype=bool)
    mask[n:] = True
    return _single("hemisphere", pts, k, pts[:, 2], -2.0 * pts[:, 2], seed=seed, boundary=mask)


# ----------------------------------------------------------------------------------------
# curves (d = 1)
# ----------------------------------------------------------------------------------------
def circle(n: int = 4000, seed: int = 6, k: int = 6, sampling: str = "random") -> Cloud:
    """Unit circle in R^2 (Sec. 4.2). sampling: "uniform" (equispaced angles, rotated by a random
    offset) or "random" (angles ~ U[0, 2pi)). f = sin(2t), Delta f = -4 sin(2t); the paper's
    solve uses U = -sin(2t) with -Delta U = -4 sin(2t)."""
    rng = np.random.default_rng(seed)
    if sampling == "uniform":
        t = rng.uniform(0.0, 2.0 * np.pi) + 2.0 * np.pi * np.arange(n) / n
    else:
        t = rng.uniform(0.0, 2.0 * np.pi, n)
    p = np.stack([np.cos(t), np.sin(t)], axis=1)
    return _single("circle", p, k, np.sin(2 * t), -4.0 * np.sin(2 * t), seed=seed,
                   sampling=sampling, d=1)


def helix(n: int = 4000, seed: int = 7, k: int = 8, pitch: float = 0.3,
          turns: float = 2.0) -> Cloud:
    """Helix (cos t, sin t, pitch t), t ~ U[0, 2pi turns) (an open curve). Arclength
    s = t sqrt(1 + pitch^2); f = sin(2t), Delta f = d^2 f / ds^2 = -4 sin(2t) / (1 + pitch^2)
    (the rows near the two ends see one-sided neighbourhoods)."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, 2.0 * np.pi * turns, n)
    p = np.stack([np.cos(t), np.sin(t), pitch * t], axis=1)
    return _single("helix", p, k, np.sin(2 * t), -4.0 * np.sin(2 * t) / (1.0 + pitch ** 2),
                   seed=seed, pitch=pitch, turns=turns, d=1)


# ----------------------------------------------------------------------------------------
# torus in R^3
# ----------------------------------------------------------------------------------------
def torus(n: int = 200_000, seed: int = 2, k: int = 24, R: float = 1.0, r: float = 0.4,
          nonuniform: bool = True) -> Cloud:
    """Torus ((R + r cos t) cos p, (R + r cos t) sin p, r sin t).

    p ~ U[0, 2pi). t is drawn by rejection from U[0, 2pi) with acceptance (1 + 0.5 cos t)/1.5,
    so the density in t is proportional to 1 + 0.5 cos t (t = 0 is the outer equator).
    f = cos(3p) sin(t), evaluated at the clean angles.
    """
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    th = np.empty(n)
    filled = 0
    while filled < n:
        cand = rng.uniform(0.0, 2.0 * np.pi, 2 * (n - filled) + 64)
        if nonuniform:
            acc = rng.uniform(0.0, 1.0, cand.shape[0]) < (1.0 + 0.5 * np.cos(cand)) / 1.5
            cand = cand[acc]
        take = min(n - filled, cand.shape[0])
        th[filled:filled + take] = cand[:take]
        filled += take
    rho = R + r * np.cos(th)
    p = np.stack([rho * np.cos(ph), rho * np.sin(ph), r * np.sin(th)], axis=1)
    f = np.cos(3 * ph) * np.sin(th)
    lap = np.cos(3 * ph) * (-np.sin(th) / r**2 - np.sin(th) * np.cos(th) / (r * rho)
                            - 9.0 * np.sin(th) / rho**2)
    return _single("torus", p, k, f, lap, seed=seed, R=R, r=r, nonuniform=nonuniform)


# ----------------------------------------------------------------------------------------
# flat torus in R^4
# ----------------------------------------------------------------------------------------
def flat_torus4(n: int = 1_000_000, seed: int = 4, k: int = 32, noise: float = 1e-4) -> Cloud:
    """(cos t, sin t, cos p, sin p) + noise * N(0, I4); f = cos(2t) cos(3p), Delta f = -13 f."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, 2.0 * np.pi, n)
    p = rng.uniform(0.0, 2.0 * np.pi, n)
    x = np.stack([np.cos(t), np.sin(t), np.cos(p), np.sin(p)], axis=1)
    if noise > 0:
        x = x + noise * rng.standard_normal((n, 4))
    f = np.cos(2 * t) * np.cos(3 * p)
    return _single("flat_torus4", x, k, f, -13.0 * f, seed=seed, noise=noise)


# ----------------------------------------------------------------------------------------
# implicit surfaces (ellipsoids) and their exact Laplacians
# ----------------------------------------------------------------------------------------
def implicit_laplacian(grad_phi, hess_phi, grad_f, hess_f):
    """Delta_S f on the level set phi = 0 (all inputs per point).

    grad_phi [N,3], hess_phi [N,3,3], grad_f [N,3], hess_f [N,3,3].
    n = grad phi/|grad phi|; div n = (tr Hphi - n^T Hphi n)/|grad phi|;
    Delta_S f = tr Hf - n^T Hf n - (div n)(n . grad f).
    """
    gn = np.linalg.norm(grad_phi, axis=1)
    nrm = grad_phi / gn[:, None]
    nHn_phi = np.einsum("ni,nij,nj->n", nrm, hess_phi, nrm)
    div_n = (np.trace(hess_phi, axis1=1, axis2=2) - nHn_phi) / gn
    nHn_f = np.einsum("ni,nij,nj->n", nrm, hess_f, nrm)
    return np.trace(hess_f, axis1=1, axis2=2) - nHn_f - div_n * np.einsum("ni,ni->n", nrm, grad_f)


def ellipsoid_functions(points: np.ndarray, axes: np.ndarray):
    """f in {x, y, z, xy} and their exact Laplacians on the ellipsoid sum (x_k/a_k)^2 = 1."""
    n = points.shape[0]
    a2 = np.asarray(axes, dtype=np.float64) ** 2
    grad_phi = 2.0 * points / a2
    hess_phi = np.broadcast_to(np.diag(2.0 / a2), (n, 3, 3))
    fs, laps = [], []
    zero_h = np.zeros((n, 3, 3))
    for c in range(3):
        g = np.zeros((n, 3))
        g[:, c] = 1.0
        fs.append(points[:, c])
        laps.append(implicit_laplacian(grad_phi, hess_phi, g, zero_h))
    g = np.stack([points[:, 1], points[:, 0], np.zeros(n)], axis=1)
    h = np.zeros((n, 3, 3))
    h[:, 0, 1] = h[:, 1, 0] = 1.0
    fs.append(points[:, 0] * points[:, 1])
    laps.append(implicit_laplacian(grad_phi, hess_phi, g, h))
    return np.stack(fs, axis=1), np.stack(laps, axis=1)


def ellipsoid_batch(n_clouds: int = 256, seed: int = 3, k: int = 20, n_min: int = 1000,
                    n_max: int = 100_000) -> Cloud:
    """Many ellipsoids: axes ~ U[0.5, 2]^3, sizes round(exp(U[ln n_min, ln n_max])).

    Points are a normalised Gaussian scaled by the axes (so they lie exactly on the
    ellipsoid; the density is not area-uniform). Four right-hand sides: x, y, z, xy.
    """
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_clouds))).astype(np.int64)
    axes = rng.uniform(0.5, 2.0, (n_clouds, 3))
    pts, fs, laps = [], [], []
    for c in range(n_clouds):
        s = sphere_points(int(sizes[c]), rng) * axes[c]
        f, lap = ellipsoid_functions(s, axes[c])
        pts.append(s)
        fs.append(f)
        laps.append(lap)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return Cloud("ellipsoid_batch", np.ascontiguousarray(np.concatenate(pts)), offsets, k,
                 np.concatenate(fs), np.concatenate(laps),
                 dict(seed=seed, axes=axes, sizes=sizes))


# ----------------------------------------------------------------------------------------
# small structured inputs used by the pins
# ----------------------------------------------------------------------------------------
def random_plane(n: int, n_ambient: int, seed: int, extent: float = 1.0):
    """n points uniform on a random 2-plane through a random offset in R^n_ambient.

    Returns (points, basis [2, n_ambient] orthonormal, offset [n_ambient]).
    """
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n_ambient, n_ambient)))
    basis = q[:, :2].T
    off = rng.standard_normal(n_ambient)
    uv = rng.uniform(-extent, extent, (n, 2))
    return off + uv @ basis, basis, off


def line_example(k_spacing: float, n_ambient: int = 2, direction=None, offset=None):
    """The paper's 1-D worked example: 5 equispaced samples x = -2k, -k, 0, k, 2k on a line."""
    d = np.zeros(n_ambient)
    d[0] = 1.0
    if direction is not None:
        d = np.asarray(direction, dtype=np.float64)
        d = d / np.linalg.norm(d)
    o = np.zeros(n_ambient) if offset is None else np.asarray(offset, dtype=np.float64)
    t = k_spacing * np.arange(-2, 3, dtype=np.float64)
    return o + t[:, None] * d[None, :]


# ----------------------------------------------------------------------------------------
# serving stream
# ----------------------------------------------------------------------------------------
def _random_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    return q * np.sign(np.diag(r))


def serving_stream(duration_s: float = 30.0, rate_hz: float = 200.0, seed: int = 5,
                   k: int = 24, n_min: int = 5000, n_max: int = 500_000, noise: float = 1e-3,
                   n_apply: int = 8, max_requests: int | None = None):
    """Poisson arrivals of random clouds. Yields dicts with arrival time, points, RHS list.

    Shape is uniform over {sphere r ~ U[0.5, 2], ellipsoid axes ~ U[0.5, 2]^3,
    torus R ~ U[0.8, 1.5], r = R U[0.2, 0.5]}, randomly rotated; sizes log-uniform in
    [n_min, n_max]; Gaussian noise sigma = noise; n_apply smooth right-hand sides.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    count = 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s or (max_requests is not None and count >= max_requests):
            return
        n = int(np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        shape = int(rng.integers(0, 3))
        if shape == 0:
            p = sphere_points(n, rng) * rng.uniform(0.5, 2.0)
        elif shape == 1:
            p = sphere_points(n, rng) * rng.uniform(0.5, 2.0, 3)
        else:
            Rm = rng.uniform(0.8, 1.5)
            rm = Rm * rng.uniform(0.2, 0.5)
            th = rng.uniform(0, 2 * np.pi, n)
            ph = rng.uniform(0, 2 * np.pi, n)
            rho = Rm + rm * np.cos(th)
            p = np.stack([rho * np.cos(ph), rho * np.sin(ph), rm * np.sin(th)], axis=1)
        p = p @ _random_rotation(rng).T + noise * rng.standard_normal((n, 3))
        w = rng.standard_normal((n_apply, 3))
        rhs = np.stack([np.sin(p @ w[j]) for j in range(n_apply)], axis=1)
        yield dict(arrival=t, points=np.ascontiguousarray(p), k=k, rhs=rhs,
                   shape=["sphere", "ellipsoid", "torus"][shape], id=count)
        count += 1


# ----------------------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------------------
CONFIGS = {
    "sphere_2k": dict(fn=sphere, kw=dict(n=2000, seed=1, k=20)),
    "torus_200k": dict(fn=torus, kw=dict(n=200_000, seed=2, k=24)),
    "ellipsoids_256": dict(fn=ellipsoid_batch, kw=dict(n_clouds=256, seed=3, k=20)),
    "flat_torus4_1m": dict(fn=flat_torus4, kw=dict(n=1_000_000, seed=4, k=32)),
    "circle_100k": dict(fn=circle, kw=dict(n=100_000, seed=6, k=6)),
}


def config(name: str, **override) -> Cloud:
    c = CONFIGS[name]
    kw = dict(c["kw"])
    kw.update(override)
    return c["fn"](**kw)
