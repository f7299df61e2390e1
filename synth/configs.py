"""Seeded synthetic low-rank-on-graph workloads.

Each builder returns a :class:`Problem`: the full graphs (L_r, L_c), the
sampling sets (Omega_r, Omega_c), the sampled matrix Y~ = Y[Omega_r][:, Omega_c]
(Section III, sampling matrices of eq. (Mc)), the compressed graphs rebuilt
as K-NN graphs on the sampled points (Section IV.A offers this rebuild beside
Kron reduction; Section VII.A rebuilds with FLANN) and their largest
eigenvalues, which the step size of Algorithm 1 needs (Section IV.B).

Nothing here runs the solvers. The data follow Definition 1: X is built from
the first k Laplacian eigenvectors of the row and column graphs, then noise
and sparse outliers are added.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

from .graphs import knn_laplacian, laplacian_lmax, low_eigvecs

__all__ = ["Problem", "round_count", "make_problem", "cfg1_tiny", "cfg2_face",
           "cfg3_video", "cfg5_batch", "small_problem", "grid_coords",
           "circle_coords", "helix_coords", "cluster_digits", "digits_points"]


@dataclasses.dataclass
class Problem:
    name: str
    p: int
    n: int
    Lr: sp.csr_matrix          # p x p, FP64, symmetric PSD
    Lc: sp.csr_matrix          # n x n
    omega_r: np.ndarray        # int32, sorted, unique, in [0, p)
    omega_c: np.ndarray        # int32, sorted, unique, in [0, n)
    Ytil: np.ndarray           # rho_r x rho_c FP64 (row-major)
    Lr_til: sp.csr_matrix      # rho_r x rho_r
    Lc_til: sp.csr_matrix      # rho_c x rho_c
    lmax_r_til: float
    lmax_c_til: float
    gamma_r: float = 1.0
    gamma_c: float = 1.0
    fista_iters: int = 500
    tol: float = 1e-10
    X_true: np.ndarray | None = None   # low-rank part (informational only)
    Y: np.ndarray | None = None        # full data (not needed by the solvers)
    meta: dict = dataclasses.field(default_factory=dict)  # workload-specific extras

    @property
    def rho_r(self) -> int:
        return int(self.omega_r.size)

    @property
    def rho_c(self) -> int:
        return int(self.omega_c.size)


def round_count(frac: float, dim: int, minimum: int = 1) -> int:
    """rho = round(frac * dim), round half to even, at least `minimum`."""
    return max(minimum, int(round(frac * dim)))


def grid_coords(h: int, w: int) -> np.ndarray:
    """Pixel (row, col) coordinates of an h x w image in raster order."""
    r, c = np.divmod(np.arange(h * w), w)
    return np.stack([r, c], axis=1).astype(np.float64)


def circle_coords(n: int, rng: np.random.Generator, noise_std: float) -> np.ndarray:
    th = 2.0 * np.pi * np.arange(n) / n
    pts = np.stack([np.cos(th), np.sin(th), np.zeros(n)], axis=1)
    return pts + noise_std * rng.standard_normal(pts.shape)


def helix_coords(p: int) -> np.ndarray:
    t = np.linspace(0.0, 4.0 * np.pi, p)
    return np.stack([np.cos(t), np.sin(t), t / (4.0 * np.pi)], axis=1)


def _sample(rng: np.random.Generator, dim: int, count: int) -> np.ndarray:
    return np.sort(rng.choice(dim, size=count, replace=False)).astype(np.int32)


def make_problem(name: str, row_coords: np.ndarray, col_coords: np.ndarray,
                 rank: int, rng: np.random.Generator, *,
                 sv: np.ndarray, noise_std: float = 0.0,
                 outlier_frac: float = 0.0, outlier_amp: float = 1.0,
                 frac_r: float = 0.1, frac_c: float = 0.1, min_rho: int = 1,
                 K: int = 10, kind: str = "normalized",
                 gamma_r: float = 1.0, gamma_c: float = 1.0,
                 fista_iters: int = 500, tol: float = 1e-10,
                 extra=None, keep_full: bool = False) -> Problem:
    """Generic low-rank-on-graphs instance (Definition 1 plus noise)."""
    p, n = row_coords.shape[0], col_coords.shape[0]
    Lr, _ = knn_laplacian(row_coords, K, kind)
    Lc, _ = knn_laplacian(col_coords, K, kind)
    Ur = low_eigvecs(Lr, rank)
    Vc = low_eigvecs(Lc, rank)
    X = (Ur * sv[None, :]) @ Vc.T
    Y = X.copy()
    if noise_std > 0:
        Y += noise_std * rng.standard_normal(Y.shape)
    if outlier_frac > 0:
        cnt = int(round(outlier_frac * p * n))
        pos = rng.choice(p * n, size=cnt, replace=False)
        Y.reshape(-1)[pos] += rng.uniform(-outlier_amp, outlier_amp, size=cnt)
    if extra is not None:
        extra(Y, rng)
    rho_r = round_count(frac_r, p, min_rho)
    rho_c = round_count(frac_c, n, min_rho)
    om_r = _sample(rng, p, rho_r)
    om_c = _sample(rng, n, rho_c)
    Ytil = np.ascontiguousarray(Y[np.ix_(om_r, om_c)])
    Lr_t, _ = knn_laplacian(row_coords[om_r], min(K, rho_r - 1), kind)
    Lc_t, _ = knn_laplacian(col_coords[om_c], min(K, rho_c - 1), kind)
    return Problem(name=name, p=p, n=n, Lr=Lr, Lc=Lc, omega_r=om_r,
                   omega_c=om_c, Ytil=Ytil, Lr_til=Lr_t, Lc_til=Lc_t,
                   lmax_r_til=laplacian_lmax(Lr_t), lmax_c_til=laplacian_lmax(Lc_t),
                   gamma_r=gamma_r, gamma_c=gamma_c, fista_iters=fista_iters,
                   tol=tol, X_true=X if keep_full else None,
                   Y=Y if keep_full else None)


def cfg1_tiny(seed: int = 0) -> Problem:
    """p=100 (helix rows) x n=200 (noisy unit circle columns), rank 5,
    N(0,1e-2) noise, 5% outliers in +-1, 50 x 100 samples, gamma = 1,
    500 FISTA iterations, decoder residual 1e-10. FP64."""
    rng = np.random.default_rng(seed)
    cols = circle_coords(200, rng, noise_std=0.1)
    rows = helix_coords(100)
    sv = rng.standard_normal(5)
    return make_problem("cfg1_tiny", rows, cols, 5, rng, sv=sv, noise_std=0.1,
                        outlier_frac=0.05, frac_r=0.5, frac_c=0.5,
                        fista_iters=500, tol=1e-10, keep_full=True)


def _scaled_sv(rng, k, p, n):
    # singular values that give entries of order one
    return math.sqrt(p * n) * rng.uniform(0.5, 1.0, size=k) / math.sqrt(k)


def _smooth_fields(rng, h, w, count, blur):
    from scipy.ndimage import gaussian_filter
    out = np.empty((count, h * w))
    for i in range(count):
        f = gaussian_filter(rng.standard_normal((h, w)), blur, mode="wrap")
        out[i] = (f / f.std()).ravel()
    return out


def cfg2_face(seed: int = 0, n: int = 1000, shape=(112, 92)) -> Problem:
    """Face-shaped stand-in: p = 112*92 pixels (2-D coordinate features),
    n samples that are smooth random fields placed along a latent circle,
    rank 10, 10% outliers in +-1, 10% row and column sampling."""
    rng = np.random.default_rng(seed)
    h, w = shape
    rows = grid_coords(h, w)
    base = _smooth_fields(rng, h, w, 3, 3.0)
    th = 2.0 * np.pi * np.arange(n) / n
    cols = (np.cos(th)[:, None] * base[0] + np.sin(th)[:, None] * base[1]
            + 0.05 * rng.standard_normal((n, 1)) * base[2])
    p = h * w
    sv = _scaled_sv(rng, 10, p, n)
    return make_problem("cfg2_face", rows, cols, 10, rng, sv=sv,
                        outlier_frac=0.10, frac_r=0.1, frac_c=0.1,
                        fista_iters=500, tol=1e-10)


def _blobs(h, w, nframes, frac, rng):
    """Moving 8x8 blobs covering about `frac` of all entries, values U(0.5, 1)."""
    nb = max(1, int(round(frac * h * w / 64.0)))
    pos = rng.uniform([0, 0], [h - 8, w - 8], size=(nb, 2))
    vel = rng.uniform(-1.5, 1.5, size=(nb, 2))

    def add(Y, rng2):
        for t in range(nframes):
            for b in range(nb):
                r0, c0 = pos[b]
                r0, c0 = int(r0), int(c0)
                idx = ((np.arange(r0, r0 + 8)[:, None] * w)
                       + np.arange(c0, c0 + 8)[None, :]).ravel()
                Y[idx, t] += rng2.uniform(0.5, 1.0, size=64)
            pos[:] += vel
            for ax, lim in ((0, h - 8), (1, w - 8)):
                lo = pos[:, ax] < 0
                hi = pos[:, ax] > lim
                vel[lo | hi, ax] *= -1
                pos[:, ax] = np.clip(pos[:, ax], 0, lim)
    return add


def cfg3_video(seed: int = 0, shape=(128, 160), nframes: int = 4096,
               frac: float = 0.05, keep_full: bool = False) -> Problem:
    """Video-shaped stand-in: p = 128*160 pixels, n = 4096 frames (10-NN on the
    frame-time coordinate: a band graph), rank-5 background plus moving 8x8
    blobs on 2% of entries with values U(0.5, 1), 5% row/column sampling."""
    rng = np.random.default_rng(seed)
    h, w = shape
    rows = grid_coords(h, w)
    cols = np.arange(nframes, dtype=np.float64)[:, None]
    p = h * w
    sv = _scaled_sv(rng, 5, p, nframes)
    return make_problem("cfg3_video", rows, cols, 5, rng, sv=sv,
                        extra=_blobs(h, w, nframes, 0.02, rng),
                        frac_r=frac, frac_c=frac, fista_iters=500, tol=1e-10,
                        keep_full=keep_full)


def small_problem(seed: int, p_shape=(12, 10), n: int = 150, rank: int = 4,
                  frac: float = 0.3, gamma=(1.0, 1.0), kind="normalized",
                  K: int = 10, fista_iters: int = 100, tol: float = 1e-10,
                  col_kind: str = "circle", keep_full: bool = False) -> Problem:
    """Scaled-down instance for parity tests: pixel-grid rows, circle or band
    columns. Sizes are free so that tests can span tiles and ragged tails."""
    rng = np.random.default_rng(seed)
    rows = grid_coords(*p_shape)
    if col_kind == "circle":
        cols = circle_coords(n, rng, noise_std=0.05)
    else:
        cols = np.arange(n, dtype=np.float64)[:, None]
    p = rows.shape[0]
    sv = _scaled_sv(rng, rank, p, n)
    return make_problem(f"small_{seed}", rows, cols, rank, rng, sv=sv,
                        noise_std=0.05, outlier_frac=0.05, frac_r=frac,
                        frac_c=frac, min_rho=K + 2, K=K, kind=kind,
                        gamma_r=gamma[0], gamma_c=gamma[1],
                        fista_iters=fista_iters, tol=tol, keep_full=keep_full)


def cfg5_batch(seed: int = 0, count: int = 64, scale: float = 1.0):
    """Batched workload: `count` instances with p log-uniform in [500, 4000]
    and n log-uniform in [200, 2000] (both multiplied by `scale`), rank 3..10,
    helix rows / circle columns, 5% outliers, 10% sampling (at least 20), and a
    4 x 4 gamma grid in {0.1, 1, 10, 100}. Returns (instances, gamma_grid)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        p = int(round(math.exp(rng.uniform(math.log(500), math.log(4000))) * scale))
        n = int(round(math.exp(rng.uniform(math.log(200), math.log(2000))) * scale))
        p, n = max(p, 40), max(n, 40)
        k = int(rng.integers(3, 11))
        rows = helix_coords(p)
        cols = circle_coords(n, rng, noise_std=0.05)
        sv = _scaled_sv(rng, k, p, n)
        out.append(make_problem(f"cfg5_{i}", rows, cols, k, rng, sv=sv,
                                noise_std=0.0, outlier_frac=0.05, frac_r=0.1,
                                frac_c=0.1, min_rho=20, fista_iters=100,
                                tol=1e-6))
    grid = [(gr, gc) for gr in (0.1, 1.0, 10.0, 100.0)
            for gc in (0.1, 1.0, 10.0, 100.0)]
    return out, grid


def cluster_digits(seed: int = 0, n: int = 70000, side: int = 28, k: int = 10,
                   frac_c: float = 0.05, K: int = 10, spread: float = 1.0) -> Problem:
    """Clustering stand-in with the shape of the paper's large digit set
    (p = 28 x 28 pixel features, n = 70000 samples, k = 10 classes; the
    paper compresses such sets along the samples only, so every row is kept
    and 5% of the columns are sampled).

    Samples sit in a 3-D latent space around k class centres (std `spread`,
    centres uniform in [0, 12]^3), and the column graph is the 10-NN graph on
    those latent points. A sample's data column is its class template (a
    smooth random image) plus a rank-3 within-class variation, Gaussian noise
    (std 0.1) and 5% outliers U(-1, 1). The row graph is the 10-NN graph of
    the pixel grid. Only the sampled columns are generated (Algorithm 3 needs
    no other data). meta: labels (n true classes) and init (k sampled column
    positions drawn at random, the seeds of k-means)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 12.0, size=(k, 3))
    labels = rng.integers(0, k, size=n)
    lat = centres[labels] + spread * rng.standard_normal((n, 3))
    lat_all = lat
    rows = grid_coords(side, side)
    p = side * side
    Lr, _ = knn_laplacian(rows, K)
    Lc, _ = knn_laplacian(lat, K)
    rho_c = round_count(frac_c, n, K + 2)
    om_c = _sample(rng, n, rho_c)
    om_r = np.arange(p, dtype=np.int32)
    templates = _smooth_fields(rng, side, side, k, 2.0)
    var = _smooth_fields(rng, side, side, 3, 2.0)
    lab_s = labels[om_c]
    Y = (templates[lab_s] + 0.3 * rng.standard_normal((rho_c, 3)) @ var
         + 0.1 * rng.standard_normal((rho_c, p))).T
    cnt = int(round(0.05 * p * rho_c))
    pos = rng.choice(p * rho_c, size=cnt, replace=False)
    Y.reshape(-1)[pos] += rng.uniform(-1.0, 1.0, size=cnt)
    Ytil = np.ascontiguousarray(Y)
    Lc_t, _ = knn_laplacian(lat[om_c], min(K, rho_c - 1))
    init = np.sort(rng.choice(rho_c, size=k, replace=False)).astype(np.int32)
    return Problem(name="cluster_digits", p=p, n=n, Lr=Lr, Lc=Lc, omega_r=om_r, omega_c=om_c,
                   Ytil=Ytil, Lr_til=Lr, Lc_til=Lc_t, lmax_r_til=laplacian_lmax(Lr),
                   lmax_c_til=laplacian_lmax(Lc_t), gamma_r=1.0, gamma_c=1.0,
                   fista_iters=500, tol=1e-10,
                   meta=dict(labels=labels, init=init, k=k, latent=lat_all))


def digits_points(seed: int = 0, n: int = 70000, side: int = 28, k: int = 10,
                  dtype=np.float64) -> tuple[np.ndarray, np.ndarray]:
    """Digit-shaped point set for graph construction between samples: n
    points of dimension side^2 in k classes. A point is its class template (a
    smooth random image, unit standard deviation) plus a rank-3 smooth
    within-class variation (std 0.3 per factor) and Gaussian noise (std 0.1).
    Returns (points n x side^2, labels)."""
    rng = np.random.default_rng(seed)
    templates = _smooth_fields(rng, side, side, k, 2.0)
    var = _smooth_fields(rng, side, side, 3, 2.0)
    labels = rng.integers(0, k, size=n)
    pts = np.empty((n, side * side), dtype=dtype)
    for s0 in range(0, n, 10000):
        s1 = min(n, s0 + 10000)
        m = s1 - s0
        pts[s0:s1] = (templates[labels[s0:s1]] + 0.3 * rng.standard_normal((m, 3)) @ var
                      + 0.1 * rng.standard_normal((m, side * side)))
    return pts, labels
