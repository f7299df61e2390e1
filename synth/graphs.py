"""K-nearest-neighbour graphs and their Laplacians for synthetic inputs.

Graph construction is the first stage of the method (Section I, the K-NN
Gaussian-kernel graph and the Laplacians L = D - W and
L_n = D^{-1/2} (D - W) D^{-1/2}; Table I step 1). It is input preparation,
not part of the solvers: both the HIP library and the CPU oracle receive the
Laplacians built here as CSR matrices.

Readings taken where the paper leaves a choice open:
  * self is never its own neighbour; edges are the union of the directed
    K-NN relations ("or vice versa");
  * ties in distance are broken by node index;
  * sigma is the mean Euclidean distance from each node to its K nearest
    neighbours, and W_ij = exp(-d_ij^2 / sigma^2);
  * every CSR row stores its diagonal entry, column indices are sorted.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.spatial import cKDTree

__all__ = ["knn_indices", "knn_laplacian", "laplacian_lmax", "low_eigvecs"]


def knn_indices(coords: np.ndarray, K: int) -> tuple[np.ndarray, np.ndarray]:
    """Return (idx, dist) of the K nearest neighbours of every point.

    idx, dist have shape (N, K); rows are sorted by (distance, index) and
    exclude the point itself.
    """
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    if coords.ndim == 1:
        coords = coords[:, None]
    N, d = coords.shape
    if N <= K:
        raise ValueError(f"need more than K={K} points, got {N}")
    kq = min(N, K + 1 + 8)
    if d <= 16:
        tree = cKDTree(coords)
        _, cand = tree.query(coords, k=kq)
    else:
        # high-dimensional points: exact brute force in row blocks
        sq = np.einsum("ij,ij->i", coords, coords)
        cand = np.empty((N, kq), dtype=np.int64)
        for s in range(0, N, 512):
            e = min(N, s + 512)
            d2 = sq[s:e, None] + sq[None, :] - 2.0 * coords[s:e] @ coords.T
            cand[s:e] = np.argpartition(d2, kq - 1, axis=1)[:, :kq]
    cand = np.asarray(cand, dtype=np.int64)
    # exact squared distances of the candidates, recomputed directly
    diff = coords[cand] - coords[:, None, :]
    d2 = np.einsum("ijk,ijk->ij", diff, diff)
    self_mask = cand == np.arange(N)[:, None]
    d2 = np.where(self_mask, np.inf, d2)
    order = np.lexsort((cand, d2), axis=1)
    cand = np.take_along_axis(cand, order, axis=1)[:, :K]
    d2 = np.take_along_axis(d2, order, axis=1)[:, :K]
    if not np.all(np.isfinite(d2)):
        raise ValueError("duplicate-free neighbour search failed")
    return cand, np.sqrt(d2)


def knn_laplacian(coords: np.ndarray, K: int = 10, kind: str = "normalized",
                  sigma: float | None = None) -> tuple[sp.csr_matrix, float]:
    """Symmetric K-NN Gaussian-kernel graph Laplacian as FP64 CSR.

    Returns (L, sigma). kind is "normalized" (L_n) or "combinatorial" (D - W).
    """
    idx, dist = knn_indices(coords, K)
    N = idx.shape[0]
    if sigma is None:
        sigma = float(dist.mean())
    w = np.exp(-(dist ** 2) / sigma ** 2)
    rows = np.repeat(np.arange(N), K)
    W = sp.coo_matrix((w.ravel(), (rows, idx.ravel())), shape=(N, N)).tocsr()
    W = W.maximum(W.T).tocsr()  # union of the directed K-NN relations
    W.setdiag(0.0)
    W.eliminate_zeros()
    deg = np.asarray(W.sum(axis=1)).ravel()
    if np.any(deg <= 0):
        raise ValueError("isolated node in K-NN graph")
    if kind == "combinatorial":
        L = sp.diags(deg) - W
    elif kind == "normalized":
        dm = 1.0 / np.sqrt(deg)
        L = sp.identity(N, format="csr") - sp.diags(dm) @ W @ sp.diags(dm)
    else:
        raise ValueError(kind)
    L = sp.csr_matrix(L)
    L.sum_duplicates()
    L.sort_indices()
    # make the operator exactly symmetric in floating point
    L = ((L + L.T) * 0.5).tocsr()
    L.sort_indices()
    if kind == "normalized":
        L.setdiag(1.0)
    return L, sigma


def laplacian_lmax(L: sp.spmatrix) -> float:
    """Largest eigenvalue (= spectral norm, L is PSD) of a Laplacian."""
    N = L.shape[0]
    if N <= 2000:
        return float(np.linalg.eigvalsh(L.toarray())[-1])
    v = spla.eigsh(L.tocsc(), k=1, which="LA", tol=1e-14,
                   v0=np.ones(N) / np.sqrt(N), return_eigenvectors=False)
    return float(v[-1])


def low_eigvecs(L: sp.spmatrix, k: int) -> np.ndarray:
    """First k eigenvectors (smallest eigenvalues) of a Laplacian, N x k."""
    N = L.shape[0]
    if N <= 400:
        _, V = np.linalg.eigh(L.toarray())
        return np.ascontiguousarray(V[:, :k])
    vals, V = spla.eigsh(L.tocsc(), k=k, sigma=-1e-3, which="LM",
                         v0=np.ones(N) / np.sqrt(N))
    order = np.argsort(vals)
    return np.ascontiguousarray(V[:, order])
