"""K-nearest-neighbour graphs and their Laplacians -- FP64 oracle (test
infrastructure only: only tests, the smoke check and the CPU baseline of the
benchmark use this module).

Definition (Section II, graphs between the rows or columns of a matrix;
Section VII-A, graph construction): every point y_i is joined to its K
nearest neighbours y_j in Euclidean distance; the weighted adjacency is
symmetric, W_ij = exp(-||y_i - y_j||^2 / sigma^2) when y_j is one of the K
nearest neighbours of y_i or y_i one of those of y_j, and 0 otherwise; D is
the diagonal of row sums of W; the combinatorial Laplacian is L = D - W and
the normalised one L_n = D^{-1/2} (D - W) D^{-1/2}.

Readings where the paper leaves a choice open:
  * a point is not its own neighbour;
  * neighbours are ordered by (squared distance, index): among equal
    distances the lower index comes first (this decides the K-th neighbour
    on regular grids);
  * sigma is the mean Euclidean distance from each point to its K nearest
    neighbours (the paper sets sigma^2 from the mean K-NN distance; the
    reading used throughout this repository takes that mean as sigma);
  * squared distances are sums over coordinates of squared differences,
    accumulated in coordinate order;
  * the normalised Laplacian has a unit diagonal and off-diagonal entries
    -W_ij / sqrt(D_ii D_jj); a point with D_ii = 0 cannot occur for K >= 1.

Everything is brute force: all N^2 distances, in row blocks.

Parity status: pinned (against a k-d tree search of the scipy library on
points with distinct distances; a five-point example on a line worked by
hand, including a tie; the pixel-grid tie-break; Laplacian invariants:
symmetry, zero row sums, positive semi-definiteness, the normalised form and
its null vector D^{1/2} 1, spectrum within [0, 2]).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["knn", "sigma_of", "adjacency", "laplacian", "knn_graph", "query_knn"]


def query_knn(points, queries, K: int):
    """The K nearest neighbours of the points with indices `queries` among
    all points (itself excluded), by (squared distance, index). Returns
    (idx (Q x K) int64, d2 (Q x K) FP64)."""
    Y = np.asarray(points, dtype=np.float64)
    if Y.ndim == 1:
        Y = Y[:, None]
    N = Y.shape[0]
    if not 1 <= K < N:
        raise ValueError("need 1 <= K < N")
    queries = np.asarray(queries, dtype=np.int64)
    idx = np.empty((queries.size, K), dtype=np.int64)
    d2o = np.empty((queries.size, K))
    block = max(1, min(512, int(2e7 // max(N * Y.shape[1], 1))))
    for s in range(0, queries.size, block):
        q = queries[s:s + block]
        d2 = np.zeros((q.size, N))
        for k in range(Y.shape[1]):              # coordinate order
            diff = Y[q, k][:, None] - Y[None, :, k]
            d2 += diff * diff
        d2[np.arange(q.size), q] = np.inf         # not its own neighbour
        for a in range(q.size):
            # every point up to the K-th smallest distance (ties included),
            # then the (distance, index) order decides
            t = np.partition(d2[a], K - 1)[K - 1]
            cand = np.flatnonzero(d2[a] <= t)
            order = np.lexsort((cand, d2[a, cand]))[:K]
            idx[s + a] = cand[order]
            d2o[s + a] = d2[a, cand[order]]
    return idx, d2o


def knn(points, K: int):
    """K nearest neighbours of every point: (idx (N x K), d2 (N x K))."""
    Y = np.asarray(points, dtype=np.float64)
    N = Y.shape[0]
    return query_knn(Y, np.arange(N), K)


def sigma_of(d2) -> float:
    """Mean Euclidean distance over all K-NN pairs."""
    return float(np.mean(np.sqrt(np.asarray(d2, dtype=np.float64))))


def adjacency(idx, d2, sigma: float) -> sp.csr_matrix:
    """Symmetric W: the Gaussian weight exp(-d^2/sigma^2) on every pair that
    is a K-NN relation in either direction (union). Each pair is stored once
    per direction, also when its weight underflows to zero."""
    idx = np.asarray(idx, dtype=np.int64)
    N, K = idx.shape
    rows = np.repeat(np.arange(N), K)
    w = np.exp(-np.asarray(d2, dtype=np.float64).ravel() / (sigma * sigma))
    r = np.concatenate([rows, idx.ravel()])
    c = np.concatenate([idx.ravel(), rows])
    v = np.concatenate([w, w])
    # a pair listed from both ends carries the same weight (the distance is
    # symmetric); keep one copy
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    first = np.ones(r.size, dtype=bool)
    first[1:] = (r[1:] != r[:-1]) | (c[1:] != c[:-1])
    r, c, v = r[first], c[first], v[first]
    indptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(indptr, r + 1, 1)
    return sp.csr_matrix((v, c, np.cumsum(indptr)), shape=(N, N))


def laplacian(W: sp.csr_matrix, kind: str = "normalized") -> sp.csr_matrix:
    """L = D - W (combinatorial) or D^{-1/2} (D - W) D^{-1/2} (normalised),
    with every diagonal entry stored."""
    W = sp.csr_matrix(W, dtype=np.float64)
    N = W.shape[0]
    deg = np.asarray(W.sum(axis=1)).ravel()
    if kind == "combinatorial":
        L = sp.diags(deg) - W
    elif kind == "normalized":
        if np.any(deg <= 0):
            raise ValueError("isolated point: the normalised Laplacian is undefined")
        Wc = W.tocoo()
        vals = -Wc.data / np.sqrt(deg[Wc.row] * deg[Wc.col])
        L = sp.csr_matrix((vals, (Wc.row, Wc.col)), shape=(N, N)) + sp.identity(N)
    else:
        raise ValueError(kind)
    L = sp.csr_matrix(L)
    L.sum_duplicates()
    L.sort_indices()
    return L


def knn_graph(points, K: int = 10, kind: str = "normalized"):
    """Laplacian of the K-NN Gaussian-kernel graph of the rows of `points`.
    Returns (L, sigma, idx, d2)."""
    idx, d2 = knn(points, K)
    s = sigma_of(d2)
    if not s > 0:
        raise ValueError("every neighbour distance is zero: sigma = 0")
    return laplacian(adjacency(idx, d2, s), kind), s, idx, d2
