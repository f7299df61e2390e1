"""Approximate decoder for clustering -- FP64 oracle (test infrastructure
only: only tests, the smoke check and the CPU baseline of the benchmark use
this module).

Method (Section VI, Algorithm 3). The columns of the FRPCAG estimate X~
(rho_r x rho_c) are the sampled data points (rho_c points of dimension
rho_r):

  1. k-means on those points gives labels, i.e. the indicator matrix
     C~ in {0,1}^(rho_c x k) with C~[i, j] = 1 iff point i is in cluster j;
  2. each indicator column is upsampled over the column graph,
     min c^T L_c c subject to c[omega_c] = c~ (eq. approx_c), whose solution
     by the graph-upsampling lemma is c[omega_c] = c~ and
     c[omega_c-bar] = -L_c(bar, bar)^{-1} L_c(bar, omega_c) c~;
  3. max pooling per row: sample i gets the cluster j of the largest C[i, j].

k-means is Lloyd's iteration from caller-given initial centroids (the paper
names k-means without an initialisation; any random draw is therefore an
input): assign every point to the nearest centroid in squared Euclidean
distance (ties to the lower cluster index), move every centroid to the mean
of its points (a cluster left empty keeps its centroid), and stop when no
assignment changes or after max_iter updates. Max pooling breaks ties the
same way. A component of the unsampled column graph with no edge to a sample
gets C = 0 and therefore cluster 0.

Parity status: pinned (k-means against the known partition of separated
blobs and against a brute-force search over every 2-partition of a tiny set;
the Lloyd fixed-point conditions; exact labels on a graph whose components
each hold the samples of one cluster; rows of C summing to one for a
combinatorial Laplacian; sampled columns keeping their k-means labels).
"""
from __future__ import annotations

import numpy as np

from . import approx as _approx

__all__ = ["kmeans", "indicators", "max_pool", "cluster_decode"]


def kmeans(points, init_centroids, max_iter: int = 100):
    """Step 1: Lloyd's k-means. points: N x d, init_centroids: k x d.
    Returns (labels (N,), centroids (k x d), updates run)."""
    P = np.asarray(points, dtype=np.float64)
    C = np.array(init_centroids, dtype=np.float64, copy=True)
    k = C.shape[0]
    labels = None
    it = 0
    while True:
        D = ((P[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)   # N x k
        new = np.argmin(D, axis=1)                                # first minimum on ties
        if labels is not None and np.array_equal(new, labels):
            break
        labels = new
        if it >= max_iter:
            break
        for j in range(k):
            members = labels == j
            if members.any():
                C[j] = P[members].mean(axis=0)
        it += 1
    return labels, C, it


def indicators(labels, k: int):
    """C~: one column per cluster, C~[i, labels[i]] = 1."""
    labels = np.asarray(labels)
    out = np.zeros((labels.size, k))
    out[np.arange(labels.size), labels] = 1.0
    return out


def max_pool(C):
    """Step 3: the column of the largest entry of every row (first on ties)."""
    return np.argmax(np.asarray(C), axis=1)


def cluster_decode(Xt, n, omega_c, Lc, init_idx, max_iter: int = 100):
    """Algorithm 3. Xt: rho_r x rho_c; init_idx: the k sampled points (column
    positions in Xt) that seed the centroids. Returns (labels (n,), info)
    with info = dict(C (n x k), sample_labels (rho_c,), kmeans_iters)."""
    Xt = np.asarray(Xt, dtype=np.float64)
    pts = Xt.T
    init_idx = np.asarray(init_idx, dtype=np.int64)
    k = init_idx.size
    lab, cen, it = kmeans(pts, pts[init_idx], max_iter)
    C = _approx.upsample(Lc, omega_c, indicators(lab, k))
    return max_pool(C), dict(C=C, sample_labels=lab, centroids=cen, kmeans_iters=it)
