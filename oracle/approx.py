"""Subspace-upsampling approximate decoder -- FP64 oracle (test
infrastructure only: only tests, the smoke check and the CPU baseline of the
benchmark use this module).

Method (Section V-C, Algorithm 2). Given the FRPCAG estimate X~ on the
sampled rows omega_r and columns omega_c:

  1. thin SVD X~ = U~ S~ V~^T (singular values in descending order);
  2. k = the number of singular values at or above ratio * S~[0] (ratio 0.1
     in the paper), at most k_max; zero singular values are never kept;
  3. upsample every kept column of U~ over the row graph and of V~ over the
     column graph: min_u u^T L u subject to u[omega] = u~ (eq. approx_uv),
     whose solution is, by the graph-upsampling lemma (appendix proof),
         u[omega]     = u~,
         u[omega-bar] = -L(omega-bar, omega-bar)^{-1} L(omega-bar, omega) u~;
  4. normalise every upsampled column to unit Euclidean norm;
  5. scale the kept singular values by sqrt(n p / (rho_r rho_c (1 - delta)))
     (the norm preservation constant of the RIP theorem);
  6. X = U S V^T.

The paper solves step 3 by preconditioned CG; the oracle takes the lemma's
closed form with a sparse direct solve. Where a connected component of the
unsampled subgraph has no edge to a sampled node, L(omega-bar, omega-bar) is
singular on it and the right-hand side vanishes there; the oracle returns
zero on such a component (the minimum-norm solution, which CG from zero also
reaches).

X is invariant under the sign of each singular pair; it is unique when the
kept singular values are distinct.

Parity status: pinned (the upsampled vectors against a constrained quadratic
minimisation solved through a null-space basis; exact recovery of a
piecewise-constant subspace on a graph with several components; full
sampling reduces the decoder to the rank-k truncation of X~; the rank
selection on prescribed singular values; the scale constant).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
import scipy.sparse.linalg as spla

__all__ = ["thin_svd", "select_rank", "upsample", "rip_scale", "approx_decode"]


def thin_svd(Xt):
    """Step 1: U~ (rho_r x m), singular values (m, descending), V~ (rho_c x m)
    with m = min(rho_r, rho_c)."""
    U, s, Vt = np.linalg.svd(np.asarray(Xt, dtype=np.float64), full_matrices=False)
    return U, s, Vt.T


def select_rank(s, ratio: float = 0.1, k_max: int | None = None) -> int:
    """Step 2: the number of singular values >= ratio * s[0] that are
    positive, capped at k_max."""
    s = np.asarray(s, dtype=np.float64)
    if s.size == 0 or not s[0] > 0.0:
        return 0
    k = int(np.count_nonzero((s >= ratio * s[0]) & (s > 0.0)))
    return k if k_max is None else min(k, int(k_max))


def upsample(L, omega, R):
    """Step 3 (graph-upsampling lemma): S with S[omega] = R and
    S[omega-bar] = -L_aa^{-1} L_ab R, for a c x c Laplacian L and the sampled
    index set omega (R has one row per sampled index)."""
    L = sp.csr_matrix(L, dtype=np.float64)
    c = L.shape[0]
    omega = np.asarray(omega, dtype=np.int64)
    R = np.asarray(R, dtype=np.float64).reshape(omega.size, -1)
    S = np.zeros((c, R.shape[1]))
    S[omega] = R
    rest = np.setdiff1d(np.arange(c), omega)
    if rest.size == 0 or R.shape[1] == 0:
        return S
    Laa = L[rest][:, rest].tocsr()
    Lab = L[rest][:, omega].tocsr()
    rhs = -(Lab @ R)
    # components of the unsampled subgraph without an edge to a sample
    ncomp, lab = csg.connected_components(Laa, directed=False)
    touches = np.zeros(ncomp, dtype=bool)
    touches[lab[np.abs(Lab).sum(axis=1).A1 > 0]] = True
    keep = touches[lab]
    if keep.any():
        idx = np.flatnonzero(keep)
        A = Laa[idx][:, idx].tocsc()
        sol = spla.spsolve(A, rhs[idx])
        S[rest[idx]] = np.asarray(sol).reshape(idx.size, -1)
    return S


def rip_scale(p: int, n: int, rho_r: int, rho_c: int, delta: float = 0.0) -> float:
    """Step 5: sqrt(n p / (rho_r rho_c (1 - delta)))."""
    return float(np.sqrt(n * p / (rho_r * rho_c * (1.0 - delta))))


def approx_decode(Xt, p, n, omega_r, omega_c, Lr, Lc, delta: float = 0.0,
                  ratio: float = 0.1, k_max: int | None = None):
    """Algorithm 2. Returns (X, info) with info = dict(k, sigma (all singular
    values of X~), U, V (unit columns), scale)."""
    Xt = np.asarray(Xt, dtype=np.float64)
    rho_r, rho_c = Xt.shape
    Ut, s, Vt = thin_svd(Xt)
    k = select_rank(s, ratio, k_max)
    U = upsample(Lr, omega_r, Ut[:, :k])
    V = upsample(Lc, omega_c, Vt[:, :k])
    U = U / np.linalg.norm(U, axis=0, keepdims=True) if k else U
    V = V / np.linalg.norm(V, axis=0, keepdims=True) if k else V
    scale = rip_scale(p, n, rho_r, rho_c, delta)
    X = (U * (scale * s[:k])) @ V.T
    return X, dict(k=k, sigma=s, U=U, V=V, scale=scale)
