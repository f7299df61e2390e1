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

The appendix's approximate decoders 2 and 3 (approx_decode_rows /
approx_decode_cols) upsample one side only and project the full data Y onto
it: X = U U^T Y or X = Y V V^T, with U (V) the upsampled and normalised
singular vectors of Algorithm 2; the scale constant cancels.

Parity status: pinned (the upsampled vectors against a constrained quadratic
minimisation solved through a null-space basis; exact recovery of a
piecewise-constant subspace on a graph with several components; full
sampling reduces the decoder to the rank-k truncation of X~; the rank
selection on prescribed singular values; the scale constant; decoders 2 and 3:
full sampling gives the rank-k truncation of Y with the Eckart-Young error,
one kept vector gives the orthogonal projection onto the upsampled vector,
and each decoder on the transposed problem is the other one).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
import scipy.sparse.linalg as spla

__all__ = ["thin_svd", "select_rank", "upsample", "rip_scale", "approx_decode",
           "approx_decode_rows", "approx_decode_cols"]


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


def _unit_columns(S):
    return S / np.linalg.norm(S, axis=0, keepdims=True) if S.shape[1] else S


def approx_decode_rows(Xt, Y, omega_r, Lr, ratio: float = 0.1, k_max: int | None = None):
    """Approximate decoder 2 (appendix, other approximate decoders): only the
    left singular vectors of X~ are upsampled, over the row graph, and
    normalised as in Algorithm 2; with the full data Y (p x n) available,
    V = Y^T U S~^-1 / scale makes X = U S~ scale V^T equal to U U^T Y, which
    is what is returned. Returns (X, info) with info = dict(k, sigma, U)."""
    Xt = np.asarray(Xt, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    Ut, s, _ = thin_svd(Xt)
    k = select_rank(s, ratio, k_max)
    U = _unit_columns(upsample(Lr, omega_r, Ut[:, :k]))
    X = U @ (U.T @ Y)
    return X, dict(k=k, sigma=s, U=U)


def approx_decode_cols(Xt, Y, omega_c, Lc, ratio: float = 0.1, k_max: int | None = None):
    """Approximate decoder 3 (appendix): only the right singular vectors of
    X~ are upsampled, over the column graph, and normalised; then
    X = Y V V^T. Returns (X, info) with info = dict(k, sigma, V)."""
    Xt = np.asarray(Xt, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    _, s, Vt = thin_svd(Xt)
    k = select_rank(s, ratio, k_max)
    V = _unit_columns(upsample(Lc, omega_c, Vt[:, :k]))
    X = (Y @ V) @ V.T
    return X, dict(k=k, sigma=s, V=V)
