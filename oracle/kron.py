"""Kron reduction of a graph Laplacian onto the sampled nodes -- FP64 oracle
(test infrastructure only: only tests, the smoke check and the CPU baseline
of the benchmark use this module).

Definition (Section IV-A, graphs for compressed data): with Omega the
sampled nodes and Omega-bar the rest, the compressed Laplacian is the Schur
complement

    L~ = L(Omega, Omega) - L(Omega, Omega-bar) L(Omega-bar, Omega-bar)^-1
                           L(Omega-bar, Omega),

rows and columns in the order of omega. L(Omega-bar, Omega-bar) is singular
on a connected component of the unsampled subgraph that has no edge to a
sampled node; such a component contributes nothing to the second term (the
right-hand side vanishes on it), which is the reading taken here and the
value the minimum-norm solution gives.

The second term is computed with a dense solve for small graphs and a sparse
LU factorisation of L(Omega-bar, Omega-bar) (per connected part that touches
Omega) otherwise; both are library steps of the definition.

Parity status: pinned (a path and a star eliminated by hand: series
conductance and the star-mesh transform; the reduced combinatorial Laplacian
is again a Laplacian: symmetric, zero row sums, non-positive off-diagonal,
positive semi-definite; no edge between sampled nodes joined by no path
through unsampled nodes; the quadratic form equals the minimum energy over
the unsampled values, found by a general-purpose minimiser; full sampling
returns L; eliminating in two steps equals eliminating at once).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
import scipy.sparse.linalg as spla

__all__ = ["kron_reduce"]


def kron_reduce(L, omega) -> np.ndarray:
    """Dense rho x rho Kron reduction of the Laplacian L onto the nodes
    omega (in that order)."""
    L = sp.csr_matrix(L, dtype=np.float64)
    c = L.shape[0]
    omega = np.asarray(omega, dtype=np.int64)
    rest = np.setdiff1d(np.arange(c), omega)
    L_oo = L[omega][:, omega].toarray()
    if rest.size == 0:
        return L_oo
    L_or = L[omega][:, rest].tocsr()           # rho x |rest|
    L_rr = L[rest][:, rest].tocsr()
    B = L_or.T.tocsc()                          # L(Omega-bar, Omega)
    ncomp, lab = csg.connected_components(L_rr, directed=False)
    touches = np.zeros(ncomp, dtype=bool)
    touches[lab[np.abs(B).sum(axis=1).A1 > 0]] = True
    keep = np.flatnonzero(touches[lab])
    if keep.size == 0:
        return L_oo
    A = L_rr[keep][:, keep]
    rhs = B[keep].toarray()
    if keep.size <= 1500:
        Xs = np.linalg.solve(A.toarray(), rhs)
    else:
        Xs = spla.splu(A.tocsc()).solve(rhs)
    return L_oo - L_or[:, keep] @ Xs
