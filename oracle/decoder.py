"""Alternate decoder -- FP64 oracle (test infrastructure only).

Problem (eq. alternatedecoder, Section V.B):

    min_X ||M_r X M_c - X~||_F^2 + gc tr(X L_c X^T) + gr tr(X^T L_r X)

with the 0/1 sampling matrices of eq. (Mc): M_r is rho_r x p with
M_r[i, j] = 1 iff j = omega_r[i]; M_c is n x rho_c with M_c[i, j] = 1 iff
i = omega_c[j]. Setting the gradient to zero gives the normal equations

    A(X) := (m_r m_c^T) o X + gr L_r X + gc X L_c = B := M_r^T X~ M_c^T,

because M_r^T M_r = diag(m_r) and M_c M_c^T = diag(m_c) when the sampled
indices are distinct. A is symmetric positive semi-definite; it is definite
when every (row component, column component) pair of the two graphs holds a
sampled entry and gr, gc > 0. The paper solves this system by conjugate
gradient (end of Section V.B); the oracle computes its exact solution.

Solvers provided (all reach the same unique solution up to rounding):
  * solve_dense   -- Cholesky of the explicit pn x pn Kronecker matrix
                     (tiny sizes);
  * solve_sparse  -- sparse LU of the same matrix (small/medium sizes);
  * solve_cg      -- textbook conjugate gradient on the operator form from
                     X0 = 0 to a relative residual of 1e-13 (any size).
When A is singular (gr = gc = 0 with partial sampling) CG from zero returns
the minimum-norm solution, which is the scattered X~ itself.

Backward: with Lambda = A^{-1} G (A symmetric), the gradient of a loss l(X)
with G = dl/dX is dl/dX~ = M_r Lambda M_c (a gather), dl/dgr = -<Lambda, L_r X>
and dl/dgc = -<Lambda, X L_c>, from differentiating A(gamma) X = B.

Parity status: pinned (three independent solvers agree; the full-sampling
eigen closed form; the gamma = 0 and nullspace identities; symmetry and
definiteness of A; stationarity of the paper's objective by finite
differences; backward by central finite differences, a dense inverse and the
adjoint identity).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import scipy.linalg as sla

__all__ = ["sampling_matrices", "masks", "rhs", "apply_A", "kron_matrix",
           "solve_dense", "solve_sparse", "solve_cg", "decode", "objective",
           "decode_backward", "cg_kappa_estimate"]


def sampling_matrices(p: int, n: int, omega_r, omega_c):
    """Explicit M_r (rho_r x p) and M_c (n x rho_c) of eq. (Mc)."""
    omega_r = np.asarray(omega_r)
    omega_c = np.asarray(omega_c)
    Mr = np.zeros((omega_r.size, p))
    Mr[np.arange(omega_r.size), omega_r] = 1.0
    Mc = np.zeros((n, omega_c.size))
    Mc[omega_c, np.arange(omega_c.size)] = 1.0
    return Mr, Mc


def masks(p: int, n: int, omega_r, omega_c):
    """m_r = diag(M_r^T M_r), m_c = diag(M_c M_c^T) as 0/1 FP64 vectors."""
    m_r = np.zeros(p)
    m_r[np.asarray(omega_r)] = 1.0
    m_c = np.zeros(n)
    m_c[np.asarray(omega_c)] = 1.0
    return m_r, m_c


def rhs(Xtil: np.ndarray, p: int, n: int, omega_r, omega_c) -> np.ndarray:
    """B = M_r^T X~ M_c^T: X~ scattered into a zero p x n matrix."""
    B = np.zeros((p, n))
    B[np.ix_(np.asarray(omega_r), np.asarray(omega_c))] = Xtil
    return B


def apply_A(X, m_r, m_c, Lr, Lc, gr, gc) -> np.ndarray:
    """A(X) = (m_r m_c^T) o X + gr L_r X + gc X L_c."""
    return (np.outer(m_r, m_c) * X) + gr * (Lr @ X) + gc * (Lc @ X.T).T


def objective(X, Xtil, omega_r, omega_c, Lr, Lc, gr, gc) -> float:
    """The decoder objective of eq. alternatedecoder, with explicit M_r, M_c."""
    p, n = X.shape
    Mr, Mc = sampling_matrices(p, n, omega_r, omega_c)
    R = Mr @ X @ Mc - Xtil
    LcX = Lc @ X.T
    return float(np.sum(R * R) + gc * np.sum(X.T * LcX)
                 + gr * np.sum(X * (Lr @ X)))


def kron_matrix(p, n, m_r, m_c, Lr, Lc, gr, gc) -> sp.csr_matrix:
    """The pn x pn matrix of A acting on column-major vec(X):
    diag(vec(m_r m_c^T)) + gr (I_n kron L_r) + gc (L_c kron I_p)."""
    D = sp.diags(np.outer(m_r, m_c).ravel(order="F"))
    K = (D + gr * sp.kron(sp.identity(n), Lr) + gc * sp.kron(Lc, sp.identity(p)))
    return sp.csr_matrix(K)


def solve_dense(B, m_r, m_c, Lr, Lc, gr, gc) -> np.ndarray:
    """Exact solution by Cholesky of the explicit Kronecker matrix."""
    p, n = B.shape
    K = kron_matrix(p, n, m_r, m_c, Lr, Lc, gr, gc).toarray()
    c = sla.cho_factor(K, lower=True)
    x = sla.cho_solve(c, B.ravel(order="F"))
    return x.reshape((p, n), order="F")


def solve_sparse(B, m_r, m_c, Lr, Lc, gr, gc) -> np.ndarray:
    """Exact solution by sparse LU of the Kronecker matrix."""
    p, n = B.shape
    K = kron_matrix(p, n, m_r, m_c, Lr, Lc, gr, gc).tocsc()
    x = spla.splu(K, permc_spec="COLAMD").solve(B.ravel(order="F"))
    return x.reshape((p, n), order="F")


def solve_cg(B, m_r, m_c, Lr, Lc, gr, gc, tol: float = 1e-13,
             max_iter: int = 200000, X0=None, return_info: bool = False):
    """Textbook conjugate gradient on A(X) = B (Hestenes-Stiefel form).

    Starts from X0 (default zero) and stops when ||B - A(X)||_F <= tol ||B||_F
    (recursive residual). Returns X, or (X, info) with iterations, the true
    relative residual and the CG coefficients (for a condition estimate)."""
    Lr = sp.csr_matrix(Lr)
    Lc = sp.csr_matrix(Lc)
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.float64)
    R = B - apply_A(X, m_r, m_c, Lr, Lc, gr, gc) if X0 is not None else B.copy()
    P = R.copy()
    rr = float(np.sum(R * R))
    bb = float(np.sum(B * B))
    alphas, betas = [], []
    it = 0
    if bb == 0.0:
        X = np.zeros_like(B)
    else:
        while it < max_iter and rr > tol * tol * bb:
            Q = apply_A(P, m_r, m_c, Lr, Lc, gr, gc)
            pq = float(np.sum(P * Q))
            if pq <= 0.0:
                raise np.linalg.LinAlgError("operator is not positive definite on the Krylov space")
            alpha = rr / pq
            X += alpha * P
            R -= alpha * Q
            rr_new = float(np.sum(R * R))
            beta = rr_new / rr
            P = R + beta * P
            rr = rr_new
            alphas.append(alpha)
            betas.append(beta)
            it += 1
    if not return_info:
        return X
    true_res = np.linalg.norm(B - apply_A(X, m_r, m_c, Lr, Lc, gr, gc))
    info = dict(iters=it, rel_residual=float(true_res / np.sqrt(bb)) if bb > 0 else 0.0,
                alphas=np.array(alphas), betas=np.array(betas))
    return X, info


def cg_kappa_estimate(alphas, betas) -> float:
    """Condition-number estimate of A from the Lanczos tridiagonal matrix that
    the CG coefficients define."""
    k = len(alphas)
    if k == 0:
        return 1.0
    d = np.empty(k)
    e = np.empty(max(k - 1, 0))
    for j in range(k):
        d[j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j < k - 1:
            e[j] = np.sqrt(betas[j]) / alphas[j]
    ev = sla.eigh_tridiagonal(d, e, eigvals_only=True)
    return float(ev[-1] / ev[0]) if ev[0] > 0 else float("inf")


def decode(Xtil, p, n, omega_r, omega_c, Lr, Lc, gr, gc, method: str = "auto",
           tol: float = 1e-13):
    """Alternate-decoder solution X (p x n) for the sampled estimate X~."""
    m_r, m_c = masks(p, n, omega_r, omega_c)
    B = rhs(np.asarray(Xtil, dtype=np.float64), p, n, omega_r, omega_c)
    if method == "auto":
        method = "dense" if p * n <= 4000 else ("sparse" if p * n <= 150000 else "cg")
    if method == "dense":
        return solve_dense(B, m_r, m_c, Lr, Lc, gr, gc)
    if method == "sparse":
        return solve_sparse(B, m_r, m_c, Lr, Lc, gr, gc)
    if method == "cg":
        return solve_cg(B, m_r, m_c, Lr, Lc, gr, gc, tol=tol)
    raise ValueError(method)


def decode_backward(G, X, p, n, omega_r, omega_c, Lr, Lc, gr, gc,
                    method: str = "auto"):
    """Adjoint of the decode map at the solution X for the upstream gradient
    G = dl/dX. Returns (dX~, dgr, dgc)."""
    m_r, m_c = masks(p, n, omega_r, omega_c)
    G = np.asarray(G, dtype=np.float64)
    if method == "auto":
        method = "dense" if p * n <= 4000 else ("sparse" if p * n <= 150000 else "cg")
    solver = {"dense": solve_dense, "sparse": solve_sparse, "cg": solve_cg}[method]
    Lam = solver(G, m_r, m_c, Lr, Lc, gr, gc)
    dXtil = Lam[np.ix_(np.asarray(omega_r), np.asarray(omega_c))]
    dgr = -float(np.sum(Lam * (Lr @ X)))
    dgc = -float(np.sum(Lam * (Lc @ X.T).T))
    return dXtil, dgr, dgc
