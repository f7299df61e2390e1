"""FRPCAG on the sampled matrix, solved by FISTA -- FP64 oracle (test
infrastructure only).

Problem (eq. frpcag_small, Section IV.B, with phi the l1 norm):

    min_X  ||Y - X||_1 + gamma_c tr(X L_c X^T) + gamma_r tr(X^T L_r X)

g(Z) is the smooth graph term, its gradient is 2 (gamma_c Z L_c + gamma_r L_r Z),
the prox of lambda ||Y - .||_1 is a soft threshold centred on Y, and the step
is lambda = 1 / beta' with beta' = 2 gamma_c ||L_c||_2 + 2 gamma_r ||L_r||_2
(all Section IV.B). FISTA is Algorithm 1.

Parity status: pinned (prox by brute-force scalar minimisation, g by the
edge-sum form of the Dirichlet energy, the gradient by finite differences
and Euler's identity, FISTA by the gamma = 0 and nullspace fixed points,
monotone ISTA descent, the Beck-Teboulle rate bound and the KKT conditions).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["smooth_term", "grad_smooth", "prox_l1_centered", "step_size",
           "objective", "fista", "momentum_sequence"]


def smooth_term(Z: np.ndarray, Lr: sp.spmatrix, Lc: sp.spmatrix,
                gamma_r: float, gamma_c: float) -> float:
    """g(Z) = gamma_c tr(Z L_c Z^T) + gamma_r tr(Z^T L_r Z)  (Section IV.B)."""
    ZLc = (Lc @ Z.T).T          # Z L_c (L_c symmetric)
    LrZ = Lr @ Z
    return float(gamma_c * np.sum(Z * ZLc) + gamma_r * np.sum(Z * LrZ))


def grad_smooth(Z: np.ndarray, Lr: sp.spmatrix, Lc: sp.spmatrix,
                gamma_r: float, gamma_c: float) -> np.ndarray:
    """grad g(Z) = 2 (gamma_c Z L_c + gamma_r L_r Z)  (Section IV.B)."""
    return 2.0 * (gamma_c * (Lc @ Z.T).T + gamma_r * (Lr @ Z))


def prox_l1_centered(Z: np.ndarray, Y: np.ndarray, lam: float) -> np.ndarray:
    """prox_{lam ||Y - .||_1}(Z) = Y + sgn(Z - Y) o max(|Z - Y| - lam, 0)
    (Section IV.B)."""
    D = Z - Y
    return Y + np.sign(D) * np.maximum(np.abs(D) - lam, 0.0)


def step_size(gamma_r: float, gamma_c: float, lmax_r: float, lmax_c: float) -> float:
    """lambda = 1 / beta', beta' = 2 gamma_c ||L_c||_2 + 2 gamma_r ||L_r||_2.

    Returns 0.0 when beta' = 0 (no graph term: the minimiser is Y itself)."""
    beta = 2.0 * gamma_c * lmax_c + 2.0 * gamma_r * lmax_r
    return 0.0 if beta == 0.0 else 1.0 / beta


def objective(X: np.ndarray, Y: np.ndarray, Lr, Lc, gamma_r, gamma_c) -> float:
    """F(X) = ||Y - X||_1 + g(X)  (eq. frpcag_small with phi = l1)."""
    return float(np.abs(Y - X).sum()) + smooth_term(X, Lr, Lc, gamma_r, gamma_c)


def momentum_sequence(J: int) -> np.ndarray:
    """t_1 = 1, t_{j+1} = (1 + sqrt(1 + 4 t_j^2)) / 2 (Algorithm 1); returns
    t_1 .. t_{J+1}."""
    t = np.empty(J + 1)
    t[0] = 1.0
    for j in range(J):
        t[j + 1] = (1.0 + np.sqrt(1.0 + 4.0 * t[j] * t[j])) / 2.0
    return t


def fista(Y: np.ndarray, Lr, Lc, gamma_r: float, gamma_c: float,
          lmax_r: float, lmax_c: float, J: int, eps: float = 0.0,
          momentum: bool = True, record=None):
    """Algorithm 1 (FISTA for FRPCAG).

    Start from Z_1 = Y, S_0 = Y, t_1 = 1. Each iteration takes a gradient step
    on g, applies the prox of the l1 term, updates t and extrapolates Z. The
    loop stops after J iterations, or earlier when
    ||Z_{j+1} - Z_j||_F^2 < eps ||Z_j||_F^2 (only when eps > 0).

    Output: the last prox iterate S_j (the paper's printed output symbol is
    undefined; S_j is the standard FISTA output). With momentum=False the
    extrapolation is dropped (ISTA), used only by the descent pin.

    Returns (S, iterations_run). `record`, if a dict, receives S_j at the
    iterations listed in its keys.
    """
    Y = np.asarray(Y, dtype=np.float64)
    lam = step_size(gamma_r, gamma_c, lmax_r, lmax_c)
    if lam == 0.0 or J == 0:
        return Y.copy(), 0
    Z = Y.copy()
    S_prev = Y.copy()
    t = 1.0
    S = Y
    for j in range(1, J + 1):
        S = prox_l1_centered(Z - lam * grad_smooth(Z, Lr, Lc, gamma_r, gamma_c), Y, lam)
        if momentum:
            t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
            Z_next = S + ((t - 1.0) / t_next) * (S - S_prev)
        else:
            t_next = 1.0
            Z_next = S
        if record is not None and j in record:
            record[j] = S.copy()
        if eps > 0.0:
            if np.sum((Z_next - Z) ** 2) < eps * np.sum(Z ** 2):
                return S, j
        S_prev, Z, t = S, Z_next, t_next
    return S, J
