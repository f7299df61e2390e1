"""Pins of the FP64 oracle against facts the paper and mathematics fix.

Nothing here compares the oracle with itself: each check uses brute force, a
closed form, an invariant or an independent algorithm, chosen so that a
dropped term, a wrong sign, a wrong index or a transposed operand fails.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import minimize

import synth
from oracle import frpcag as F
from oracle import decoder as D


def _tiny(seed=3, p_shape=(4, 5), n=12, frac=0.5, kind="normalized", gamma=(1.0, 1.0)):
    return synth.small_problem(seed, p_shape=p_shape, n=n, rank=2, frac=frac,
                               gamma=gamma, kind=kind, K=3)


# ---------------------------------------------------------------- generator

def test_laplacian_invariants():
    rng = np.random.default_rng(0)
    pts = rng.standard_normal((60, 3))
    L, sigma = synth.knn_laplacian(pts, 10, "combinatorial")
    Ln, sigma_n = synth.knn_laplacian(pts, 10, "normalized")
    assert sigma == sigma_n
    A, An = L.toarray(), Ln.toarray()
    assert np.array_equal(A, A.T) and np.array_equal(An, An.T)
    W = -(A - np.diag(np.diag(A)))
    assert np.all(W >= 0)
    deg = W.sum(axis=1)
    # L = D - W with L 1 = 0; every node keeps at least its K out-neighbours
    assert np.allclose(np.diag(A), deg, rtol=1e-13)
    assert np.allclose(A @ np.ones(60), 0, atol=1e-12)
    assert np.all((W > 0).sum(axis=1) >= 10)
    # Gaussian weights of the K-NN edges
    d = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=2)
    nz = W > 0
    assert np.allclose(W[nz], np.exp(-d[nz] ** 2 / sigma ** 2), rtol=1e-13)
    # L_n = D^{-1/2} (D - W) D^{-1/2}, nullspace D^{1/2} 1, spectrum in [0, 2]
    Dm = np.diag(1 / np.sqrt(deg))
    assert np.allclose(An, Dm @ A @ Dm, atol=1e-14)
    assert np.allclose(An @ np.sqrt(deg), 0, atol=1e-12)
    for M in (A, An):
        ev = np.linalg.eigvalsh(M)
        assert ev[0] > -1e-12
    ev = np.linalg.eigvalsh(An)
    assert ev[-1] <= 2.0 + 1e-12
    assert abs(synth.laplacian_lmax(Ln) - ev[-1]) < 1e-12


def test_knn_tie_break_on_grid():
    idx, dist = synth.knn_indices(synth.grid_coords(6, 7), 4)
    # the four distance-1 neighbours of an interior pixel, ascending index
    i = 2 * 7 + 3
    assert list(idx[i]) == [i - 7, i - 1, i + 1, i + 7]
    assert np.allclose(dist[i], 1.0)


# ---------------------------------------------------------------- prox

def test_prox_matches_bruteforce_scalar_minimisation():
    rng = np.random.default_rng(1)
    grid = np.linspace(-4, 4, 800001)
    for _ in range(25):
        z, y = rng.uniform(-2, 2, 2)
        lam = rng.uniform(0.01, 1.5)
        obj = lam * np.abs(grid - y) + 0.5 * (grid - z) ** 2
        x_bf = grid[np.argmin(obj)]
        x = F.prox_l1_centered(np.array([z]), np.array([y]), lam)[0]
        assert abs(x - x_bf) <= 2e-5
    # edge cases: z = y, and |z - y| = lambda exactly
    assert F.prox_l1_centered(np.array([0.7]), np.array([0.7]), 0.3)[0] == 0.7
    assert F.prox_l1_centered(np.array([1.0]), np.array([0.5]), 0.5)[0] == 0.5
    assert F.prox_l1_centered(np.array([0.0]), np.array([0.5]), 0.5)[0] == 0.5


# ---------------------------------------------------------------- smooth term

def test_smooth_term_equals_edge_sum_dirichlet_energy():
    # tr(V^T L V) = 1/2 sum_ik W_ik ||v_i - v_k||^2 for L = D - W, and
    # tr(V^T L_n V) = 1/2 sum_ik W_ik ||v_i / sqrt(d_i) - v_k / sqrt(d_k)||^2
    rng = np.random.default_rng(2)
    pr, pc = rng.standard_normal((9, 2)), rng.standard_normal((13, 3))
    Z = rng.standard_normal((9, 13))

    def energy(W, V, normalized):
        deg = W.sum(axis=1)
        Vs = V / np.sqrt(deg)[:, None] if normalized else V
        e = 0.0
        for i in range(W.shape[0]):
            for k in range(W.shape[0]):
                if W[i, k] != 0:
                    e += 0.5 * W[i, k] * np.sum((Vs[i] - Vs[k]) ** 2)
        return e

    for kind in ("combinatorial", "normalized"):
        Lr, _ = synth.knn_laplacian(pr, 4, kind)
        Lc, _ = synth.knn_laplacian(pc, 4, kind)
        Wr = -synth.knn_laplacian(pr, 4, "combinatorial")[0].toarray()
        Wc = -synth.knn_laplacian(pc, 4, "combinatorial")[0].toarray()
        np.fill_diagonal(Wr, 0)
        np.fill_diagonal(Wc, 0)
        norm = kind == "normalized"
        g_edge = 0.7 * energy(Wc, Z.T, norm) + 1.9 * energy(Wr, Z, norm)
        assert np.isclose(F.smooth_term(Z, Lr, Lc, 1.9, 0.7), g_edge, rtol=1e-12)


def test_gradient_by_finite_differences_and_euler_identity():
    P = _tiny()
    rng = np.random.default_rng(4)
    Z = rng.standard_normal(P.Ytil.shape)
    gr, gc = 1.3, 0.4
    Gz = F.grad_smooth(Z, P.Lr_til, P.Lc_til, gr, gc)
    for _ in range(5):
        V = rng.standard_normal(Z.shape)
        h = 1e-3
        fd = (F.smooth_term(Z + h * V, P.Lr_til, P.Lc_til, gr, gc)
              - F.smooth_term(Z - h * V, P.Lr_til, P.Lc_til, gr, gc)) / (2 * h)
        assert np.isclose(fd, np.sum(Gz * V), rtol=1e-9, atol=1e-10)
    assert np.isclose(np.sum(Gz * Z), 2 * F.smooth_term(Z, P.Lr_til, P.Lc_til, gr, gc), rtol=1e-12)


def test_step_size_is_exact_lipschitz_constant():
    P = _tiny()
    gr, gc = 0.8, 2.5
    r, c = P.Ytil.shape
    # Hessian of g on column-major vec(Z): 2 (gc L_c kron I + gr I kron L_r)
    H = 2 * (gc * np.kron(P.Lc_til.toarray(), np.eye(r)) + gr * np.kron(np.eye(c), P.Lr_til.toarray()))
    lip = np.linalg.eigvalsh(H)[-1]
    lam = F.step_size(gr, gc, P.lmax_r_til, P.lmax_c_til)
    assert np.isclose(1.0 / lam, lip, rtol=1e-10)
    assert F.step_size(0.0, 0.0, 1.0, 1.0) == 0.0


# ---------------------------------------------------------------- FISTA

def test_fista_gamma_zero_and_zero_iterations_return_Y():
    P = _tiny()
    S, it = F.fista(P.Ytil, P.Lr_til, P.Lc_til, 0.0, 0.0, P.lmax_r_til, P.lmax_c_til, 50)
    assert np.array_equal(S, P.Ytil) and it == 0
    S, it = F.fista(P.Ytil, P.Lr_til, P.Lc_til, 1.0, 1.0, P.lmax_r_til, P.lmax_c_til, 0)
    assert np.array_equal(S, P.Ytil)


@pytest.mark.parametrize("kind", ["combinatorial", "normalized"])
def test_fista_nullspace_data_is_a_fixed_point(kind):
    P = _tiny(kind=kind)
    zr = np.linalg.eigh(P.Lr_til.toarray())[1][:, 0]
    zc = np.linalg.eigh(P.Lc_til.toarray())[1][:, 0]
    Y = 3.0 * np.outer(zr, zc)
    S, _ = F.fista(Y, P.Lr_til, P.Lc_til, 2.0, 5.0, P.lmax_r_til, P.lmax_c_til, 40)
    assert np.allclose(S, Y, atol=1e-12)


def test_ista_objective_decreases_monotonically():
    P = _tiny(seed=5)
    args = (P.Lr_til, P.Lc_til, 1.0, 3.0, P.lmax_r_til, P.lmax_c_til)
    rec = {j: None for j in range(1, 61)}
    F.fista(P.Ytil, *args, 60, momentum=False, record=rec)
    vals = [F.objective(rec[j], P.Ytil, P.Lr_til, P.Lc_til, 1.0, 3.0) for j in range(1, 61)]
    assert np.all(np.diff(vals) <= 1e-12 * max(1.0, abs(vals[0])))


def _reference_minimum(Y, Lr, Lc, gr, gc):
    """Independent solver: split X - Y = Pp - Pn with Pp, Pn >= 0 and run
    bound-constrained L-BFGS-B on the smooth reformulation."""
    shape = Y.shape
    m = Y.size
    Lr_d, Lc_d = Lr.toarray(), Lc.toarray()

    def fun(v):
        Pp = v[:m].reshape(shape)
        Pn = v[m:].reshape(shape)
        X = Y + Pp - Pn
        g = gc * np.sum(X * (X @ Lc_d)) + gr * np.sum(X * (Lr_d @ X))
        gx = 2 * (gc * X @ Lc_d + gr * Lr_d @ X)
        f = Pp.sum() + Pn.sum() + g
        return f, np.concatenate([(1 + gx).ravel(), (1 - gx).ravel()])

    res = minimize(fun, np.zeros(2 * m), jac=True, method="L-BFGS-B",
                   bounds=[(0, None)] * (2 * m),
                   options=dict(maxiter=20000, maxfun=40000, ftol=1e-15, gtol=1e-12))
    return res.fun


def test_fista_reaches_independent_minimum_with_rate_bound_and_kkt():
    P = _tiny(seed=6, p_shape=(3, 4), n=10, frac=0.7)
    gr, gc = 0.6, 1.7
    Lr, Lc = P.Lr_til, P.Lc_til
    Y = P.Ytil
    args = (Lr, Lc, gr, gc, P.lmax_r_til, P.lmax_c_til)
    Xs, _ = F.fista(Y, *args, 30000)
    Fstar = F.objective(Xs, Y, Lr, Lc, gr, gc)
    F_ref = _reference_minimum(Y, Lr, Lc, gr, gc)
    assert abs(Fstar - F_ref) <= 1e-8 * max(1.0, abs(F_ref))
    assert Fstar <= F_ref + 1e-10
    # Beck-Teboulle: F(S_k) - F* <= 2 beta' ||S_0 - X*||^2 / (k + 1)^2
    beta = 1.0 / F.step_size(gr, gc, P.lmax_r_til, P.lmax_c_til)
    rec = {k: None for k in range(1, 301)}
    F.fista(Y, *args, 300, record=rec)
    d0 = np.sum((Y - Xs) ** 2)
    for k in range(1, 301):
        gap = F.objective(rec[k], Y, Lr, Lc, gr, gc) - Fstar
        assert gap <= 2 * beta * d0 / (k + 1) ** 2 + 1e-9
    # KKT: 0 in grad g(X) + d||X - Y||_1
    G = F.grad_smooth(Xs, Lr, Lc, gr, gc)
    off = np.abs(Xs - Y) > 1e-7
    assert np.all(np.abs(G[off] - np.sign(Y - Xs)[off]) < 1e-4)
    assert np.all(np.abs(G[~off]) <= 1 + 1e-4)


def test_momentum_sequence_closed_form_growth():
    t = F.momentum_sequence(2000)
    assert t[0] == 1.0
    # t_{j+1}^2 - t_{j+1} = t_j^2 exactly in exact arithmetic, and t_j >= (j+1)/2
    assert np.allclose(t[1:] ** 2 - t[1:], t[:-1] ** 2, rtol=1e-12)
    j = np.arange(1, 2002)
    assert np.all(t >= (j + 1) / 2 - 1e-12)


# ---------------------------------------------------------------- decoder

def _dec_problem(seed=7, p_shape=(5, 6), n=20, frac=0.4, gamma=(0.7, 1.3), kind="normalized"):
    P = synth.small_problem(seed, p_shape=p_shape, n=n, rank=3, frac=frac,
                            gamma=gamma, kind=kind, K=4)
    rng = np.random.default_rng(seed + 100)
    Xtil = rng.standard_normal((P.rho_r, P.rho_c))
    return P, Xtil


def test_three_independent_solvers_agree():
    P, Xtil = _dec_problem()
    m_r, m_c = D.masks(P.p, P.n, P.omega_r, P.omega_c)
    B = D.rhs(Xtil, P.p, P.n, P.omega_r, P.omega_c)
    args = (m_r, m_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c)
    Xd = D.solve_dense(B, *args)
    Xs = D.solve_sparse(B, *args)
    Xc, info = D.solve_cg(B, *args, return_info=True)
    scale = np.linalg.norm(Xd)
    assert np.linalg.norm(Xs - Xd) <= 1e-11 * scale
    assert np.linalg.norm(Xc - Xd) <= 1e-9 * scale
    assert info["rel_residual"] <= 1e-12


def test_decoder_solution_is_stationary_for_the_paper_objective():
    P, Xtil = _dec_problem(seed=8)
    X = D.decode(Xtil, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c)
    f0 = D.objective(X, Xtil, P.omega_r, P.omega_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c)
    rng = np.random.default_rng(9)
    for _ in range(5):
        V = rng.standard_normal(X.shape)
        h = 1e-3
        fp = D.objective(X + h * V, Xtil, P.omega_r, P.omega_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c)
        fm = D.objective(X - h * V, Xtil, P.omega_r, P.omega_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c)
        assert abs(fp - fm) / (2 * h) <= 1e-8 * np.linalg.norm(V) * max(1.0, abs(f0))
        assert fp > f0 and fm > f0


def test_operator_symmetric_definite_and_matches_kronecker():
    P, _ = _dec_problem(seed=10, p_shape=(3, 4), n=9, frac=0.5)
    m_r, m_c = D.masks(P.p, P.n, P.omega_r, P.omega_c)
    N = P.p * P.n
    M = np.empty((N, N))
    for k in range(N):
        E = np.zeros(N)
        E[k] = 1.0
        M[:, k] = D.apply_A(E.reshape(P.p, P.n), m_r, m_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c).ravel()
    assert np.allclose(M, M.T, atol=1e-14)
    assert np.linalg.eigvalsh(M)[0] > 0
    K = D.kron_matrix(P.p, P.n, m_r, m_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c).toarray()
    # K acts on column-major vec, M on row-major vec
    perm = np.arange(N).reshape(P.p, P.n).ravel(order="F")
    assert np.allclose(K, M[np.ix_(perm, perm)], atol=1e-14)


def _full(seed=11, gamma=(0.9, 2.1)):
    P = synth.small_problem(seed, p_shape=(4, 5), n=15, rank=2, frac=1.0, gamma=gamma, K=4)
    assert P.rho_r == P.p and P.rho_c == P.n
    return P


def test_full_sampling_eigen_closed_form():
    P = _full()
    rng = np.random.default_rng(12)
    Xtil = rng.standard_normal((P.p, P.n))
    X = D.decode(Xtil, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c)
    lr, Pr = np.linalg.eigh(P.Lr.toarray())
    lc, Qc = np.linalg.eigh(P.Lc.toarray())
    Xcf = Pr @ ((Pr.T @ Xtil @ Qc) / (1 + P.gamma_r * lr[:, None] + P.gamma_c * lc[None, :])) @ Qc.T
    assert np.allclose(X, Xcf, atol=1e-12)


def test_full_sampling_identities():
    P = _full(gamma=(0.0, 0.0))
    rng = np.random.default_rng(13)
    Xtil = rng.standard_normal((P.p, P.n))
    X = D.decode(Xtil, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, 0.0, 0.0)
    assert np.allclose(X, Xtil, atol=1e-13)
    zr = np.linalg.eigh(P.Lr.toarray())[1][:, 0]
    zc = np.linalg.eigh(P.Lc.toarray())[1][:, 0]
    Xt = np.outer(zr, zc)
    for g in [(0.5, 3.0), (10.0, 0.1)]:
        X = D.decode(Xt, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, *g)
        assert np.allclose(X, Xt, atol=1e-12)


def test_singular_decoder_cg_returns_scattered_samples():
    P, Xtil = _dec_problem(seed=14)
    m_r, m_c = D.masks(P.p, P.n, P.omega_r, P.omega_c)
    B = D.rhs(Xtil, P.p, P.n, P.omega_r, P.omega_c)
    X, info = D.solve_cg(B, m_r, m_c, P.Lr, P.Lc, 0.0, 0.0, return_info=True)
    assert np.allclose(X, B, atol=1e-15) and info["iters"] == 1


def test_sampling_matrices_follow_eq_Mc():
    Mr, Mc = D.sampling_matrices(6, 7, [1, 4], [0, 3, 6])
    Y = np.arange(42.0).reshape(6, 7)
    assert np.array_equal(Mr @ Y @ Mc, Y[np.ix_([1, 4], [0, 3, 6])])
    m_r, m_c = D.masks(6, 7, [1, 4], [0, 3, 6])
    assert np.array_equal(np.diag(Mr.T @ Mr), m_r) and np.array_equal(np.diag(Mc @ Mc.T), m_c)
    assert np.array_equal(D.rhs(Mr @ Y @ Mc, 6, 7, [1, 4], [0, 3, 6]), Mr.T @ (Mr @ Y @ Mc) @ Mc.T)


def test_cg_condition_estimate_matches_dense_spectrum():
    P, Xtil = _dec_problem(seed=15, p_shape=(3, 4), n=9, frac=0.5)
    m_r, m_c = D.masks(P.p, P.n, P.omega_r, P.omega_c)
    B = D.rhs(Xtil, P.p, P.n, P.omega_r, P.omega_c)
    B = B + np.random.default_rng(0).standard_normal(B.shape)  # excite all modes
    _, info = D.solve_cg(B, m_r, m_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c, tol=1e-14, return_info=True)
    ev = np.linalg.eigvalsh(D.kron_matrix(P.p, P.n, m_r, m_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c).toarray())
    kappa = D.cg_kappa_estimate(info["alphas"], info["betas"])
    assert np.isclose(kappa, ev[-1] / ev[0], rtol=1e-3)


# ---------------------------------------------------------------- backward

def _loss(X, Xt):
    return float(np.sum((X - Xt) ** 2))


def test_backward_matches_central_finite_differences():
    P, Xtil = _dec_problem(seed=16)
    rng = np.random.default_rng(17)
    Xt = rng.standard_normal((P.p, P.n))
    args = (P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc)

    def L(Xti, gr, gc):
        return _loss(D.decode(Xti, *args, gr, gc), Xt)

    gr, gc = P.gamma_r, P.gamma_c
    X = D.decode(Xtil, *args, gr, gc)
    G = 2 * (X - Xt)
    dX, dgr, dgc = D.decode_backward(G, X, *args, gr, gc)
    h = 1e-4
    V = rng.standard_normal(Xtil.shape)
    fd = (L(Xtil + h * V, gr, gc) - L(Xtil - h * V, gr, gc)) / (2 * h)
    assert np.isclose(fd, np.sum(dX * V), rtol=1e-7)
    fd_r = (L(Xtil, gr + h, gc) - L(Xtil, gr - h, gc)) / (2 * h)
    fd_c = (L(Xtil, gr, gc + h) - L(Xtil, gr, gc - h)) / (2 * h)
    assert np.isclose(fd_r, dgr, rtol=1e-6)
    assert np.isclose(fd_c, dgc, rtol=1e-6)


def test_backward_dense_jacobian_and_adjoint_identity():
    # the dense-Kronecker gradient at p = 60, n = 80 with 50% sampling
    P = synth.small_problem(18, p_shape=(6, 10), n=80, rank=3, frac=0.5, gamma=(1.0, 1.0))
    assert (P.p, P.n, P.rho_r, P.rho_c) == (60, 80, 30, 40)
    rng = np.random.default_rng(19)
    Xtil = rng.standard_normal((P.rho_r, P.rho_c))
    G = rng.standard_normal((P.p, P.n))
    m_r, m_c = D.masks(P.p, P.n, P.omega_r, P.omega_c)
    K = D.kron_matrix(P.p, P.n, m_r, m_c, P.Lr, P.Lc, 1.0, 1.0).toarray()
    Kinv = np.linalg.inv(K)
    # scatter matrix S: column-major vec(B) = S column-major vec(Xtil)
    S = np.zeros((P.p * P.n, P.rho_r * P.rho_c))
    for b in range(P.rho_c):
        for a in range(P.rho_r):
            S[P.omega_c[b] * P.p + P.omega_r[a], b * P.rho_r + a] = 1.0
    J = Kinv @ S  # Jacobian of vec(X) w.r.t. vec(Xtil)
    dX_dense = (J.T @ G.ravel(order="F")).reshape((P.rho_r, P.rho_c), order="F")
    X = D.decode(Xtil, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, 1.0, 1.0, method="sparse")
    dX, dgr, dgc = D.decode_backward(G, X, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, 1.0, 1.0)
    assert np.allclose(dX, dX_dense, atol=1e-10)
    # dX/dgr = -A^{-1} (L_r X): dense route
    LrX = (P.Lr @ X).ravel(order="F")
    assert np.isclose(dgr, -G.ravel(order="F") @ (Kinv @ LrX), rtol=1e-9)
    # adjoint identity <A^{-1} G, B> = <G, A^{-1} B>
    B = rng.standard_normal((P.p, P.n))
    lhs = np.sum(D.solve_sparse(G, m_r, m_c, P.Lr, P.Lc, 1.0, 1.0) * B)
    rhs_ = np.sum(G * D.solve_sparse(B, m_r, m_c, P.Lr, P.Lc, 1.0, 1.0))
    assert np.isclose(lhs, rhs_, rtol=1e-10)


def test_fista_beck_teboulle_lyapunov_energy_is_nonincreasing():
    # With the momentum of Algorithm 1, E_k = (2/L) t_k^2 (F(S_k) - F*) +
    # ||t_k S_k - (t_k - 1) S_{k-1} - X*||^2 never increases (the key lemma of
    # the FISTA rate proof; L = beta', S_0 = Y). Any other extrapolation breaks it.
    P = _tiny(seed=6, p_shape=(3, 4), n=10, frac=0.7)
    for gr, gc in ((0.6, 1.7), (5.0, 5.0)):
        _lyapunov_check(P, gr, gc)


def _lyapunov_check(P, gr, gc):
    Lr, Lc, Y = P.Lr_til, P.Lc_til, P.Ytil
    args = (Lr, Lc, gr, gc, P.lmax_r_til, P.lmax_c_til)
    Xs, _ = F.fista(Y, *args, 60000)
    Fstar = F.objective(Xs, Y, Lr, Lc, gr, gc)
    beta = 1.0 / F.step_size(gr, gc, P.lmax_r_til, P.lmax_c_til)
    K = 200
    rec = {k: None for k in range(1, K + 1)}
    S_out, _ = F.fista(Y, *args, K, record=rec)
    assert np.array_equal(S_out, rec[K])  # output = last prox iterate S_K
    rec[0] = Y
    t = F.momentum_sequence(K)  # t[k-1] = t_k
    E = []
    for k in range(1, K + 1):
        tk = t[k - 1]
        u = tk * rec[k] - (tk - 1) * rec[k - 1] - Xs
        E.append(2 / beta * tk ** 2 * (F.objective(rec[k], Y, Lr, Lc, gr, gc) - Fstar) + np.sum(u * u))
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-9 * E[0])


# ---------------------------------------------------------------- FISTA early stop

def test_fista_eps_stop_on_nullspace_data_after_one_iteration():
    # nullspace data: grad g = 0, so S_1 = Y and Z_2 = S_1 = Z_1; the relative
    # change is 0 < eps at the first test, the output is S_1 = Y
    P = _tiny(kind="normalized")
    zr = np.linalg.eigh(P.Lr_til.toarray())[1][:, 0]
    zc = np.linalg.eigh(P.Lc_til.toarray())[1][:, 0]
    Y = -1.5 * np.outer(zr, zc)
    S, it = F.fista(Y, P.Lr_til, P.Lc_til, 1.0, 2.0, P.lmax_r_til, P.lmax_c_til, 50, eps=1e-30)
    assert it == 1
    assert np.allclose(S, Y, atol=1e-13)


@pytest.mark.parametrize("seed,gamma", [(5, (1.0, 3.0)), (8, (0.4, 0.9))])
def test_fista_eps_stop_rule_index_and_output(seed, gamma):
    # Algorithm 1 stops at the first j with ||Z_{j+1} - Z_j||^2 < eps ||Z_j||^2
    # and returns S_j. The Z sequence is rebuilt from the recorded prox
    # iterates S_j with the momentum step Z_{j+1} = S_j + ((t_j - 1)/t_{j+1})
    # (S_j - S_{j-1}), S_0 = Z_1 = Y, and the t_j of the pinned momentum
    # sequence; every eps placed just above / just below a recorded ratio
    # must stop exactly there / one iteration later (strict inequality).
    P = _tiny(seed=seed)
    gr, gc = gamma
    args = (P.Lr_til, P.Lc_til, gr, gc, P.lmax_r_til, P.lmax_c_til)
    J = 80
    rec = {j: None for j in range(1, J + 1)}
    F.fista(P.Ytil, *args, J, record=rec)
    t = F.momentum_sequence(J)               # t[j-1] = t_j
    S = [P.Ytil] + [rec[j] for j in range(1, J + 1)]
    Z = [None, P.Ytil]                       # Z[j] = Z_j
    for j in range(1, J + 1):
        Z.append(S[j] + ((t[j - 1] - 1.0) / t[j]) * (S[j] - S[j - 1]))
    ratio = np.array([np.sum((Z[j + 1] - Z[j]) ** 2) / np.sum(Z[j] ** 2)
                      for j in range(1, J + 1)])
    assert np.all(np.isfinite(ratio)) and ratio.max() > 0

    def first_stop(eps):
        hit = np.nonzero(ratio < eps)[0]
        return int(hit[0]) + 1 if hit.size else J

    checked = 0
    for j in (2, 5, 11, 23, 40, 67):
        for eps in (ratio[j - 1] * (1 + 1e-9), ratio[j - 1] * (1 - 1e-9)):
            want = first_stop(eps)
            S_out, it = F.fista(P.Ytil, *args, J, eps=eps)
            assert it == want, (j, eps, it, want)
            assert np.array_equal(S_out, S[want])
            checked += 1
    # the stop index really moves with eps (the pin is not vacuous)
    assert len({first_stop(r * (1 + 1e-9)) for r in ratio}) > 5
    assert checked == 12


def test_fista_eps_stop_is_strict_on_zero_data():
    # Y = 0: every iterate is 0, so the test compares 0 < eps * 0, which is
    # false for the strict rule; all J iterations run
    P = _tiny()
    Y = np.zeros_like(P.Ytil)
    S, it = F.fista(Y, P.Lr_til, P.Lc_til, 1.0, 1.0, P.lmax_r_til, P.lmax_c_til, 7, eps=0.5)
    assert it == 7 and not S.any()
