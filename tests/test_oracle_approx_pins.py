"""Pins of the approximate-decoder oracle (Section V-C, Algorithm 2) against
facts that do not come from the oracle itself."""
import numpy as np
import scipy.sparse as sp

from oracle import approx as OA


def _random_laplacian(c, rng, density=0.35, comps=None):
    """Combinatorial Laplacian of a random weighted graph; with comps (a list
    of node-index arrays) edges only join nodes of the same component, and a
    path inside each component keeps it connected."""
    W = np.zeros((c, c))
    groups = comps if comps is not None else [np.arange(c)]
    for g in groups:
        g = np.asarray(g)
        for a, b in zip(g[:-1], g[1:]):
            W[a, b] = W[b, a] = rng.uniform(0.5, 1.5)
        for i in g:
            for j in g:
                if i < j and rng.random() < density:
                    W[i, j] = W[j, i] = rng.uniform(0.1, 2.0)
    return sp.csr_matrix(np.diag(W.sum(1)) - W)


def test_upsample_solves_the_constrained_quadratic_program():
    # min tr(S^T L S) s.t. S[omega] = R, solved through its KKT system
    # [2L  E^T; E  0] [S; mu] = [0; R] (E selects the sampled rows) -- the
    # Lagrangian route, not the Schur complement the lemma uses
    rng = np.random.default_rng(1)
    c = 14
    L = _random_laplacian(c, rng)
    omega = np.array([1, 5, 6, 11])
    R = rng.standard_normal((omega.size, 3))
    S = OA.upsample(L, omega, R)
    E = np.zeros((omega.size, c))
    E[np.arange(omega.size), omega] = 1.0
    K = np.block([[2.0 * L.toarray(), E.T], [E, np.zeros((omega.size, omega.size))]])
    rhs = np.vstack([np.zeros((c, 3)), R])
    ref = np.linalg.solve(K, rhs)[:c]
    assert np.abs(S - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(S[omega], R)
    # and it is a minimum: feasible perturbations raise the objective
    f = lambda X: np.trace(X.T @ (L @ X))
    free = np.setdiff1d(np.arange(c), omega)
    for _ in range(5):
        D = np.zeros_like(S)
        D[free] = rng.standard_normal((free.size, 3))
        assert f(S + 1e-3 * D) > f(S)


def test_upsample_recovers_piecewise_constant_signals_exactly():
    # a signal constant on each connected component lies in the null space
    # of L (lambda = 0): one sample per component recovers it exactly; a
    # component without samples gets the minimum-norm value 0
    rng = np.random.default_rng(2)
    comps = [np.arange(0, 7), np.arange(7, 15), np.arange(15, 19), np.arange(19, 24)]
    L = _random_laplacian(24, rng, comps=comps)
    vals = np.array([2.5, -1.0, 0.75, 9.0])
    truth = np.concatenate([np.full(g.size, v) for g, v in zip(comps, vals)])
    omega = np.array([3, 8, 9, 16])  # nothing from the last component
    S = OA.upsample(L, omega, truth[omega][:, None])[:, 0]
    assert np.abs(S[:19] - truth[:19]).max() <= 1e-12
    assert np.all(S[19:] == 0.0)


def test_select_rank_on_prescribed_singular_values():
    rng = np.random.default_rng(3)
    sig = np.array([10.0, 5.0, 1.5, 0.9, 0.2])
    Q1, _ = np.linalg.qr(rng.standard_normal((9, 5)))
    Q2, _ = np.linalg.qr(rng.standard_normal((7, 5)))
    _, s, _ = OA.thin_svd((Q1 * sig) @ Q2.T)
    assert s.size == 7
    assert np.allclose(s[:5], sig, rtol=1e-13) and np.all(s[5:] <= 1e-13)
    assert OA.select_rank(s, 0.1) == 3        # threshold 1.0 keeps 10, 5, 1.5
    assert OA.select_rank(s, 0.01) == 5
    assert OA.select_rank(s, 0.1, k_max=2) == 2
    assert OA.select_rank(np.zeros(4), 0.1) == 0
    assert OA.select_rank(np.array([3.0, 0.0]), 0.0) == 1  # zero values never kept
    assert OA.select_rank(np.array([10.0, 1.0, 0.5]), 0.1) == 2  # "at or above" the threshold


def test_rip_scale_closed_form():
    assert OA.rip_scale(100, 200, 50, 100) == 2.0
    assert abs(OA.rip_scale(100, 200, 50, 100, delta=0.75) - 4.0) <= 1e-15


def test_full_sampling_gives_the_rank_k_truncation():
    # omega = everything: U = U~, V = V~, scale 1 (delta = 0), so X is the
    # best rank-k approximation of X~ (Eckart-Young: the squared error is the
    # sum of the dropped squared singular values); keeping every value
    # returns X~ itself
    rng = np.random.default_rng(4)
    p, n = 11, 8
    Lr = _random_laplacian(p, rng)
    Lc = _random_laplacian(n, rng)
    sig = np.array([6.0, 3.0, 2.0, 0.4, 0.3, 0.1, 0.05, 0.01])
    Q1, _ = np.linalg.qr(rng.standard_normal((p, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Xt = (Q1 * sig) @ Q2.T
    X, info = OA.approx_decode(Xt, p, n, np.arange(p), np.arange(n), Lr, Lc, ratio=0.1)
    assert info["k"] == 3 and info["scale"] == 1.0      # threshold 0.6 keeps 6, 3, 2
    assert np.linalg.matrix_rank(X, tol=1e-9) == 3
    assert abs(np.linalg.norm(Xt - X) ** 2 - np.sum(sig[3:] ** 2)) <= 1e-12
    X_all, info = OA.approx_decode(Xt, p, n, np.arange(p), np.arange(n), Lr, Lc, ratio=0.0)
    assert info["k"] == n
    assert np.abs(X_all - Xt).max() <= 1e-12


def test_block_constant_matrix_is_recovered_exactly():
    # rows: two components of 10 nodes, columns: two of 8; X is constant a
    # on (A1, B1), b on (A2, B2), 0 elsewhere. Half of every component is
    # sampled, so X~ has singular values a sqrt(20), b sqrt(20) with sampled
    # indicator vectors; upsampling extends them to the full indicators,
    # normalisation makes them 1/sqrt(10) and 1/sqrt(8), and the scale
    # sqrt(np / (rho_r rho_c)) = 2 restores X exactly
    rng = np.random.default_rng(5)
    A = [np.arange(0, 10), np.arange(10, 20)]
    B = [np.arange(0, 8), np.arange(8, 16)]
    Lr = _random_laplacian(20, rng, comps=A)
    Lc = _random_laplacian(16, rng, comps=B)
    a, b = 3.0, 0.7
    X = np.zeros((20, 16))
    X[np.ix_(A[0], B[0])] = a
    X[np.ix_(A[1], B[1])] = b
    om_r = np.sort(np.concatenate([rng.choice(g, 5, replace=False) for g in A]))
    om_c = np.sort(np.concatenate([rng.choice(g, 4, replace=False) for g in B]))
    Xt = X[np.ix_(om_r, om_c)]
    Xd, info = OA.approx_decode(Xt, 20, 16, om_r, om_c, Lr, Lc)
    assert info["k"] == 2
    assert np.allclose(info["sigma"][:2], [a * np.sqrt(20), b * np.sqrt(20)], rtol=1e-13)
    assert info["scale"] == 2.0
    assert np.abs(Xd - X).max() <= 1e-12
    # delta enters only through the scale: 1 / sqrt(1 - 0.36) = 1.25
    Xd2, _ = OA.approx_decode(Xt, 20, 16, om_r, om_c, Lr, Lc, delta=0.36)
    assert np.abs(Xd2 - 1.25 * X).max() <= 1e-12
    # the row and column graphs are not interchangeable
    Lr_bad = _random_laplacian(20, rng, comps=[np.arange(0, 5), np.arange(5, 20)])
    Xbad, _ = OA.approx_decode(Xt, 20, 16, om_r, om_c, Lr_bad, Lc)
    assert np.abs(Xbad - X).max() > 1e-3


# ---------------------------------------------------------- decoders 2 and 3

def test_one_side_decoders_full_sampling_give_the_rank_k_truncation_of_Y():
    # omega = everything and X~ = Y: U = U~ (orthonormal), so U U^T Y and
    # Y V V^T are the best rank-k approximation of Y (Eckart-Young)
    rng = np.random.default_rng(11)
    p, n = 13, 9
    Lr = _random_laplacian(p, rng)
    Lc = _random_laplacian(n, rng)
    sig = np.array([9.0, 5.0, 3.0, 2.5, 0.5, 0.2, 0.1, 0.05, 0.02])
    Q1, _ = np.linalg.qr(rng.standard_normal((p, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Y = (Q1 * sig) @ Q2.T
    for fn, L, om in ((OA.approx_decode_rows, Lr, np.arange(p)),
                      (OA.approx_decode_cols, Lc, np.arange(n))):
        X, info = fn(Y, Y, om, L, ratio=0.25)
        assert info["k"] == 4                      # threshold 2.25 keeps 9, 5, 3, 2.5
        assert np.linalg.matrix_rank(X, tol=1e-9) == 4
        assert abs(np.linalg.norm(Y - X) ** 2 - np.sum(sig[4:] ** 2)) <= 1e-12


def test_one_kept_vector_gives_the_orthogonal_projection():
    # k = 1: X = u u^T Y / ||u||^2 with u the upsampled leading vector: the
    # residual Y - X is orthogonal to u and X has rank one along u
    rng = np.random.default_rng(12)
    p, n = 30, 17
    Lr = _random_laplacian(p, rng)
    Lc = _random_laplacian(n, rng)
    om_r = np.sort(rng.choice(p, 9, replace=False))
    om_c = np.sort(rng.choice(n, 6, replace=False))
    Y = rng.standard_normal((p, n))
    Xt = np.outer(rng.standard_normal(9), rng.standard_normal(6)) + 1e-3 * rng.standard_normal((9, 6))
    X, info = OA.approx_decode_rows(Xt, Y, om_r, Lr, ratio=0.5)
    assert info["k"] == 1
    u = OA.upsample(Lr, om_r, np.linalg.svd(Xt)[0][:, :1])[:, 0]
    assert np.abs(u @ (Y - X)).max() <= 1e-12 * np.abs(Y).max() * np.linalg.norm(u)
    assert np.linalg.matrix_rank(X, tol=1e-10) == 1
    assert np.abs(X - np.outer(u, u @ Y) / (u @ u)).max() <= 1e-12
    X3, info3 = OA.approx_decode_cols(Xt, Y, om_c, Lc, ratio=0.5)
    v = OA.upsample(Lc, om_c, np.linalg.svd(Xt)[2][:1].T)[:, 0]
    assert info3["k"] == 1 and np.abs((Y - X3) @ v).max() <= 1e-12 * np.abs(Y).max() * np.linalg.norm(v)


def test_decoder_3_is_decoder_2_of_the_transposed_problem():
    rng = np.random.default_rng(13)
    p, n = 25, 19
    Lr = _random_laplacian(p, rng)
    Lc = _random_laplacian(n, rng)
    om_r = np.sort(rng.choice(p, 8, replace=False))
    om_c = np.sort(rng.choice(n, 7, replace=False))
    Y = rng.standard_normal((p, n))
    Xt = Y[np.ix_(om_r, om_c)] + 0.1 * rng.standard_normal((8, 7))
    X3, i3 = OA.approx_decode_cols(Xt, Y, om_c, Lc, ratio=0.2)
    X2t, i2 = OA.approx_decode_rows(Xt.T, Y.T, om_c, Lc, ratio=0.2)
    assert i3["k"] == i2["k"] >= 2
    assert np.abs(X3 - X2t.T).max() <= 1e-12 * np.abs(X3).max()
