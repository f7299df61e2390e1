"""Pins of the Kron-reduction oracle (Section IV-A, graphs for compressed
data) against facts that do not come from the oracle itself."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import minimize

from oracle import kron as OK


def _lap(W):
    W = np.asarray(W, dtype=float)
    return sp.csr_matrix(np.diag(W.sum(1)) - W)


def _random_graph(c, rng, density=0.25):
    W = np.zeros((c, c))
    for a in range(c - 1):                       # a path keeps it connected
        W[a, a + 1] = W[a + 1, a] = rng.uniform(0.5, 1.5)
    for i in range(c):
        for j in range(i + 2, c):
            if rng.random() < density:
                W[i, j] = W[j, i] = rng.uniform(0.1, 2.0)
    return W


def test_path_elimination_is_series_conductance():
    # 0 -(2)- 1 -(3)- 2 with node 1 eliminated: one edge of weight 2 * 3 / 5
    W = np.zeros((3, 3))
    W[0, 1] = W[1, 0] = 2.0
    W[1, 2] = W[2, 1] = 3.0
    R = OK.kron_reduce(_lap(W), [0, 2])
    assert np.allclose(R, 1.2 * np.array([[1.0, -1.0], [-1.0, 1.0]]), atol=1e-15)


def test_star_elimination_is_the_star_mesh_transform():
    # centre 0 with leaves of weights 1, 2, 4 (sum 7): the leaves become a
    # complete graph with weights w_i w_j / 7
    w = np.array([1.0, 2.0, 4.0])
    W = np.zeros((4, 4))
    W[0, 1:] = W[1:, 0] = w
    R = OK.kron_reduce(_lap(W), [1, 2, 3])
    mesh = np.outer(w, w) / 7.0
    np.fill_diagonal(mesh, 0.0)
    assert np.allclose(R, np.diag(mesh.sum(1)) - mesh, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_reduced_laplacian_is_a_laplacian(seed):
    rng = np.random.default_rng(seed)
    c = 40
    L = _lap(_random_graph(c, rng))
    om = np.sort(rng.choice(c, 12, replace=False))
    R = OK.kron_reduce(L, om)
    assert np.allclose(R, R.T, atol=1e-13)
    assert np.allclose(R.sum(1), 0.0, atol=1e-12)
    off = R - np.diag(np.diag(R))
    assert np.all(off <= 1e-13)
    assert np.linalg.eigvalsh(R)[0] > -1e-12


def test_no_edge_without_a_path_through_unsampled_nodes():
    # a - c - b with a, b, c sampled and an unsampled pendant u on c, plus an
    # unsampled node v joining c and d: a and b only meet through c, so the
    # reduced graph has no a-b edge; c and d meet through v, so they do
    a, b, c, d, u, v = range(6)
    W = np.zeros((6, 6))
    for i, j, x in ((a, c, 1.0), (c, b, 2.0), (c, u, 0.7), (c, v, 1.3), (v, d, 0.9)):
        W[i, j] = W[j, i] = x
    om = [a, b, c, d]
    R = OK.kron_reduce(_lap(W), om)
    assert R[0, 1] == 0.0 and R[1, 0] == 0.0
    assert R[2, 3] < 0.0


def test_quadratic_form_is_the_minimum_energy_extension():
    # x~^T L~ x~ = min over the unsampled values of x^T L x with x = x~ on
    # omega, the minimum found by a general-purpose minimiser
    rng = np.random.default_rng(5)
    c = 18
    L = _lap(_random_graph(c, rng, 0.3)).toarray()
    om = np.sort(rng.choice(c, 6, replace=False))
    rest = np.setdiff1d(np.arange(c), om)
    R = OK.kron_reduce(sp.csr_matrix(L), om)
    for _ in range(3):
        xt = rng.standard_normal(om.size)

        def energy(y):
            x = np.empty(c)
            x[om] = xt
            x[rest] = y
            return x @ L @ x, 2 * (L @ x)[rest]

        res = minimize(energy, np.zeros(rest.size), jac=True, method="BFGS",
                       options=dict(gtol=1e-12, maxiter=10000))
        assert abs(res.fun - xt @ R @ xt) <= 1e-9 * max(1.0, abs(res.fun))


def test_full_sampling_returns_L_and_two_step_elimination():
    rng = np.random.default_rng(6)
    c = 30
    L = _lap(_random_graph(c, rng))
    assert np.allclose(OK.kron_reduce(L, np.arange(c)), L.toarray(), atol=0)
    om = np.sort(rng.choice(c, 8, replace=False))
    mid = np.sort(np.union1d(om, rng.choice(np.setdiff1d(np.arange(c), om), 10, replace=False)))
    R1 = OK.kron_reduce(L, om)
    L_mid = OK.kron_reduce(L, mid)
    pos = np.searchsorted(mid, om)
    R2 = OK.kron_reduce(sp.csr_matrix(L_mid), pos)
    assert np.allclose(R1, R2, atol=1e-12)


def test_unsampled_component_without_samples_contributes_nothing():
    # nodes 3, 4 form a component with no sampled node: the reduction onto
    # {0, 1, 2} equals the reduction of the other component alone
    W = np.zeros((5, 5))
    W[0, 1] = W[1, 0] = 1.0
    W[1, 2] = W[2, 1] = 2.0
    W[3, 4] = W[4, 3] = 5.0
    R = OK.kron_reduce(_lap(W), [0, 1, 2])
    assert np.allclose(R, _lap(W[:3, :3]).toarray(), atol=0)
