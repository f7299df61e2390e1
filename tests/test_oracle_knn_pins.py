"""Pins of the K-NN graph oracle (Section II graph construction) against
facts that do not come from the oracle itself."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.spatial import cKDTree

from oracle import knn as OK


def test_five_points_on_a_line_by_hand():
    # points 0, 1, 3, 6, 10 with K = 2, worked by hand:
    #   0 -> {1 (d 1), 3 (d 3)}; 1 -> {0 (1), 3 (2)}; 3 -> {1 (2), then 0 and 6
    #   tie at 3: the lower index, point 0}; 6 -> {3 (3), 10 (4)}; 10 -> {6 (4), 3 (7)}
    #   sigma = (1+3 + 1+2 + 2+3 + 3+4 + 4+7) / 10 = 3
    #   edges (union): 0-1, 0-2, 1-2, 2-3, 3-4, 2-4 with w = exp(-d^2 / 9)
    pts = np.array([[0.0], [1.0], [3.0], [6.0], [10.0]])
    L, s, idx, d2 = OK.knn_graph(pts, 2, "combinatorial")
    assert [list(r) for r in idx] == [[1, 2], [0, 2], [1, 0], [2, 4], [3, 2]]
    assert s == 3.0
    W = np.zeros((5, 5))
    for (a, b), d in {(0, 1): 1, (0, 2): 3, (1, 2): 2, (2, 3): 3, (3, 4): 4, (2, 4): 7}.items():
        W[a, b] = W[b, a] = np.exp(-d * d / 9.0)
    assert np.allclose(L.toarray(), np.diag(W.sum(1)) - W, rtol=0, atol=1e-15)
    assert L.nnz == 5 + 12
    Ln, _, _, _ = OK.knn_graph(pts, 2, "normalized")
    dm = 1 / np.sqrt(W.sum(1))
    assert np.allclose(Ln.toarray(), np.eye(5) - dm[:, None] * W * dm[None, :], atol=1e-15)


def test_matches_kdtree_on_points_with_distinct_distances():
    rng = np.random.default_rng(0)
    for N, d, K in [(300, 3, 10), (257, 2, 7), (120, 9, 5), (50, 1, 3)]:
        pts = rng.standard_normal((N, d))
        idx, d2 = OK.knn(pts, K)
        dist, ref = cKDTree(pts).query(pts, k=K + 1)
        assert np.array_equal(ref[:, 0], np.arange(N))       # itself first
        assert np.array_equal(idx, ref[:, 1:])
        assert np.allclose(np.sqrt(d2), dist[:, 1:], rtol=1e-13, atol=0)


def test_query_subset_equals_full_rows():
    rng = np.random.default_rng(1)
    pts = rng.uniform(size=(400, 4))
    idx, d2 = OK.knn(pts, 6)
    q = np.array([0, 17, 399, 200])
    i2, e2 = OK.query_knn(pts, q, 6)
    assert np.array_equal(i2, idx[q]) and np.array_equal(e2, d2[q])


def test_pixel_grid_tie_break_by_index():
    h, w = 7, 9
    r, c = np.divmod(np.arange(h * w), w)
    pts = np.stack([r, c], 1).astype(float)
    idx, d2 = OK.knn(pts, 10)
    i = 3 * w + 4        # interior pixel
    # 4 at distance 1, 4 at sqrt 2, then two of the four at distance 2: the
    # two of lowest index (up and left)
    assert list(idx[i]) == [i - w, i - 1, i + 1, i + w,
                            i - w - 1, i - w + 1, i + w - 1, i + w + 1,
                            i - 2 * w, i - 2]
    assert list(d2[i]) == [1.0] * 4 + [2.0] * 4 + [4.0] * 2


@pytest.mark.parametrize("kind", ["combinatorial", "normalized"])
def test_laplacian_invariants(kind):
    rng = np.random.default_rng(2)
    pts = rng.standard_normal((150, 3))
    L, s, idx, d2 = OK.knn_graph(pts, 10, kind)
    A = L.toarray()
    assert np.array_equal(A, A.T)
    Wm = -(A - np.diag(np.diag(A)))
    assert np.all(Wm >= 0)
    # every point keeps at least its K out-neighbours, and each edge is a
    # K-NN relation in some direction
    nb = (Wm > 0)
    assert np.all(nb.sum(1) >= 10)
    rel = np.zeros_like(nb)
    rel[np.repeat(np.arange(150), 10), idx.ravel()] = True
    assert np.array_equal(nb, rel | rel.T)
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > -1e-12
    if kind == "combinatorial":
        assert np.allclose(A @ np.ones(150), 0, atol=1e-13)
        # Gaussian weights of the distances
        d = np.linalg.norm(pts[:, None] - pts[None], axis=2)
        assert np.allclose(Wm[nb], np.exp(-d[nb] ** 2 / s ** 2), rtol=1e-13)
        assert np.isclose(s, np.mean(np.sort(d + np.diag([np.inf] * 150), 1)[:, :10]), rtol=1e-14)
    else:
        assert np.allclose(np.diag(A), 1.0)
        Lc, _, _, _ = OK.knn_graph(pts, 10, "combinatorial")
        deg = np.diag(Lc.toarray())
        assert np.allclose(A, Lc.toarray() / np.sqrt(np.outer(deg, deg)), atol=1e-15)
        assert np.allclose(A @ np.sqrt(deg), 0, atol=1e-13)
        assert ev[-1] <= 2 + 1e-12


def test_duplicate_points_and_zero_sigma():
    # duplicates sit at distance 0 and are ordered by index; all-equal
    # points leave sigma = 0, which has no Gaussian kernel
    pts = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 0.0], [5.0, 5.0], [0.0, 0.0]])
    idx, d2 = OK.knn(pts, 2)
    assert list(idx[0]) == [2, 4] and list(idx[2]) == [0, 4] and list(idx[4]) == [0, 2]
    with pytest.raises(ValueError):
        OK.knn_graph(np.zeros((6, 2)), 3)


def test_adjacency_keeps_underflowed_weights():
    # 40 points 0.01 apart and one point 1000 away, K = 1: sigma is about 24,
    # so the far point's only edge has weight exp(-1680) = 0 in FP64; it is
    # stored as an explicit zero, not dropped
    pts = np.concatenate([0.01 * np.arange(40), [1000.0]])[:, None]
    idx, d2 = OK.knn(pts, 1)
    assert idx[40, 0] == 39
    W = OK.adjacency(idx, d2, OK.sigma_of(d2))
    assert W[40, 39] == 0.0 and W[39, 40] == 0.0
    assert W.indptr[41] - W.indptr[40] == 1 and W.indices[W.indptr[40]] == 39
    assert sp.issparse(W) and np.array_equal((W != 0).toarray(), (W != 0).toarray().T)
