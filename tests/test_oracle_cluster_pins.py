"""Pins of the clustering-decoder oracle (Section VI, Algorithm 3) against
facts that do not come from the oracle itself."""
import itertools

import numpy as np
import scipy.sparse as sp

from oracle import cluster as OC


def _line_laplacian(idx_groups, n, rng):
    """Combinatorial Laplacian (D - W) of disjoint weighted paths, one per
    group of node indices."""
    W = np.zeros((n, n))
    for g in idx_groups:
        for a, b in zip(g[:-1], g[1:]):
            W[a, b] = W[b, a] = rng.uniform(0.5, 1.5)
    return sp.csr_matrix(np.diag(W.sum(1)) - W)


def test_kmeans_recovers_separated_blobs_and_their_means():
    rng = np.random.default_rng(0)
    centers = np.array([[0.0, 0.0, 0.0], [10.0, 0.0, 0.0], [0.0, 10.0, 5.0]])
    truth = np.repeat(np.arange(3), [7, 9, 6])
    pts = centers[truth] + 0.3 * rng.standard_normal((truth.size, 3))
    init = pts[[0, 7, 16]]  # one point of each blob
    lab, cen, it = OC.kmeans(pts, init)
    assert np.array_equal(lab, truth)
    for j in range(3):
        assert np.allclose(cen[j], pts[truth == j].mean(axis=0), rtol=0, atol=1e-14)
    assert 1 <= it <= 3


def test_kmeans_fixed_point_conditions():
    # at convergence every point is nearest to its own centroid (brute force
    # over all centroids) and every non-empty centroid is its members' mean
    rng = np.random.default_rng(1)
    pts = rng.standard_normal((60, 4))
    lab, cen, _ = OC.kmeans(pts, pts[:5], max_iter=500)
    for i, x in enumerate(pts):
        d = [float(np.dot(x - c, x - c)) for c in cen]
        assert d[lab[i]] == min(d)
    for j in range(5):
        if np.any(lab == j):
            assert np.allclose(cen[j], pts[lab == j].mean(axis=0), atol=1e-14)


def test_kmeans_matches_brute_force_two_partition():
    # 9 points in two groups: the best 2-partition by brute force (all
    # 2^9 assignments, within-cluster sum of squares) is what Lloyd reaches
    rng = np.random.default_rng(2)
    pts = np.vstack([rng.normal(0.0, 0.5, (4, 2)), rng.normal(4.0, 0.5, (5, 2))])

    def sse(lab):
        return sum(((pts[lab == j] - pts[lab == j].mean(0)) ** 2).sum()
                   for j in (0, 1) if np.any(lab == j))

    best = min((np.array(a) for a in itertools.product((0, 1), repeat=9)), key=sse)
    lab, _, _ = OC.kmeans(pts, pts[[0, 8]])
    assert np.array_equal(lab, best) or np.array_equal(lab, 1 - best)


def test_indicators_and_max_pool():
    lab = np.array([2, 0, 1, 2])
    C = OC.indicators(lab, 3)
    assert C.shape == (4, 3) and np.array_equal(C.sum(1), np.ones(4))
    assert np.array_equal(OC.max_pool(C), lab)
    assert np.array_equal(OC.max_pool(np.array([[0.2, 0.7, 0.7], [0.5, 0.5, 0.1]])), [1, 0])


def test_cluster_decode_on_component_graph_is_exact():
    # the column graph has one component per cluster and every component is
    # sampled (the lambda = 0 case of the clustering theorem): the
    # upsampled indicators are exactly one-hot and every label is right; a
    # fifth component without samples gets C = 0 and label 0
    rng = np.random.default_rng(3)
    sizes = [30, 25, 40, 20]
    groups, start = [], 0
    for s in sizes:
        groups.append(np.arange(start, start + s))
        start += s
    orphan = np.arange(start, start + 6)
    n = start + 6
    Lc = _line_laplacian(groups + [orphan], n, rng)
    truth = np.concatenate([np.full(s, j) for j, s in enumerate(sizes)] + [np.zeros(6, int)])
    omega_c = np.sort(np.concatenate([rng.choice(g, 6, replace=False) for g in groups]))
    rho_r = 12
    means = rng.normal(0.0, 8.0, (4, rho_r))
    Xt = (means[truth[omega_c]] + 0.2 * rng.standard_normal((omega_c.size, rho_r))).T
    init = [int(np.flatnonzero(truth[omega_c] == j)[0]) for j in range(4)]
    labels, info = OC.cluster_decode(Xt, n, omega_c, Lc, init)
    assert np.array_equal(info["sample_labels"], truth[omega_c])
    assert np.array_equal(labels, truth)
    C = info["C"]
    assert np.abs(C[:start] - OC.indicators(truth[:start], 4)).max() <= 1e-12
    assert np.all(C[start:] == 0.0)


def test_upsampled_indicators_form_a_partition_of_unity():
    # with a combinatorial Laplacian the constant vector is harmonic, so the
    # upsampled indicators of a connected graph sum to one on every row, and
    # the sampled rows keep their k-means labels
    rng = np.random.default_rng(4)
    n = 80
    Lc = _line_laplacian([np.arange(n)], n, rng)
    Lc = Lc + _line_laplacian([rng.permutation(n)], n, rng)  # a second path: loops
    omega_c = np.sort(rng.choice(n, 20, replace=False))
    Xt = rng.standard_normal((6, 20))
    labels, info = OC.cluster_decode(Xt, n, omega_c, Lc, [0, 1, 2])
    C = info["C"]
    assert np.abs(C.sum(axis=1) - 1.0).max() <= 1e-12
    assert np.array_equal(labels[omega_c], info["sample_labels"])
    # the k-means inside the decoder ran to its fixed point on these
    # unstructured points: centroids are their members' means, labels nearest
    pts, lab, cen = Xt.T, info["sample_labels"], info["centroids"]
    assert info["kmeans_iters"] >= 1
    for j in range(3):
        if np.any(lab == j):
            assert np.allclose(cen[j], pts[lab == j].mean(axis=0), atol=1e-14)
    assert np.array_equal(lab, np.argmin(((pts[:, None] - cen[None]) ** 2).sum(2), axis=1))


def test_kmeans_update_cap_by_hand():
    # 1-D points 0, 2, 3, 7, 10 with seeds 0 and 2, worked by hand:
    #   assignment to (0, 2)        -> 0 1 1 1 1, means (0, 5.5)
    #   assignment to (0, 5.5)      -> 0 0 1 1 1, means (1, 20/3)
    #   assignment to (1, 20/3)     -> 0 0 0 1 1, means (5/3, 8.5)
    #   assignment to (5/3, 8.5)    -> unchanged: converged after 3 updates
    pts = np.array([[0.0], [2.0], [3.0], [7.0], [10.0]])
    seeds = pts[[0, 1]]
    want = {
        0: ([0, 1, 1, 1, 1], [0.0, 2.0]),
        1: ([0, 0, 1, 1, 1], [0.0, 5.5]),
        2: ([0, 0, 0, 1, 1], [1.0, 20.0 / 3.0]),
        3: ([0, 0, 0, 1, 1], [5.0 / 3.0, 8.5]),
        100: ([0, 0, 0, 1, 1], [5.0 / 3.0, 8.5]),
    }
    for cap, (lab_w, cen_w) in want.items():
        lab, cen, it = OC.kmeans(pts, seeds, max_iter=cap)
        assert list(lab) == lab_w, cap
        assert np.allclose(cen[:, 0], cen_w, rtol=0, atol=1e-15), cap
        assert it == min(cap, 3)
