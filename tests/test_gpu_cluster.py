"""Clustering decoder (Algorithm 3) on the GPU against the FP64 oracle.

k-means labels and iteration counts must match exactly (the inputs keep the
nearest and second-nearest centroid of every point apart by far more than
rounding). The upsampled indicators C are checked by their backward error:
the true residual of the device's C in the oracle's system
L(bar, bar) c = -L(bar, omega) c~, relative to the right-hand side, must be
at most 1e-10 (the device CG stops at a recursive residual of 1e-12). The
forward error is that times cond(L(bar, bar)), which grows with the graph:
1e-5 absolute on entries in [0, 1] is the bar. Max pooling must agree
wherever the oracle's two largest entries of a row differ by more than 4x
the measured forward error; where they do not, the device's choice must be
one of the near-tied maxima."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import paper_1602_02070_amd as cp
import synth
from oracle import cluster as OC

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _margins(pts, cen, lab):
    d = ((pts[:, None, :] - cen[None]) ** 2).sum(2)
    own = d[np.arange(len(lab)), lab]
    d[np.arange(len(lab)), lab] = np.inf
    return (d.min(1) - own) / np.maximum(own, 1e-300)


def _check(P, Xt_in, mode, init, km_iter=100):
    dt = torch.float64 if mode == "fp64" else torch.float32
    ref_lab, ref = OC.cluster_decode(Xt_in, P.n, P.omega_c, P.Lc, init, km_iter)
    assert _margins(Xt_in.T, ref["centroids"], ref["sample_labels"]).min() > 1e-6
    lab, slab, C, info = cp.cluster_decode(torch.from_numpy(Xt_in).to(dt).cuda(),
                                           torch.from_numpy(P.omega_c).cuda(), P.n,
                                           cp.Graph.from_scipy(P.Lc), init, km_iter, tol=TOL,
                                           want_C=True)
    assert info["status"] == 0
    assert info["kmeans_iters"] == ref["kmeans_iters"]
    assert np.array_equal(slab.cpu().numpy(), ref["sample_labels"])
    Ch = C.cpu().numpy()
    # backward error in the oracle's own system
    L = sp.csr_matrix(P.Lc)
    rest = np.setdiff1d(np.arange(P.n), P.omega_c)
    Ctil = OC.indicators(ref["sample_labels"], len(init))
    b = -(L[rest][:, P.omega_c] @ Ctil)
    r = L[rest][:, rest] @ Ch[rest] - b
    bn = np.linalg.norm(b, axis=0)
    back = np.max(np.linalg.norm(r, axis=0)[bn > 0] / bn[bn > 0]) if np.any(bn > 0) else 0.0
    assert back <= 1e-10, back
    assert np.array_equal(Ch[P.omega_c], Ctil)
    err = np.abs(Ch - ref["C"]).max()
    assert err <= 1e-5
    got = lab.cpu().numpy()
    Cs = np.sort(ref["C"], axis=1)
    gap = Cs[:, -1] - Cs[:, -2] if Cs.shape[1] > 1 else np.full(P.n, np.inf)
    margin = 4.0 * err + 1e-12
    clear = gap > margin
    assert np.array_equal(got[clear], ref_lab[clear])
    rows = np.flatnonzero(~clear)
    assert np.all(ref["C"][rows, got[rows]] >= Cs[rows, -1] - margin)
    print(f"[cluster] backward error {back:.1e}", flush=True)
    return info, err, int((~clear).sum())


@pytest.mark.parametrize("mode", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(3000, 8, 5, 0.1), (5000, 12, 7, 0.05), (1200, 6, 3, 0.2)],
                         ids=["n3000", "n5000", "n1200"])
def test_cluster_decode_matches_oracle(shape, mode):
    n, side, k, frac = shape
    P = synth.cluster_digits(0, n=n, side=side, k=k, frac_c=frac)
    print(f"[case] cluster {mode} n {n} p {P.p} rho_c {P.rho_c} k {k}", flush=True)
    Xt = P.Ytil if mode == "fp64" else P.Ytil.astype(np.float32).astype(np.float64)
    info, err, ties = _check(P, Xt, mode, P.meta["init"])
    print(f"[cluster] kmeans {info['kmeans_iters']} it, CG {info['cg_iters']} it, "
          f"C err {err:.1e}, near-ties {ties}", flush=True)


def test_cluster_decode_kmeans_cap_and_single_cluster():
    P = synth.cluster_digits(1, n=2000, side=8, k=4, frac_c=0.1)
    print("[case] cluster kmeans_max_iter 0 and 1", flush=True)
    for km in (0, 1):
        info, _, _ = _check(P, P.Ytil, "fp64", P.meta["init"], km_iter=km)
        assert info["kmeans_iters"] == km
    print("[case] cluster k = 1", flush=True)
    lab, slab, C, info = cp.cluster_decode(torch.from_numpy(P.Ytil).cuda(),
                                           torch.from_numpy(P.omega_c).cuda(), P.n,
                                           cp.Graph.from_scipy(P.Lc), [3], want_C=True)
    assert info["status"] == 0
    assert torch.count_nonzero(lab).item() == 0 and torch.count_nonzero(slab).item() == 0
    # one indicator equal to one on every sample: its harmonic extension is
    # the solution of the full upsampling system, finite everywhere
    assert torch.isfinite(C).all()


def test_cluster_decode_component_graph_is_exact():
    # one component per cluster, every component sampled, plus an unsampled
    # component: exact labels, C one-hot, the orphan rows 0 (label 0)
    rng = np.random.default_rng(3)
    sizes = [300, 250, 400, 200]
    groups, start = [], 0
    Ls = []
    for s in sizes:
        groups.append(np.arange(start, start + s))
        Ls.append(synth.knn_laplacian(np.linspace(0, 1, s)[:, None], 4, kind="combinatorial")[0])
        start += s
    Ls.append(synth.knn_laplacian(np.linspace(0, 1, 60)[:, None], 4, kind="combinatorial")[0])
    n = start + 60
    Lc = sp.block_diag(Ls).tocsr()
    truth = np.concatenate([np.full(s, j) for j, s in enumerate(sizes)] + [np.zeros(60, int)])
    om = np.sort(np.concatenate([rng.choice(g, 25, replace=False) for g in groups])).astype(np.int32)
    means = rng.normal(0.0, 8.0, (4, 16))
    Xt = (means[truth[om]] + 0.2 * rng.standard_normal((om.size, 16))).T.copy()
    init = [int(np.flatnonzero(truth[om] == j)[0]) for j in range(4)]
    print("[case] cluster component graph", flush=True)
    lab, slab, C, info = cp.cluster_decode(torch.from_numpy(Xt).cuda(), torch.from_numpy(om).cuda(),
                                           n, cp.Graph.from_scipy(Lc), init, tol=TOL, want_C=True)
    assert info["status"] == 0
    assert np.array_equal(lab.cpu().numpy(), truth)
    Ch = C.cpu().numpy()
    assert np.abs(Ch[:start] - OC.indicators(truth[:start], 4)).max() <= 1e-9
    assert np.all(Ch[start:] == 0.0)


def test_cluster_decode_digits_shape():
    # the full clustering workload: 784 x 70000, 5% of the samples, k = 10
    P = synth.cluster_digits(0)
    print(f"[case] cluster digits {P.p}x{P.n}, rho_c {P.rho_c}", flush=True)
    Xt = P.Ytil.astype(np.float32).astype(np.float64)
    info, err, ties = _check(P, Xt, "fp32", P.meta["init"])
    print(f"[cluster] digits: kmeans {info['kmeans_iters']} it, CG {info['cg_iters']} it, "
          f"{info['ms']:.1f} ms, C err {err:.1e}, near-ties {ties}", flush=True)


def test_cluster_decode_many_clusters():
    # 33 clusters: the indicator panels are 64 columns wide
    P = synth.cluster_digits(2, n=4000, side=8, k=33, frac_c=0.1)
    print(f"[case] cluster k 33: n {P.n} rho_c {P.rho_c}", flush=True)
    info, err, ties = _check(P, P.Ytil, "fp64", P.meta["init"])
    print(f"[cluster] k 33: kmeans {info['kmeans_iters']} it, CG {info['cg_iters']} it, "
          f"C err {err:.1e}, near-ties {ties}", flush=True)
