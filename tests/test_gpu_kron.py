"""Kron reduction on the GPU (cpca_kron_reduce) against the FP64 oracle
(oracle/kron.py, Section IV-A).

Bar: the device solves every column of L(bar, bar)^-1 L(bar, Omega) by PCG to
||r|| <= 1e-12 ||b||; the oracle factorises. The error of a column is at
most cond(L(bar, bar)) * 1e-12, below 1e-8 relative to max |L~| on these
graphs."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import paper_1602_02070_amd as cp
import synth
from tests.gpu_util import video_problem
from oracle import kron as OK

pytestmark = pytest.mark.gpu


def _run(L, om, tol=1e-12):
    R, info = cp.kron_reduce(cp.Graph.from_scipy(L), torch.from_numpy(np.asarray(om, np.int32)).cuda(),
                             tol=tol)
    return R.cpu().numpy(), info


def _check(L, om, bar=1e-8):
    ref = OK.kron_reduce(L, om)
    got, info = _run(L, om)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"[kron] n {L.shape[0]} rho {len(om)}: max err {err:.2e}, {info['iters']} CG it, "
          f"{info['ms']:.1f} ms", flush=True)
    assert info["status"] == 0
    assert err <= bar
    assert np.array_equal(got, got.T)
    return got


@pytest.mark.parametrize("kind", ["combinatorial", "normalized"])
@pytest.mark.parametrize("seed,shape,frac", [(80, (9, 13), 0.3), (81, (12, 10), 0.05),
                                             (82, (20, 24), 0.2), (83, (7, 7), 0.9)])
def test_kron_matches_oracle_on_pixel_graphs(kind, seed, shape, frac):
    rng = np.random.default_rng(seed)
    L, _ = synth.knn_laplacian(synth.grid_coords(*shape), 10, kind)
    n = L.shape[0]
    om = np.sort(rng.choice(n, max(1, int(round(frac * n))), replace=False))
    R = _check(L, om)
    if kind == "combinatorial":
        assert np.abs(R.sum(1)).max() <= 1e-8 * np.abs(R).max()


def test_kron_more_than_64_columns_and_isolated_parts():
    # 150 sampled nodes (three column batches) on a graph with a component
    # that holds no sample, and a sampled node with no unsampled neighbour
    rng = np.random.default_rng(3)
    L1, _ = synth.knn_laplacian(rng.standard_normal((400, 3)), 8, "combinatorial")
    L2, _ = synth.knn_laplacian(rng.standard_normal((30, 2)), 4, "combinatorial")
    L = sp.block_diag([L1, L2, sp.csr_matrix((1, 1))]).tocsr()
    om = np.sort(np.concatenate([rng.choice(400, 149, replace=False), [430]]))
    _check(L, om)


def test_kron_video_row_graph_full_size():
    # the 128 x 160 pixel graph of the video-shaped workload reduced onto its
    # 1024 sampled rows (16 column batches), as the compressed row graph
    print("[case] kron video rows", flush=True)
    P = video_problem()
    _check(P.Lr, P.omega_r, bar=1e-8)
