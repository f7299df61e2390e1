"""Subspace-upsampling approximate decoder (Algorithm 2) on the GPU against
the FP64 oracle.

Bars: singular values to 1e-12 relative (one-sided Jacobi vs LAPACK); the
decoded X to 1e-8 relative in FP64, since the oracle solves the upsampling
systems exactly and the device CG stops at ||r|| <= 1e-12 ||b||, an error of
at most cond(L_aa) * 1e-12 (cond is below 1e3 on these graphs); 2e-6 in
FP32, where the output is rounded once more (the input is the same
FP32-rounded X~ on both sides)."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import paper_1602_02070_amd as cp
import synth
from oracle import approx as OA
from tests.gpu_util import dev_problem, host, rel, video_problem

pytestmark = pytest.mark.gpu

# (seed, pixel grid of the rows, n, sampling fraction): rho_r >= rho_c and
# rho_r < rho_c (both SVD orientations), odd min(rho_r, rho_c), n odd / even /
# a multiple of 4, several CG workgroups per graph
CASES = [(60, (9, 13), 130, 0.4), (61, (12, 10), 77, 0.5), (62, (5, 11), 45, 0.6),
         (63, (20, 24), 301, 0.2), (64, (40, 48), 1100, 0.1), (65, (7, 7), 2000, 0.05)]
TOL = 1e-12


def _input(P, mode):
    return P.Ytil if mode == "fp64" else P.Ytil.astype(np.float32).astype(np.float64)


def _gap(s, ratio):
    s = np.asarray(s)
    return float(np.min(np.abs(s[s > 0] / s[0] - ratio)))


@pytest.mark.parametrize("mode", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
def test_approx_decode_matches_oracle(case, mode):
    seed, shape, n, frac = case
    P = synth.small_problem(seed, p_shape=shape, n=n, frac=frac, rank=4)
    print(f"[case] approx {mode} seed {seed}: {P.p}x{P.n}, Xtil {P.Ytil.shape}", flush=True)
    dt = torch.float64 if mode == "fp64" else torch.float32
    d = dev_problem(P, dt)
    X_ref, ref = OA.approx_decode(_input(P, mode), P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc,
                                  delta=0.2, ratio=0.1)
    assert _gap(ref["sigma"], 0.1) > 1e-6  # the rank decision is not a rounding tie
    X, sig, info = cp.approx_decode(d["Ytil"], d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"],
                                    delta=0.2, sigma_ratio=0.1, tol=TOL)
    assert info["status"] == 0
    assert info["k"] == ref["k"]
    assert abs(info["scale"] - ref["scale"]) <= 1e-15 * ref["scale"]
    assert np.abs(np.asarray(sig) - ref["sigma"]).max() <= 1e-12 * ref["sigma"][0]
    assert info["rel_residual_r"] <= TOL and info["rel_residual_c"] <= TOL
    e = rel(host(X), X_ref)
    print(f"[approx] k {info['k']} sweeps {info['svd_sweeps']} iters {info['iters_r']}/"
          f"{info['iters_c']} rel.err {e:.2e}", flush=True)
    assert e <= (1e-8 if mode == "fp64" else 2e-6)


def test_approx_decode_full_sampling_and_k_cap():
    P = synth.small_problem(61, p_shape=(12, 10), n=77, frac=0.5, rank=4)
    rng = np.random.default_rng(0)
    Xt = rng.standard_normal((P.p, P.n)) + 3.0 * np.outer(rng.standard_normal(P.p),
                                                          rng.standard_normal(P.n))
    om_r = np.arange(P.p, dtype=np.int32)
    om_c = np.arange(P.n, dtype=np.int32)
    Lr, Lc = cp.Graph.from_scipy(P.Lr), cp.Graph.from_scipy(P.Lc)
    dXt = torch.from_numpy(Xt).cuda()
    for ratio, k_max in ((0.1, 64), (0.0, 3), (0.3, 64)):
        print(f"[case] approx full sampling ratio {ratio} k_max {k_max}", flush=True)
        X_ref, ref = OA.approx_decode(Xt, P.p, P.n, om_r, om_c, P.Lr, P.Lc, ratio=ratio,
                                      k_max=k_max)
        X, _, info = cp.approx_decode(dXt, torch.from_numpy(om_r).cuda(),
                                      torch.from_numpy(om_c).cuda(), P.p, P.n, Lr, Lc,
                                      sigma_ratio=ratio, k_max=k_max, tol=TOL)
        assert info["status"] == 0 and info["k"] == ref["k"]
        # nothing to upsample: X is the rank-k truncation of X~ (scale 1)
        assert info["iters_r"] == 0 and info["iters_c"] == 0
        assert rel(host(X), X_ref) <= 1e-12


def test_approx_decode_unsampled_component_and_zero_input():
    # rows: two connected components, only the first one sampled. The second
    # has no edge to a sample, so its rows are the minimum-norm value 0.
    rng = np.random.default_rng(7)
    pa, pb, n = 30, 25, 40
    # points on a line: each K-NN graph is connected
    La, _ = synth.knn_laplacian(np.linspace(0, 1, pa)[:, None], 6)
    Lb, _ = synth.knn_laplacian(np.linspace(0, 1, pb)[:, None], 6)
    Lr_s = sp.block_diag([La, Lb]).tocsr()
    Lc_s, _ = synth.knn_laplacian(np.linspace(0, 1, n)[:, None], 6)
    om_r = np.sort(rng.choice(pa, 12, replace=False)).astype(np.int32)
    om_c = np.sort(rng.choice(n, 15, replace=False)).astype(np.int32)
    Xt = rng.standard_normal((12, 15))
    Lr, Lc = cp.Graph.from_scipy(Lr_s), cp.Graph.from_scipy(Lc_s)
    dr, dc = torch.from_numpy(om_r).cuda(), torch.from_numpy(om_c).cuda()
    print("[case] approx unsampled component", flush=True)
    X_ref, ref = OA.approx_decode(Xt, pa + pb, n, om_r, om_c, Lr_s, Lc_s, ratio=0.2)
    X, _, info = cp.approx_decode(torch.from_numpy(Xt).cuda(), dr, dc, pa + pb, n, Lr, Lc,
                                  sigma_ratio=0.2, tol=TOL)
    assert info["status"] == 0 and info["k"] == ref["k"]
    Xh = host(X)
    assert np.all(Xh[pa:] == 0.0)
    assert rel(Xh, X_ref) <= 1e-8
    print("[case] approx zero input", flush=True)
    X0, sig0, info0 = cp.approx_decode(torch.zeros((12, 15), dtype=torch.float32).cuda(), dr, dc,
                                       pa + pb, n, Lr, Lc)
    assert info0["status"] == 0 and info0["k"] == 0
    assert np.all(np.asarray(sig0) == 0.0)
    assert torch.count_nonzero(X0).item() == 0


def test_approx_decode_recovers_block_constant_matrix_exactly():
    # two row and two column components, half of each sampled: the oracle's
    # closed-form case, where Algorithm 2 returns the matrix itself. The
    # Laplacians are combinatorial (D - W), whose null space on a component
    # is the constant vector (also the case with a non-unit diagonal, so the
    # Jacobi preconditioner is not the identity)
    rng = np.random.default_rng(5)
    A = [np.arange(0, 60), np.arange(60, 120)]
    B = [np.arange(0, 44), np.arange(44, 88)]
    La = [synth.knn_laplacian(np.linspace(0, 1, g.size)[:, None], 5, kind="combinatorial")[0]
          for g in A]
    Lb = [synth.knn_laplacian(np.linspace(0, 1, g.size)[:, None], 5, kind="combinatorial")[0]
          for g in B]
    Lr_s, Lc_s = sp.block_diag(La).tocsr(), sp.block_diag(Lb).tocsr()
    X = np.zeros((120, 88))
    X[np.ix_(A[0], B[0])] = 3.0
    X[np.ix_(A[1], B[1])] = 0.7
    om_r = np.sort(np.concatenate([rng.choice(g, 30, replace=False) for g in A])).astype(np.int32)
    om_c = np.sort(np.concatenate([rng.choice(g, 22, replace=False) for g in B])).astype(np.int32)
    Xt = X[np.ix_(om_r, om_c)]
    print("[case] approx block-constant recovery", flush=True)
    Xd, _, info = cp.approx_decode(torch.from_numpy(Xt).cuda(), torch.from_numpy(om_r).cuda(),
                                   torch.from_numpy(om_c).cuda(), 120, 88,
                                   cp.Graph.from_scipy(Lr_s), cp.Graph.from_scipy(Lc_s),
                                   tol=TOL)
    assert info["status"] == 0 and info["k"] == 2 and info["scale"] == 2.0
    assert np.abs(host(Xd) - X).max() <= 1e-9


def test_approx_decode_video_shape_sampled_entries():
    # the full 20480 x 4096 video-shaped workload (FP32 output) against the
    # oracle's U, V and scale at 20000 random entries
    P = video_problem()
    print(f"[case] approx video {P.p}x{P.n}, Xtil {P.Ytil.shape}", flush=True)
    d = dev_problem(P, torch.float32)
    Xt_in = _input(P, "fp32")
    Ut, s, Vt = OA.thin_svd(Xt_in)
    k = OA.select_rank(s, 0.1)
    assert _gap(s, 0.1) > 1e-6
    U = OA.upsample(P.Lr, P.omega_r, Ut[:, :k])
    V = OA.upsample(P.Lc, P.omega_c, Vt[:, :k])
    U /= np.linalg.norm(U, axis=0)
    V /= np.linalg.norm(V, axis=0)
    w = OA.rip_scale(P.p, P.n, *P.Ytil.shape) * s[:k]
    X, sig, info = cp.approx_decode(d["Ytil"], d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"],
                                    tol=1e-10)
    assert info["status"] == 0 and info["k"] == k
    assert np.abs(np.asarray(sig) - s).max() <= 1e-12 * s[0]
    rng = np.random.default_rng(1)
    ii = rng.integers(0, P.p, 20000)
    jj = rng.integers(0, P.n, 20000)
    ref = np.einsum("ec,c,ec->e", U[ii], w, V[jj])
    got = X[torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda()].double().cpu().numpy()
    e = rel(got, ref)
    print(f"[approx] video k {k} sweeps {info['svd_sweeps']} iters {info['iters_r']}/"
          f"{info['iters_c']} {info['ms']:.1f} ms, sampled rel.err {e:.2e}", flush=True)
    assert e <= 1e-5


@pytest.mark.parametrize("k_max", [20, 40])
def test_approx_decode_wide_column_layouts(k_max):
    # k = 20 and 40 kept values: the CG panels are 32 and 64 columns wide and
    # the rank-k output takes its one-column-per-thread path (KP > 16)
    P = synth.small_problem(66, p_shape=(16, 18), n=310, frac=0.3, rank=4)
    print(f"[case] approx wide layout k_max {k_max}: {P.p}x{P.n}, Xtil {P.Ytil.shape}", flush=True)
    d = dev_problem(P, torch.float64)
    X_ref, ref = OA.approx_decode(P.Ytil, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc,
                                  ratio=0.0, k_max=k_max)
    assert ref["k"] == k_max
    X, sig, info = cp.approx_decode(d["Ytil"], d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"],
                                    sigma_ratio=0.0, k_max=k_max, tol=TOL)
    assert info["status"] == 0 and info["k"] == k_max
    # the 40 leading singular values of this matrix are distinct (X is unique)
    s = ref["sigma"][:k_max]
    assert np.min(np.diff(-s) / s[0]) > 1e-8
    e = rel(host(X), X_ref)
    print(f"[approx] wide k {k_max}: rel.err {e:.2e}", flush=True)
    assert e <= 1e-8
