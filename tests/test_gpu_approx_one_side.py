"""Approximate decoders 2 and 3 of the appendix on the GPU
(cpca_approx_decode2 / 3) against the FP64 oracle (approx_decode_rows /
approx_decode_cols): one graph side upsampled, the full data projected.

Bars as for Algorithm 2: the decoded X to 1e-8 relative in FP64 (per-column
CG to 1e-12 against the oracle's direct solve) and 2e-6 in FP32 (output and
input rounded once)."""
import numpy as np
import pytest
import torch

import paper_1602_02070_amd as cp
import synth
from oracle import approx as OA
from tests.gpu_util import host, rel, video_problem

pytestmark = pytest.mark.gpu

CASES = [(70, (9, 13), 130, 0.4), (71, (12, 10), 77, 0.5), (72, (5, 11), 45, 0.6),
         (73, (20, 24), 301, 0.2), (74, (40, 48), 1100, 0.1), (75, (7, 7), 2000, 0.05)]
TOL = 1e-12


def _gap(s, ratio):
    s = np.asarray(s)
    return float(np.min(np.abs(s[s > 0] / s[0] - ratio)))


def _r32(a):
    return np.asarray(a).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("side", ["rows", "cols"])
@pytest.mark.parametrize("mode", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
def test_one_side_decoders_match_oracle(case, mode, side):
    seed, shape, n, frac = case
    P = synth.small_problem(seed, p_shape=shape, n=n, frac=frac, rank=4, keep_full=True)
    print(f"[case] decoder {'2' if side == 'rows' else '3'} {mode} seed {seed}: {P.p}x{P.n}",
          flush=True)
    dt = torch.float64 if mode == "fp64" else torch.float32
    Xt = P.Ytil if mode == "fp64" else _r32(P.Ytil)
    Y = P.Y if mode == "fp64" else _r32(P.Y)
    if side == "rows":
        X_ref, ref = OA.approx_decode_rows(Xt, Y, P.omega_r, P.Lr, ratio=0.1, k_max=16)
        om, L = P.omega_r, P.Lr
    else:
        X_ref, ref = OA.approx_decode_cols(Xt, Y, P.omega_c, P.Lc, ratio=0.1, k_max=16)
        om, L = P.omega_c, P.Lc
    assert _gap(ref["sigma"], 0.1) > 1e-6
    X, sig, info = cp.approx_decode_one_side(
        side, torch.from_numpy(Xt).to(dt).cuda(), torch.from_numpy(om).cuda(), P.p, P.n,
        cp.Graph.from_scipy(L), torch.from_numpy(Y).to(dt).cuda(), sigma_ratio=0.1, k_max=16,
        tol=TOL)
    assert info["status"] == 0 and info["k"] == ref["k"] and info["scale"] == 1.0
    assert np.abs(np.asarray(sig) - ref["sigma"]).max() <= 1e-12 * ref["sigma"][0]
    used = info["rel_residual_r"] if side == "rows" else info["rel_residual_c"]
    other = info["iters_c"] if side == "rows" else info["iters_r"]
    assert used <= TOL and other == 0
    e = rel(host(X), X_ref)
    print(f"[one-side] k {info['k']} iters {info['iters_r']}/{info['iters_c']} rel.err {e:.2e}",
          flush=True)
    assert e <= (1e-8 if mode == "fp64" else 2e-6)


def test_one_side_decoders_full_sampling_truncate_Y():
    # every row and column sampled and X~ = Y: decoder 2 and 3 both return the
    # rank-k truncation of Y (nothing is upsampled)
    P = synth.small_problem(71, p_shape=(12, 10), n=77, frac=0.5, rank=4, keep_full=True)
    print("[case] one-side full sampling", flush=True)
    Y = P.Y
    U, s, Vt = np.linalg.svd(Y, full_matrices=False)
    k = int(np.count_nonzero(s >= 0.1 * s[0]))
    trunc = (U[:, :k] * s[:k]) @ Vt[:k]
    dY = torch.from_numpy(Y).cuda()
    for side, om, L in (("rows", np.arange(P.p, dtype=np.int32), P.Lr),
                        ("cols", np.arange(P.n, dtype=np.int32), P.Lc)):
        X, _, info = cp.approx_decode_one_side(side, dY, torch.from_numpy(om).cuda(), P.p, P.n,
                                               cp.Graph.from_scipy(L), dY, sigma_ratio=0.1,
                                               k_max=16, tol=TOL)
        assert info["status"] == 0 and info["k"] == k
        assert rel(host(X), trunc) <= 1e-11


@pytest.fixture(scope="module")
def video_full():
    return video_problem()


@pytest.mark.parametrize("side", ["rows", "cols"])
def test_one_side_decoders_video_full_size(video_full, side):
    # the video-shaped workload, 20480 x 4096, with the FP32 full data: one
    # launch configuration of each projection at its real shape
    P = video_full
    print(f"[case] decoder {'2' if side == 'rows' else '3'} video full size", flush=True)
    Xt, Y = _r32(P.Ytil), _r32(P.Y)
    if side == "rows":
        X_ref, ref = OA.approx_decode_rows(Xt, Y, P.omega_r, P.Lr, ratio=0.1, k_max=16)
        om, L = P.omega_r, P.Lr
    else:
        X_ref, ref = OA.approx_decode_cols(Xt, Y, P.omega_c, P.Lc, ratio=0.1, k_max=16)
        om, L = P.omega_c, P.Lc
    X, sig, info = cp.approx_decode_one_side(
        side, torch.from_numpy(Xt).float().cuda(), torch.from_numpy(om).cuda(), P.p, P.n,
        cp.Graph.from_scipy(L), torch.from_numpy(Y).float().cuda(), sigma_ratio=0.1, k_max=16,
        tol=1e-10)
    assert info["status"] == 0 and info["k"] == ref["k"]
    e = rel(host(X), X_ref)
    print(f"[one-side] video {side}: k {info['k']}, CG {info['iters_r']}/{info['iters_c']}, "
          f"rel.err {e:.2e}, {info['ms']:.1f} ms", flush=True)
    assert e <= 2e-6
