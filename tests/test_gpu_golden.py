"""Full-size parity on the video-shaped workload (p = 128 * 160, n = 4096, 5%
row/column sampling): the GPU pipeline, in the launch configuration bench.py
times, against FP64 oracle values of X sampled at 20 000 fixed positions
(tests/golden/video_oracle_samples.npz, written by
tests/golden/make_video_golden.py from synth and oracle only). The stored
input fingerprint guards against a change of the generated inputs; the oracle
residual is 1.1e-13 with a condition-number estimate of 7.0e3, so the stored
values are within about 1e-9 of the exact solution."""
import os

import numpy as np
import pytest
import torch

import paper_1602_02070_amd as cp
import synth
from tests.golden.make_video_golden import fingerprint

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "video_oracle_samples.npz")


@pytest.fixture(scope="module")
def video():
    if not os.path.exists(GOLD):
        pytest.skip("golden samples have not been generated")
    g = np.load(GOLD)
    P = synth.cfg3_video(0)
    # the generators' eigen-solvers round differently on different hosts (last
    # bits); a change beyond that means the inputs are not the stored ones
    assert np.allclose(fingerprint(P), g["fingerprint"], rtol=1e-9, atol=0.0), \
        "generated inputs changed"
    return P, g


@pytest.mark.parametrize("mode,tol,bar", [("fp32_ir", 1e-8, 1e-5), ("fp64", 1e-11, 1e-7)])
def test_video_full_size_matches_oracle_samples(video, mode, tol, bar):
    P, g = video
    print(f"[case] golden video {mode}", flush=True)
    dev = torch.device("cuda", 0)
    dt = torch.float64 if mode == "fp64" else torch.float32
    Lr, Lc = cp.Graph.from_scipy(P.Lr), cp.Graph.from_scipy(P.Lc)
    Lrt, Lct = cp.Graph.from_scipy(P.Lr_til), cp.Graph.from_scipy(P.Lc_til)
    Y = torch.from_numpy(P.Ytil).to(dt).to(dev)
    Xt, fi = cp.frpcag(Y, Lrt, Lct, P.gamma_r, P.gamma_c, P.lmax_r_til, P.lmax_c_til,
                       max_iter=500)
    X, di = cp.decode(Xt, torch.from_numpy(P.omega_r).to(dev), torch.from_numpy(P.omega_c).to(dev),
                      P.p, P.n, Lr, Lc, P.gamma_r, P.gamma_c, tol=tol, max_iter=50000, mode=mode)
    assert di["status"] == 0 and di["rel_residual"] <= tol
    idx = torch.from_numpy(g["idx"]).to(dev)
    got = X.reshape(-1)[idx].double().cpu().numpy()
    ref = g["vals"]
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    norm = float(X.double().norm())
    print(f"[golden] {mode}: sampled rel.err {err:.3e}, ||X|| {norm:.6e} vs {float(g['norm']):.6e}",
          flush=True)
    assert err <= bar
    assert abs(norm - float(g["norm"])) <= bar * float(g["norm"])
