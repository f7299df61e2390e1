"""Full-size parity against stored FP64 oracle values.

* Video-shaped workload (p = 128 * 160, n = 4096, 5% row/column sampling):
  the GPU pipeline, in the launch configuration bench.py times, against the
  oracle's X sampled at 20 000 fixed positions
  (tests/golden/video_oracle_samples.npz, from make_video_golden.py). The
  oracle residual is 1.1e-13 with a condition-number estimate of 7.0e3, so
  the stored values are within about 1e-9 of the exact solution. One fused
  product at this shape is also checked entry by entry against the oracle's
  operator, in both element types and both panel kernels.
* Face-shaped workload (10304 x 1000, 10% sampling): FISTA output and X
  against oracle samples (face_oracle_samples.npz, make_face_golden.py).
* Batched workload: eight tasks at full size, among them the largest
  instance at gamma = (100, 100) and (0.1, 100), against oracle samples
  (batch_oracle_samples.npz, make_batch_golden.py).

Every golden file is written by a committed script that calls only synth and
oracle; a stored input fingerprint guards against a change of the generated
inputs."""
import os

import numpy as np
import pytest
import torch

import paper_1602_02070_amd as cp
import synth
from tests.gpu_util import video_problem
from oracle import decoder as OD
from tests.golden.make_batch_golden import fingerprint as batch_fingerprint
from tests.golden.make_face_golden import fingerprint as face_fingerprint
from tests.golden.make_video_golden import fingerprint

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "video_oracle_samples.npz")


@pytest.fixture(scope="module")
def video():
    if not os.path.exists(GOLD):
        pytest.skip("golden samples have not been generated")
    g = np.load(GOLD)
    P = video_problem()
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


# ------------------------------------------------------------------ full-size product

_APPLY_REF = {}


def _apply_reference(P, mode):
    """FP64 oracle product on a seeded full-size operand (rounded to FP32 for
    the FP32 kernels) and an elementwise rounding scale sum |terms|."""
    if mode not in _APPLY_REF:
        rng = np.random.default_rng(5)
        Pm = rng.standard_normal((P.p, P.n))
        if mode == "fp32":
            Pm = Pm.astype(np.float32).astype(np.float64)
        m_r, m_c = OD.masks(P.p, P.n, P.omega_r, P.omega_c)
        ref = OD.apply_A(Pm, m_r, m_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c)
        scale = OD.apply_A(np.abs(Pm), m_r, m_c, abs(P.Lr), abs(P.Lc), P.gamma_r, P.gamma_c)
        _APPLY_REF[mode] = (Pm, ref, scale, float(np.sum(Pm * ref)))
    return _APPLY_REF[mode]


@pytest.mark.parametrize("mode", ["fp32", "fp64"])
@pytest.mark.parametrize("kernel", ["panel_lo", "panel"])
def test_video_full_size_product_elementwise(video, mode, kernel):
    # one fused product at 20480 x 4096 in the panel kernels' real launch
    # geometry (the panel tables, panels per workgroup and per-XCD ranges
    # that the CG uses on this operand), every entry against the oracle
    P, _ = video
    print(f"[case] full-size product {mode} {kernel}", flush=True)
    dev = torch.device("cuda", 0)
    dt = torch.float64 if mode == "fp64" else torch.float32
    Pm, ref, scale, pq_ref = _apply_reference(P, mode)
    Lr, Lc = cp.Graph.from_scipy(P.Lr), cp.Graph.from_scipy(P.Lc)
    om_r = torch.from_numpy(P.omega_r).to(dev)
    om_c = torch.from_numpy(P.omega_c).to(dev)
    cp.set_apply_config(0, -1, kernel=kernel)
    try:
        Q, pq = cp.apply_operator(torch.from_numpy(Pm).to(dt).to(dev), Lr, Lc, P.gamma_r,
                                  P.gamma_c, om_r, om_c, mode=mode)
    finally:
        cp.set_apply_config(0, -1)
    got = Q.double().cpu().numpy()
    u = 2.0 ** -24 if mode == "fp32" else 2.0 ** -53
    # at most 64 rounding steps per output (K_r + K_c + 2 products and sums)
    bad = np.abs(got - ref) > 64 * u * scale
    worst = float(np.max(np.abs(got - ref) / np.maximum(scale, 1e-300)))
    print(f"[product] {mode} {kernel}: max |err| / sum|terms| = {worst:.2e} "
          f"({worst / u:.1f} u), <P,Q> rel.err {abs(pq - pq_ref) / abs(pq_ref):.2e}", flush=True)
    assert not bad.any(), f"{int(bad.sum())} entries outside the rounding bound"
    pq_tol = 1e-5 if mode == "fp32" else 1e-12
    assert abs(pq - pq_ref) <= pq_tol * abs(pq_ref)


# ------------------------------------------------------------------ face shape

FACE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "face_oracle_samples.npz")


@pytest.fixture(scope="module")
def face():
    if not os.path.exists(FACE):
        pytest.skip("face golden samples have not been generated")
    g = np.load(FACE)
    P = synth.cfg2_face(0)
    assert np.allclose(face_fingerprint(P), g["fingerprint"], rtol=1e-9, atol=0.0), \
        "generated inputs changed"
    return P, g


@pytest.mark.parametrize("mode,tol,res_bar,bar", [("fp32_ir", 1e-8, 1e-8, 1e-5),
                                                  ("fp32", 1e-6, 2e-5, 1e-4),
                                                  ("fp64", 1e-11, 1e-11, 1e-7)])
def test_face_full_size_matches_oracle_samples(face, mode, tol, res_bar, bar):
    # the face-shaped workload (10304 x 1000, 10% sampling): FISTA 500
    # iterations on the FP32 (or FP64) sampled matrix, then the decoder.
    # Plain FP32 CG stops on its recursive residual, whose true FP64 value
    # stalls at a few 1e-6 here; its error is reported against a looser bar
    # (the 1e-5 bar is for the refined FP32 mode).
    P, g = face
    print(f"[case] golden face {mode}", flush=True)
    dev = torch.device("cuda", 0)
    dt = torch.float64 if mode == "fp64" else torch.float32
    Lr, Lc = cp.Graph.from_scipy(P.Lr), cp.Graph.from_scipy(P.Lc)
    Lrt, Lct = cp.Graph.from_scipy(P.Lr_til), cp.Graph.from_scipy(P.Lc_til)
    Y = torch.from_numpy(P.Ytil).to(dt).to(dev)
    Xt, _ = cp.frpcag(Y, Lrt, Lct, P.gamma_r, P.gamma_c, P.lmax_r_til, P.lmax_c_til,
                      max_iter=500)
    got_t = Xt.reshape(-1)[torch.from_numpy(g["idx_t"]).to(dev)].double().cpu().numpy()
    err_t = np.linalg.norm(got_t - g["vals_t"]) / np.linalg.norm(g["vals_t"])
    X, di = cp.decode(Xt, torch.from_numpy(P.omega_r).to(dev), torch.from_numpy(P.omega_c).to(dev),
                      P.p, P.n, Lr, Lc, P.gamma_r, P.gamma_c, tol=tol, max_iter=50000, mode=mode)
    assert di["status"] == 0 and di["rel_residual"] <= res_bar
    got = X.reshape(-1)[torch.from_numpy(g["idx"]).to(dev)].double().cpu().numpy()
    err = np.linalg.norm(got - g["vals"]) / np.linalg.norm(g["vals"])
    norm = float(X.double().norm())
    print(f"[golden] face {mode}: X~ sampled rel.err {err_t:.3e}; X sampled rel.err {err:.3e} "
          f"({di['iters']} it, FP64 residual {di['rel_residual']:.1e}), ||X|| {norm:.6e} vs "
          f"{float(g['norm']):.6e}", flush=True)
    assert err_t <= (1e-6 if mode != "fp64" else 1e-11)
    assert err <= bar
    assert abs(norm - float(g["norm"])) <= bar * float(g["norm"])


# ------------------------------------------------------------------ batched subset

BATCH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                     "batch_oracle_samples.npz")


def test_batched_full_size_subset_matches_oracle_samples():
    # eight tasks of the batched workload (64 instances x 4 x 4 gammas) at
    # their full sizes, among them the largest instance at gamma = (100, 100)
    # and (0.1, 100): one batched FP32 + refinement run, FISTA 100 iterations,
    # decoder to 1e-8, against FP64 oracle samples of every task's X
    if not os.path.exists(BATCH):
        pytest.skip("batched golden samples have not been generated")
    g = np.load(BATCH)
    print("[case] golden batched subset", flush=True)
    probs, _ = synth.cfg5_batch(0)
    tasks = [(int(k), float(a), float(b)) for k, a, b in g["tasks"]]
    used = sorted({k for k, _, _ in tasks})
    dev = torch.device("cuda", 0)
    inst = []
    for k in used:
        P = probs[k]
        t0 = next(t for t, (kk, _, _) in enumerate(tasks) if kk == k)
        assert np.allclose(batch_fingerprint(P), g[f"t{t0}_fingerprint"], rtol=1e-9, atol=0.0), \
            f"generated inputs of instance {k} changed"
        G = {a: cp.Graph.from_scipy(getattr(P, a)) for a in ("Lr", "Lc", "Lr_til", "Lc_til")}
        inst.append(cp.Instance(P.p, P.n, torch.from_numpy(P.omega_r).to(dev),
                                torch.from_numpy(P.omega_c).to(dev), G["Lr"], G["Lc"],
                                G["Lr_til"], G["Lc_til"], P.lmax_r_til, P.lmax_c_til,
                                torch.from_numpy(P.Ytil).float().to(dev)))
    btasks = [(used.index(k), gr, gc) for k, gr, gc in tasks]
    Xs, _, infos = cp.solve_batched(inst, btasks, fista_iters=100, tol=1e-8, max_iter=50000,
                                    mode="fp32_ir")
    for t, ((k, gr, gc), X, info) in enumerate(zip(tasks, Xs, infos)):
        assert info["status"] == 0, (t, info)
        idx = torch.from_numpy(g[f"t{t}_idx"]).to(dev)
        got = X.reshape(-1)[idx].double().cpu().numpy()
        ref = g[f"t{t}_vals"]
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        nerr = abs(float(X.double().norm()) - float(g[f"t{t}_norm"])) / float(g[f"t{t}_norm"])
        print(f"[golden] batch task {t}: instance {k} {probs[k].p}x{probs[k].n} gamma ({gr}, {gc}):"
              f" sampled rel.err {err:.2e}, norm rel.err {nerr:.2e}, {info['iters']} it "
              f"(oracle kappa {float(g[f't{t}_kappa']):.1e})", flush=True)
        assert err <= 1e-5 and nerr <= 1e-5, (t, k, gr, gc, err, nerr)
