"""Batched solves (many instances of uneven sizes, gamma grids) against the
single-problem calls and against the FP64 oracle."""
import ctypes
import os

import numpy as np
import pytest
import torch

import paper_1602_02070_amd as cp
from paper_1602_02070_amd import _lib
import synth
from oracle import decoder as OD
from oracle import frpcag as OF
from tests.gpu_util import dev_problem, host, rel

pytestmark = pytest.mark.gpu

SHAPES = [((6, 7), 45), ((9, 13), 130), ((5, 11), 77), ((12, 10), 201), ((4, 9), 38)]
GRID = [(0.5, 0.3), (0.5, 3.0), (5.0, 0.3), (5.0, 3.0)]
J = 60


@pytest.fixture(scope="module")
def batch():
    probs = [synth.small_problem(40 + k, p_shape=s, n=n, frac=0.4, rank=3)
             for k, (s, n) in enumerate(SHAPES)]
    return probs


def _instances(probs, dtype):
    out = []
    for P in probs:
        d = dev_problem(P, dtype)
        out.append(cp.Instance(P.p, P.n, d["om_r"], d["om_c"], d["Lr"], d["Lc"], d["Lr_til"],
                               d["Lc_til"], P.lmax_r_til, P.lmax_c_til, d["Ytil"]))
    return out


def _tasks(probs):
    return [(k, gr, gc) for k in range(len(probs)) for gr, gc in GRID]


@pytest.mark.parametrize("mode", ["fp64", "fp32_ir"])
def test_batched_matches_single_calls_and_oracle(batch, mode):
    print(f"[case] batched {mode}", flush=True)
    dt = torch.float64 if mode == "fp64" else torch.float32
    inst = _instances(batch, dt)
    tasks = _tasks(batch)
    tol = 1e-12 if mode == "fp64" else 1e-10
    Xs, Xts, infos = cp.solve_batched(inst, tasks, fista_iters=J, tol=tol, mode=mode,
                                      want_xtil=True)
    assert all(i["status"] == 0 for i in infos)
    for t, (k, gr, gc) in enumerate(tasks):
        P, I = batch[k], inst[k]
        Xt1, _ = cp.frpcag(I.Ytil, I.Lr_til, I.Lc_til, gr, gc, P.lmax_r_til, P.lmax_c_til,
                           max_iter=J)
        X1, _ = cp.decode(Xt1, I.omega_r, I.omega_c, P.p, P.n, I.Lr, I.Lc, gr, gc, tol=tol,
                          mode=mode)
        assert rel(host(Xts[t]), host(Xt1)) <= 1e-12
        assert rel(host(Xs[t]), host(X1)) <= (1e-9 if mode == "fp64" else 1e-6)
        # oracle: FISTA then the exact decoder on the (rounded) estimate
        Y = P.Ytil if mode == "fp64" else P.Ytil.astype(np.float32).astype(np.float64)
        Xt_ref, _ = OF.fista(Y, P.Lr_til, P.Lc_til, gr, gc, P.lmax_r_til, P.lmax_c_til, J)
        if mode != "fp64":
            Xt_ref = Xt_ref.astype(np.float32).astype(np.float64)
        X_ref = OD.decode(Xt_ref, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, gr, gc)
        assert rel(host(Xs[t]), X_ref) <= (1e-8 if mode == "fp64" else 1e-5), (t, k, gr, gc)


def test_batched_deterministic_and_autotuned(batch):
    print("[case] batched determinism + autotune", flush=True)
    inst = _instances(batch, torch.float32)
    tasks = _tasks(batch)
    a, _, _ = cp.solve_batched(inst, tasks, fista_iters=J, tol=1e-10)
    b, _, _ = cp.solve_batched(inst, tasks, fista_iters=J, tol=1e-10)
    assert all(torch.equal(x, y) for x, y in zip(a, b))
    cp.set_apply_config(-1, -1)
    try:
        c, _, infos = cp.solve_batched(inst, tasks, fista_iters=J, tol=1e-10)
        assert all(i["status"] == 0 for i in infos)
        for x, y in zip(a, c):
            assert rel(host(x), host(y)) <= 1e-6
        # single-problem autotune path as well
        P = batch[3]
        I = inst[3]
        X1, _ = cp.decode(I.Ytil, I.omega_r, I.omega_c, P.p, P.n, I.Lr, I.Lc, 1.0, 1.0, tol=1e-10)
    finally:
        cp.set_apply_config(0, -1)
    X2, _ = cp.decode(I.Ytil, I.omega_r, I.omega_c, P.p, P.n, I.Lr, I.Lc, 1.0, 1.0, tol=1e-10)
    assert rel(host(X1), host(X2)) <= 1e-6


def _handle_with_env(env):
    """A new library handle on the current stream, created under `env`."""
    lib = _lib.load()
    hp = ctypes.c_void_p()
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        st = lib.cpca_create(ctypes.byref(hp),
                             ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream)))
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v
    assert st == 0
    return hp.value


@pytest.mark.parametrize("mode", ["fp64", "fp32_ir"])
def test_batched_tail_compaction_changes_nothing(batch, mode, capfd):
    # the block tables shrink to the running tasks as tasks converge; every
    # task keeps its own blocks and reduction order, so the outputs and
    # iteration counts must be bit-identical to a run with full tables
    print(f"[case] batched tail compaction {mode}", flush=True)
    dt = torch.float64 if mode == "fp64" else torch.float32
    inst = _instances(batch, dt)
    tasks = _tasks(batch)
    tol = 1e-13 if mode == "fp64" else 1e-10
    lib = _lib.load()
    h_on = _handle_with_env({"CPCA_DEBUG": "1"})
    h_off = _handle_with_env({"CPCA_BATCH_COMPACT": "0"})
    try:
        # leave FP32 data in the first handle's workspace: the padding
        # columns of the CG vectors must not carry it into the dot products
        # (the second handle's workspace is new)
        cp.solve_batched(_instances(batch, torch.float32), tasks, fista_iters=J, tol=1e-10,
                         mode="fp32_ir", h=h_on)
        torch.cuda.synchronize()
        capfd.readouterr()
        a, _, ia = cp.solve_batched(inst, tasks, fista_iters=J, tol=tol, mode=mode, h=h_on)
        torch.cuda.synchronize()
        log = capfd.readouterr().err
        b, _, ib = cp.solve_batched(inst, tasks, fista_iters=J, tol=tol, mode=mode, h=h_off)
        torch.cuda.synchronize()
    finally:
        lib.cpca_destroy(h_on)
        lib.cpca_destroy(h_off)
    n_comp = log.count("tables compacted")
    its = [i["iters"] for i in ia]
    print(f"[compaction] iterations {min(its)}..{max(its)}, {n_comp} compactions", flush=True)
    assert n_comp >= 1
    assert all(i["status"] == 0 for i in ia)
    assert [i["iters"] for i in ib] == its
    assert [i["outer_iters"] for i in ib] == [i["outer_iters"] for i in ia]
    assert all(torch.equal(x, y) for x, y in zip(a, b))


def test_batched_iteration_cap_reports_noconv(batch):
    inst = _instances(batch[:2], torch.float64)
    with pytest.warns(RuntimeWarning):
        Xs, _, infos = cp.solve_batched(inst, [(0, 1.0, 1.0), (1, 10.0, 10.0)], fista_iters=5,
                                        tol=1e-14, max_iter=3, mode="fp64")
    assert all(i["status"] == 2 and i["iters"] == 3 for i in infos)


@pytest.fixture(scope="module")
def anisotropic():
    # instance 5 of the batched workload (2077 x 287, helix rows, circle
    # columns): at gamma = (0.1, 100) the system is too ill-conditioned for a
    # plain FP32 CG recursion to keep its direction across residual
    # replacements; the solver must restart and still converge
    probs, _ = synth.cfg5_batch(0, count=6)
    return probs[5]


def test_fp32_ir_converges_on_anisotropic_gammas(anisotropic):
    P = anisotropic
    print(f"[case] anisotropic gammas {P.p}x{P.n}", flush=True)
    d = dev_problem(P, torch.float32)
    gam = (0.1, 100.0)
    X32, i32 = cp.decode(d["Ytil"], d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], *gam,
                         tol=1e-8, max_iter=50000, mode="fp32_ir")
    assert i32["status"] == 0 and i32["rel_residual"] <= 1e-8
    X64, i64 = cp.decode(d["Ytil"].double(), d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"],
                         *gam, tol=1e-12, max_iter=100000, mode="fp64")
    assert i64["status"] == 0
    e32 = rel(host(X32), host(X64))
    print(f"[anisotropic] fp32_ir {i32['iters']} it / {i32['outer_iters']} replacements, "
          f"fp64 {i64['iters']} it, rel.diff {e32:.2e}", flush=True)
    assert e32 <= 1e-5
    # the same task in a batch next to easy ones
    inst = [cp.Instance(P.p, P.n, d["om_r"], d["om_c"], d["Lr"], d["Lc"], d["Lr_til"],
                        d["Lc_til"], P.lmax_r_til, P.lmax_c_til, d["Ytil"])]
    tasks = [(0, 0.1, 100.0), (0, 1.0, 1.0), (0, 100.0, 0.1)]
    Xs, _, infos = cp.solve_batched(inst, tasks, fista_iters=20, tol=1e-8, max_iter=50000,
                                    mode="fp32_ir")
    assert all(i["status"] == 0 for i in infos)
    Xt1, _ = cp.frpcag(d["Ytil"], d["Lr_til"], d["Lc_til"], 0.1, 100.0, P.lmax_r_til,
                       P.lmax_c_til, max_iter=20)
    X1, _ = cp.decode(Xt1.double(), d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 0.1, 100.0,
                      tol=1e-12, max_iter=100000, mode="fp64")
    assert rel(host(Xs[0]), host(X1)) <= 1e-5
