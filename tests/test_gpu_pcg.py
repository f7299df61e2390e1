"""The decoder's two-level preconditioned CG (aggregation coarse space,
pcg.hpp; forced on at every size here with CPCA_PRECOND=1) against the FP64
oracle and against plain CG (CPCA_PRECOND=0).

Both reach the unique solution of the decoder's normal equations, so both are
held to the oracle at the same tolerance; the preconditioned solve must need
fewer iterations where the graphs are large enough for the coarse level to
matter."""
import contextlib
import os

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import paper_1602_02070_amd as cp
import synth
from oracle import decoder as OD
from tests.gpu_util import dev_problem, host, rel

pytestmark = pytest.mark.gpu


@contextlib.contextmanager
def precond(value):
    old = os.environ.get("CPCA_PRECOND")
    os.environ["CPCA_PRECOND"] = value
    try:
        yield
    finally:
        if old is None:
            del os.environ["CPCA_PRECOND"]
        else:
            os.environ["CPCA_PRECOND"] = old


def plain_cg():
    return precond("0")


@pytest.fixture(autouse=True)
def preconditioned_at_every_size():
    # these problems are smaller than the default threshold of the coarse
    # level (2^20 entries): force it on, plain CG is asked for explicitly
    with precond("1"):
        yield


def _solve(P, d, Xtil, gam, mode, tol):
    dt = torch.float64 if mode == "fp64" else torch.float32
    Xt = torch.from_numpy(Xtil).to(dt).cuda()
    return cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], *gam, tol=tol,
                     mode=mode)


@pytest.mark.parametrize("seed,shape,n,gam,frac,col_kind", [
    (11, (12, 10), 150, (1.0, 1.0), 0.3, "circle"),     # 120 rows: a few aggregates, 3 column ranges
    (12, (7, 19), 257, (10.0, 0.1), 0.2, "band"),       # n not a multiple of 4 or of 64
    (13, (33, 20), 65, (0.1, 10.0), 0.4, "circle"),     # two column ranges, the second of one column
    (14, (6, 6), 40, (1.0, 1.0), 0.5, "band"),          # 36 rows: two aggregates, one column range
    (15, (40, 41), 512, (1.0, 1.0), 0.05, "band"),      # video-like sampling
])
def test_pcg_matches_oracle_and_plain_cg(seed, shape, n, gam, frac, col_kind):
    P = synth.small_problem(seed, p_shape=shape, n=n, frac=frac, gamma=gam, col_kind=col_kind)
    print(f"[case] pcg seed={seed} p={P.p} n={P.n} gamma={gam}", flush=True)
    d = dev_problem(P)
    rng = np.random.default_rng(seed)
    Xtil = P.Ytil + 0.1 * rng.standard_normal(P.Ytil.shape)
    ref = OD.decode(Xtil, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, *gam)
    X, info = _solve(P, d, Xtil, gam, "fp64", 1e-13)
    assert info["status"] == 0
    assert rel(host(X), ref) <= 1e-8
    with plain_cg():
        Xp, infop = _solve(P, d, Xtil, gam, "fp64", 1e-13)
    assert infop["status"] == 0
    assert rel(host(Xp), ref) <= 1e-8
    assert rel(host(X), host(Xp)) <= 1e-8
    ref32 = OD.decode(Xtil.astype(np.float32).astype(np.float64), P.p, P.n, P.omega_r,
                      P.omega_c, P.Lr, P.Lc, *gam)
    for mode in ("fp32", "fp32_ir"):
        X32, info32 = _solve(P, d, Xtil, gam, mode, 1e-5 if mode == "fp32" else 1e-11)
        assert info32["status"] == 0, mode
        assert rel(host(X32), ref32) <= (1e-3 if mode == "fp32" else 1e-5), mode
    if P.p * P.n >= 20000:
        assert info["iters"] < infop["iters"], (info["iters"], infop["iters"])


def test_pcg_cuts_iterations_on_a_banded_problem():
    # a 48 x 61 pixel grid and a 1024-frame time line at 5 % sampling: the
    # coarse level must at least halve the iteration count
    P = synth.small_problem(21, p_shape=(48, 61), n=1024, frac=0.05, gamma=(1.0, 1.0),
                            col_kind="band")
    print("[case] pcg banded 2928 x 1024", flush=True)
    d = dev_problem(P)
    Xtil = P.Ytil
    ref = OD.decode(Xtil, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, 1.0, 1.0)
    X, info = _solve(P, d, Xtil, (1.0, 1.0), "fp64", 1e-12)
    with plain_cg():
        Xp, infop = _solve(P, d, Xtil, (1.0, 1.0), "fp64", 1e-12)
    print(f"[pcg] iterations {info['iters']} preconditioned, {infop['iters']} plain", flush=True)
    assert rel(host(X), ref) <= 1e-9 and rel(host(Xp), ref) <= 1e-9
    assert 2 * info["iters"] <= infop["iters"]


def test_pcg_gamma_zero_on_one_side_falls_back_to_plain_cg():
    # gamma_r = 0: the coarse operator is not built (plain CG); the result is
    # still the oracle's
    P = synth.small_problem(22, p_shape=(12, 10), n=150, frac=0.3, gamma=(0.0, 1.0))
    print("[case] pcg gamma_r = 0", flush=True)
    d = dev_problem(P)
    ref = OD.decode(P.Ytil, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, 0.0, 1.0)
    X, info = _solve(P, d, P.Ytil, (0.0, 1.0), "fp64", 1e-13)
    with plain_cg():
        Xp, infop = _solve(P, d, P.Ytil, (0.0, 1.0), "fp64", 1e-13)
    assert info["status"] == 0 and rel(host(X), ref) <= 1e-8
    assert info["iters"] == infop["iters"] and torch.equal(X, Xp)


def _isolate(L, i):
    """The Laplacian L with node i cut off (its edges removed, the degrees
    of its neighbours lowered): row and column i become zero."""
    L = sp.lil_matrix(L)
    for j in list(L.rows[i]):
        if j != i:
            L[j, j] = L[j, j] + L[i, j]
            L[j, i] = 0.0
            L[i, j] = 0.0
    L[i, i] = 0.0
    L = sp.csr_matrix(L)
    L.eliminate_zeros()
    return L


@pytest.mark.parametrize("sampled", [True, False])
def test_pcg_combinatorial_laplacians_with_isolated_nodes(sampled):
    # an isolated row node and an isolated column node (zero Laplacian rows).
    # Sampled: the operator stays definite and the coarse level is used.
    # Unsampled: a component without samples makes the operator singular;
    # the coarse level is dropped and plain CG from zero gives the
    # minimum-norm solution, as the oracle's CG does.
    P = synth.small_problem(23, p_shape=(9, 11), n=120, frac=0.3, gamma=(1.0, 1.0),
                            kind="combinatorial")
    om_r, om_c = P.omega_r, P.omega_c
    if sampled:
        i, j0 = int(om_r[3]), int(om_c[2])
    else:
        i = int(np.setdiff1d(np.arange(P.p), om_r)[3])
        j0 = int(np.setdiff1d(np.arange(P.n), om_c)[2])
    Lr, Lc = _isolate(P.Lr, i), _isolate(P.Lc, j0)
    print(f"[case] pcg isolated nodes, sampled={sampled}", flush=True)
    Gr, Gc = cp.Graph.from_scipy(Lr), cp.Graph.from_scipy(Lc)
    ref = OD.decode(P.Ytil, P.p, P.n, om_r, om_c, Lr, Lc, 1.0, 1.0, method="cg", tol=1e-14)
    Xt = torch.from_numpy(P.Ytil).cuda()
    tr, tc = torch.from_numpy(om_r).cuda(), torch.from_numpy(om_c).cuda()
    X, info = cp.decode(Xt, tr, tc, P.p, P.n, Gr, Gc, 1.0, 1.0, tol=1e-13)
    assert info["status"] == 0
    assert rel(host(X), ref) <= 1e-8
    if not sampled:
        with plain_cg():
            Xp, infop = cp.decode(Xt, tr, tc, P.p, P.n, Gr, Gc, 1.0, 1.0, tol=1e-13)
        assert info["iters"] == infop["iters"] and torch.equal(X, Xp)


def test_pcg_repeated_decodes_reuse_the_coarse_inverse_and_follow_gamma():
    # the same operator with new gammas rebuilds the coarse inverse; going
    # back to the first gammas gives bit-identical results
    P = synth.small_problem(24, p_shape=(12, 12), n=150, frac=0.3, gamma=(1.0, 1.0),
                            col_kind="band")
    print("[case] pcg gamma changes", flush=True)
    d = dev_problem(P)
    outs = []
    for gam in [(1.0, 1.0), (10.0, 0.5), (1.0, 1.0)]:
        ref = OD.decode(P.Ytil, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, *gam)
        X, info = _solve(P, d, P.Ytil, gam, "fp64", 1e-13)
        assert info["status"] == 0 and rel(host(X), ref) <= 1e-8, gam
        outs.append(X)
    assert torch.equal(outs[0], outs[2])
