"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Sizes are chosen so the oracle finishes in seconds while the GPU launches
still span several row blocks, several 64-column SELL slices and ragged
tails in both dimensions."""
import warnings

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import paper_1602_02070_amd as cp
from paper_1602_02070_amd import _lib
import synth
from oracle import decoder as OD
from oracle import frpcag as OF
from tests.gpu_util import dev_problem, host, rel

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def cfg1():
    return synth.cfg1_tiny(0)


def _rand_sym_csr(n, rng, deg_lo=0, deg_hi=30, empty_frac=0.1):
    """Random symmetric sparse matrix with skewed degrees and empty rows."""
    rows, cols = [], []
    for i in range(n):
        if rng.random() < empty_frac:
            continue
        d = int(min(n - 1, rng.integers(deg_lo, deg_hi) * (1 + 5 * (rng.random() < 0.05))))
        nb = rng.choice(n, size=d, replace=False)
        rows += [i] * d
        cols += list(nb)
    A = sp.coo_matrix((rng.standard_normal(len(rows)), (rows, cols)), shape=(n, n)).tocsr()
    A = (A + A.T).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


APPLY_SHAPES = [(1, 1), (7, 70), (63, 129), (130, 257), (300, 513), (1000, 64), (64, 1100)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", APPLY_SHAPES)
def test_apply_matches_oracle_random_graphs(shape, dtype):
    p, n = shape
    _announce(f"apply {p}x{n} {dtype}")
    rng = np.random.default_rng(p * 1000 + n)
    Lr = _rand_sym_csr(p, rng)
    Lc = _rand_sym_csr(n, rng)
    om_r = np.sort(rng.choice(p, size=max(1, p // 3), replace=False)).astype(np.int32)
    om_c = np.sort(rng.choice(n, size=max(1, n // 4), replace=False)).astype(np.int32)
    P = rng.standard_normal((p, n))
    gr, gc = 0.7, 1.9
    m_r, m_c = OD.masks(p, n, om_r, om_c)
    Q_ref = OD.apply_A(P, m_r, m_c, Lr, Lc, gr, gc)
    Pt = torch.from_numpy(P).to(dtype).cuda()
    Q, pq = cp.apply_operator(Pt, cp.Graph.from_scipy(Lr), cp.Graph.from_scipy(Lc), gr, gc,
                              torch.from_numpy(om_r).cuda(), torch.from_numpy(om_c).cuda())
    Qh = host(Q)
    scale = np.abs(Q_ref).max() + 1e-30
    tol = 1e-13 if dtype == torch.float64 else 3e-6
    assert np.abs(Qh - Q_ref).max() <= tol * scale * 10
    Ph = host(Pt)
    assert np.isclose(pq, np.sum(Ph * OD.apply_A(Ph, m_r, m_c, Lr, Lc, gr, gc)),
                      rtol=1e-12 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("n", [333, 600, 1100])
@pytest.mark.parametrize("R,lds,kernel", [(0, -1, "auto"), (0, -1, "strip"), (0, -1, "panel"),
                                          (0, -1, "panel_lo"), (0, -1, "rows"), (1, 1, "auto"), (2, 1, "auto"),
                                          (4, 1, "auto"), (8, 1, "auto"), (1, 0, "auto"),
                                          (4, 0, "auto")])
def test_apply_every_launch_shape(R, lds, kernel, n):
    # n = 333: scalar columns; 600 / 1100: 16-byte vectors, ragged; the circle
    # column graph is banded (plus wrap-around entries in the sliced-ELL
    # remainder). With the default shape (R = 0) the band goes to the kernel
    # named by `kernel` (auto: row panels) with a partial last strip and a
    # partial last panel group / row chunk; R = 1, 2, 4 with LDS take the
    # row kernel with the band in LDS
    _announce(f"apply launch shape R={R} lds={lds} kernel={kernel} n={n}")
    P_ = synth.small_problem(3, p_shape=(11, 13), n=n, rank=3, frac=0.3)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((P_.p, P_.n))
    m_r, m_c = OD.masks(P_.p, P_.n, P_.omega_r, P_.omega_c)
    ref = OD.apply_A(X, m_r, m_c, P_.Lr, P_.Lc, 1.3, 0.4)
    d = dev_problem(P_)
    cp.set_apply_config(R, lds, kernel)
    try:
        for dtype, tol in ((torch.float64, 1e-13), (torch.float32, 2e-6)):
            Q, _ = cp.apply_operator(torch.from_numpy(X).to(dtype).cuda(), d["Lr"], d["Lc"], 1.3,
                                     0.4, d["om_r"], d["om_c"])
            assert np.abs(host(Q) - ref).max() <= tol * np.abs(ref).max() * 10
    finally:
        cp.set_apply_config(0, -1)


@pytest.mark.parametrize("kernel", ["panel", "panel_lo", "strip", "rows"])
@pytest.mark.parametrize("shape,n,K", [((48, 61), 1024, 10), ((30, 37), 1000, 10),
                                       ((20, 25), 512, 20)])
def test_apply_banded_many_panels(kernel, shape, n, K):
    # A pixel-grid L_r (many panels: 48 x 61 = 2928 rows, panels of up to 64
    # rows) and a banded time-line L_c; the last case has about 25 entries per
    # L_r row, beyond the panel table, so "panel" falls back to column strips.
    # Both element types; FP64 against the oracle at rounding level.
    _announce(f"apply banded kernel={kernel} grid={shape} n={n} K={K}")
    import scipy.sparse as sps
    Lr, _ = synth.knn_laplacian(synth.grid_coords(*shape), K)
    Lc, _ = synth.knn_laplacian(np.arange(float(n))[:, None], 10)
    p = Lr.shape[0]
    rng = np.random.default_rng(11)
    om_r = np.sort(rng.choice(p, p // 7, replace=False)).astype(np.int32)
    om_c = np.sort(rng.choice(n, n // 9, replace=False)).astype(np.int32)
    X = rng.standard_normal((p, n))
    m_r, m_c = OD.masks(p, n, om_r, om_c)
    gr, gc = 0.8, 2.5
    ref = OD.apply_A(X, m_r, m_c, Lr, Lc, gr, gc)
    cp.set_apply_config(0, -1, kernel)
    try:
        for dtype, tol in ((torch.float64, 1e-13), (torch.float32, 2e-6)):
            Xt = torch.from_numpy(X).to(dtype).cuda()
            Q, pq = cp.apply_operator(Xt, cp.Graph.from_scipy(Lr), cp.Graph.from_scipy(Lc), gr,
                                      gc, torch.from_numpy(om_r).cuda(),
                                      torch.from_numpy(om_c).cuda())
            Xh = host(Xt)
            refd = OD.apply_A(Xh, m_r, m_c, Lr, Lc, gr, gc)
            assert np.abs(host(Q) - refd).max() <= tol * np.abs(refd).max() * 10
            assert np.isclose(pq, np.sum(Xh * refd), rtol=1e-12 if dtype == torch.float64 else 1e-5)
        assert sps.issparse(Lr)
    finally:
        cp.set_apply_config(0, -1)


@pytest.mark.parametrize("kernel", ["panel", "panel_lo"])
def test_apply_panels_on_unstructured_rows(kernel):
    # An irregular L_r (5-NN graph of 1500 random points in 3-D, plus 37
    # isolated rows and a two-row component) with a banded L_c of ragged
    # width: the panels grow along irregular neighbourhoods, so rows stay
    # resident in LDS in irregular slot patterns across each panel group
    _announce(f"apply panels on unstructured rows kernel={kernel}")
    rng = np.random.default_rng(23)
    Lg, _ = synth.knn_laplacian(rng.standard_normal((1500, 3)), 5)
    assert (np.diff(Lg.tocsr().indptr) - 1).max() <= 16  # panel tables apply
    pair = sp.csr_matrix(np.array([[1.0, -1.0], [-1.0, 1.0]]))
    Lr = sp.block_diag([Lg, sp.csr_matrix((37, 37)), pair], format="csr")
    n = 777
    Lc, _ = synth.knn_laplacian(np.arange(float(n))[:, None], 10)
    p = Lr.shape[0]
    om_r = np.sort(rng.choice(p, p // 5, replace=False)).astype(np.int32)
    om_c = np.sort(rng.choice(n, n // 6, replace=False)).astype(np.int32)
    m_r, m_c = OD.masks(p, n, om_r, om_c)
    gr, gc = 1.3, 0.7
    X = rng.standard_normal((p, n))
    cp.set_apply_config(0, -1, kernel)
    try:
        for dtype, tol in ((torch.float64, 1e-13), (torch.float32, 2e-6)):
            Xt = torch.from_numpy(X).to(dtype).cuda()
            Q, pq = cp.apply_operator(Xt, cp.Graph.from_scipy(Lr), cp.Graph.from_scipy(Lc), gr,
                                      gc, torch.from_numpy(om_r).cuda(),
                                      torch.from_numpy(om_c).cuda())
            Xh = host(Xt)
            refd = OD.apply_A(Xh, m_r, m_c, Lr, Lc, gr, gc)
            assert np.abs(host(Q) - refd).max() <= tol * np.abs(refd).max() * 10
            assert np.isclose(pq, np.sum(Xh * refd), rtol=1e-12 if dtype == torch.float64 else 1e-5)
    finally:
        cp.set_apply_config(0, -1)


def test_fista_trajectory_matches_oracle(cfg1):
    P = cfg1
    d = dev_problem(P)
    args = (P.Lr_til, P.Lc_til, P.gamma_r, P.gamma_c, P.lmax_r_til, P.lmax_c_til)
    rec = {j: None for j in (1, 2, 10, 100, 500)}
    OF.fista(P.Ytil, *args, 500, record=rec)
    for J in rec:
        _announce(f"fista cfg1 J={J}")
        X, info = cp.frpcag(d["Ytil"], d["Lr_til"], d["Lc_til"], P.gamma_r, P.gamma_c,
                            P.lmax_r_til, P.lmax_c_til, max_iter=J)
        assert info["iters"] == J
        assert rel(host(X), rec[J]) <= 1e-11
        assert np.isclose(info["objective"],
                          OF.objective(rec[J], P.Ytil, P.Lr_til, P.Lc_til, P.gamma_r, P.gamma_c),
                          rtol=1e-11)


@pytest.mark.parametrize("seed,shape,n,gam", [(1, (12, 10), 150, (1.0, 1.0)),
                                              (2, (9, 23), 333, (10.0, 0.1)),
                                              (3, (40, 30), 90, (0.5, 3.0))])
def test_fista_parity_small_problems(seed, shape, n, gam):
    P = synth.small_problem(seed, p_shape=shape, n=n, frac=0.5, gamma=gam, fista_iters=200)
    _announce(f"fista small seed={seed} {P.rho_r}x{P.rho_c}")
    d = dev_problem(P)
    ref, _ = OF.fista(P.Ytil, P.Lr_til, P.Lc_til, *gam, P.lmax_r_til, P.lmax_c_til, 200)
    X, _ = cp.frpcag(d["Ytil"], d["Lr_til"], d["Lc_til"], *gam, P.lmax_r_til, P.lmax_c_til, 200)
    assert rel(host(X), ref) <= 1e-11
    # FP32 input/output, FP64 state
    X32, _ = cp.frpcag(d["Ytil"].float(), d["Lr_til"], d["Lc_til"], *gam, P.lmax_r_til,
                       P.lmax_c_til, 200)
    ref32, _ = OF.fista(P.Ytil.astype(np.float32).astype(np.float64), P.Lr_til, P.Lc_til, *gam,
                        P.lmax_r_til, P.lmax_c_til, 200)
    assert rel(host(X32), ref32) <= 1e-6


def test_fista_eps_stopping_matches_oracle(cfg1):
    P = cfg1
    d = dev_problem(P)
    for eps in (1e-4, 1e-6):
        _announce(f"fista eps={eps}")
        ref, it = OF.fista(P.Ytil, P.Lr_til, P.Lc_til, 1.0, 1.0, P.lmax_r_til, P.lmax_c_til,
                           2000, eps=eps)
        X, info = cp.frpcag(d["Ytil"], d["Lr_til"], d["Lc_til"], 1.0, 1.0, P.lmax_r_til,
                            P.lmax_c_til, max_iter=2000, eps=eps)
        assert info["iters"] == it
        assert rel(host(X), ref) <= 1e-11


def test_fista_gamma_zero_returns_Y(cfg1):
    d = dev_problem(cfg1)
    X, info = cp.frpcag(d["Ytil"], d["Lr_til"], d["Lc_til"], 0.0, 0.0, 0.0, 0.0, max_iter=50)
    assert torch.equal(X, d["Ytil"]) and info["iters"] == 0


def _decode_ref(P, Xtil, gr, gc):
    return OD.decode(Xtil, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, gr, gc)


def test_decode_cfg1_all_modes(cfg1):
    P = cfg1
    d = dev_problem(P)
    Xtil, _ = OF.fista(P.Ytil, P.Lr_til, P.Lc_til, 1.0, 1.0, P.lmax_r_til, P.lmax_c_til, 500)
    ref = _decode_ref(P, Xtil, 1.0, 1.0)
    Xt = torch.from_numpy(Xtil).cuda()
    _announce("decode cfg1 fp64")
    X, info = cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0, tol=1e-12)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-11
    assert rel(host(X), ref) <= 1e-9
    _announce("decode cfg1 fp32_ir")
    X, info = cp.decode(Xt.float(), d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0,
                        tol=1e-10, mode="fp32_ir")
    assert info["status"] == 0 and info["rel_residual"] <= 1e-10
    ref32 = _decode_ref(P, Xtil.astype(np.float32).astype(np.float64), 1.0, 1.0)
    assert rel(host(X), ref32) <= 1e-5
    _announce("decode cfg1 fp32")
    X, info = cp.decode(Xt.float(), d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0,
                        tol=1e-5, mode="fp32")
    assert info["status"] == 0
    assert rel(host(X), ref32) <= 1e-3


@pytest.mark.parametrize("seed,shape,n,gam,frac", [
    (4, (12, 10), 150, (1.0, 1.0), 0.3),
    (5, (7, 19), 257, (10.0, 0.1), 0.2),
    (6, (33, 20), 65, (0.1, 10.0), 0.4),
    (7, (10, 10), 300, (100.0, 100.0), 0.25),
])
def test_decode_parity_small(seed, shape, n, gam, frac):
    P = synth.small_problem(seed, p_shape=shape, n=n, frac=frac, gamma=gam)
    _announce(f"decode small seed={seed} p={P.p} n={P.n} gamma={gam}")
    d = dev_problem(P)
    rng = np.random.default_rng(seed)
    Xtil = P.Ytil + 0.1 * rng.standard_normal(P.Ytil.shape)
    ref = _decode_ref(P, Xtil, *gam)
    Xt = torch.from_numpy(Xtil).cuda()
    X, info = cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], *gam, tol=1e-13)
    assert info["status"] == 0
    assert rel(host(X), ref) <= 1e-8
    X32, info = cp.decode(Xt.float(), d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], *gam,
                          tol=1e-11, mode="fp32_ir")
    assert info["status"] == 0
    ref32 = _decode_ref(P, Xtil.astype(np.float32).astype(np.float64), *gam)
    assert rel(host(X32), ref32) <= 1e-5


def test_decode_warm_start_and_zero_rhs(cfg1):
    P = cfg1
    d = dev_problem(P)
    rng = np.random.default_rng(1)
    Xtil = rng.standard_normal((P.rho_r, P.rho_c))
    ref = _decode_ref(P, Xtil, 1.0, 1.0)
    Xt = torch.from_numpy(Xtil).cuda()
    X0 = torch.from_numpy(ref + 1e-3 * rng.standard_normal(ref.shape)).cuda()
    _announce("decode warm start fp64")
    X, info = cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0,
                        tol=1e-12, X0=X0)
    assert rel(host(X), ref) <= 1e-9
    X, info2 = cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0, tol=1e-12)
    assert info["iters"] < info2["iters"]
    _announce("decode warm start fp32_ir")
    X, info = cp.decode(Xt.float(), d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0,
                        tol=1e-10, X0=X0.float())
    assert rel(host(X), ref) <= 1e-5
    _announce("decode zero rhs")
    for mode in ("fp64", "fp32", "fp32_ir"):
        dt = torch.float64 if mode == "fp64" else torch.float32
        X, info = cp.decode(torch.zeros_like(Xt, dtype=dt), d["om_r"], d["om_c"], P.p, P.n,
                            d["Lr"], d["Lc"], 1.0, 1.0, mode=mode)
        assert info["status"] == 0 and torch.count_nonzero(X) == 0


def test_decode_singular_gamma_zero_returns_scatter(cfg1):
    P = cfg1
    d = dev_problem(P)
    Xt = torch.from_numpy(P.Ytil).cuda()
    X, info = cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 0.0, 0.0)
    B = OD.rhs(P.Ytil, P.p, P.n, P.omega_r, P.omega_c)
    # one CG step: X = alpha B with alpha = <B,B>/<B,A B> = 1 up to summation order
    assert info["iters"] == 1 and rel(host(X), B) <= 1e-14


def test_decode_is_deterministic(cfg1):
    P = cfg1
    d = dev_problem(P)
    Xt = torch.from_numpy(P.Ytil).cuda()
    for mode in ("fp64", "fp32_ir"):
        dt = torch.float64 if mode == "fp64" else torch.float32
        a, _ = cp.decode(Xt.to(dt), d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0)
        b, _ = cp.decode(Xt.to(dt), d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0)
        assert torch.equal(a, b)


def test_backward_matches_oracle():
    P = synth.small_problem(18, p_shape=(6, 10), n=80, rank=3, frac=0.5, gamma=(1.0, 1.0))
    _announce("backward p=60 n=80")
    d = dev_problem(P)
    rng = np.random.default_rng(3)
    Xtil = rng.standard_normal((P.rho_r, P.rho_c))
    Xtrue = rng.standard_normal((P.p, P.n))
    X = _decode_ref(P, Xtil, 1.0, 1.0)
    G = 2 * (X - Xtrue)
    dX_ref, dgr_ref, dgc_ref = OD.decode_backward(G, X, P.p, P.n, P.omega_r, P.omega_c, P.Lr,
                                                  P.Lc, 1.0, 1.0)
    dX, dgr, dgc, info = cp.decode_backward(torch.from_numpy(G).cuda(), torch.from_numpy(X).cuda(),
                                            d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"],
                                            1.0, 1.0, tol=1e-13)
    assert rel(host(dX), dX_ref) <= 1e-9
    assert np.isclose(dgr, dgr_ref, rtol=1e-9) and np.isclose(dgc, dgc_ref, rtol=1e-9)
    dX, dgr, dgc, info = cp.decode_backward(torch.from_numpy(G).float().cuda(),
                                            torch.from_numpy(X).float().cuda(), d["om_r"],
                                            d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0,
                                            tol=1e-10, mode="fp32_ir")
    assert rel(host(dX), dX_ref) <= 1e-5
    assert np.isclose(dgr, dgr_ref, rtol=1e-5) and np.isclose(dgc, dgc_ref, rtol=1e-5)


def test_autograd_decode_matches_finite_differences():
    P = synth.small_problem(18, p_shape=(6, 10), n=80, rank=3, frac=0.5, gamma=(1.0, 1.0))
    _announce("autograd decode")
    d = dev_problem(P)
    rng = np.random.default_rng(4)
    Xtrue = torch.from_numpy(rng.standard_normal((P.p, P.n))).cuda()
    prob = cp.DecodeProblem(d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], tol=1e-13)
    Xt = torch.from_numpy(P.Ytil).cuda().requires_grad_(True)
    gr = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    gc = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = ((cp.Decode.apply(Xt, gr, gc, prob) - Xtrue) ** 2).sum()
    loss.backward()

    def L(Xtil, a, b):
        X = OD.decode(Xtil, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, a, b)
        return float(np.sum((X - host(Xtrue)) ** 2))

    h = 1e-4
    V = rng.standard_normal(P.Ytil.shape)
    fd = (L(P.Ytil + h * V, 1, 1) - L(P.Ytil - h * V, 1, 1)) / (2 * h)
    assert np.isclose(float((Xt.grad.double().cpu().numpy() * V).sum()), fd, rtol=1e-6)
    fd_r = (L(P.Ytil, 1 + h, 1) - L(P.Ytil, 1 - h, 1)) / (2 * h)
    fd_c = (L(P.Ytil, 1, 1 + h) - L(P.Ytil, 1, 1 - h)) / (2 * h)
    assert np.isclose(gr.grad.item(), fd_r, rtol=1e-6)
    assert np.isclose(gc.grad.item(), fd_c, rtol=1e-6)


def test_invalid_inputs_are_rejected_on_device(cfg1):
    P = cfg1
    d = dev_problem(P)
    Xt = torch.from_numpy(P.Ytil).cuda()
    dup = d["om_r"].clone()
    dup[1] = dup[0]
    with pytest.raises(cp.CpcaError, match="repeated"):
        cp.decode(Xt, dup, d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0)
    bad = cp.Graph(d["Lr"].rowptr, d["Lr"].colind.clone(), d["Lr"].vals, P.p)
    bad.colind[3] = P.p + 5
    with pytest.raises(cp.CpcaError, match="out of"):
        cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, bad, d["Lc"], 1.0, 1.0)
    with pytest.raises(cp.CpcaError, match="gamma"):
        cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], -1.0, 1.0)
    # iteration cap: ENOCONV returns the last iterate with a warning
    with pytest.warns(RuntimeWarning):
        X, info = cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0,
                            tol=1e-14, max_iter=3)
    assert info["status"] == 2 and info["iters"] == 3


def test_autotuned_pipeline_matches_oracle():
    # with autotuning on, the FISTA and CG products run in the shapes the
    # tuner picks on the live operands; results stay at parity
    P = synth.small_problem(21, p_shape=(20, 24), n=400, rank=4, frac=0.3, fista_iters=150,
                            col_kind="band")
    _announce(f"autotuned pipeline {P.p}x{P.n}")
    d = dev_problem(P)
    ref_t, _ = OF.fista(P.Ytil, P.Lr_til, P.Lc_til, P.gamma_r, P.gamma_c, P.lmax_r_til,
                        P.lmax_c_til, 150)
    ref = OD.decode(ref_t, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c)
    cp.set_apply_config(-1, -1)
    try:
        for _ in range(2):  # the second call takes the cached choices
            Xt, _ = cp.frpcag(d["Ytil"], d["Lr_til"], d["Lc_til"], P.gamma_r, P.gamma_c,
                              P.lmax_r_til, P.lmax_c_til, max_iter=150)
            assert rel(host(Xt), ref_t) <= 1e-11
            X, info = cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], P.gamma_r,
                                P.gamma_c, tol=1e-12, mode="fp64")
            assert info["status"] == 0 and rel(host(X), ref) <= 1e-9
            X32, _ = cp.decode(Xt.float(), d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"],
                               P.gamma_r, P.gamma_c, tol=1e-9)
            assert rel(host(X32), ref) <= 1e-6
    finally:
        cp.set_apply_config(0, -1)


def _decode_both(Xtil, om_r, om_c, p, n, Lr, Lc, gr, gc):
    """GPU decode in FP64 and FP32_IR with the default launch shapes."""
    Lrg, Lcg = cp.Graph.from_scipy(Lr), cp.Graph.from_scipy(Lc)
    r = torch.from_numpy(om_r).cuda()
    c = torch.from_numpy(om_c).cuda()
    X64, i64 = cp.decode(torch.from_numpy(Xtil).cuda(), r, c, p, n, Lrg, Lcg, gr, gc, tol=1e-13,
                         mode="fp64")
    X32, i32 = cp.decode(torch.from_numpy(Xtil).float().cuda(), r, c, p, n, Lrg, Lcg, gr, gc,
                         tol=1e-9)
    return host(X64), i64, host(X32), i32


@pytest.mark.parametrize("single", ["row", "column"])
def test_decode_single_row_or_column(single):
    # one node on one side: its Laplacian is the empty 1 x 1 matrix
    import scipy.sparse as sps
    _announce(f"degenerate single {single}")
    rng = np.random.default_rng(31)
    L1 = sps.csr_matrix((1, 1))
    Lother, _ = synth.knn_laplacian(synth.circle_coords(300, rng, noise_std=0.05), 10)
    if single == "row":
        p, n, Lr, Lc = 1, 300, L1, Lother
        om_r = np.array([0], np.int32)
        om_c = np.sort(rng.choice(n, 60, replace=False)).astype(np.int32)
    else:
        p, n, Lr, Lc = 300, 1, Lother, L1
        om_r = np.sort(rng.choice(p, 60, replace=False)).astype(np.int32)
        om_c = np.array([0], np.int32)
    Xtil = rng.standard_normal((len(om_r), len(om_c)))
    ref = OD.decode(Xtil, p, n, om_r, om_c, Lr, Lc, 0.7, 1.3)
    X64, i64, X32, i32 = _decode_both(Xtil, om_r, om_c, p, n, Lr, Lc, 0.7, 1.3)
    assert i64["status"] == 0 and i32["status"] == 0
    assert rel(X64, ref) <= 1e-10
    assert rel(X32, ref) <= 1e-6


def test_decode_with_isolated_nodes_in_both_graphs():
    # rows / columns of degree 0 (empty CSR rows): the panel tables hold no
    # entries for them; sampled isolated rows keep the system definite
    import scipy.sparse as sps
    _announce("degenerate isolated nodes")
    rng = np.random.default_rng(32)
    Lg, _ = synth.knn_laplacian(synth.grid_coords(12, 14), 10)
    Lr = sps.block_diag([Lg, sps.csr_matrix((5, 5))], format="csr")
    Lb, _ = synth.knn_laplacian(np.arange(596.0)[:, None], 10)
    Lc = sps.block_diag([Lb, sps.csr_matrix((4, 4))], format="csr")
    p, n = Lr.shape[0], Lc.shape[0]
    om_r = np.sort(np.concatenate([rng.choice(168, 40, replace=False),
                                   np.arange(168, 173)])).astype(np.int32)
    om_c = np.sort(np.concatenate([rng.choice(596, 90, replace=False),
                                   np.arange(596, 600)])).astype(np.int32)
    Xtil = rng.standard_normal((len(om_r), len(om_c)))
    ref = OD.decode(Xtil, p, n, om_r, om_c, Lr, Lc, 1.1, 0.6, method="cg", tol=1e-13)
    for kernel in ("panel", "panel_lo", "strip", "rows"):
        cp.set_apply_config(0, -1, kernel)
        try:
            X64, i64, X32, i32 = _decode_both(Xtil, om_r, om_c, p, n, Lr, Lc, 1.1, 0.6)
        finally:
            cp.set_apply_config(0, -1)
        assert i64["status"] == 0 and i32["status"] == 0, kernel
        assert rel(X64, ref) <= 1e-9, kernel
        assert rel(X32, ref) <= 1e-6, kernel


def test_full_sampling_without_regularisation_returns_samples():
    # every entry sampled and gamma = 0: the system is the identity, X = X~
    _announce("degenerate full sampling gamma 0")
    P = synth.small_problem(33, p_shape=(9, 12), n=200, frac=1.0)
    rng = np.random.default_rng(33)
    Xtil = rng.standard_normal((P.p, P.n))
    om_r = np.arange(P.p, dtype=np.int32)
    om_c = np.arange(P.n, dtype=np.int32)
    X64, i64, X32, i32 = _decode_both(Xtil, om_r, om_c, P.p, P.n, P.Lr, P.Lc, 0.0, 0.0)
    assert i64["status"] == 0 and i64["iters"] <= 1
    assert np.array_equal(X64, Xtil)
    assert rel(X32, Xtil) <= 1e-7


def test_cfg4_fp32_gradient_at_config1_shapes():
    # differentiation workload at the tiny shapes (p = 100, n = 200, 50 x 100
    # samples): loss ||decode(Y~) - X_true||_F^2 with the gradient for Y~ in
    # FP32 and for both gammas in FP64, through the autograd Function, against
    # the oracle's adjoint and central finite differences (h = 1e-4) of the
    # oracle's loss; and the FP32 adjoint at p = 60, n = 80 against the dense
    # Kronecker gradient
    P = synth.cfg1_tiny(0)
    _announce("cfg4 fp32 gradient 100x200")
    d = dev_problem(P, torch.float32)
    Xtrue = P.X_true
    prob = cp.DecodeProblem(d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], tol=1e-10,
                            mode="fp32_ir")
    Y = d["Ytil"].clone().requires_grad_(True)
    gr = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    gc = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    X = cp.Decode.apply(Y, gr, gc, prob)
    assert X.dtype == torch.float32
    loss = ((X.double() - torch.from_numpy(Xtrue).cuda()) ** 2).sum()
    loss.backward()
    assert Y.grad.dtype == torch.float32

    Yr = P.Ytil.astype(np.float32).astype(np.float64)
    X_ref = OD.decode(Yr, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, 1.0, 1.0)
    dY_ref, dgr_ref, dgc_ref = OD.decode_backward(2 * (X_ref - Xtrue), X_ref, P.p, P.n,
                                                  P.omega_r, P.omega_c, P.Lr, P.Lc, 1.0, 1.0)
    e = rel(host(Y.grad), dY_ref)
    print(f"[cfg4] dY~ rel.err {e:.2e}, dgr {gr.grad.item():.8e} vs {dgr_ref:.8e}, "
          f"dgc {gc.grad.item():.8e} vs {dgc_ref:.8e}", flush=True)
    assert e <= 1e-5
    assert np.isclose(gr.grad.item(), dgr_ref, rtol=1e-5)
    assert np.isclose(gc.grad.item(), dgc_ref, rtol=1e-5)

    def L(Yt, a, b):
        Xd = OD.decode(Yt, P.p, P.n, P.omega_r, P.omega_c, P.Lr, P.Lc, a, b)
        return float(np.sum((Xd - Xtrue) ** 2))

    h = 1e-4
    rng = np.random.default_rng(9)
    for _ in range(3):
        V = rng.standard_normal(P.Ytil.shape)
        fd = (L(Yr + h * V, 1, 1) - L(Yr - h * V, 1, 1)) / (2 * h)
        assert np.isclose(float((host(Y.grad) * V).sum()), fd, rtol=1e-5)
    fd_r = (L(Yr, 1 + h, 1) - L(Yr, 1 - h, 1)) / (2 * h)
    fd_c = (L(Yr, 1, 1 + h) - L(Yr, 1, 1 - h)) / (2 * h)
    assert np.isclose(gr.grad.item(), fd_r, rtol=1e-5)
    assert np.isclose(gc.grad.item(), fd_c, rtol=1e-5)

    # dense Kronecker adjoint at p = 60, n = 80, FP32 tensors
    P2 = synth.small_problem(18, p_shape=(6, 10), n=80, rank=3, frac=0.5, gamma=(1.0, 1.0))
    d2 = dev_problem(P2, torch.float32)
    rng = np.random.default_rng(10)
    Xt2 = rng.standard_normal((P2.rho_r, P2.rho_c)).astype(np.float32).astype(np.float64)
    X2 = OD.decode(Xt2, P2.p, P2.n, P2.omega_r, P2.omega_c, P2.Lr, P2.Lc, 1.0, 1.0,
                   method="dense")
    G2 = 2 * (X2 - rng.standard_normal((P2.p, P2.n)))
    ref2 = OD.decode_backward(G2, X2, P2.p, P2.n, P2.omega_r, P2.omega_c, P2.Lr, P2.Lc, 1.0, 1.0,
                              method="dense")
    dX, dgr, dgc, _ = cp.decode_backward(torch.from_numpy(G2).float().cuda(),
                                         torch.from_numpy(X2).float().cuda(), d2["om_r"],
                                         d2["om_c"], P2.p, P2.n, d2["Lr"], d2["Lc"], 1.0, 1.0,
                                         tol=1e-10, mode="fp32_ir")
    assert rel(host(dX), ref2[0]) <= 1e-5
    assert np.isclose(dgr, ref2[1], rtol=1e-5) and np.isclose(dgc, ref2[2], rtol=1e-5)


# ------------------------------------------------------------------ norm estimate, error paths

def _graph(L):
    return cp.Graph.from_scipy(sp.csr_matrix(L))


def test_laplacian_lmax_matches_dense_spectrum():
    # device power iteration (outside the parity contract) against the dense
    # spectrum: normalised and combinatorial Laplacians, a sampled video-size
    # pixel graph, a path graph (clustered top of the spectrum)
    _announce("laplacian lmax")
    P1 = synth.cfg1_tiny(0)
    Pc = synth.small_problem(12, p_shape=(9, 11), n=120, kind="combinatorial")
    rng = np.random.default_rng(2)
    Lv, _ = synth.knn_laplacian(synth.grid_coords(128, 160)[np.sort(rng.choice(20480, 1024, replace=False))], 10)
    m = 300
    W = sp.diags([np.ones(m - 1), np.ones(m - 1)], [-1, 1])
    Lpath = sp.diags(np.asarray(W.sum(axis=1)).ravel()) - W
    for name, L in [("cfg1 rows", P1.Lr_til), ("cfg1 cols", P1.Lc_til), ("comb rows", Pc.Lr),
                    ("comb cols", Pc.Lc), ("video sampled rows", Lv), ("path", Lpath)]:
        ref = np.linalg.eigvalsh(sp.csr_matrix(L).toarray())[-1]
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", RuntimeWarning)
            lm, info = cp.laplacian_lmax(_graph(L))
        print(f"[lmax] {name}: {lm:.12f} vs {ref:.12f} ({info['iters']} products, "
              f"status {info['status']})", flush=True)
        if info["status"] == 0:
            assert abs(lm - ref) <= 1e-8 * ref, name
        assert lm <= ref * (1 + 1e-12)
        assert abs(lm - ref) <= 1e-4 * ref, name


def test_frpcag_with_estimated_norms_stays_at_parity(cfg1):
    # lmax <= 0 asks the library for the norms; 500 FISTA iterations with the
    # estimates stay close to the run with the exact values and to the oracle
    P = cfg1
    _announce("frpcag estimated lmax")
    d = dev_problem(P)
    exact, _ = cp.frpcag(d["Ytil"], d["Lr_til"], d["Lc_til"], 1.0, 1.0, P.lmax_r_til,
                         P.lmax_c_til, max_iter=500)
    est, info = cp.frpcag(d["Ytil"], d["Lr_til"], d["Lc_til"], 1.0, 1.0, 0.0, -1.0, max_iter=500)
    ref, _ = OF.fista(P.Ytil, P.Lr_til, P.Lc_til, 1.0, 1.0, P.lmax_r_til, P.lmax_c_til, 500)
    e1, e2 = rel(host(est), host(exact)), rel(host(est), ref)
    print(f"[lmax] FISTA with estimated norms: rel.diff {e1:.2e} vs exact-norm run, "
          f"{e2:.2e} vs oracle", flush=True)
    assert info["status"] == 0 and e1 <= 1e-6 and e2 <= 1e-6
    # gamma = 0 on one side: that norm is not needed and not estimated
    a, _ = cp.frpcag(d["Ytil"], d["Lr_til"], d["Lc_til"], 0.0, 1.0, 0.0, P.lmax_c_til, 50)
    b, _ = OF.fista(P.Ytil, P.Lr_til, P.Lc_til, 0.0, 1.0, 0.0, P.lmax_c_til, 50)
    assert rel(host(a), b) <= 1e-12


@pytest.mark.parametrize("mode", ["fp64", "fp32", "fp32_ir"])
def test_indefinite_operator_reports_enotspd(cfg1, mode):
    # L_r = -5 I makes <B, A B> < 0 at the first CG step: the breakdown is
    # reported as CPCA_ENOTSPD, every kernel returns, and the handle works on
    P = cfg1
    _announce(f"enotspd {mode}")
    d = dev_problem(P)
    dt = torch.float64 if mode == "fp64" else torch.float32
    neg = _graph(-5.0 * sp.identity(P.p))
    Xt = torch.from_numpy(P.Ytil).to(dt).cuda()
    with pytest.raises(cp.CpcaError) as e:
        cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, neg, d["Lc"], 1.0, 1.0, mode=mode)
    assert e.value.status == _lib.ENOTSPD, str(e.value)
    X, info = cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0,
                        tol=1e-10, mode=mode)
    ref = _decode_ref(P, P.Ytil.astype(np.float32).astype(np.float64) if mode != "fp64"
                      else P.Ytil, 1.0, 1.0)
    assert info["status"] == 0 and rel(host(X), ref) <= (1e-9 if mode == "fp64" else 1e-5)


@pytest.mark.parametrize("mode", ["fp64", "fp32", "fp32_ir"])
def test_nan_input_reports_enan(cfg1, mode):
    # a NaN in X~ (decoder) or in Y~ (FISTA) ends the iteration with CPCA_ENAN
    P = cfg1
    _announce(f"enan {mode}")
    d = dev_problem(P)
    dt = torch.float64 if mode == "fp64" else torch.float32
    Xt = torch.from_numpy(P.Ytil).to(dt).cuda()
    Xt[3, 7] = float("nan")
    with pytest.raises(cp.CpcaError) as e:
        cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0, mode=mode)
    assert e.value.status == _lib.ENAN, str(e.value)
    Xt[3, 7] = float("inf")
    with pytest.raises(cp.CpcaError) as e:
        cp.frpcag(Xt, d["Lr_til"], d["Lc_til"], 1.0, 1.0, P.lmax_r_til, P.lmax_c_til, 20,
                  mode=mode)
    assert e.value.status == _lib.ENAN, str(e.value)
    X, info = cp.decode(torch.from_numpy(P.Ytil).to(dt).cuda(), d["om_r"], d["om_c"], P.p, P.n,
                        d["Lr"], d["Lc"], 1.0, 1.0, tol=1e-10, mode=mode)
    assert info["status"] == 0


# ------------------------------------------------------------------ operator-image cache

def _debug_handle():
    import ctypes
    import os
    lib = _lib.load()
    hp = ctypes.c_void_p()
    old = os.environ.get("CPCA_DEBUG")
    os.environ["CPCA_DEBUG"] = "1"
    try:
        st = lib.cpca_create(ctypes.byref(hp),
                             ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream)))
    finally:
        if old is None:
            del os.environ["CPCA_DEBUG"]
        else:
            os.environ["CPCA_DEBUG"] = old
    assert st == 0
    return hp.value


@pytest.mark.parametrize("mode", ["fp64", "fp32_ir"])
def test_operator_image_cache_reuse_and_invalidation(mode, capfd):
    # a second decode on the same operator reuses the staged image and gives
    # the same bits; changing one value of L_r in place (same pointers), or
    # one sampled index, is seen by the content key and restages the image
    P = synth.small_problem(23, p_shape=(16, 20), n=300, rank=3, frac=0.3, col_kind="band")
    _announce(f"image cache {mode}")
    d = dev_problem(P)
    dt = torch.float64 if mode == "fp64" else torch.float32
    Xt = torch.from_numpy(P.Ytil).to(dt).cuda()
    h = _debug_handle()
    tol = 1e-12 if mode == "fp64" else 1e-10
    bar = 1e-9 if mode == "fp64" else 1e-5
    Xr = P.Ytil if mode == "fp64" else P.Ytil.astype(np.float32).astype(np.float64)
    try:
        capfd.readouterr()
        X1, _ = cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0, tol=tol,
                          mode=mode, h=h)
        X2, _ = cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0, tol=tol,
                          mode=mode, h=h)
        torch.cuda.synchronize()
        log = capfd.readouterr().err
        assert log.count("operator image staged") == 1 and log.count("operator image reused") == 1
        assert torch.equal(X1, X2)
        # values of L_r changed in place (same pointers): a PSD rank-one
        # increment on one edge, 0.05 (e_i + e_j)(e_i + e_j)^T
        Lr2 = P.Lr.copy().tolil()
        i, j = 5, int(P.Lr[5].indices[-1])
        assert i != j
        for a, b in ((i, i), (j, j), (i, j), (j, i)):
            Lr2[a, b] = P.Lr[a, b] + 0.05
        Lr2 = Lr2.tocsr()
        Lr2.sort_indices()
        assert np.array_equal(Lr2.indices, P.Lr.indices)
        d["Lr"].vals.copy_(torch.from_numpy(Lr2.data))
        X3, i3 = cp.decode(Xt, d["om_r"], d["om_c"], P.p, P.n, d["Lr"], d["Lc"], 1.0, 1.0,
                           tol=tol, mode=mode, h=h)
        torch.cuda.synchronize()
        log = capfd.readouterr().err
        assert "operator image staged" in log and "reused" not in log
        ref3 = OD.decode(Xr, P.p, P.n, P.omega_r, P.omega_c, Lr2, P.Lc, 1.0, 1.0)
        assert i3["status"] == 0 and rel(host(X3), ref3) <= bar
        # one sampled column index changed: restaged, and the new operator used
        om_c2 = P.omega_c.copy()
        free = np.setdiff1d(np.arange(P.n), om_c2)
        om_c2[-1] = free[-1]
        order = np.argsort(om_c2)
        om_c2 = om_c2[order]
        Xt2 = Xt[:, torch.from_numpy(order).cuda()].contiguous()
        X4, i4 = cp.decode(Xt2, d["om_r"], torch.from_numpy(om_c2).cuda(), P.p, P.n, d["Lr"],
                           d["Lc"], 1.0, 1.0, tol=tol, mode=mode, h=h)
        torch.cuda.synchronize()
        log = capfd.readouterr().err
        assert "operator image staged" in log
        ref4 = OD.decode(Xr[:, order], P.p, P.n, P.omega_r, om_c2, Lr2, P.Lc, 1.0, 1.0)
        assert i4["status"] == 0 and rel(host(X4), ref4) <= bar
    finally:
        _lib.load().cpca_destroy(h)
