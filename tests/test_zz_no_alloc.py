"""The no-allocation product (cpca_apply_noalloc) against cpca_apply, both
called through the C ABI: the same kernels on a static scratch array instead
of the handle's workspace must give the same result, on consecutive calls
whose second input is smaller, with no change of the device's free memory."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import paper_1602_02070_amd as cp
from paper_1602_02070_amd import _lib
import synth

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _call(fn, h, mode, P, Q, om_r, om_c, Lr, Lc, gr, gc):
    pq = ctypes.c_double()
    p, n = P.shape
    st = fn(h, _lib.MODES[mode], _ptr(P), _ptr(Q), p, n, _ptr(om_r), om_r.numel(), _ptr(om_c),
            om_c.numel(), ctypes.byref(Lr.desc), ctypes.byref(Lc.desc), gr, gc, ctypes.byref(pq))
    return st, pq.value


def _case(P, mode, seed):
    dt = torch.float64 if mode == "fp64" else torch.float32
    rng = np.random.default_rng(seed)
    X = torch.from_numpy(rng.standard_normal((P.p, P.n))).to(dt).cuda()
    return (X, cp.Graph.from_scipy(P.Lr), cp.Graph.from_scipy(P.Lc),
            torch.from_numpy(P.omega_r).cuda(), torch.from_numpy(P.omega_c).cuda())


@pytest.mark.parametrize("mode", ["fp32", "fp64"])
def test_noalloc_apply_matches_apply_on_consecutive_calls(mode):
    print(f"[case] apply_noalloc {mode}", flush=True)
    lib = _lib.load()
    h = cp.handle()
    # a banded column graph (row-panel kernel) spanning several panels and
    # strips, then a smaller problem on a circle graph (row kernel)
    big = synth.small_problem(31, p_shape=(48, 61), n=1100, col_kind="band")
    small = synth.small_problem(32, p_shape=(9, 13), n=77)
    warm = _case(small, mode, 0)
    Qw = torch.empty_like(warm[0])
    assert _call(lib.cpca_apply_noalloc, h, mode, warm[0], Qw, warm[3], warm[4], warm[1],
                 warm[2], 1.0, 1.0)[0] == _lib.OK
    torch.cuda.synchronize()
    for k, (P, gr, gc) in enumerate([(big, 0.7, 1.3), (small, 2.0, 0.5)]):
        X, Lr, Lc, om_r, om_c = _case(P, mode, 10 + k)
        Q_ref = torch.full_like(X, float("nan"))
        Q = torch.full_like(X, float("nan"))
        st, pq_ref = _call(lib.cpca_apply, h, mode, X, Q_ref, om_r, om_c, Lr, Lc, gr, gc)
        assert st == _lib.OK, _lib.last_error()
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        st, pq = _call(lib.cpca_apply_noalloc, h, mode, X, Q, om_r, om_c, Lr, Lc, gr, gc)
        assert st == _lib.OK, _lib.last_error()
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        print(f"[noalloc] {mode} {P.p}x{P.n}: <P,Q> {pq:.15e} vs {pq_ref:.15e}, free memory "
              f"{free0} -> {free1}", flush=True)
        assert free1 == free0
        assert torch.equal(Q, Q_ref)
        assert pq == pq_ref


def test_noalloc_apply_rejects_an_operator_beyond_the_scratch():
    # a random symmetric L_r of about 3.6 M non-zeros needs about 44 MB as FP64
    # CSR, beyond the 32 MiB scratch; the column graph links only columns 20
    # apart (no band, so no row-panel tables are built)
    print("[case] apply_noalloc size limit", flush=True)
    lib = _lib.load()
    h = cp.handle()
    p, n = 300000, 40
    rng = np.random.default_rng(3)
    A = sp.random(p, p, density=6.0 / p, random_state=rng, format="csr")
    Lr = cp.Graph.from_scipy((A + A.T).tocsr())
    j = np.arange(20)
    W = sp.csr_matrix((np.ones(40), (np.r_[j, j + 20], np.r_[j + 20, j])), shape=(n, n))
    Lc = cp.Graph.from_scipy(sp.identity(n, format="csr") - 0.5 * W)
    X = torch.zeros((p, n), dtype=torch.float64, device="cuda")
    Q = torch.zeros_like(X)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    st, _ = _call(lib.cpca_apply_noalloc, h, "fp64", X, Q, e, e, Lr, Lc, 1.0, 1.0)
    assert st == _lib.EINVAL and "scratch holds" in _lib.last_error(), _lib.last_error()
    assert not Q.any()
