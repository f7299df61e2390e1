"""C-ABI checks that run without a GPU: the library loads, exports every
function include/cpca.h declares, and rejects bad arguments on the host
before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1602_02070_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1602_02070_amd import _build
        _build.build()
    return _lib.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cpca.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cpca_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTS)


def test_version(lib):
    assert re.match(rb"^\d+\.\d+\.\d+$", lib.cpca_version())


def _a(x, dt):
    return np.ascontiguousarray(x, dtype=dt)


def test_check_csr_host(lib):
    rp, ci, v = _a([0, 2, 3, 5], np.int32), _a([0, 1, 1, 0, 2], np.int32), _a([2, -1, 1, -1, 1.], np.float64)
    ok = lib.cpca_check_csr_host(3, 5, rp.ctypes.data, ci.ctypes.data, v.ctypes.data)
    assert ok == _lib.OK and _lib.last_error() == ""
    bad_idx = _a([0, 1, 3, 0, 2], np.int32)
    assert lib.cpca_check_csr_host(3, 5, rp.ctypes.data, bad_idx.ctypes.data, v.ctypes.data) == _lib.EINVAL
    assert "column index 3" in _lib.last_error()
    dec = _a([0, 2, 1, 5], np.int32)
    assert lib.cpca_check_csr_host(3, 5, dec.ctypes.data, ci.ctypes.data, v.ctypes.data) == _lib.EINVAL
    assert "decreases" in _lib.last_error()
    end = _a([0, 2, 3, 4], np.int32)
    assert lib.cpca_check_csr_host(3, 5, end.ctypes.data, ci.ctypes.data, v.ctypes.data) == _lib.EINVAL
    nan = _a([2, np.nan, 1, -1, 1.], np.float64)
    assert lib.cpca_check_csr_host(3, 5, rp.ctypes.data, ci.ctypes.data, nan.ctypes.data) == _lib.EINVAL
    assert "non-finite" in _lib.last_error()
    assert lib.cpca_check_csr_host(0, 0, rp.ctypes.data, ci.ctypes.data, v.ctypes.data) == _lib.EINVAL
    # empty rows are structurally valid
    rp2 = _a([0, 0, 1, 1], np.int32)
    assert lib.cpca_check_csr_host(3, 1, rp2.ctypes.data, _a([2], np.int32).ctypes.data, None) == _lib.OK


def test_check_index_set_host(lib):
    ok = _a([4, 0, 2], np.int32)
    assert lib.cpca_check_index_set_host(3, 5, ok.ctypes.data) == _lib.OK
    dup = _a([4, 0, 4], np.int32)
    assert lib.cpca_check_index_set_host(3, 5, dup.ctypes.data) == _lib.EINVAL
    assert "repeated" in _lib.last_error()
    oob = _a([4, 5], np.int32)
    assert lib.cpca_check_index_set_host(2, 5, oob.ctypes.data) == _lib.EINVAL
    neg = _a([-1], np.int32)
    assert lib.cpca_check_index_set_host(1, 5, neg.ctypes.data) == _lib.EINVAL
    assert lib.cpca_check_index_set_host(6, 5, ok.ctypes.data) == _lib.EINVAL
    assert lib.cpca_check_index_set_host(0, 5, None) == _lib.OK


def _csr(n, nnz=1):
    # descriptor with non-null (host, never dereferenced) pointers
    buf = (ctypes.c_int32 * 8)()
    vals = (ctypes.c_double * 8)()
    return _lib.CpcaCsr(n, nnz, ctypes.addressof(buf), ctypes.addressof(buf),
                        ctypes.addressof(vals)), (buf, vals)


def test_entry_points_reject_bad_scalars_before_device_work(lib):
    info = _lib.CpcaInfo()
    dummy = ctypes.c_void_p(16)
    Lr, k1 = _csr(10)
    Lc, k2 = _csr(20)
    args_ok = dict(mode=0, rho_r=5, rho_c=6, p=10, n=20, gr=1.0, gc=1.0, tol=1e-8, it=100)

    def dec(**kw):
        a = dict(args_ok, **kw)
        return lib.cpca_decode(None, a["mode"], dummy, a["rho_r"], a["rho_c"], dummy, dummy,
                               a["p"], a["n"], ctypes.byref(Lr), ctypes.byref(Lc), a["gr"],
                               a["gc"], a["tol"], a["it"], None, dummy, ctypes.byref(info))

    cases = [(dict(mode=7), "mode"), (dict(p=0), "size"), (dict(rho_r=11), "samples"),
             (dict(gr=-1.0), "gamma_r"), (dict(gc=float("nan")), "gamma_c"),
             (dict(tol=0.0), "tol"), (dict(it=0), "max_iter"), (dict(n=21), "Lc")]
    for kw, word in cases:
        assert dec(**kw) == _lib.EINVAL, kw
        assert word in _lib.last_error(), (kw, _lib.last_error())
    # every check passes: the null handle is the remaining problem
    assert dec() == _lib.EINVAL and "null handle" in _lib.last_error()

    def fr(**kw):
        a = dict(dict(rr=10, rc=20, gr=1.0, gc=1.0, lr=1.5, lc=1.5, it=10, eps=0.0), **kw)
        return lib.cpca_frpcag(None, 0, dummy, a["rr"], a["rc"], ctypes.byref(Lr), ctypes.byref(Lc),
                               a["gr"], a["gc"], a["lr"], a["lc"], a["it"], a["eps"], dummy,
                               ctypes.byref(info))

    for kw, word in [(dict(lr=float("nan")), "lmax"), (dict(it=-1), "max_iter"), (dict(eps=-1.0), "eps"),
                     (dict(rr=11), "Lr_til"), (dict(gc=float("inf")), "gamma_c")]:
        assert fr(**kw) == _lib.EINVAL, kw
        assert word in _lib.last_error(), (kw, _lib.last_error())
    assert fr(gr=0.0, lr=0.0) == _lib.EINVAL and "null handle" in _lib.last_error()
    # lmax <= 0 asks for the device estimate: it passes the argument checks
    assert fr(lr=0.0, lc=-1.0) == _lib.EINVAL and "null handle" in _lib.last_error()
    lm = ctypes.c_double()
    for kw, word in [(dict(tol=0.0), "tol"), (dict(tol=1.0), "tol"), (dict(it=0), "max_iter")]:
        a = dict(dict(tol=1e-9, it=100), **kw)
        assert lib.cpca_laplacian_lmax(None, ctypes.byref(Lr), a["tol"], a["it"], ctypes.byref(lm),
                                       ctypes.byref(info)) == _lib.EINVAL, kw
        assert word in _lib.last_error(), (kw, _lib.last_error())
    assert lib.cpca_laplacian_lmax(None, ctypes.byref(Lr), 1e-9, 100, None, None) == _lib.EINVAL
    assert lib.cpca_laplacian_lmax(None, ctypes.byref(Lr), 1e-9, 100, ctypes.byref(lm),
                                   None) == _lib.EINVAL and "null handle" in _lib.last_error()
    assert lib.cpca_create(None, None) == _lib.EINVAL
    assert lib.cpca_destroy(None) == _lib.OK


def test_approx_decode_rejects_bad_arguments_before_device_work(lib):
    info = _lib.CpcaApproxInfo()
    dummy = ctypes.c_void_p(16)
    Lr, k1 = _csr(10)
    Lc, k2 = _csr(20)
    base = dict(mode=1, rho_r=5, rho_c=6, p=10, n=20, delta=0.0, ratio=0.1, kmax=16, tol=1e-10,
                it=100)

    def call(**kw):
        a = dict(base, **kw)
        return lib.cpca_approx_decode(None, a["mode"], dummy, a["rho_r"], a["rho_c"], dummy, dummy,
                                      a["p"], a["n"], ctypes.byref(Lr), ctypes.byref(Lc),
                                      a["delta"], a["ratio"], a["kmax"], a["tol"], a["it"], dummy,
                                      None, ctypes.byref(info))

    cases = [(dict(mode=5), "mode"), (dict(n=0), "size"), (dict(rho_c=21), "samples"),
             (dict(delta=1.0), "delta"), (dict(delta=-0.1), "delta"),
             (dict(ratio=1.5), "sigma_ratio"), (dict(ratio=float("nan")), "sigma_ratio"),
             (dict(kmax=0), "k_max"), (dict(kmax=65), "k_max"), (dict(tol=-1.0), "tol"),
             (dict(it=-1), "max_iter"), (dict(p=11), "Lr")]
    for kw, word in cases:
        assert call(**kw) == _lib.EINVAL, kw
        assert word in _lib.last_error(), (kw, _lib.last_error())
    assert call() == _lib.EINVAL and "null handle" in _lib.last_error()
    assert call(it=0, ratio=0.0, kmax=64) == _lib.EINVAL and "null handle" in _lib.last_error()


def test_cluster_decode_rejects_bad_arguments_before_device_work(lib):
    info = _lib.CpcaClusterInfo()
    dummy = ctypes.c_void_p(16)
    Lc, keep = _csr(50)
    base = dict(mode=0, rho_r=8, rho_c=20, n=50, k=4, km=100, tol=1e-10, it=100)

    def call(**kw):
        a = dict(base, **kw)
        return lib.cpca_cluster_decode(None, a["mode"], dummy, a["rho_r"], a["rho_c"], dummy,
                                       a["n"], ctypes.byref(Lc), a["k"], dummy, a["km"], a["tol"],
                                       a["it"], dummy, None, None, ctypes.byref(info))

    cases = [(dict(mode=3), "mode"), (dict(rho_r=0), "size"), (dict(rho_c=51), "samples"),
             (dict(n=51), "Lc"), (dict(k=0), "k must"), (dict(k=65), "k must"),
             (dict(k=21), "k must"), (dict(km=-1), "kmeans_max_iter"), (dict(tol=0.0), "tol"),
             (dict(it=-1), "max_iter")]
    for kw, word in cases:
        assert call(**kw) == _lib.EINVAL, kw
        assert word in _lib.last_error(), (kw, _lib.last_error())
    assert call() == _lib.EINVAL and "null handle" in _lib.last_error()


def test_knn_graph_rejects_bad_arguments_before_device_work(lib):
    info = _lib.CpcaInfo()
    dummy = ctypes.c_void_p(16)
    nnz = ctypes.c_int64()
    sig = ctypes.c_double()
    base = dict(N=100, d=3, K=10, norm=1, cap=100 * 21)

    def call(**kw):
        a = dict(base, **kw)
        return lib.cpca_knn_graph(None, dummy, a["N"], a["d"], a["K"], a["norm"], dummy, dummy,
                                  dummy, a["cap"], ctypes.byref(nnz), ctypes.byref(sig), None,
                                  ctypes.byref(info))

    cases = [(dict(N=1), "N must"), (dict(d=0), "d must"), (dict(K=0), "K must"),
             (dict(K=29), "K must"), (dict(N=10, K=10, cap=210), "K must"),
             (dict(norm=2), "normalized"), (dict(cap=100 * 21 - 1), "nnz_cap")]
    for kw, word in cases:
        assert call(**kw) == _lib.EINVAL, kw
        assert word in _lib.last_error(), (kw, _lib.last_error())
    assert call() == _lib.EINVAL and "null handle" in _lib.last_error()


def test_one_side_decoders_reject_bad_arguments_before_device_work(lib):
    info = _lib.CpcaApproxInfo()
    dummy = ctypes.c_void_p(16)
    Lr, k1 = _csr(10)
    Lc, k2 = _csr(20)
    base = dict(mode=1, rho_r=5, rho_c=6, p=10, n=20, ratio=0.1, kmax=16, tol=1e-10, it=100,
                Y=dummy)
    for fn, L, dimkey in ((lib.cpca_approx_decode2, Lr, "p"), (lib.cpca_approx_decode3, Lc, "n")):
        def call(**kw):
            a = dict(base, **kw)
            return fn(None, a["mode"], dummy, a["rho_r"], a["rho_c"], dummy, a["p"], a["n"],
                      ctypes.byref(L), a["Y"], a["ratio"], a["kmax"], a["tol"], a["it"], dummy,
                      None, ctypes.byref(info))

        cases = [(dict(mode=5), "mode"), (dict(n=0), "size"), (dict(rho_c=21), "samples"),
                 (dict(ratio=1.5), "sigma_ratio"), (dict(kmax=0), "k_max"),
                 (dict(kmax=17), "k_max"), (dict(tol=-1.0), "tol"), (dict(it=-1), "max_iter"),
                 (dict(Y=None), "null Y"), ({dimkey: 11}, "L")]
        for kw, word in cases:
            assert call(**kw) == _lib.EINVAL, kw
            assert word in _lib.last_error(), (kw, _lib.last_error())
        assert call() == _lib.EINVAL and "null handle" in _lib.last_error()


def test_kron_reduce_rejects_bad_arguments_before_device_work(lib):
    info = _lib.CpcaInfo()
    dummy = ctypes.c_void_p(16)
    L, keep = _csr(30)

    def call(rho=5, tol=1e-12, it=100, om=dummy, out=dummy):
        return lib.cpca_kron_reduce(None, ctypes.byref(L), om, rho, tol, it, out, ctypes.byref(info))

    for kw, word in [(dict(rho=0), "rho"), (dict(rho=31), "rho"), (dict(tol=0.0), "tol"),
                     (dict(it=-1), "max_iter"), (dict(om=None), "null"), (dict(out=None), "null")]:
        assert call(**kw) == _lib.EINVAL, kw
        assert word in _lib.last_error(), (kw, _lib.last_error())
    assert call() == _lib.EINVAL and "null handle" in _lib.last_error()
