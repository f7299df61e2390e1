"""Python binding of the CPCA solver library: argument marshalling only.

Every computation runs in libcpca.so (HIP kernels for gfx950); PyTorch
provides device memory and the current stream. Tensors must be CUDA (ROCm)
tensors, contiguous, row-major.
"""
from __future__ import annotations

import ctypes
import dataclasses
import warnings

import numpy as np
import torch

from . import _lib
from ._lib import CpcaApproxInfo, CpcaClusterInfo, CpcaCsr, CpcaInfo, CpcaInstance, CpcaTask

__all__ = ["CpcaError", "Graph", "handle", "frpcag", "laplacian_lmax", "knn_graph", "decode",
           "decode_backward", "approx_decode_one_side", "kron_reduce",
           "apply_operator", "Decode", "DecodeProblem", "profiling", "get_profile",
           "mode_for", "set_apply_config", "Instance", "solve_batched"]


class CpcaError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.last_error()
        super().__init__(f"{where}: {_lib.STATUS_NAMES.get(status, status)}: {msg}")


def _check(status: int, where: str, allow_noconv: bool = True) -> int:
    if status == _lib.OK:
        return status
    if status == _lib.ENOCONV and allow_noconv:
        warnings.warn(f"{where}: iteration limit reached ({_lib.last_error()})", RuntimeWarning)
        return status
    raise CpcaError(status, where)


# ------------------------------------------------------------------ handles
_handles: dict = {}


def handle(device=None, stream=None) -> int:
    """Library handle bound to (device, stream); cached per pair."""
    lib = _lib.load()
    dev = torch.device("cuda", torch.cuda.current_device() if device is None
                       else torch.device(device).index or 0)
    with torch.cuda.device(dev):
        s = torch.cuda.current_stream(dev) if stream is None else stream
        key = (dev.index, int(s.cuda_stream))
        h = _handles.get(key)
        if h is None:
            hp = ctypes.c_void_p()
            _check(lib.cpca_create(ctypes.byref(hp), ctypes.c_void_p(int(s.cuda_stream))),
                   "cpca_create", allow_noconv=False)
            h = hp.value
            _handles[key] = h
        return h


def profiling(enable: bool, h=None) -> None:
    lib = _lib.load()
    _check(lib.cpca_set_profiling(h or handle(), int(bool(enable))), "cpca_set_profiling")


KERNELS = {"auto": -1, "rows": 0, "strip": 1, "panel": 2, "panel_lo": 3}


def set_apply_config(rows_per_block: int = 0, use_lds: int = -1, kernel: str = "auto",
                     h=None) -> None:
    """Launch shape of the fused two-sided product (0 / -1 = automatic).

    kernel: preference for a banded L_c, one of "auto", "rows", "strip",
    "panel", "panel_lo" (see cpca_set_apply_config)."""
    lib = _lib.load()
    _check(lib.cpca_set_apply_config(h or handle(), int(rows_per_block), int(use_lds),
                                     KERNELS[kernel]),
           "cpca_set_apply_config", allow_noconv=False)


def get_profile(family: str, h=None) -> tuple[int, float]:
    lib = _lib.load()
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(lib.cpca_get_profile(h or handle(), family.encode(), ctypes.byref(n), ctypes.byref(ms)),
           "cpca_get_profile")
    return n.value, ms.value


# -------------------------------------------------------------------- graphs
class Graph:
    """Square CSR matrix (a graph Laplacian) resident on the GPU:
    int32 row pointers and column indices, FP64 values."""

    def __init__(self, rowptr: torch.Tensor, colind: torch.Tensor, vals: torch.Tensor, n: int):
        self.rowptr = rowptr.to(torch.int32).contiguous()
        self.colind = colind.to(torch.int32).contiguous()
        self.vals = vals.to(torch.float64).contiguous()
        self.n = int(n)
        self.nnz = int(self.colind.numel())
        self._desc = CpcaCsr(self.n, self.nnz, self.rowptr.data_ptr(), self.colind.data_ptr(),
                             self.vals.data_ptr())

    @classmethod
    def from_scipy(cls, L, device="cuda") -> "Graph":
        L = L.tocsr()
        L.sort_indices()
        return cls(torch.from_numpy(np.asarray(L.indptr, dtype=np.int32)).to(device),
                   torch.from_numpy(np.asarray(L.indices, dtype=np.int32)).to(device),
                   torch.from_numpy(np.asarray(L.data, dtype=np.float64)).to(device),
                   L.shape[0])

    @property
    def desc(self) -> CpcaCsr:
        return self._desc

    def to_scipy(self):
        """Host copy as a scipy.sparse CSR matrix."""
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals.cpu().numpy(), self.colind.cpu().numpy(),
                              self.rowptr.cpu().numpy()), shape=(self.n, self.n))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def mode_for(dtype: torch.dtype, mode: str | None) -> str:
    if mode is not None:
        if mode not in _lib.MODES:
            raise ValueError(f"unknown mode {mode!r}")
        return mode
    if dtype == torch.float64:
        return "fp64"
    if dtype == torch.float32:
        return "fp32_ir"
    raise TypeError(f"unsupported dtype {dtype}")


def _dtype_of(mode: str) -> torch.dtype:
    return torch.float64 if mode == "fp64" else torch.float32


def _need(t: torch.Tensor, name: str, dtype: torch.dtype, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.contiguous()


def _index(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    return t.to(torch.int32).contiguous()


# ------------------------------------------------------------------- solvers
def frpcag(Ytil: torch.Tensor, Lr_til: Graph, Lc_til: Graph, gamma_r: float, gamma_c: float,
           lmax_r: float, lmax_c: float, max_iter: int = 500, eps: float = 0.0,
           mode: str | None = None):
    """FISTA for FRPCAG on the sampled matrix (Algorithm 1). Returns (X~, info)."""
    mode = mode_for(Ytil.dtype, mode)
    Y = _need(Ytil, "Ytil", _dtype_of(mode))
    rr, rc = Y.shape
    out = torch.empty_like(Y)
    info = CpcaInfo()
    st = _lib.load().cpca_frpcag(handle(Y.device), _lib.MODES[mode], _ptr(Y), rr, rc,
                                 ctypes.byref(Lr_til.desc), ctypes.byref(Lc_til.desc),
                                 float(gamma_r), float(gamma_c), float(lmax_r), float(lmax_c),
                                 int(max_iter), float(eps), _ptr(out), ctypes.byref(info))
    _check(st, "cpca_frpcag")
    return out, info.as_dict()


def laplacian_lmax(L: Graph, tol: float = 1e-9, max_iter: int = 50000, device=None):
    """Largest eigenvalue of a PSD CSR matrix by FP64 power iteration on the
    device (the FISTA step's norm, Section IV.B). Returns (lmax, info)."""
    lmax = ctypes.c_double()
    info = CpcaInfo()
    st = _lib.load().cpca_laplacian_lmax(handle(device or L.rowptr.device), ctypes.byref(L.desc),
                                         float(tol), int(max_iter), ctypes.byref(lmax),
                                         ctypes.byref(info))
    _check(st, "cpca_laplacian_lmax")
    return lmax.value, info.as_dict()


def knn_graph(points: torch.Tensor, K: int = 10, kind: str = "normalized",
              want_knn: bool = False):
    """Laplacian of the K-NN Gaussian-kernel graph of the rows of `points`
    (N x d, FP64, on the GPU): Section II. kind: "normalized" or
    "combinatorial". Returns (Graph, info) with info = dict(sigma, nnz, ms,
    knn (N x K int32 neighbour indices, if want_knn))."""
    Y = _need(points, "points", torch.float64)
    if Y.dim() != 2:
        raise ValueError("points must be N x d")
    N, d = Y.shape
    if kind not in ("normalized", "combinatorial"):
        raise ValueError(f"unknown kind {kind!r}")
    cap = N * (2 * int(K) + 1)
    rowptr = torch.empty(N + 1, dtype=torch.int32, device=Y.device)
    colind = torch.empty(cap, dtype=torch.int32, device=Y.device)
    vals = torch.empty(cap, dtype=torch.float64, device=Y.device)
    knn = torch.empty((N, int(K)), dtype=torch.int32, device=Y.device) if want_knn else None
    nnz = ctypes.c_int64()
    sigma = ctypes.c_double()
    info = CpcaInfo()
    st = _lib.load().cpca_knn_graph(handle(Y.device), _ptr(Y), N, d, int(K),
                                    int(kind == "normalized"), _ptr(rowptr), _ptr(colind),
                                    _ptr(vals), cap, ctypes.byref(nnz), ctypes.byref(sigma),
                                    _ptr(knn), ctypes.byref(info))
    _check(st, "cpca_knn_graph", allow_noconv=False)
    m = nnz.value
    G = Graph(rowptr, colind[:m].clone(), vals[:m].clone(), N)
    out = dict(sigma=sigma.value, nnz=m, ms=info.ms)
    if want_knn:
        out["knn"] = knn
    return G, out


def kron_reduce(L: Graph, omega: torch.Tensor, tol: float = 1e-12, max_iter: int = 20000):
    """Kron reduction of L onto the nodes omega (Section IV-A): the dense
    rho x rho FP64 Schur complement, rows and columns in the order of omega.
    Returns (L~, info)."""
    om = _index(omega, "omega")
    rho = om.numel()
    out = torch.empty((rho, rho), dtype=torch.float64, device=om.device)
    info = CpcaInfo()
    st = _lib.load().cpca_kron_reduce(handle(om.device), ctypes.byref(L.desc), _ptr(om), rho,
                                      float(tol), int(max_iter), _ptr(out), ctypes.byref(info))
    _check(st, "cpca_kron_reduce")
    return out, info.as_dict()


def decode(Xtil: torch.Tensor, omega_r: torch.Tensor, omega_c: torch.Tensor, p: int, n: int,
           Lr: Graph, Lc: Graph, gamma_r: float, gamma_c: float, tol: float = 1e-10,
           max_iter: int = 20000, mode: str | None = None, X0: torch.Tensor | None = None,
           out: torch.Tensor | None = None, h=None):
    """Alternate decoder by CG (Section V.B). Returns (X, info)."""
    mode = mode_for(Xtil.dtype, mode)
    dt = _dtype_of(mode)
    Xt = _need(Xtil, "Xtil", dt)
    om_r = _index(omega_r, "omega_r")
    om_c = _index(omega_c, "omega_c")
    if Xt.shape != (om_r.numel(), om_c.numel()):
        raise ValueError("Xtil shape must be (len(omega_r), len(omega_c))")
    X0c = None if X0 is None else _need(X0, "X0", dt, (p, n))
    if out is None:
        out = torch.empty((p, n), dtype=dt, device=Xt.device)
    else:
        out = _need(out, "out", dt, (p, n))
    info = CpcaInfo()
    st = _lib.load().cpca_decode(h or handle(Xt.device), _lib.MODES[mode], _ptr(Xt), Xt.shape[0],
                                 Xt.shape[1], _ptr(om_r), _ptr(om_c), int(p), int(n),
                                 ctypes.byref(Lr.desc), ctypes.byref(Lc.desc), float(gamma_r),
                                 float(gamma_c), float(tol), int(max_iter), _ptr(X0c), _ptr(out),
                                 ctypes.byref(info))
    _check(st, "cpca_decode")
    return out, info.as_dict()


def approx_decode(Xtil: torch.Tensor, omega_r: torch.Tensor, omega_c: torch.Tensor, p: int,
                  n: int, Lr: Graph, Lc: Graph, delta: float = 0.0, sigma_ratio: float = 0.1,
                  k_max: int = 64, tol: float = 1e-10, max_iter: int = 20000,
                  mode: str | None = None, out: torch.Tensor | None = None, h=None):
    """Subspace-upsampling approximate decoder (Section V.C, Algorithm 2).

    Returns (X, sigma, info): X is p x n, sigma the singular values of Xtil
    (descending, FP64 host array), info the call's cpca_approx_info."""
    mode = mode_for(Xtil.dtype, mode)
    dt = _dtype_of(mode)
    Xt = _need(Xtil, "Xtil", dt)
    om_r = _index(omega_r, "omega_r")
    om_c = _index(omega_c, "omega_c")
    if Xt.shape != (om_r.numel(), om_c.numel()):
        raise ValueError("Xtil shape must be (len(omega_r), len(omega_c))")
    if out is None:
        out = torch.empty((p, n), dtype=dt, device=Xt.device)
    else:
        out = _need(out, "out", dt, (p, n))
    sigma = (ctypes.c_double * max(1, min(Xt.shape)))()
    info = CpcaApproxInfo()
    st = _lib.load().cpca_approx_decode(h or handle(Xt.device), _lib.MODES[mode], _ptr(Xt),
                                        Xt.shape[0], Xt.shape[1], _ptr(om_r), _ptr(om_c), int(p),
                                        int(n), ctypes.byref(Lr.desc), ctypes.byref(Lc.desc),
                                        float(delta), float(sigma_ratio), int(k_max), float(tol),
                                        int(max_iter), _ptr(out), sigma, ctypes.byref(info))
    _check(st, "cpca_approx_decode")
    return out, [sigma[i] for i in range(min(Xt.shape))], info.as_dict()


def approx_decode_one_side(side: str, Xtil: torch.Tensor, omega: torch.Tensor, p: int, n: int,
                           L: Graph, Y: torch.Tensor, sigma_ratio: float = 0.1, k_max: int = 16,
                           tol: float = 1e-10, max_iter: int = 20000, mode: str | None = None,
                           out: torch.Tensor | None = None, h=None):
    """Approximate decoders 2 and 3 of the appendix: side "rows" upsamples
    the left singular vectors of X~ over L_r and returns X = U U^T Y; side
    "cols" upsamples the right ones over L_c and returns X = Y V V^T. Y is
    the full p x n data. Returns (X, sigma, info) as approx_decode."""
    if side not in ("rows", "cols"):
        raise ValueError("side must be 'rows' or 'cols'")
    mode = mode_for(Xtil.dtype, mode)
    dt = _dtype_of(mode)
    Xt = _need(Xtil, "Xtil", dt)
    Yd = _need(Y, "Y", dt, (p, n))
    om = _index(omega, "omega")
    if out is None:
        out = torch.empty((p, n), dtype=dt, device=Xt.device)
    else:
        out = _need(out, "out", dt, (p, n))
    sigma = (ctypes.c_double * max(1, min(Xt.shape)))()
    info = CpcaApproxInfo()
    fn = _lib.load().cpca_approx_decode2 if side == "rows" else _lib.load().cpca_approx_decode3
    st = fn(h or handle(Xt.device), _lib.MODES[mode], _ptr(Xt), Xt.shape[0], Xt.shape[1], _ptr(om),
            int(p), int(n), ctypes.byref(L.desc), _ptr(Yd), float(sigma_ratio), int(k_max),
            float(tol), int(max_iter), _ptr(out), sigma, ctypes.byref(info))
    _check(st, "cpca_approx_decode2" if side == "rows" else "cpca_approx_decode3")
    return out, [sigma[i] for i in range(min(Xt.shape))], info.as_dict()


def cluster_decode(Xtil: torch.Tensor, omega_c: torch.Tensor, n: int, Lc: Graph, init,
                   kmeans_max_iter: int = 100, tol: float = 1e-10, max_iter: int = 20000,
                   mode: str | None = None, want_C: bool = False, h=None):
    """Approximate decoder for clustering (Section VI, Algorithm 3).

    init: the k seed columns of Xtil (positions in [0, rho_c)). Returns
    (labels (n, int32), sample_labels (rho_c, int32), C (n x k FP64) or None,
    info)."""
    mode = mode_for(Xtil.dtype, mode)
    dt = _dtype_of(mode)
    Xt = _need(Xtil, "Xtil", dt)
    om_c = _index(omega_c, "omega_c")
    if Xt.shape[1] != om_c.numel():
        raise ValueError("Xtil must have len(omega_c) columns")
    seeds = _index(torch.as_tensor(init, dtype=torch.int32).to(Xt.device), "init")
    k = seeds.numel()
    labels = torch.empty(n, dtype=torch.int32, device=Xt.device)
    slab = torch.empty(Xt.shape[1], dtype=torch.int32, device=Xt.device)
    C = torch.empty((n, k), dtype=torch.float64, device=Xt.device) if want_C else None
    info = CpcaClusterInfo()
    st = _lib.load().cpca_cluster_decode(h or handle(Xt.device), _lib.MODES[mode], _ptr(Xt),
                                         Xt.shape[0], Xt.shape[1], _ptr(om_c), int(n),
                                         ctypes.byref(Lc.desc), int(k), _ptr(seeds),
                                         int(kmeans_max_iter), float(tol), int(max_iter),
                                         _ptr(labels), _ptr(C), _ptr(slab), ctypes.byref(info))
    _check(st, "cpca_cluster_decode")
    return labels, slab, C, info.as_dict()


def decode_backward(G: torch.Tensor, X: torch.Tensor, omega_r, omega_c, p: int, n: int,
                    Lr: Graph, Lc: Graph, gamma_r: float, gamma_c: float, tol: float = 1e-10,
                    max_iter: int = 20000, mode: str | None = None):
    """Adjoint of `decode`. Returns (dXtil, dgamma_r, dgamma_c, info)."""
    mode = mode_for(X.dtype, mode)
    dt = _dtype_of(mode)
    Gc = _need(G, "G", dt, (p, n))
    Xc = _need(X, "X", dt, (p, n))
    om_r = _index(omega_r, "omega_r")
    om_c = _index(omega_c, "omega_c")
    dXt = torch.empty((om_r.numel(), om_c.numel()), dtype=dt, device=Xc.device)
    dgr = ctypes.c_double()
    dgc = ctypes.c_double()
    info = CpcaInfo()
    st = _lib.load().cpca_decode_backward(handle(Xc.device), _lib.MODES[mode], _ptr(Gc), _ptr(Xc),
                                          om_r.numel(), om_c.numel(), _ptr(om_r), _ptr(om_c),
                                          int(p), int(n), ctypes.byref(Lr.desc),
                                          ctypes.byref(Lc.desc), float(gamma_r), float(gamma_c),
                                          float(tol), int(max_iter), _ptr(dXt), ctypes.byref(dgr),
                                          ctypes.byref(dgc), ctypes.byref(info))
    _check(st, "cpca_decode_backward")
    return dXt, dgr.value, dgc.value, info.as_dict()


def apply_operator(P: torch.Tensor, Lr: Graph, Lc: Graph, gamma_r: float, gamma_c: float,
                   omega_r: torch.Tensor | None = None, omega_c: torch.Tensor | None = None,
                   mode: str | None = None, out: torch.Tensor | None = None):
    """Q = (m_r m_c^T) o P + gamma_r L_r P + gamma_c P L_c. Returns (Q, <P, Q>)."""
    mode = mode_for(P.dtype, mode)
    if mode == "fp32_ir":
        mode = "fp32"
    Pc = _need(P, "P", _dtype_of(mode))
    p, n = Pc.shape
    om_r = None if omega_r is None else _index(omega_r, "omega_r")
    om_c = None if omega_c is None else _index(omega_c, "omega_c")
    Q = torch.empty_like(Pc) if out is None else _need(out, "out", Pc.dtype, (p, n))
    pq = ctypes.c_double()
    st = _lib.load().cpca_apply(handle(Pc.device), _lib.MODES[mode], _ptr(Pc), _ptr(Q), p, n,
                                _ptr(om_r), 0 if om_r is None else om_r.numel(), _ptr(om_c),
                                0 if om_c is None else om_c.numel(), ctypes.byref(Lr.desc),
                                ctypes.byref(Lc.desc), float(gamma_r), float(gamma_c),
                                ctypes.byref(pq))
    _check(st, "cpca_apply", allow_noconv=False)
    return Q, pq.value


# ---------------------------------------------------------------- autograd
@dataclasses.dataclass
class DecodeProblem:
    """Everything the decoder needs besides X~ and the gammas."""
    omega_r: torch.Tensor
    omega_c: torch.Tensor
    p: int
    n: int
    Lr: Graph
    Lc: Graph
    tol: float = 1e-10
    max_iter: int = 20000
    mode: str | None = None


class Decode(torch.autograd.Function):
    """X = decode(X~, gamma_r, gamma_c) with gradients for X~ and both gammas
    (adjoint CG, A symmetric). gamma_r / gamma_c are 0-d tensors."""

    @staticmethod
    def forward(ctx, Xtil, gamma_r, gamma_c, prob: DecodeProblem):
        gr, gc = float(gamma_r), float(gamma_c)
        X, _ = decode(Xtil.detach(), prob.omega_r, prob.omega_c, prob.p, prob.n, prob.Lr,
                      prob.Lc, gr, gc, prob.tol, prob.max_iter, prob.mode)
        ctx.save_for_backward(X)
        ctx.prob = prob
        ctx.g = (gr, gc)
        ctx.gdt = (gamma_r.dtype if torch.is_tensor(gamma_r) else torch.float64,
                   gamma_c.dtype if torch.is_tensor(gamma_c) else torch.float64)
        return X

    @staticmethod
    def backward(ctx, G):
        (X,) = ctx.saved_tensors
        prob = ctx.prob
        dXt, dgr, dgc, _ = decode_backward(G.contiguous().to(X.dtype), X, prob.omega_r,
                                           prob.omega_c, prob.p, prob.n, prob.Lr, prob.Lc,
                                           ctx.g[0], ctx.g[1], prob.tol, prob.max_iter, prob.mode)
        return (dXt, torch.tensor(dgr, dtype=ctx.gdt[0], device=X.device),
                torch.tensor(dgc, dtype=ctx.gdt[1], device=X.device), None)


# ------------------------------------------------------------------ batched
@dataclasses.dataclass
class Instance:
    """One problem of a batched solve: graphs, sampling sets and sampled data
    (all on the GPU)."""
    p: int
    n: int
    omega_r: torch.Tensor
    omega_c: torch.Tensor
    Lr: Graph
    Lc: Graph
    Lr_til: Graph
    Lc_til: Graph
    lmax_r_til: float
    lmax_c_til: float
    Ytil: torch.Tensor


def solve_batched(instances, tasks, fista_iters: int = 500, tol: float = 1e-9,
                  max_iter: int = 20000, mode: str | None = None, want_xtil: bool = False,
                  raise_errors: bool = True, h=None):
    """FISTA + alternate decoder for every task (instance index, gamma_r,
    gamma_c) in one batched run. Returns (X list, X~ list or None, infos).
    With raise_errors=False a failed task is reported only in its info.
    h: library handle (default: the one of the inputs' device and the
    current stream)."""
    if not instances or not tasks:
        raise ValueError("need at least one instance and one task")
    mode = mode_for(instances[0].Ytil.dtype, mode)
    dt = _dtype_of(mode)
    keep = []
    cin = (CpcaInstance * len(instances))()
    for k, I in enumerate(instances):
        Y = _need(I.Ytil, f"instances[{k}].Ytil", dt)
        om_r = _index(I.omega_r, "omega_r")
        om_c = _index(I.omega_c, "omega_c")
        keep += [Y, om_r, om_c]
        cin[k] = CpcaInstance(int(I.p), int(I.n), om_r.numel(), om_c.numel(), om_r.data_ptr(),
                              om_c.data_ptr(), ctypes.pointer(I.Lr.desc), ctypes.pointer(I.Lc.desc),
                              ctypes.pointer(I.Lr_til.desc), ctypes.pointer(I.Lc_til.desc),
                              float(I.lmax_r_til), float(I.lmax_c_til), Y.data_ptr())
    outs, xts = [], []
    ctk = (CpcaTask * len(tasks))()
    for t, (inst, gr, gc) in enumerate(tasks):
        I = instances[inst]
        X = torch.empty((I.p, I.n), dtype=dt, device=I.Ytil.device)
        Xt = (torch.empty((I.omega_r.numel(), I.omega_c.numel()), dtype=dt, device=X.device)
              if want_xtil else None)
        outs.append(X)
        xts.append(Xt)
        ctk[t] = CpcaTask(int(inst), 0, float(gr), float(gc), X.data_ptr(),
                          None if Xt is None else Xt.data_ptr())
    infos = (CpcaInfo * len(tasks))()
    st = _lib.load().cpca_solve_batched(h or handle(instances[0].Ytil.device), _lib.MODES[mode], cin,
                                        len(instances), ctk, len(tasks), int(fista_iters),
                                        float(tol), int(max_iter), infos)
    if raise_errors:
        _check(st, "cpca_solve_batched")
    return outs, (xts if want_xtil else None), [i.as_dict() for i in infos]
