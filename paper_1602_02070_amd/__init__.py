"""MI355X-native solvers for Compressive PCA on graphs (arXiv 1602.02070).

The hot path (FISTA for FRPCAG on the sampled matrix, the alternate decoder
by conjugate gradient and its adjoint) runs in libcpca.so, hand-written HIP
for gfx950 behind a C ABI (include/cpca.h). This package is its Python
binding. The library is loaded on first use; a missing build raises.
"""
from .api import (CpcaError, Decode, DecodeProblem, Graph, apply_operator,  # noqa: F401
                  decode, decode_backward, frpcag, get_profile, handle, mode_for,
                  profiling, set_apply_config, Instance, solve_batched, approx_decode,
                  cluster_decode, laplacian_lmax, knn_graph,
                  approx_decode_one_side, kron_reduce)

__version__ = "0.1.0"
