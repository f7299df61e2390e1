"""Plain FP64 CPU oracle for the CPCA hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package. The HIP library never calls it and shares
no code with it.

Contents (each function cites the passage it follows):
  frpcag  -- the FRPCAG objective (eq. frpcag_small), the smooth part g and
             its gradient, the prox of the l1 data term, the step size and
             FISTA (Algorithm 1, Section IV.B);
  decoder -- the alternate decoder (eq. alternatedecoder, Section V.B): its
             normal-equation operator, right-hand side, exact solution by a
             dense Kronecker factorisation, a sparse direct factorisation or
             textbook conjugate gradient, and the adjoint (backward) of the
             decode map;
  approx  -- the subspace-upsampling approximate decoder (Algorithm 2,
             Section V.C): thin SVD, rank selection, graph upsampling by the
             closed form of its lemma, normalisation, RIP scaling.
  cluster -- the approximate decoder for clustering (Algorithm 3, Section
             VI): Lloyd's k-means from given seeds, upsampling of the cluster
             indicators over the column graph, max pooling.
  kron    -- Kron reduction of a Laplacian onto the sampled nodes (Section
             IV-A): the Schur complement, written out.
  knn     -- K-nearest-neighbour Gaussian-kernel graphs and their
             combinatorial / normalised Laplacians (Section II, graph
             construction in Section VII-A), by brute force.

Every floating-point computation is FP64. Parity status of each function is
stated in its docstring; all functions here are pinned by tests that check
them against closed forms, brute force or invariants fixed by the paper.
"""
from . import frpcag, decoder, approx, cluster, knn, kron  # noqa: F401
