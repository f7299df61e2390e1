/*
 * cpca.h -- C ABI of the MI355X (gfx950) library for the graph-regularised
 * low-rank solvers of Compressive PCA on graphs (Shahid, Perraudin, Puy,
 * Vandergheynst, arXiv 1602.02070).
 *
 * Notation (Sections II-V of the paper):
 *   Y, X          p x n data / low-rank matrices; rows are features (row graph
 *                 G_r, Laplacian L_r, p x p), columns are samples (column graph
 *                 G_c, Laplacian L_c, n x n).
 *   Omega_r/_c    sampled row / column indices (eq. (Mc)), rho_r = |Omega_r|,
 *                 rho_c = |Omega_c|; Y~ = M_r Y M_c is rho_r x rho_c and its
 *                 row a / column b is row Omega_r[a] / column Omega_c[b] of Y.
 *   L~_r, L~_c    Laplacians of the graphs on the sampled rows / columns.
 *
 * Conventions shared by every entry point:
 *   - Dense matrices are row-major (the column index is contiguous) and live
 *     in caller-owned DEVICE memory. Inputs are never modified; outputs
 *     (*_out) are written on CPCA_OK and, for iterative calls, on
 *     CPCA_ENOCONV (then they hold the last iterate).
 *   - Element type follows the mode: double for CPCA_FP64, float for
 *     CPCA_FP32 and CPCA_FP32_IR. CSR values are always double.
 *   - CSR matrices (cpca_csr) are square, symmetric positive semi-definite
 *     (graph Laplacians), int32 row pointers / column indices in device
 *     memory, with at most INT32_MAX non-zeros. Symmetry is assumed, not
 *     checked: row j of L_c is used as column j. Structure (monotone row
 *     pointers, indices in range) and finiteness are checked on every call.
 *   - Index sets are int32 device arrays whose entries are distinct and in
 *     range (checked on every call).
 *   - Every call is synchronous with respect to the host: it enqueues work
 *     on the handle's stream and returns after that work has finished, so
 *     `info` is valid on return. Calls on one handle must not overlap.
 *   - Argument checks happen before any device work; CPCA_EINVAL leaves the
 *     outputs untouched. cpca_last_error() describes the last failure of the
 *     calling thread.
 *   - No exception or abort crosses this interface.
 */
#ifndef CPCA_H
#define CPCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpca_handle_s* cpca_handle;

typedef enum {
  CPCA_OK = 0,
  CPCA_EINVAL = 1,   /* invalid argument (nothing was written)               */
  CPCA_ENOCONV = 2,  /* max_iter reached before the tolerance                */
  CPCA_ENOTSPD = 3,  /* CG breakdown: <p, A p> <= 0 (operator not definite)  */
  CPCA_ENAN = 4,     /* NaN or Inf met during the iteration                  */
  CPCA_EHIP = 5,     /* HIP runtime error                                    */
  CPCA_ENOMEM = 6    /* device or pinned-host allocation failed              */
} cpca_status;

typedef enum {
  CPCA_FP64 = 0,     /* everything in FP64                                   */
  CPCA_FP32 = 1,     /* FP32 vectors and sparse products, FP64 CG scalars    */
  CPCA_FP32_IR = 2   /* FP32 CG with FP64 residual replacement: the solution
                        accumulates in FP64 and the FP32 residual is replaced
                        by the FP64 residual B - A(X) whenever it has dropped
                        by 100x (the search direction is kept)             */
} cpca_mode;

typedef struct {
  int64_t n;               /* order of the square matrix                     */
  int64_t nnz;             /* number of stored entries                       */
  const int32_t* rowptr;   /* n + 1 entries, rowptr[0] = 0, rowptr[n] = nnz  */
  const int32_t* colind;   /* nnz column indices in [0, n)                   */
  const double* vals;      /* nnz values                                     */
} cpca_csr;

typedef struct {
  int32_t iters;           /* FISTA iterations run / total CG iterations     */
  int32_t outer_iters;     /* FP64 residual replacements (CPCA_FP32_IR)      */
  int32_t status;          /* same value as the call's return code           */
  int32_t reserved;
  double rel_residual;     /* decode: FP64 ||B - A(X)||_F / ||B||_F of the
                              returned X; frpcag: last ||Z+ - Z||^2/||Z||^2  */
  double objective;        /* frpcag: objective of eq. (frpcag_small) at the
                              returned X~; decode: 0                          */
  double ms;               /* wall time of the call                          */
} cpca_info;

/* Library version string ("major.minor.patch"). */
const char* cpca_version(void);

/* Message describing the last failure on the calling thread ("" if none). */
const char* cpca_last_error(void);

/*
 * Create a handle bound to the current HIP device and to `hip_stream`
 * (a hipStream_t; NULL means the legacy default stream). The handle owns all
 * workspace; it grows on demand and is released by cpca_destroy.
 * Errors: EINVAL (h == NULL), EHIP, ENOMEM.
 */
cpca_status cpca_create(cpca_handle* h, void* hip_stream);
cpca_status cpca_destroy(cpca_handle h);

/* Re-bind the handle to another stream of the same device. */
cpca_status cpca_set_stream(cpca_handle h, void* hip_stream);

/*
 * FRPCAG on the sampled matrix by FISTA (Section IV.B, Algorithm 1):
 *
 *   min_X ||Y~ - X||_1 + gamma_c tr(X L~_c X^T) + gamma_r tr(X^T L~_r X)
 *
 * Ytil        rho_r x rho_c input (double for FP64, float otherwise).
 * Lr_til      rho_r x rho_r Laplacian; Lc_til rho_c x rho_c Laplacian.
 * gamma_r/_c  >= 0 and finite.
 * lmax_r/_c   spectral norms ||L~_r||_2, ||L~_c||_2 (largest eigenvalues),
 *             finite. The step is 1/beta' with
 *             beta' = 2 gamma_c lmax_c + 2 gamma_r lmax_r; beta' = 0 returns Y~.
 *             A value <= 0 where the matching gamma is > 0 makes the library
 *             estimate that norm itself, as cpca_laplacian_lmax does with
 *             tol 1e-9 and at most 50000 products (the paper leaves the
 *             method open; such runs are outside the parity contract,
 *             which passes the exact values).
 * max_iter    J >= 0. eps >= 0: stop after iteration j when
 *             ||Z_{j+1} - Z_j||_F^2 < eps ||Z_j||_F^2; eps = 0 runs exactly J
 *             iterations.
 * Xtil_out    rho_r x rho_c output: the last prox iterate S_j.
 * The iteration state is FP64 in every mode (the FP32 modes only convert the
 * input and the output).
 * Returns OK (also when J iterations ran with eps > 0 unmet), EINVAL, ENAN,
 * EHIP, ENOMEM.
 */
cpca_status cpca_frpcag(cpca_handle h, cpca_mode mode,
                        const void* Ytil, int64_t rho_r, int64_t rho_c,
                        const cpca_csr* Lr_til, const cpca_csr* Lc_til,
                        double gamma_r, double gamma_c,
                        double lmax_r, double lmax_c,
                        int32_t max_iter, double eps,
                        void* Xtil_out, cpca_info* info);

/*
 * Largest eigenvalue of a symmetric positive semi-definite CSR matrix (a
 * graph Laplacian), i.e. its spectral norm, which sets the FISTA step of
 * Section IV.B. FP64 power iteration on the device from a fixed
 * pseudo-random positive start vector: w = L v, theta = <v, w> with
 * ||v|| = 1, stop when ||w - theta v|| <= tol * theta (an eigenvalue then
 * lies within tol * theta of theta) or after max_iter products.
 * L           square CSR in device memory (structure checked as everywhere).
 * tol         in (0, 1); max_iter >= 1.
 * lmax        host pointer, receives theta (also on ENOCONV).
 * info        iters = products run, rel_residual = ||w - theta v|| / theta.
 * The estimate approaches the largest eigenvalue from below; a start vector
 * orthogonal to its eigenvector (probability zero) would give another one.
 * Returns OK, ENOCONV (max_iter reached first), EINVAL, ENAN, EHIP, ENOMEM.
 */
cpca_status cpca_laplacian_lmax(cpca_handle h, const cpca_csr* L, double tol,
                                int32_t max_iter, double* lmax, cpca_info* info);

/*
 * K-nearest-neighbour graph Laplacian of a point set (Section II: each point
 * is joined to its K nearest neighbours in Euclidean distance; the
 * symmetric adjacency carries W_ij = exp(-||y_i - y_j||^2 / sigma^2) on every
 * pair related in either direction; L = D - W, or D^{-1/2} (D - W) D^{-1/2}
 * when normalized; Section VII-A takes K = 10 and sets sigma from the mean
 * K-NN distance).
 * points      N x d row-major FP64 (device): row i is y_i (a row or column
 *             of the data matrix, or any feature vector).
 * K           1 <= K <= min(28, N - 1).
 * normalized  1: L_n (unit diagonal), 0: combinatorial L.
 * rowptr_out  N + 1 int32 (device); colind_out / vals_out hold at least
 *             nnz_cap >= N (2K + 1) entries (device); the CSR rows are sorted
 *             by column and store the diagonal; *nnz_out (host) receives the
 *             number used (N + N K + the entries added by the union).
 * sigma_out   host: the mean Euclidean distance over the N K neighbour pairs.
 * knn_out     optional N x K int32 (device): the neighbours of each point by
 *             (squared distance, index), or NULL.
 * Readings: a point is not its own neighbour; equal distances are ordered by
 * index; sigma is the mean K-NN distance itself. Candidates are selected with
 * squared distances from FP64 MFMA Gram tiles (||y_i||^2 + ||y_j||^2 -
 * 2 <y_i, y_j>); the K kept ones are re-ranked with squared distances summed
 * directly over coordinates in FP64, which are also the ones weighted.
 * Returns OK, EINVAL (also when sigma = 0: every neighbour distance is zero;
 * nothing is written then), ENAN (NaN or Inf in the points), EHIP, ENOMEM.
 */
cpca_status cpca_knn_graph(cpca_handle h, const double* points, int64_t N, int64_t d,
                           int32_t K, int32_t normalized, int32_t* rowptr_out,
                           int32_t* colind_out, double* vals_out, int64_t nnz_cap,
                           int64_t* nnz_out, double* sigma_out, int32_t* knn_out,
                           cpca_info* info);

/*
 * Kron reduction of a graph Laplacian onto sampled nodes (Section IV-A,
 * graphs for compressed data):
 *   L~ = L(Omega, Omega) - L(Omega, Omega-bar) L(Omega-bar, Omega-bar)^-1 L(Omega-bar, Omega).
 * It equals the sampled rows of L S, where S upsamples the unit vectors on
 * Omega (S = I there, -L(bar, bar)^-1 L(bar, Omega) elsewhere); S is solved
 * by the upsampling PCG of cpca_approx_decode, 64 columns at a time, each
 * column to ||r|| <= tol ||b||. A component of the unsampled subgraph with no
 * edge to Omega contributes nothing. The result is symmetrised,
 * (L~ + L~^T) / 2, and is generally dense (the paper notes the fill-in).
 * L           n x n symmetric PSD Laplacian (device CSR, FP64 values).
 * omega       rho distinct int32 node indices (device); rows and columns of
 *             the output follow this order.
 * rho         1 <= rho <= min(n, 65536).
 * tol > 0, max_iter >= 0: per-column CG stop and cap.
 * Lred_out    rho x rho row-major FP64 (device).
 * info        iters = largest CG iteration count, rel_residual = largest
 *             final per-column recursive residual.
 * Returns OK, EINVAL, ENOCONV (cap reached; the output is written), ENOTSPD,
 * ENAN, EHIP, ENOMEM.
 */
cpca_status cpca_kron_reduce(cpca_handle h, const cpca_csr* L, const int32_t* omega,
                             int64_t rho, double tol, int32_t max_iter,
                             double* Lred_out, cpca_info* info);

/*
 * Alternate decoder (Section V.B, eq. alternatedecoder) solved by conjugate
 * gradient on its normal equations
 *
 *   (m_r m_c^T) o X + gamma_r L_r X + gamma_c X L_c = M_r^T X~ M_c^T,
 *
 * where m_r / m_c are the 0/1 indicators of Omega_r / Omega_c.
 * From 2^20 entries on (environment CPCA_PRECOND=1: at every size, =0:
 * never) CG is preconditioned by a two-level aggregation coarse space (row
 * aggregates of L_r times ranges of 64 columns; the coarse operator is built
 * and inverted on the device on the first call for an operator and gamma
 * pair, then reused) plus a weighted Jacobi part. The solution is the same; info.iters counts the
 * preconditioned iterations. Operators that are singular (a gamma of 0, a
 * connected component of either graph without a sampled node) are solved by
 * plain CG.
 * Xtil        rho_r x rho_c (row a, column b belongs at (omega_r[a], omega_c[b])).
 * omega_r/_c  rho_r / rho_c distinct int32 indices in [0, p) / [0, n).
 * Lr, Lc      p x p and n x n Laplacians; gamma_r/_c >= 0 and finite.
 * tol         > 0: stop when ||B - A(X)||_F <= tol ||B||_F, measured on the CG
 *             recursive residual (FP64 and FP32 modes) or on the true FP64
 *             residual computed at each replacement (FP32_IR).
 *             info.rel_residual always reports the true FP64 residual of the
 *             returned X.
 * max_iter    > 0: cap on CG iterations (FP32_IR: in total, with at most 40
 *             residual replacements).
 * X0          optional p x n warm start (NULL: zero).
 * X_out       p x n solution.
 * Returns OK, EINVAL, ENOCONV, ENOTSPD (gamma = 0 with partial sampling can
 * make A singular; CG from zero still returns the minimum-norm solution when
 * the right-hand side is consistent), ENAN, EHIP, ENOMEM.
 */
cpca_status cpca_decode(cpca_handle h, cpca_mode mode,
                        const void* Xtil, int64_t rho_r, int64_t rho_c,
                        const int32_t* omega_r, const int32_t* omega_c,
                        int64_t p, int64_t n,
                        const cpca_csr* Lr, const cpca_csr* Lc,
                        double gamma_r, double gamma_c,
                        double tol, int32_t max_iter,
                        const void* X0, void* X_out, cpca_info* info);

/*
 * Adjoint of cpca_decode. Given G = dl/dX at the decoder solution X, solves
 * A Lambda = G (A is symmetric) with the same solver and returns
 *   dXtil_out = Lambda[Omega_r, Omega_c]            (rho_r x rho_c),
 *   *dgamma_r = -<Lambda, L_r X>,  *dgamma_c = -<Lambda, X L_c>   (FP64),
 * which follow from differentiating A(gamma) X = M_r^T X~ M_c^T.
 * G, X: p x n device arrays of the mode's type; dgamma_r/_c: host pointers.
 */
cpca_status cpca_decode_backward(cpca_handle h, cpca_mode mode,
                                 const void* G, const void* X,
                                 int64_t rho_r, int64_t rho_c,
                                 const int32_t* omega_r, const int32_t* omega_c,
                                 int64_t p, int64_t n,
                                 const cpca_csr* Lr, const cpca_csr* Lc,
                                 double gamma_r, double gamma_c,
                                 double tol, int32_t max_iter,
                                 void* dXtil_out, double* dgamma_r,
                                 double* dgamma_c, cpca_info* info);

/*
 * Subspace-upsampling approximate decoder (Section V.C, Algorithm 2). With
 * the thin SVD X~ = U~ S~ V~^T (singular values descending):
 *   1. k = the number of singular values >= sigma_ratio * S~[0] that are
 *      positive (the paper takes sigma_ratio = 0.1), at most k_max;
 *   2. each kept column u~ of U~ is upsampled over L_r (and each v~ of V~
 *      over L_c) as min u^T L u subject to u[omega] = u~ (eq. approx_uv),
 *      whose solution (the graph-upsampling lemma) keeps u~ on omega and
 *      solves L(omega-bar, omega-bar) u = -L(omega-bar, omega) u~ on the rest
 *      (Jacobi-preconditioned CG per column, FP64);
 *   3. the upsampled columns are normalised to unit norm, the singular values
 *      scaled by sqrt(n p / (rho_r rho_c (1 - delta))), and
 *      X = U diag(scaled S~[:k]) V^T is written.
 * The SVD (one-sided Jacobi), the CG and all scalars are FP64 in every mode;
 * the FP32 modes convert the input and round the output.
 * Xtil        rho_r x rho_c (row a, column b belongs at (omega_r[a], omega_c[b])),
 *             min(rho_r, rho_c) <= 4096.
 * omega_r/_c  rho_r / rho_c distinct int32 indices in [0, p) / [0, n).
 * Lr, Lc      p x p and n x n Laplacians (symmetric PSD; values used in
 *             place on the device). Where a connected component of the
 *             unsampled nodes has no edge to a sampled node, its rows get the
 *             minimum-norm value 0.
 * delta       RIP constant in [0, 1).
 * sigma_ratio in [0, 1]; k_max in [1, 64].
 * tol         > 0: per-column CG stop ||r|| <= tol ||b|| (recursive residual).
 * max_iter    >= 0: cap on CG iterations (both graphs run together).
 * X_out       p x n output (mode type). sigma_out: optional HOST array of
 *             min(rho_r, rho_c) doubles receiving all singular values of X~,
 *             descending.
 * X is unique when the kept singular values are distinct (the sign of each
 * singular pair cancels).
 * Returns OK, EINVAL, ENOCONV (CG cap reached or the SVD did not converge in
 * 40 sweeps; X is written either way), ENOTSPD, ENAN, EHIP, ENOMEM.
 */
typedef struct {
  int32_t k;               /* kept singular values                           */
  int32_t svd_sweeps;      /* Jacobi sweeps run                              */
  int32_t iters_r;         /* CG iterations, row graph (largest column)      */
  int32_t iters_c;         /* CG iterations, column graph                    */
  int32_t status;          /* same value as the call's return code           */
  int32_t reserved;
  double rel_residual_r;   /* largest per-column ||r|| / ||b||, row graph    */
  double rel_residual_c;   /* same, column graph                             */
  double scale;            /* sqrt(n p / (rho_r rho_c (1 - delta)))          */
  double ms;               /* wall time of the call                          */
} cpca_approx_info;

cpca_status cpca_approx_decode(cpca_handle h, cpca_mode mode,
                               const void* Xtil, int64_t rho_r, int64_t rho_c,
                               const int32_t* omega_r, const int32_t* omega_c,
                               int64_t p, int64_t n,
                               const cpca_csr* Lr, const cpca_csr* Lc,
                               double delta, double sigma_ratio, int32_t k_max,
                               double tol, int32_t max_iter,
                               void* X_out, double* sigma_out,
                               cpca_approx_info* info);

/*
 * Approximate decoders 2 and 3 (appendix, other approximate decoders): with
 * the full data matrix Y available, only one subspace is upsampled.
 *   decoder 2 (cpca_approx_decode2): the kept left singular vectors of X~
 *     (k as in cpca_approx_decode) are upsampled over L_r and normalised to
 *     unit columns U; X = U U^T Y.
 *   decoder 3 (cpca_approx_decode3): the kept right singular vectors are
 *     upsampled over L_c and normalised to V; X = Y V V^T.
 * The paper writes these as X = U S~ s V^T with V = Y^T U S~^-1 / s (and the
 * mirror image); the RIP scale s cancels, so delta is not an argument.
 * Xtil        rho_r x rho_c (mode type), min(rho_r, rho_c) <= 4096.
 * omega_r/_c  the sampled rows (decoder 2) or columns (decoder 3), distinct.
 * Lr / Lc     the p x p or n x n Laplacian of that side (device, FP64 values).
 * Y           p x n full data (mode type, device).
 * sigma_ratio in [0, 1]; k_max in [1, 16].
 * tol, max_iter, X_out, sigma_out as in cpca_approx_decode; info reports the
 * upsampled side's CG iterations and residuals (the other side's are 0) and
 * scale = 1.
 * The SVD, the CG and the projections accumulate in FP64; Y is read once and
 * X written once (two streaming passes plus partial sums of p x k or k x n).
 * Returns OK, EINVAL, ENOCONV, ENOTSPD, ENAN, EHIP, ENOMEM.
 */
cpca_status cpca_approx_decode2(cpca_handle h, cpca_mode mode,
                                const void* Xtil, int64_t rho_r, int64_t rho_c,
                                const int32_t* omega_r, int64_t p, int64_t n,
                                const cpca_csr* Lr, const void* Y,
                                double sigma_ratio, int32_t k_max, double tol,
                                int32_t max_iter, void* X_out, double* sigma_out,
                                cpca_approx_info* info);
cpca_status cpca_approx_decode3(cpca_handle h, cpca_mode mode,
                                const void* Xtil, int64_t rho_r, int64_t rho_c,
                                const int32_t* omega_c, int64_t p, int64_t n,
                                const cpca_csr* Lc, const void* Y,
                                double sigma_ratio, int32_t k_max, double tol,
                                int32_t max_iter, void* X_out, double* sigma_out,
                                cpca_approx_info* info);

/*
 * Approximate decoder for clustering (Section VI, Algorithm 3). The rho_c
 * columns of X~ are the sampled points (dimension rho_r):
 *   1. k-means (Lloyd) from the k seed points init[0..k): assign each point
 *      to the nearest centroid in squared Euclidean distance (ties to the
 *      lower index), move each centroid to the mean of its points (an empty
 *      cluster keeps its centroid), until no assignment changes or after
 *      kmeans_max_iter updates;
 *   2. each cluster indicator column is upsampled over L_c as
 *      min c^T L_c c subject to c[omega_c] = c~ (eq. approx_c): the graph-
 *      upsampling lemma, solved by Jacobi-preconditioned CG per column (FP64);
 *   3. max pooling: sample i gets the column of its largest C[i, j] (ties to
 *      the lower index).
 * k-means, the CG and C are FP64 in every mode; the mode sets X~'s type.
 * Xtil        rho_r x rho_c (column b is sample omega_c[b]).
 * omega_c     rho_c distinct int32 indices in [0, n) (device).
 * Lc          n x n Laplacian (symmetric PSD, used in place on the device).
 *             Rows of a component with no sample get C = 0 (label 0).
 * k           clusters, in [1, 64] and <= rho_c.
 * init        k distinct int32 positions in [0, rho_c) (device): the seeds.
 * kmeans_max_iter >= 0; tol > 0 (per-column ||r|| <= tol ||b||); max_iter >= 0.
 * labels_out  n int32 cluster labels (device).
 * C_out       optional n x k FP64 upsampled indicators (device), or NULL.
 * sample_labels_out  optional rho_c int32 k-means labels (device), or NULL.
 * Returns OK, EINVAL, ENOCONV (CG cap; outputs are written either way),
 * ENOTSPD, ENAN, EHIP, ENOMEM.
 */
typedef struct {
  int32_t kmeans_iters;    /* centroid updates run                           */
  int32_t cg_iters;        /* CG iterations (largest column)                 */
  int32_t status;          /* same value as the call's return code           */
  int32_t reserved;
  double rel_residual;     /* largest per-column ||r|| / ||b||               */
  double ms;               /* wall time of the call                          */
} cpca_cluster_info;

cpca_status cpca_cluster_decode(cpca_handle h, cpca_mode mode,
                                const void* Xtil, int64_t rho_r, int64_t rho_c,
                                const int32_t* omega_c, int64_t n,
                                const cpca_csr* Lc, int32_t k, const int32_t* init,
                                int32_t kmeans_max_iter, double tol, int32_t max_iter,
                                int32_t* labels_out, double* C_out,
                                int32_t* sample_labels_out, cpca_cluster_info* info);

/*
 * One application of the decoder operator (the fused two-sided sparse
 * product of eq. alternatedecoder's normal equations):
 *   Q = (m_r m_c^T) o P + gamma_r L_r P + gamma_c P L_c,  *pq = <P, Q> (FP64).
 * With rho_r = rho_c = 0 (omega pointers may then be NULL) the mask term is
 * zero. P, Q: p x n of the mode's type (FP32_IR behaves as FP32). pq may be
 * NULL.
 */
cpca_status cpca_apply(cpca_handle h, cpca_mode mode, const void* P, void* Q,
                       int64_t p, int64_t n,
                       const int32_t* omega_r, int64_t rho_r,
                       const int32_t* omega_c, int64_t rho_c,
                       const cpca_csr* Lr, const cpca_csr* Lc,
                       double gamma_r, double gamma_c, double* pq);

/*
 * cpca_apply without device memory allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, result and kernels as cpca_apply; the
 * staged operator image (L_r, L_c in the kernel layouts, masks, row-panel
 * tables) and the partial sums go to a static device array of 32 MiB per
 * GPU (held from the first cpca_create on that GPU until the process ends)
 * instead of the handle's workspace, which is neither used nor grown.
 * Nothing in the array has to start at zero: each call overwrites the image
 * and every partial it reads. All handles on one GPU share the array, so
 * calls that overlap on one GPU (several host threads or streams) race and
 * must be serialised by the caller. Host memory for the staging is still
 * taken from the C++ heap; no device or pinned allocation is made, and
 * profiling events are not recorded for this call.
 * Errors as cpca_apply, plus EINVAL when the operator image and partial sums
 * need more than 32 MiB (for example about 2.5 M non-zeros of L_r in FP64);
 * the message states both sizes.
 */
cpca_status cpca_apply_noalloc(cpca_handle h, cpca_mode mode, const void* P, void* Q,
                               int64_t p, int64_t n,
                               const int32_t* omega_r, int64_t rho_r,
                               const int32_t* omega_c, int64_t rho_c,
                               const cpca_csr* Lr, const cpca_csr* Lc,
                               double gamma_r, double gamma_c, double* pq);

/*
 * Host-side structural checks, exposed so that they can be exercised
 * without a GPU. Pointers are HOST memory here.
 *   cpca_check_csr_host: rowptr monotone with rowptr[0] = 0 and
 *     rowptr[n] = nnz, every column index in [0, n), every value finite
 *     (vals may be NULL to skip the value check).
 *   cpca_check_index_set_host: `count` distinct indices in [0, dim).
 * Return OK or EINVAL (message in cpca_last_error).
 */
cpca_status cpca_check_csr_host(int64_t n, int64_t nnz, const int32_t* rowptr,
                                const int32_t* colind, const double* vals);
cpca_status cpca_check_index_set_host(int64_t count, int64_t dim,
                                      const int32_t* idx);

/*
 * Per-kernel timing with HIP events recorded on the handle's stream around
 * every launch of the named kernel family. Families: "apply" (the fused
 * two-sided sparse product with the CG epilogue), "update" (the CG x/r
 * update), "fista" (the fused FISTA step), "other" (the fused product with
 * any other epilogue: residual, objective, adjoint dots, plain apply),
 * "rankk" (the rank-k output product of cpca_approx_decode); with the
 * coarse-level preconditioner "update" is the r update with the coarse
 * partial sums, "pupdate" the x/p update and "coarse" the three small
 * coarse-level launches of an iteration, timed as one span.
 * Enabling resets the counters.
 * cpca_get_profile returns the number of timed launches and their summed
 * duration in milliseconds.
 */
cpca_status cpca_set_profiling(cpca_handle h, int32_t enable);
cpca_status cpca_get_profile(cpca_handle h, const char* family,
                             int64_t* launches, double* total_ms);

/*
 * Launch shape of the fused two-sided product on this handle:
 * rows_per_block in {-1, 0, 1, 2, 4, 8}: 0 = built-in default, -1 = autotune
 * (each new shape is timed over the candidate shapes on the first solve and
 * the fastest is kept in the handle; with the environment variable
 * CPCA_TUNE_CACHE naming a file, choices are also appended to it and read
 * back by cpca_create). use_lds in {-1, 0, 1}: -1 = automatic, 1 = stage the
 * workgroup's rows in LDS when they fit in 64 KiB, 0 = gather the X L_c
 * operands from global memory. kernel in {-1, 0, 1, 2, 3} is the preference
 * for a banded L_c (most entries within 8 or 16 of the diagonal): -1 =
 * automatic (row panels where L_r rows hold at most 16 off-diagonal entries,
 * else column strips; for bands up to 8 wide the panel variant of 3), 0 = row
 * kernel, 1 = column strips, 2 = row panels that prefetch the next panel into
 * registers (two waves per SIMD; falls back to column strips when a row of
 * L_r is too long), 3 = row panels that load each panel just before staging
 * it (three waves per SIMD, bands up to 8 wide; the autotuner times both).
 * Shapes differ only in the
 * order in which an output's terms are summed (the row-panel kernel adds the
 * diagonal of L_r first) and in the grid-level reduction order of the CG
 * scalars; every shape is deterministic run to run.
 */
cpca_status cpca_set_apply_config(cpca_handle h, int32_t rows_per_block, int32_t use_lds,
                                  int32_t kernel);

/*
 * Batched solves (many instances of uneven sizes, each swept over several
 * (gamma_r, gamma_c) pairs): for every task, FISTA on the instance's sampled
 * matrix (Algorithm 1, fista_iters iterations, eps = 0) followed by the
 * alternate decoder on its full graphs, both with the task's gammas. In
 * FP32 modes the sampled estimate X~ is rounded to float between the two
 * stages, exactly as a cpca_frpcag call followed by cpca_decode would do.
 *
 * All tasks are resident on the device together and advance through
 * batched kernels (one launch covers every task); FISTA and chunks of CG
 * iterations are captured as HIP graphs and replayed until every task has
 * converged. Memory: about (5 FP64 + 4 FP32) words per decoded entry in
 * FP32_IR mode, summed over tasks.
 *
 * instances   n_instances descriptors; all pointers are device memory with
 *             the same conventions as cpca_frpcag / cpca_decode.
 * tasks       n_tasks descriptors: instance index, gammas (>= 0), X_out
 *             (p x n, required) and Xtil_out (rho_r x rho_c, may be NULL).
 * tol, max_iter  as in cpca_decode (per task).
 * infos       optional host array of n_tasks results.
 * Returns OK when every task converged; otherwise the first error status
 * among the tasks (ENOCONV if that is the only problem). Outputs are written
 * for every task either way.
 */
typedef struct {
  int64_t p, n;                 /* full matrix size                           */
  int64_t rho_r, rho_c;         /* sample counts                              */
  const int32_t* omega_r;       /* sampled rows, distinct, in [0, p)          */
  const int32_t* omega_c;       /* sampled columns, distinct, in [0, n)       */
  const cpca_csr* Lr;           /* p x p Laplacian                            */
  const cpca_csr* Lc;           /* n x n Laplacian                            */
  const cpca_csr* Lr_til;       /* rho_r x rho_r Laplacian of sampled rows    */
  const cpca_csr* Lc_til;       /* rho_c x rho_c Laplacian of sampled columns */
  double lmax_r_til, lmax_c_til;/* their largest eigenvalues (finite; <= 0:    */
                                /* estimated on the device, as in cpca_frpcag) */
  const void* Ytil;             /* rho_r x rho_c sampled data                 */
} cpca_instance;

typedef struct {
  int32_t instance;             /* index into the instance array              */
  int32_t reserved;
  double gamma_r, gamma_c;      /* used by FISTA and by the decoder           */
  void* X_out;                  /* p x n decoded matrix (mode dtype)          */
  void* Xtil_out;               /* rho_r x rho_c FISTA output or NULL         */
} cpca_task;

cpca_status cpca_solve_batched(cpca_handle h, cpca_mode mode,
                               const cpca_instance* instances, int32_t n_instances,
                               const cpca_task* tasks, int32_t n_tasks,
                               int32_t fista_iters, double tol, int32_t max_iter,
                               cpca_info* infos);

#ifdef __cplusplus
}
#endif

#endif /* CPCA_H */
