// The approximate decoders on gfx950: cpca_approx_decode (subspace
// upsampling, Algorithm 2, Section V-C) and cpca_cluster_decode (clustering,
// Algorithm 3, Section VI: k-means on the columns of X~, the same
// upsampling CG on the cluster indicators over L_c, max pooling).
//
// Algorithm 2:
//   1. Thin SVD of X~ by one-sided (Hestenes) Jacobi: the rows of
//      W = X~^T (rho_r >= rho_c) or W = X~ (rho_r < rho_c) are orthogonalised
//      pairwise, in round-robin order (every round rotates m/2 disjoint
//      pairs, one workgroup per pair; m - 1 rounds make a sweep, captured as
//      one HIP graph and replayed until a sweep rotates nothing). The same
//      rotations applied to the identity give the other singular vectors.
//   2. k = the number of singular values >= ratio * sigma_max (positive,
//      at most k_max), chosen on the device with the order of the values.
//   3. Graph upsampling of the k kept left vectors over L_r and right
//      vectors over L_c: the lemma of Section V-C gives the unknown rows as
//      the solution of L(omega-bar, omega-bar) u = -L(omega-bar, omega) u~,
//      solved by Jacobi-preconditioned CG, one independent CG per column,
//      both graphs in the same launches, chunks of iterations as HIP graphs.
//   4.-6. Column norms, the RIP scale sqrt(n p / (rho_r rho_c (1 - delta)))
//      and X = U S V^T as one rank-k product that streams X to HBM.
//
// Everything before the last step works on small arrays and is latency
// bound; the last step writes the p x n output once and is HBM bound.
#include "common.hpp"

namespace {

constexpr int kApproxKMax = 64;       // largest k (columns per row in the CG layout)
constexpr int kMaxSweeps = 40;        // Jacobi sweeps before giving up
constexpr int kUpChunk = 16;          // CG iterations per graph replay
constexpr int kUpMaxBlocks = 4096;    // workgroups per graph side in the streaming CG kernels
constexpr int kSvdMaxM = 4096;        // min(rho_r, rho_c) held in LDS by the rank kernel

// ------------------------------------------------------------ block sums
// Sum of NV values over the workgroup (kThreads threads); every thread gets
// the totals.
template <int NV>
__device__ void block_sum(double (&v)[NV]) {
  __shared__ double red[NV][kMaxWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[k][wid] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < kMaxWaves; ++w) s += red[k][w];
    v[k] = s;
  }
  __syncthreads();
}

// Per-column sums over a workgroup whose thread t holds column t % KP (KP a
// power of two <= 64): a fixed-order tree in LDS, so results do not depend
// on timing. On return red[c] holds the sum of column c (c < KP).
__device__ void column_tree(double* red, int KP) {
  for (int s = kThreads / 2; s >= KP; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
  }
  __syncthreads();
}

// ------------------------------------------------------------- SVD kernels
// W (m x len) from X~ (rho_r x rho_c, row-major, type TI): W = X~^T when
// trans, else X~. Q = I (m x m).
template <typename TI>
__global__ void __launch_bounds__(kThreads)
k_jac_load(double* __restrict__ W, double* __restrict__ Q, const TI* __restrict__ Xt, int rho_r,
           int rho_c, int trans, int m) {
  const size_t N = (size_t)rho_r * rho_c;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const size_t i = e / rho_c, j = e - i * rho_c;
    const double v = (double)Xt[e];
    if (trans) W[j * rho_r + i] = v;
    else W[e] = v;
  }
  const size_t M2 = (size_t)m * m;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < M2; e += stride)
    Q[e] = (e / m == e % m) ? 1.0 : 0.0;
}

// ||W||_F^2 (one workgroup); rotations leave it unchanged.
__global__ void __launch_bounds__(kThreads)
k_jac_fro(const double* __restrict__ W, size_t N, double* __restrict__ fro2) {
  double s[1] = {0.0};
  for (size_t e = threadIdx.x; e < N; e += kThreads) s[0] += W[e] * W[e];
  block_sum<1>(s);
  if (threadIdx.x == 0) fro2[0] = s[0];
}

// One round of one-sided Jacobi: workgroup b rotates the pair of rows
// pairs[b] of W (length len) so that they become orthogonal, and applies the
// same rotation to the rows of Q (length m). Pairs whose normalised inner
// product is at most tol are left alone, and so are rows whose squared norm
// is at most floor_rel * ||W||_F^2: those are rounding noise of a
// rank-deficient X~, and rotating them against each other would never stop.
// count gathers the rotations done.
__global__ void __launch_bounds__(kThreads)
k_jac_round(double* __restrict__ W, double* __restrict__ Q, int m, int len,
            const int2* __restrict__ pairs, double tol, const double* __restrict__ fro2,
            double floor_rel, int* __restrict__ count) {
  const int2 pr = pairs[blockIdx.x];
  if (pr.x >= m || pr.y >= m) return;  // the idle slot of an odd m
  double* wa = W + (size_t)pr.x * len;
  double* wb = W + (size_t)pr.y * len;
  double s[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < len; i += kThreads) {
    const double x = wa[i], y = wb[i];
    s[0] += x * x;
    s[1] += y * y;
    s[2] += x * y;
  }
  block_sum<3>(s);
  const double al = s[0], be = s[1], ga = s[2];
  const double floor2 = floor_rel * fro2[0];
  if (!(al > floor2 && be > floor2 && fabs(ga) > tol * sqrt(al) * sqrt(be))) return;
  // t = tan(theta), the smaller root of t^2 + 2 zeta t - 1 = 0, makes the
  // rotated rows orthogonal: (c wa - s wb) . (s wa + c wb) = 0
  const double zeta = (be - al) / (2.0 * ga);
  const double az = fabs(zeta);
  const double t = copysign(1.0 / (az + (az < 1e150 ? sqrt(1.0 + az * az) : az)), zeta);
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double sn = c * t;
  for (int i = threadIdx.x; i < len; i += kThreads) {
    const double x = wa[i], y = wb[i];
    wa[i] = c * x - sn * y;
    wb[i] = sn * x + c * y;
  }
  double* qa = Q + (size_t)pr.x * m;
  double* qb = Q + (size_t)pr.y * m;
  for (int i = threadIdx.x; i < m; i += kThreads) {
    const double x = qa[i], y = qb[i];
    qa[i] = c * x - sn * y;
    qb[i] = sn * x + c * y;
  }
  if (threadIdx.x == 0) atomicAdd(count, 1);
}

// The same round with both rows of W and of Q held in registers (EPT
// elements per thread, len <= EPT * kThreads): every load is issued before
// the first reduction, and the rotation works on the registers.
template <int EPT>
__global__ void __launch_bounds__(kThreads)
k_jac_round_reg(double* __restrict__ W, double* __restrict__ Q, int m, int len,
                const int2* __restrict__ pairs, double tol, const double* __restrict__ fro2,
                double floor_rel, int* __restrict__ count) {
  const int2 pr = pairs[blockIdx.x];
  if (pr.x >= m || pr.y >= m) return;
  double* wa = W + (size_t)pr.x * len;
  double* wb = W + (size_t)pr.y * len;
  double* qa = Q + (size_t)pr.x * m;
  double* qb = Q + (size_t)pr.y * m;
  double xa[EPT], xb[EPT], ya[EPT], yb[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = (int)threadIdx.x + e * kThreads;
    xa[e] = i < len ? wa[i] : 0.0;
    xb[e] = i < len ? wb[i] : 0.0;
    ya[e] = i < m ? qa[i] : 0.0;
    yb[e] = i < m ? qb[i] : 0.0;
  }
  double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    s[0] += xa[e] * xa[e];
    s[1] += xb[e] * xb[e];
    s[2] += xa[e] * xb[e];
  }
  block_sum<3>(s);
  const double al = s[0], be = s[1], ga = s[2];
  const double floor2 = floor_rel * fro2[0];
  if (!(al > floor2 && be > floor2 && fabs(ga) > tol * sqrt(al) * sqrt(be))) return;
  const double zeta = (be - al) / (2.0 * ga);
  const double az = fabs(zeta);
  const double t = copysign(1.0 / (az + (az < 1e150 ? sqrt(1.0 + az * az) : az)), zeta);
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double sn = c * t;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = (int)threadIdx.x + e * kThreads;
    if (i < len) {
      wa[i] = c * xa[e] - sn * xb[e];
      wb[i] = sn * xa[e] + c * xb[e];
    }
    if (i < m) {
      qa[i] = c * ya[e] - sn * yb[e];
      qb[i] = sn * ya[e] + c * yb[e];
    }
  }
  if (threadIdx.x == 0) atomicAdd(count, 1);
}

__global__ void k_zero_int(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// One workgroup: sigma_j = ||W_j||, their descending order (ties by index),
// and k. Outputs: sig[r] = r-th largest value, perm[r] = its row of W,
// kout[0] = k.
__global__ void __launch_bounds__(kThreads)
k_svd_rank(const double* __restrict__ W, int m, int len, double ratio, int kmax,
           double* __restrict__ sig, int* __restrict__ perm, int* __restrict__ kout) {
  __shared__ double sg[kSvdMaxM];
  __shared__ int kc;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  for (int j = wid; j < m; j += kMaxWaves) {
    const double* w = W + (size_t)j * len;
    double s = 0.0;
    for (int i = lane; i < len; i += kWave) s += w[i] * w[i];
    s = wave_sum(s);
    // NaN is ordered below every value, so the ranks below always form a
    // permutation
    if (lane == 0) sg[j] = s == s ? sqrt(s) : -1.0;
  }
  if (threadIdx.x == 0) kc = 0;
  __syncthreads();
  double mx = 0.0;
  for (int j = 0; j < m; ++j) mx = fmax(mx, sg[j]);
  int cnt = 0;
  for (int j = threadIdx.x; j < m; j += kThreads) {
    const double v = sg[j];
    int r = 0;
    for (int i = 0; i < m; ++i) r += (sg[i] > v || (sg[i] == v && i < j)) ? 1 : 0;
    sig[r] = v;
    perm[r] = j;
    cnt += (v > 0.0 && v >= ratio * mx) ? 1 : 0;
  }
  atomicAdd(&kc, cnt);
  __syncthreads();
  if (threadIdx.x == 0) kout[0] = min(kc, kmax);
}

// The k kept singular vectors in the CG layout (rows x KP, zero-padded):
// the long side (length len) from the rows of W divided by sigma, the short
// side (length m) from the rows of Q. lv/sv receive the long/short side.
__global__ void __launch_bounds__(kThreads)
k_svd_vectors(const double* __restrict__ W, const double* __restrict__ Q, int m, int len,
              const double* __restrict__ sig, const int* __restrict__ perm, int k, int KP,
              double* __restrict__ lv, double* __restrict__ sv) {
  const size_t NL = (size_t)len * KP, NS = (size_t)m * KP;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < NL + NS; e += stride) {
    if (e < NL) {
      const int i = (int)(e / KP), c = (int)(e % KP);
      lv[e] = c < k ? W[(size_t)perm[c] * len + i] / sig[c] : 0.0;
    } else {
      const size_t f = e - NL;
      const int i = (int)(f / KP), c = (int)(f % KP);
      sv[f] = c < k ? Q[(size_t)perm[c] * m + i] : 0.0;
    }
  }
}

// ------------------------------------------------------- upsampling by CG
// One graph side: the unknown rows (not sampled) of S solve
// L(unknown, unknown) x = -L(unknown, sampled) R column by column, one
// Jacobi-preconditioned CG per column. Vectors are c x KP row-major; the
// sampled rows of r, z, p and q stay zero. The streaming kernels (start,
// product, update, p-update) run on as many workgroups as the rows need and
// write per-workgroup partial sums of every column. A reduction kernel with
// one workgroup per (side, column) then sums them in a fixed order and takes
// every scalar decision of that column (alpha, beta, convergence,
// breakdown): each scalar has a single writer.
struct UpSide {
  const int32_t* rp = nullptr;   // CSR of the full c x c Laplacian (caller's, FP64)
  const int32_t* ci = nullptr;
  const double* v = nullptr;
  const double* dinv = nullptr;  // 1 / L_ii on unknown rows (1 where L_ii <= 0), 0 on sampled rows
  const int32_t* inv = nullptr;  // position in omega of a sampled row, -1 otherwise
  const double* R = nullptr;     // sampled values (rho x KP)
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double* S = nullptr;           // upsampled vectors (c x KP), the result
  double* pa = nullptr;          // KP x nb partials (product, norms)
  double* pb = nullptr;          // 2 x KP x nb partials (start, update)
  double* scal = nullptr;        // per column: rz, rr, bb, thr, alpha, beta (6 x kApproxKMax)
  int* state = nullptr;          // per column: done, iters (2 x kApproxKMax)
  int c = 0, nb = 0;
};

// scal / state layout
__device__ __forceinline__ double* s_rz(const UpSide& s) { return s.scal; }
__device__ __forceinline__ double* s_rr(const UpSide& s) { return s.scal + kApproxKMax; }
__device__ __forceinline__ double* s_bb(const UpSide& s) { return s.scal + 2 * kApproxKMax; }
__device__ __forceinline__ double* s_thr(const UpSide& s) { return s.scal + 3 * kApproxKMax; }
__device__ __forceinline__ double* s_alpha(const UpSide& s) { return s.scal + 4 * kApproxKMax; }
__device__ __forceinline__ double* s_beta(const UpSide& s) { return s.scal + 5 * kApproxKMax; }
__device__ __forceinline__ int* s_done(const UpSide& s) { return s.state; }
__device__ __forceinline__ int* s_iters(const UpSide& s) { return s.state + kApproxKMax; }

// The workgroup's side and its index within that side (streaming kernels).
__device__ __forceinline__ const UpSide& pick(const UpSide& a, const UpSide& b, int& local) {
  local = (int)blockIdx.x < a.nb ? (int)blockIdx.x : (int)blockIdx.x - a.nb;
  return (int)blockIdx.x < a.nb ? a : b;
}

// (L y)_row for the CG layout: sum over the CSR row of v * y[col, c].
__device__ __forceinline__ double lap_row(const UpSide& s, const double* __restrict__ y, int row,
                                          int c, int KP) {
  double acc = 0.0;
  const int e1 = s.rp[row + 1];
  for (int e = s.rp[row]; e < e1; ++e) acc += s.v[e] * y[(size_t)s.ci[e] * KP + c];
  return acc;
}

// Writes the workgroup's per-column sums of NV values per thread (thread t
// holds column t % KP) to part[g][c][lb], in a fixed-order LDS tree. The
// partials of one column are contiguous, so the reductions read them
// coalesced.
template <int NV>
__device__ void store_col_partials(const double (&acc)[NV], double* part, int lb, int nb, int KP) {
  __shared__ double red[NV][kThreads];
#pragma unroll
  for (int g = 0; g < NV; ++g) red[g][threadIdx.x] = acc[g];
  for (int st = kThreads / 2; st >= KP; st >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < st) {
#pragma unroll
      for (int g = 0; g < NV; ++g) red[g][threadIdx.x] += red[g][threadIdx.x + st];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < KP) {
#pragma unroll
    for (int g = 0; g < NV; ++g) part[((size_t)g * KP + threadIdx.x) * nb + lb] = red[g][threadIdx.x];
  }
}

// Column total of group g over the side's nb workgroups, summed by the whole
// workgroup in a fixed order (every thread receives it).
__device__ double col_sum(const double* part, int nb, int KP, int g, int c) {
  double t[1] = {0.0};
  const double* col = part + ((size_t)g * KP + c) * nb;
  for (int b = threadIdx.x; b < nb; b += kThreads) t[0] += col[b];
  block_sum<1>(t);
  return t[0];
}

// Per-column totals of every column at once (thread t receives the total of
// column t % KP); for the one-workgroup epilogue kernels.
__device__ double col_total(const double* part, int nb, int KP, int g, double* red) {
  const int c = threadIdx.x & (KP - 1);
  const int rpb = kThreads / KP;
  double s = 0.0;
  const double* col = part + ((size_t)g * KP + c) * nb;
  for (int b = (int)threadIdx.x / KP; b < nb; b += rpb) s += col[b];
  red[threadIdx.x] = s;
  column_tree(red, KP);
  const double t = red[c];
  __syncthreads();  // red is reused by the caller
  return t;
}

// Start: S = R on sampled rows (0 elsewhere), x = 0 (pass 0); b = -(L S) on
// unknown rows, r = b, z = D^-1 r, p = z, q = 0, partials <r, z>, <r, r>
// (pass 1).
__global__ void __launch_bounds__(kThreads)
k_up_start(UpSide a, UpSide b2, int KP, int pass) {
  int lb;
  const UpSide& s = pick(a, b2, lb);
  const int c = threadIdx.x & (KP - 1);
  const int rpb = kThreads / KP;
  double acc[2] = {0.0, 0.0};
  for (int row = lb * rpb + (int)threadIdx.x / KP; row < s.c; row += s.nb * rpb) {
    const size_t e = (size_t)row * KP + c;
    if (pass == 0) {
      const int pos = s.inv[row];
      s.S[e] = pos >= 0 ? s.R[(size_t)pos * KP + c] : 0.0;
      s.x[e] = 0.0;
    } else {
      const double bv = s.inv[row] >= 0 ? 0.0 : -lap_row(s, s.S, row, c, KP);
      const double zv = s.dinv[row] * bv;
      s.r[e] = bv;
      s.z[e] = zv;
      s.p[e] = zv;
      s.q[e] = 0.0;
      acc[0] += bv * zv;
      acc[1] += bv * bv;
    }
  }
  if (pass == 0) return;
  store_col_partials<2>(acc, s.pb, lb, s.nb, KP);
}

// One workgroup per (side, column): arm the scalars from the start partials.
// Columns past k, and columns with a zero right-hand side (x = 0), are done.
__global__ void __launch_bounds__(kThreads)
k_up_arm(UpSide a, UpSide b2, int KP, int k, double tol2) {
  const int side = blockIdx.x / KP, c = blockIdx.x % KP;
  const UpSide& s = side == 0 ? a : b2;
  const double rz = col_sum(s.pb, s.nb, KP, 0, c);
  const double rr = col_sum(s.pb, s.nb, KP, 1, c);
  if (threadIdx.x != 0) return;
  s_rz(s)[c] = rz;
  s_rr(s)[c] = rr;
  s_bb(s)[c] = rr;
  s_thr(s)[c] = tol2 * rr;
  s_iters(s)[c] = 0;
  s_done(s)[c] = (c >= k || !(rr > 0.0)) ? 1 : (bad(rr) || bad(rz) ? 3 : 0);
}

// q = (L p) on unknown rows of running columns; partials <p, q>.
__global__ void __launch_bounds__(kThreads)
k_up_apply(UpSide a, UpSide b2, int KP) {
  int lb;
  const UpSide& s = pick(a, b2, lb);
  const int c = threadIdx.x & (KP - 1);
  const int rpb = kThreads / KP;
  double acc[1] = {0.0};
  if (s_done(s)[c] == 0) {
    for (int row = lb * rpb + (int)threadIdx.x / KP; row < s.c; row += s.nb * rpb) {
      if (s.inv[row] >= 0) continue;  // sampled row: q stays 0
      const size_t e = (size_t)row * KP + c;
      const double qv = lap_row(s, s.p, row, c, KP);
      s.q[e] = qv;
      acc[0] += s.p[e] * qv;
    }
  }
  store_col_partials<1>(acc, s.pa, lb, s.nb, KP);
}

// One workgroup per (side, column): convergence of the previous iteration
// (<r, r> at most the threshold), breakdown (<p, q> not positive, or not
// finite), else alpha = <r, z> / <p, q>.
__global__ void __launch_bounds__(kThreads)
k_up_alpha(UpSide a, UpSide b2, int KP) {
  const int side = blockIdx.x / KP, c = blockIdx.x % KP;
  const UpSide& s = side == 0 ? a : b2;
  if (s_done(s)[c] != 0) return;  // uniform over the workgroup
  const double pq = col_sum(s.pa, s.nb, KP, 0, c);
  if (threadIdx.x != 0) return;
  if (s_rr(s)[c] <= s_thr(s)[c]) {
    s_done(s)[c] = 1;
  } else if (bad(pq) || !(pq > 0.0)) {
    s_done(s)[c] = bad(pq) ? 3 : 2;
  } else {
    s_alpha(s)[c] = s_rz(s)[c] / pq;
  }
}

// x += alpha p; r -= alpha q; z = D^-1 r on unknown rows of running columns;
// partials <r, z>, <r, r>.
__global__ void __launch_bounds__(kThreads)
k_up_update(UpSide a, UpSide b2, int KP) {
  int lb;
  const UpSide& s = pick(a, b2, lb);
  const int c = threadIdx.x & (KP - 1);
  const int rpb = kThreads / KP;
  double acc[2] = {0.0, 0.0};
  if (s_done(s)[c] == 0) {
    const double alpha = s_alpha(s)[c];
    for (int row = lb * rpb + (int)threadIdx.x / KP; row < s.c; row += s.nb * rpb) {
      if (s.inv[row] >= 0) continue;
      const size_t e = (size_t)row * KP + c;
      s.x[e] += alpha * s.p[e];
      const double rv = s.r[e] - alpha * s.q[e];
      const double zv = s.dinv[row] * rv;
      s.r[e] = rv;
      s.z[e] = zv;
      acc[0] += rv * zv;
      acc[1] += rv * rv;
    }
  }
  store_col_partials<2>(acc, s.pb, lb, s.nb, KP);
}

// One workgroup per (side, column): beta = <r, z>_new / <r, z>; the new
// scalars replace the old ones.
__global__ void __launch_bounds__(kThreads)
k_up_beta(UpSide a, UpSide b2, int KP) {
  const int side = blockIdx.x / KP, c = blockIdx.x % KP;
  const UpSide& s = side == 0 ? a : b2;
  if (s_done(s)[c] != 0) return;
  const double rz_new = col_sum(s.pb, s.nb, KP, 0, c);
  const double rr_new = col_sum(s.pb, s.nb, KP, 1, c);
  if (threadIdx.x != 0) return;
  if (bad(rz_new) || bad(rr_new)) {
    s_done(s)[c] = 3;
    return;
  }
  s_beta(s)[c] = rz_new / s_rz(s)[c];
  s_rz(s)[c] = rz_new;
  s_rr(s)[c] = rr_new;
  s_iters(s)[c] += 1;
}

// p = z + beta p on unknown rows of running columns.
__global__ void __launch_bounds__(kThreads)
k_up_pupdate(UpSide a, UpSide b2, int KP) {
  int lb;
  const UpSide& s = pick(a, b2, lb);
  const int c = threadIdx.x & (KP - 1);
  const int rpb = kThreads / KP;
  if (s_done(s)[c] != 0) return;  // no barrier below
  const double beta = s_beta(s)[c];
  for (int row = lb * rpb + (int)threadIdx.x / KP; row < s.c; row += s.nb * rpb) {
    if (s.inv[row] >= 0) continue;
    const size_t e = (size_t)row * KP + c;
    s.p[e] = s.z[e] + beta * s.p[e];
  }
}

// S = x on unknown rows (the sampled rows already hold R); partials of the
// column norms ||S_c||^2.
__global__ void __launch_bounds__(kThreads)
k_up_finish(UpSide a, UpSide b2, int KP) {
  int lb;
  const UpSide& s = pick(a, b2, lb);
  const int c = threadIdx.x & (KP - 1);
  const int rpb = kThreads / KP;
  double acc[1] = {0.0};
  for (int row = lb * rpb + (int)threadIdx.x / KP; row < s.c; row += s.nb * rpb) {
    const size_t e = (size_t)row * KP + c;
    double v = s.S[e];
    if (s.inv[row] < 0) {
      v = s.x[e];
      s.S[e] = v;
    }
    acc[0] += v * v;
  }
  store_col_partials<1>(acc, s.pa, lb, s.nb, KP);
}

// One workgroup: w_c = scale sigma_c / (||u_c|| ||v_c||) for c < k, 0 past
// k (U from side a, V from side b). Also the relative residuals.
__global__ void __launch_bounds__(kThreads)
k_up_weights(UpSide a, UpSide b2, int KP, int k, const double* __restrict__ sig, double scale,
             double* __restrict__ w, double* __restrict__ rel) {
  __shared__ double red[kThreads];
  const double nu = sqrt(col_total(a.pa, a.nb, KP, 0, red));
  const double nv = sqrt(col_total(b2.pa, b2.nb, KP, 0, red));
  const int c = threadIdx.x;
  if (c >= KP) return;
  w[c] = c < k ? scale * sig[c] / (nu * nv) : 0.0;
  // final recursive residuals
  for (int side = 0; side < 2; ++side) {
    const UpSide& s = side == 0 ? a : b2;
    const double bb = s_bb(s)[c];
    rel[side * KP + c] = c < k && bb > 0.0 ? sqrt(s_rr(s)[c] / bb) : 0.0;
  }
}

// ----------------------------------------------------------- rank-k output
// X[i, j] = sum_c U[i, c] w_c V[j, c] for i < p, j < n (row-major, leading
// dimension n, type TO). A workgroup owns a strip of kThreads * VEC
// columns and a range of rows: it keeps w * V of its columns in registers
// and streams the rows, reading each U row (KP values, the same for the
// whole workgroup) once. VEC-wide stores need n % VEC == 0.
template <typename TO, int KPT, int VEC>
__global__ void __launch_bounds__(kThreads)
k_rank_k(TO* __restrict__ X, const double* __restrict__ U, const double* __restrict__ V,
         const double* __restrict__ w, int p, int n, int KP, int rows_per, int nstrips) {
  const int strip = blockIdx.x % nstrips;
  const int rg = blockIdx.x / nstrips;
  const int j0 = (strip * kThreads + (int)threadIdx.x) * VEC;
  const int i0 = rg * rows_per;
  const int i1 = min(p, i0 + rows_per);
  double vw[VEC][KPT];
#pragma unroll
  for (int q = 0; q < VEC; ++q)
#pragma unroll
    for (int c = 0; c < KPT; ++c)
      vw[q][c] = (j0 + q < n && c < KP) ? V[(size_t)(j0 + q) * KP + c] * w[c] : 0.0;
  if (j0 >= n) return;
  for (int i = i0; i < i1; ++i) {
    const double* u = U + (size_t)i * KP;
    double uc[KPT];
#pragma unroll
    for (int c = 0; c < KPT; ++c) uc[c] = c < KP ? u[c] : 0.0;
    TO out[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < KPT; ++c) acc += uc[c] * vw[q][c];
      out[q] = (TO)acc;
    }
    TO* dst = X + (size_t)i * n + j0;
    if (VEC > 1 && j0 + VEC <= n) {
      vst<TO, VEC>(dst, out);
    } else {
#pragma unroll
      for (int q = 0; q < VEC; ++q)
        if (j0 + q < n) dst[q] = out[q];
    }
  }
}

template <typename TO>
__global__ void __launch_bounds__(kThreads) k_fill_zero(TO* __restrict__ X, size_t N) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) X[e] = TO(0);
}

// --------------------------------- one-side decoders (appendix: decoders 2, 3)
// One workgroup: w_c = 1 / ||S_c||^2 for c < k (0 past k), so that
// S diag(w) S^T = U U^T for the unit columns U = S / ||S||; rel = the final
// recursive CG residuals of the side.
__global__ void __launch_bounds__(kThreads)
k_up_unitw(UpSide a, int KP, int k, double* __restrict__ w, double* __restrict__ rel) {
  __shared__ double red[kThreads];
  const double n2 = col_total(a.pa, a.nb, KP, 0, red);
  const int c = threadIdx.x;
  if (c >= KP) return;
  w[c] = (c < k && n2 > 0.0) ? 1.0 / n2 : 0.0;
  const double bb = s_bb(a)[c];
  rel[c] = c < k && bb > 0.0 ? sqrt(s_rr(a)[c] / bb) : 0.0;
}

// Decoder 2, G = S^T Y (KP x n), first pass: workgroup (strip, chunk) sums
// rows [chunk * rows_per, ...) of S[i, c] Y[i, j] for its kThreads * VEC
// columns; partials Gp[chunk][c][j]. Each S row (KP values) is the same for
// the whole workgroup.
template <typename T, int KPT, int VEC>
__global__ void __launch_bounds__(kThreads)
k_proj_left(const T* __restrict__ Y, const double* __restrict__ S, int p, int n, int KP,
            int rows_per, int nstrips, double* __restrict__ Gp) {
  const int strip = blockIdx.x % nstrips;
  const int chunk = blockIdx.x / nstrips;
  const int j0 = (strip * kThreads + (int)threadIdx.x) * VEC;
  const int i0 = chunk * rows_per, i1 = min(p, i0 + rows_per);
  double acc[KPT][VEC];
#pragma unroll
  for (int c = 0; c < KPT; ++c)
#pragma unroll
    for (int q = 0; q < VEC; ++q) acc[c][q] = 0.0;
  if (j0 < n) {
    const bool full = j0 + VEC <= n;
    for (int i = i0; i < i1; ++i) {
      T y[VEC];
      const T* src = Y + (size_t)i * n + j0;
      if (VEC > 1 && full) {
        vld<T, VEC>(src, y);
      } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q) y[q] = j0 + q < n ? src[q] : T(0);
      }
      const double* srow = S + (size_t)i * KP;
#pragma unroll
      for (int c = 0; c < KPT; ++c) {
        const double sc = c < KP ? srow[c] : 0.0;
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[c][q] += sc * (double)y[q];
      }
    }
  }
  double* dst = Gp + (size_t)chunk * KP * n;
#pragma unroll
  for (int c = 0; c < KPT; ++c)
    if (c < KP)
#pragma unroll
      for (int q = 0; q < VEC; ++q)
        if (j0 + q < n) dst[(size_t)c * n + j0 + q] = acc[c][q];
}

// Decoder 2, second pass: Gt[j][c] = sum over chunks of Gp[chunk][c][j]
// (fixed order), written n x KP for the rank-k output kernel.
__global__ void __launch_bounds__(kThreads)
k_proj_left_sum(const double* __restrict__ Gp, int nchunks, int n, int KP, double* __restrict__ Gt) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * KP) return;
  const int j = (int)(e / KP), c = (int)(e % KP);
  double s = 0.0;
  for (int b = 0; b < nchunks; ++b) s += Gp[((size_t)b * KP + c) * n + j];
  Gt[e] = s;
}

// Decoder 3, G = Y S (p x KP), first pass: each wave owns a strip of
// 64 * VEC columns (its S rows in registers) and walks the rows of its
// workgroup's row range; per row the KP sums over the strip are reduced
// across the wave and written as partials Gp[i][wstrip][c].
template <typename T, int KPT, int VEC>
__global__ void __launch_bounds__(kThreads)
k_proj_right(const T* __restrict__ Y, const double* __restrict__ S, int p, int n, int KP,
             int rows_per, int nwg_strips, int nwstrips, double* __restrict__ Gp) {
  const int wg_strip = blockIdx.x % nwg_strips;
  const int rg = blockIdx.x / nwg_strips;
  const int lane = threadIdx.x & 63;
  const int wstrip = wg_strip * kMaxWaves + (int)threadIdx.x / 64;
  const int j0 = (wstrip * 64 + lane) * VEC;
  const int i0 = rg * rows_per, i1 = min(p, i0 + rows_per);
  if (wstrip >= nwstrips) return;  // whole wave
  double sv[VEC][KPT];
#pragma unroll
  for (int q = 0; q < VEC; ++q)
#pragma unroll
    for (int c = 0; c < KPT; ++c)
      sv[q][c] = (j0 + q < n && c < KP) ? S[(size_t)(j0 + q) * KP + c] : 0.0;
  const bool full = j0 + VEC <= n;
  for (int i = i0; i < i1; ++i) {
    T y[VEC];
    const T* src = Y + (size_t)i * n + j0;
    if (VEC > 1 && full) {
      vld<T, VEC>(src, y);
    } else {
#pragma unroll
      for (int q = 0; q < VEC; ++q) y[q] = j0 + q < n ? src[q] : T(0);
    }
    double acc[KPT];
#pragma unroll
    for (int c = 0; c < KPT; ++c) {
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < VEC; ++q) a += (double)y[q] * sv[q][c];
      acc[c] = wave_sum(a);
    }
    if (lane == 0) {
      double* dst = Gp + ((size_t)i * nwstrips + wstrip) * KP;
#pragma unroll
      for (int c = 0; c < KPT; ++c)
        if (c < KP) dst[c] = acc[c];
    }
  }
}

// Decoder 3, second pass: G[i][c] = sum over wave strips of Gp[i][s][c].
__global__ void __launch_bounds__(kThreads)
k_proj_right_sum(const double* __restrict__ Gp, int nwstrips, int p, int KP, double* __restrict__ G) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)p * KP) return;
  const int i = (int)(e / KP), c = (int)(e % KP);
  double s = 0.0;
  for (int b = 0; b < nwstrips; ++b) s += Gp[((size_t)i * nwstrips + b) * KP + c];
  G[e] = s;
}

// ------------------------------------------- Kron reduction (Section IV-A)
// The Schur complement onto the sampled nodes equals the sampled rows of
// L S, where S is the graph upsampling of the unit vectors: S = I on Omega
// and S = -L(bar, bar)^-1 L(bar, Omega) elsewhere. Columns are processed KP
// at a time: R holds unit vectors col0 .. col0 + kb - 1.
__global__ void __launch_bounds__(kThreads)
k_kron_rhs(double* __restrict__ R, int rho, int KP, int col0, int kb) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)rho * KP) return;
  const int a = (int)(e / KP), c = (int)(e % KP);
  R[e] = (c < kb && a == col0 + c) ? 1.0 : 0.0;
}

// out[a][col0 + c] = (L S)[omega[a], c] for a < rho, c < kb (rho x rho row-major).
__global__ void __launch_bounds__(kThreads)
k_kron_rows(UpSide s, const int32_t* __restrict__ omega, int rho, int KP, int col0, int kb,
            double* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)rho * KP) return;
  const int a = (int)(e / KP), c = (int)(e % KP);
  if (c >= kb) return;
  out[(size_t)a * rho + col0 + c] = lap_row(s, s.S, omega[a], c, KP);
}

// out = (out + out^T) / 2 (the two triangles agree to the CG tolerance).
__global__ void __launch_bounds__(kThreads)
k_kron_sym(double* __restrict__ out, int rho) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)rho * rho) return;
  const int i = (int)(e / rho), j = (int)(e % rho);
  if (j <= i) return;
  const double v = 0.5 * (out[(size_t)i * rho + j] + out[(size_t)j * rho + i]);
  out[(size_t)i * rho + j] = v;
  out[(size_t)j * rho + i] = v;
}

// ---------------------------------------------- clustering (Algorithm 3)
// Points (rho_c x rho_r, FP64): point j is column j of X~ (rho_r x rho_c).
template <typename TI>
__global__ void __launch_bounds__(kThreads)
k_km_points(double* __restrict__ P, const TI* __restrict__ Xt, int rho_r, int rho_c) {
  const size_t N = (size_t)rho_r * rho_c;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const size_t i = e / rho_c, j = e - i * rho_c;
    P[j * rho_r + i] = (double)Xt[e];
  }
}

// Centroids from the seed points; labels = -1 (every point changes on the
// first assignment).
__global__ void __launch_bounds__(kThreads)
k_km_seed(double* __restrict__ Cen, const double* __restrict__ P, const int* __restrict__ init,
          int k, int d, int* __restrict__ labels, int N) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)k * d; e += stride) {
    const size_t j = e / d, t = e - j * d;
    Cen[e] = P[(size_t)init[j] * d + t];
  }
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)N; e += stride)
    labels[e] = -1;
}

// Assignment (one workgroup per point): the nearest centroid in squared
// Euclidean distance, the lower index on ties; changed counts new labels.
__global__ void __launch_bounds__(kThreads)
k_km_assign(const double* __restrict__ P, const double* __restrict__ Cen, int d, int k,
            int* __restrict__ labels, int* __restrict__ changed) {
  const double* x = P + (size_t)blockIdx.x * d;
  double best = 0.0;
  int bj = -1;
  for (int j0 = 0; j0 < k; j0 += 8) {
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    for (int t = threadIdx.x; t < d; t += kThreads) {
      const double xv = x[t];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (j0 + q < k) {
          const double df = xv - Cen[(size_t)(j0 + q) * d + t];
          acc[q] += df * df;
        }
      }
    }
    block_sum<8>(acc);
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (j0 + q < k && (bj < 0 || acc[q] < best)) {
        best = acc[q];
        bj = j0 + q;
      }
  }
  if (threadIdx.x == 0 && labels[blockIdx.x] != bj) {
    labels[blockIdx.x] = bj;
    atomicAdd(changed, 1);
  }
}

// Update: centroid j (workgroup j % k, dimension slice blockIdx.x / k)
// becomes the mean of its points; an empty cluster keeps its centroid.
__global__ void __launch_bounds__(kThreads)
k_km_update(const double* __restrict__ P, double* __restrict__ Cen, const int* __restrict__ labels,
            int N, int d, int k) {
  const int j = blockIdx.x % k;
  const int t = (blockIdx.x / k) * kThreads + threadIdx.x;
  int cnt = 0;
  double sum = 0.0;
  for (int i = 0; i < N; ++i) {
    if (labels[i] == j) {
      ++cnt;
      if (t < d) sum += P[(size_t)i * d + t];
    }
  }
  if (cnt > 0 && t < d) Cen[(size_t)j * d + t] = sum / cnt;
}

// The indicator columns of the sample labels in the CG layout (rho_c x KP).
__global__ void __launch_bounds__(kThreads)
k_km_onehot(double* __restrict__ R, const int* __restrict__ labels, int N, int KP) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)N * KP; e += stride)
    R[e] = labels[e / KP] == (int)(e % KP) ? 1.0 : 0.0;
}

// Max pooling: the column of the largest of the k upsampled indicators of
// every row (the lower index on ties); optionally C itself (n x k, FP64).
__global__ void __launch_bounds__(kThreads)
k_max_pool(const double* __restrict__ S, int n, int KP, int k, int* __restrict__ out,
           double* __restrict__ C) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride) {
    const double* row = S + i * KP;
    double best = row[0];
    int bj = 0;
    for (int c = 1; c < k; ++c)
      if (row[c] > best) {
        best = row[c];
        bj = c;
      }
    out[i] = bj;
    if (C)
      for (int c = 0; c < k; ++c) C[i * k + c] = row[c];
  }
}

// ------------------------------------------------------------------- host
int pow2_at_least(int k) {
  int v = 1;
  while (v < k) v <<= 1;
  return v;
}

// Round-robin (circle) schedule: m players (plus an idle slot when m is
// odd), M - 1 rounds of M / 2 disjoint pairs, every pair met once a sweep.
std::vector<int2> round_robin(int m) {
  const int M = m + (m & 1);
  std::vector<int2> t;
  if (M < 2) return t;
  t.reserve((size_t)(M - 1) * (M / 2));
  for (int r = 0; r < M - 1; ++r) {
    auto at = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + r) % (M - 1)) + 1; };
    for (int k = 0; k < M / 2; ++k) t.push_back(make_int2(at(k), at(M - 1 - k)));
  }
  return t;
}

template <int KPT, typename TO>
hipError_t launch_rank_k_t(hipStream_t st, TO* X, const double* U, const double* V,
                           const double* w, int p, int n, int KP) {
  // 16-byte stores where the rows allow it; small KP leaves room for more
  // columns per thread
  constexpr int VW = KPT <= 16 ? (int)(16 / sizeof(TO)) : 1;  // registers: VW * KPT doubles
  const bool vec = VW > 1 && n % VW == 0;
  const int cols = kThreads * (vec ? VW : 1);
  const int nstrips = (n + cols - 1) / cols;
  // about 2048 workgroups, at least 8 rows each
  const int rows_per = std::max(8, (int)(((int64_t)p * nstrips + 2047) / 2048));
  const int ngroups = (p + rows_per - 1) / rows_per;
  const int grid = nstrips * ngroups;
  if (vec)
    k_rank_k<TO, KPT, VW><<<grid, kThreads, 0, st>>>(X, U, V, w, p, n, KP, rows_per, nstrips);
  else
    k_rank_k<TO, KPT, 1><<<grid, kThreads, 0, st>>>(X, U, V, w, p, n, KP, rows_per, nstrips);
  return hipGetLastError();
}

template <typename TO>
hipError_t launch_rank_k(hipStream_t st, TO* X, const double* U, const double* V, const double* w,
                         int p, int n, int KP) {
  switch (KP) {
    case 1: return launch_rank_k_t<1>(st, X, U, V, w, p, n, KP);
    case 2: return launch_rank_k_t<2>(st, X, U, V, w, p, n, KP);
    case 4: return launch_rank_k_t<4>(st, X, U, V, w, p, n, KP);
    case 8: return launch_rank_k_t<8>(st, X, U, V, w, p, n, KP);
    case 16: return launch_rank_k_t<16>(st, X, U, V, w, p, n, KP);
    case 32: return launch_rank_k_t<32>(st, X, U, V, w, p, n, KP);
    case 64: return launch_rank_k_t<64>(st, X, U, V, w, p, n, KP);
    default: return hipErrorInvalidValue;
  }
}

// One-side projections of decoders 2 and 3: side 0: Gt = (S^T Y)^T (n x KP),
// side 1: G = Y S (p x KP), each as a partial-sum pass plus a fixed-order sum.
// Gp must hold proj_partials(...) doubles.
inline int proj_vec(size_t elem, int n) {
  const int v = (int)(16 / elem);
  return n % v == 0 ? v : 1;
}
inline size_t proj_partials(int side, size_t elem, int p, int n, int KP) {
  const int vec = proj_vec(elem, n);
  if (side == 0) {
    const int nstrips = (n + kThreads * vec - 1) / (kThreads * vec);
    const int nchunks = std::min(std::max(1, (1024 + nstrips - 1) / nstrips), std::min(p, 128));
    return (size_t)nchunks * KP * n;
  }
  const int nwstrips = (n + 64 * vec - 1) / (64 * vec);
  return (size_t)p * nwstrips * KP;
}

template <int KPT, int VEC, typename T>
hipError_t launch_proj_v(hipStream_t st, int side, const T* Y, const double* S, int p, int n,
                         int KP, double* Gp, double* G) {
  if (side == 0) {
    const int nstrips = (n + kThreads * VEC - 1) / (kThreads * VEC);
    int nchunks = std::min(std::max(1, (1024 + nstrips - 1) / nstrips), std::min(p, 128));
    const int rows_per = (p + nchunks - 1) / nchunks;
    nchunks = (p + rows_per - 1) / rows_per;
    k_proj_left<T, KPT, VEC><<<nstrips * nchunks, kThreads, 0, st>>>(Y, S, p, n, KP, rows_per,
                                                                    nstrips, Gp);
    k_proj_left_sum<<<(int)(((size_t)n * KP + kThreads - 1) / kThreads), kThreads, 0, st>>>(
        Gp, nchunks, n, KP, G);
  } else {
    const int nwstrips = (n + 64 * VEC - 1) / (64 * VEC);
    const int nwg = (nwstrips + kMaxWaves - 1) / kMaxWaves;
    const int ngroups = std::min(std::max(1, (1024 + nwg - 1) / nwg), p);
    const int rows_per = (p + ngroups - 1) / ngroups;
    const int ng = (p + rows_per - 1) / rows_per;
    k_proj_right<T, KPT, VEC><<<nwg * ng, kThreads, 0, st>>>(Y, S, p, n, KP, rows_per, nwg,
                                                            nwstrips, Gp);
    k_proj_right_sum<<<(int)(((size_t)p * KP + kThreads - 1) / kThreads), kThreads, 0, st>>>(
        Gp, nwstrips, p, KP, G);
  }
  return hipGetLastError();
}

template <int KPT, typename T>
hipError_t launch_proj_t(hipStream_t st, int side, const T* Y, const double* S, int p, int n,
                         int KP, double* Gp, double* G) {
  constexpr int VW = (int)(16 / sizeof(T));
  if (proj_vec(sizeof(T), n) == VW) return launch_proj_v<KPT, VW, T>(st, side, Y, S, p, n, KP, Gp, G);
  return launch_proj_v<KPT, 1, T>(st, side, Y, S, p, n, KP, Gp, G);
}

template <typename T>
hipError_t launch_proj(hipStream_t st, int side, const T* Y, const double* S, int p, int n, int KP,
                       double* Gp, double* G) {
  switch (KP) {
    case 1: return launch_proj_t<1, T>(st, side, Y, S, p, n, KP, Gp, G);
    case 2: return launch_proj_t<2, T>(st, side, Y, S, p, n, KP, Gp, G);
    case 4: return launch_proj_t<4, T>(st, side, Y, S, p, n, KP, Gp, G);
    case 8: return launch_proj_t<8, T>(st, side, Y, S, p, n, KP, Gp, G);
    case 16: return launch_proj_t<16, T>(st, side, Y, S, p, n, KP, Gp, G);
    default: return hipErrorInvalidValue;
  }
}

struct SideHost {
  std::vector<int32_t> inv;
  std::vector<double> dinv;
};

// Host tables of one side: the inverse of omega and the Jacobi
// preconditioner of the unknown rows.
SideHost side_tables(const HostCsr& L, const std::vector<int32_t>& omega) {
  SideHost s;
  s.inv.assign((size_t)L.n, -1);
  for (size_t a = 0; a < omega.size(); ++a) s.inv[(size_t)omega[a]] = (int32_t)a;
  s.dinv.assign((size_t)L.n, 0.0);
  for (int64_t i = 0; i < L.n; ++i) {
    if (s.inv[(size_t)i] >= 0) continue;
    double d = 0.0;
    for (int32_t e = L.rp[(size_t)i]; e < L.rp[(size_t)i + 1]; ++e)
      if (L.ci[(size_t)e] == i) d += L.v[(size_t)e];
    s.dinv[(size_t)i] = d > 0.0 ? 1.0 / d : 1.0;
  }
  return s;
}

cpca_status fetch_indices(const char* name, const int32_t* idx, int64_t count, int64_t dim,
                          std::vector<int32_t>& out) {
  std::vector<uint8_t> mask;
  STCHK(fetch_index_set(name, idx, count, dim, mask));
  out.resize((size_t)count);
  HIPCHK(hipMemcpy(out.data(), idx, sizeof(int32_t) * count, hipMemcpyDefault));
  return CPCA_OK;
}

// Per side: done flags then iteration counts (kApproxKMax each), sides A, B.
cpca_status read_states(cpca_handle h, const UpSide& A, const UpSide& B, int nsides,
                        std::vector<int>& hs) {
  hs.assign(2 * 2 * kApproxKMax, 1);
  HIPCHK(hipMemcpyAsync(hs.data(), A.state, sizeof(int) * 2 * kApproxKMax, hipMemcpyDeviceToHost,
                        h->stream));
  if (nsides > 1)
    HIPCHK(hipMemcpyAsync(hs.data() + 2 * kApproxKMax, B.state, sizeof(int) * 2 * kApproxKMax,
                          hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return CPCA_OK;
}

// Upsampling CG over nsides graph sides (A, and B when nsides = 2) in shared
// launches: start vectors from S's sampled rows, per-column CG to
// ||r|| <= tol ||b|| or max_iter, then S on the unknown rows and the column
// norm partials. Chunks of kUpChunk iterations are replayed as a HIP graph
// on a side stream; the host reads the done flags between chunks.
cpca_status upsample_solve(cpca_handle h, const UpSide& A, const UpSide& B, int nsides, int KP,
                           int k, double tol, int max_iter, std::vector<int>& hstate) {
  TraceRange trace_("upsampling PCG");
  hipStream_t st = h->stream;
  const int gup = A.nb + (nsides > 1 ? B.nb : 0);
  k_up_start<<<gup, kThreads, 0, st>>>(A, B, KP, 0);
  LAUNCHCHK();
  k_up_start<<<gup, kThreads, 0, st>>>(A, B, KP, 1);
  LAUNCHCHK();
  k_up_arm<<<nsides * KP, kThreads, 0, st>>>(A, B, KP, k, tol * tol);
  LAUNCHCHK();
  auto all_done = [&]() {
    for (int side = 0; side < nsides; ++side)
      for (int c = 0; c < k; ++c)
        if (hstate[(size_t)side * 2 * kApproxKMax + c] == 0) return false;
    return true;
  };
  STCHK(read_states(h, A, B, nsides, hstate));
  hipStream_t cs;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipEvent_t ev;
  hipError_t err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  auto enqueue = [&](hipStream_t s2) -> hipError_t {
    k_up_apply<<<gup, kThreads, 0, s2>>>(A, B, KP);
    k_up_alpha<<<nsides * KP, kThreads, 0, s2>>>(A, B, KP);
    k_up_update<<<gup, kThreads, 0, s2>>>(A, B, KP);
    k_up_beta<<<nsides * KP, kThreads, 0, s2>>>(A, B, KP);
    k_up_pupdate<<<gup, kThreads, 0, s2>>>(A, B, KP);
    return hipGetLastError();
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (err == hipSuccess && max_iter >= kUpChunk) {
    err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    for (int j = 0; j < kUpChunk && err == hipSuccess; ++j) err = enqueue(cs);
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (err == hipSuccess) err = e2;
    if (err == hipSuccess) err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  }
  if (err == hipSuccess) err = hipEventRecord(ev, st);
  if (err == hipSuccess) err = hipStreamWaitEvent(cs, ev, 0);
  int it = 0;
  cpca_status sst = CPCA_OK;
  while (err == hipSuccess && it < max_iter && !all_done()) {
    if (exec && it + kUpChunk <= max_iter) {
      err = hipGraphLaunch(exec, cs);
      it += kUpChunk;
    } else {
      err = enqueue(cs);
      it += 1;
    }
    if (err == hipSuccess) err = hipEventRecord(ev, cs);
    if (err == hipSuccess) err = hipStreamWaitEvent(st, ev, 0);
    if (err != hipSuccess) break;
    if ((sst = read_states(h, A, B, nsides, hstate)) != CPCA_OK) break;
  }
  const hipError_t e3 = hipStreamSynchronize(cs);
  if (err == hipSuccess) err = e3;
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipEventDestroy(ev);
  (void)hipStreamDestroy(cs);
  if (err != hipSuccess) return fail(CPCA_EHIP, std::string("upsampling CG: ") + hipGetErrorString(err));
  STCHK(sst);
  k_up_finish<<<gup, kThreads, 0, st>>>(A, B, KP);
  LAUNCHCHK();
  return CPCA_OK;
}

// variant 0: Algorithm 2 (both graphs); 1: decoder 2 (row graph only,
// X = U U^T Y); 2: decoder 3 (column graph only, X = Y V V^T). The one-side
// variants take the full data Y (p x n) and ignore the absent side's
// arguments (omega, L, delta).
template <typename T>
cpca_status run_approx(cpca_handle h, const T* Xt, int64_t rho_r, int64_t rho_c,
                       const int32_t* om_r, const int32_t* om_c, int64_t p, int64_t n,
                       const cpca_csr* Lr, const cpca_csr* Lc, double delta, double ratio,
                       int32_t k_max, double tol, int32_t max_iter, T* X_out, double* sigma_out,
                       cpca_approx_info* info, int variant = 0, const T* Y = nullptr) {
  const auto t0 = std::chrono::steady_clock::now();
  HIPCHK(hipStreamSynchronize(h->stream));  // inputs may still be in flight
  const bool use_r = variant != 2, use_c = variant != 1;
  HostCsr hLr, hLc;
  std::vector<int32_t> wr, wc;
  SideHost sr, sc;
  if (use_r) {
    STCHK(fetch_csr("Lr", Lr, hLr));
    STCHK(fetch_indices("omega_r", om_r, rho_r, p, wr));
    sr = side_tables(hLr, wr);
  }
  if (use_c) {
    STCHK(fetch_csr("Lc", Lc, hLc));
    STCHK(fetch_indices("omega_c", om_c, rho_c, n, wc));
    sc = side_tables(hLc, wc);
  }

  const int trans = rho_r >= rho_c ? 1 : 0;
  const int m = (int)std::min(rho_r, rho_c);
  const int len = (int)std::max(rho_r, rho_c);
  if (m > kSvdMaxM) {
    char buf[96];
    std::snprintf(buf, sizeof buf, "approx_decode: min(rho_r, rho_c) = %d exceeds %d", m, kSvdMaxM);
    return fail(CPCA_EINVAL, buf);
  }
  const std::vector<int2> rr_tab = round_robin(m);
  const int M = m + (m & 1);
  const int npair = M / 2;
  const int KPmax = pow2_at_least(k_max);

  // ---- workspace
  double *W = nullptr, *Q = nullptr, *sig = nullptr, *lv = nullptr, *sv = nullptr, *wts = nullptr,
         *rel = nullptr, *fro2 = nullptr;
  int2* pairs = nullptr;
  int *cnt = nullptr, *perm = nullptr, *kdev = nullptr, *inv_r = nullptr, *inv_c = nullptr;
  double *dinv_r = nullptr, *dinv_c = nullptr, *gproj = nullptr, *gpart = nullptr;
  UpSide A, B;  // A: rows (L_r), B: columns (L_c)
  auto grid_for = [&](int64_t) { return kUpMaxBlocks; };  // partial buffers: the largest grid
  auto layout = [&](Arena& a) {
    W = a.take<double>((size_t)m * len);
    Q = a.take<double>((size_t)m * m);
    pairs = a.take<int2>(std::max<size_t>(rr_tab.size(), 1));
    cnt = a.take<int>(1);
    fro2 = a.take<double>(1);
    sig = a.take<double>((size_t)m);
    perm = a.take<int>((size_t)m);
    kdev = a.take<int>(1);
    lv = a.take<double>((size_t)len * KPmax);
    sv = a.take<double>((size_t)m * KPmax);
    wts = a.take<double>(kApproxKMax);
    rel = a.take<double>(2 * kApproxKMax);
    inv_r = a.take<int>((size_t)p);
    inv_c = a.take<int>((size_t)n);
    dinv_r = a.take<double>((size_t)p);
    dinv_c = a.take<double>((size_t)n);
    if (variant != 0) {
      gproj = a.take<double>((size_t)std::max(p, n) * KPmax);
      gpart = a.take<double>(proj_partials(variant - 1, sizeof(T), (int)p, (int)n, KPmax));
    }
    for (int side = 0; side < 2; ++side) {
      UpSide& s = side == 0 ? A : B;
      const int64_t c = side == 0 ? p : n;
      s.c = (int)c;
      s.nb = grid_for(c);
      const size_t N = (size_t)c * KPmax;
      s.x = a.take<double>(N);
      s.r = a.take<double>(N);
      s.z = a.take<double>(N);
      s.p = a.take<double>(N);
      s.q = a.take<double>(N);
      s.S = a.take<double>(N);
      s.pa = a.take<double>((size_t)s.nb * KPmax);
      s.pb = a.take<double>((size_t)s.nb * 2 * KPmax);
      s.scal = a.take<double>(6 * kApproxKMax);
      s.state = a.take<int>(2 * kApproxKMax);
    }
  };
  {
    Arena a;
    layout(a);
    STCHK(ensure_ws(h, a.off));
  }
  Arena ar;
  ar.base = h->ws;
  layout(ar);
  hipStream_t st = h->stream;
  if (!rr_tab.empty())
    HIPCHK(hipMemcpyAsync(pairs, rr_tab.data(), sizeof(int2) * rr_tab.size(), hipMemcpyHostToDevice, st));
  if (use_r) {
    HIPCHK(hipMemcpyAsync(inv_r, sr.inv.data(), sizeof(int) * p, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dinv_r, sr.dinv.data(), sizeof(double) * p, hipMemcpyHostToDevice, st));
  }
  if (use_c) {
    HIPCHK(hipMemcpyAsync(inv_c, sc.inv.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dinv_c, sc.dinv.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  }

  // ---- 1. one-sided Jacobi SVD
  k_jac_load<T><<<vec_grid((size_t)rho_r * rho_c), kThreads, 0, st>>>(W, Q, Xt, (int)rho_r,
                                                                       (int)rho_c, trans, m);
  LAUNCHCHK();
  k_jac_fro<<<1, kThreads, 0, st>>>(W, (size_t)m * len, fro2);
  LAUNCHCHK();
  // rotations stop once the normalised inner product of every pair is
  // within rounding of the dot products (len units in the last place); rows
  // below len ulps of ||X~||_F count as zero
  const double jac_tol = 2.220446049250313e-16 * std::max(len, 16);
  const double floor_rel = jac_tol * jac_tol;
  int sweeps = 0;
  bool svd_ok = true;
  if (npair > 0 && m > 1) {
    hipStream_t cs;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev;
    hipError_t err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (err == hipSuccess) err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (err == hipSuccess) {
      k_zero_int<<<1, 64, 0, cs>>>(cnt, 1);
      // rows of up to 2048 elements stay in registers (m <= len)
      const int ept = (len + kThreads - 1) / kThreads;
      for (int r = 0; r < M - 1; ++r) {
        const int2* pr = pairs + (size_t)r * npair;
        if (ept <= 1)
          k_jac_round_reg<1><<<npair, kThreads, 0, cs>>>(W, Q, m, len, pr, jac_tol, fro2, floor_rel, cnt);
        else if (ept <= 2)
          k_jac_round_reg<2><<<npair, kThreads, 0, cs>>>(W, Q, m, len, pr, jac_tol, fro2, floor_rel, cnt);
        else if (ept <= 4)
          k_jac_round_reg<4><<<npair, kThreads, 0, cs>>>(W, Q, m, len, pr, jac_tol, fro2, floor_rel, cnt);
        else if (ept <= 8)
          k_jac_round_reg<8><<<npair, kThreads, 0, cs>>>(W, Q, m, len, pr, jac_tol, fro2, floor_rel, cnt);
        else
          k_jac_round<<<npair, kThreads, 0, cs>>>(W, Q, m, len, pr, jac_tol, fro2, floor_rel, cnt);
      }
      err = hipGetLastError();
      hipError_t e2 = hipStreamEndCapture(cs, &graph);
      if (err == hipSuccess) err = e2;
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (err == hipSuccess) err = hipEventRecord(ev, st);
    if (err == hipSuccess) err = hipStreamWaitEvent(cs, ev, 0);
    int hc = 1;
    while (err == hipSuccess && sweeps < kMaxSweeps) {
      err = hipGraphLaunch(exec, cs);
      if (err == hipSuccess) err = hipMemcpyAsync(&hc, cnt, sizeof(int), hipMemcpyDeviceToHost, cs);
      if (err == hipSuccess) err = hipStreamSynchronize(cs);
      ++sweeps;
      if (err != hipSuccess || hc == 0) break;
    }
    if (err == hipSuccess) err = hipEventRecord(ev, cs);
    if (err == hipSuccess) err = hipStreamWaitEvent(st, ev, 0);
    const hipError_t e3 = hipStreamSynchronize(cs);
    if (err == hipSuccess) err = e3;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(cs);
    if (err != hipSuccess) return fail(CPCA_EHIP, std::string("approx_decode SVD: ") + hipGetErrorString(err));
    svd_ok = hc == 0;
  }
  // ---- 2. order of the singular values and k
  k_svd_rank<<<1, kThreads, 0, st>>>(W, m, len, ratio, k_max, sig, perm, kdev);
  LAUNCHCHK();
  std::vector<double> hsig((size_t)m);
  int k = 0;
  HIPCHK(hipMemcpyAsync(hsig.data(), sig, sizeof(double) * m, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&k, kdev, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (sigma_out) std::copy(hsig.begin(), hsig.end(), sigma_out);
  auto finish_info = [&](cpca_status s, int it_r, int it_c, double rel_r, double rel_c) {
    if (!info) return;
    info->k = k;
    info->svd_sweeps = sweeps;
    info->iters_r = it_r;
    info->iters_c = it_c;
    info->status = (int32_t)s;
    info->reserved = 0;
    info->rel_residual_r = rel_r;
    info->rel_residual_c = rel_c;
    info->scale = variant != 0 ? 1.0
                               : std::sqrt((double)n * (double)p /
                                           ((double)rho_r * (double)rho_c * (1.0 - delta)));
    info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  };
  const size_t NX = (size_t)p * n;
  if (k == 0) {
    k_fill_zero<T><<<vec_grid(NX), kThreads, 0, st>>>(X_out, NX);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(st));
    const cpca_status s = svd_ok ? CPCA_OK : CPCA_ENOCONV;
    finish_info(s, 0, 0, 0.0, 0.0);
    if (!svd_ok) return fail(CPCA_ENOCONV, "approx_decode: Jacobi SVD did not converge");
    return CPCA_OK;
  }
  const int KP = pow2_at_least(k);
  // the buffers were sized for KPmax; the grids follow the actual KP
  for (int side = 0; side < 2; ++side) {
    UpSide& s = side == 0 ? A : B;
    s.nb = (int)std::max<int64_t>(1, std::min<int64_t>(kUpMaxBlocks, ((int64_t)s.c * KP + kThreads - 1) / kThreads));
    const cpca_csr* L = side == 0 ? Lr : Lc;
    if (!L) continue;  // the absent side of a one-side decoder (never launched)
    s.rp = L->rowptr;
    s.ci = L->colind;
    s.v = L->vals;
    s.inv = side == 0 ? inv_r : inv_c;
    s.dinv = side == 0 ? dinv_r : dinv_c;
  }
  // long side = columns of W's rows: left vectors when trans, else right
  A.R = trans ? lv : sv;
  B.R = trans ? sv : lv;
  k_svd_vectors<<<vec_grid((size_t)(len + m) * KP), kThreads, 0, st>>>(W, Q, m, len, sig, perm, k, KP,
                                                                       lv, sv);
  LAUNCHCHK();

  std::vector<int> hstate;
  std::vector<double> hrel(2 * (size_t)KP, 0.0);
  int it_r = 0, it_c = 0, worst = 0;
  double rel_r = 0.0, rel_c = 0.0;
  if (variant == 0) {
    // ---- 3. upsampling, both graphs in the same launches
    STCHK(upsample_solve(h, A, B, 2, KP, k, tol, max_iter, hstate));
    // ---- 4.-6. norms, weights, X = U diag(w) V^T
    const double scale = std::sqrt((double)n * (double)p / ((double)rho_r * (double)rho_c * (1.0 - delta)));
    k_up_weights<<<1, kThreads, 0, st>>>(A, B, KP, k, sig, scale, wts, rel);
    LAUNCHCHK();
    STCHK(prof_begin(h, FAM_RANKK));
    HIPCHK(launch_rank_k<T>(st, X_out, A.S, B.S, wts, (int)p, (int)n, KP));
    STCHK(prof_end(h));
    HIPCHK(hipMemcpyAsync(hrel.data(), rel, sizeof(double) * 2 * KP, hipMemcpyDeviceToHost, st));
    STCHK(read_states(h, A, B, 2, hstate));
  } else {
    // ---- one graph side: upsample, unit columns, project the full data
    UpSide& U1 = variant == 1 ? A : B;
    UpSide& U2 = variant == 1 ? B : A;
    STCHK(upsample_solve(h, U1, U2, 1, KP, k, tol, max_iter, hstate));
    k_up_unitw<<<1, kThreads, 0, st>>>(U1, KP, k, wts, rel);
    LAUNCHCHK();
    HIPCHK(launch_proj<T>(st, variant - 1, Y, U1.S, (int)p, (int)n, KP, gpart, gproj));
    STCHK(prof_begin(h, FAM_RANKK));
    if (variant == 1)   // X = S diag(w) (S^T Y)
      HIPCHK(launch_rank_k<T>(st, X_out, U1.S, gproj, wts, (int)p, (int)n, KP));
    else                // X = (Y S) diag(w) S^T
      HIPCHK(launch_rank_k<T>(st, X_out, gproj, U1.S, wts, (int)p, (int)n, KP));
    STCHK(prof_end(h));
    HIPCHK(hipMemcpyAsync(hrel.data() + (variant == 1 ? 0 : KP), rel, sizeof(double) * KP,
                          hipMemcpyDeviceToHost, st));
    std::vector<int> hs1;
    STCHK(read_states(h, U1, U2, 1, hs1));
    // side states in the (rows, columns) order of the report
    hstate.assign(2 * 2 * kApproxKMax, 1);
    std::copy(hs1.begin(), hs1.begin() + 2 * kApproxKMax,
              hstate.begin() + (variant == 1 ? 0 : 2 * kApproxKMax));
    if (variant == 1)
      std::fill(hstate.begin() + 3 * kApproxKMax, hstate.end(), 0);   // no column iterations
    else
      std::fill(hstate.begin() + kApproxKMax, hstate.begin() + 2 * kApproxKMax, 0);
  }
  STCHK(prof_collect(h));
  for (int c = 0; c < k; ++c) {
    const int dr = hstate[(size_t)c], dc = hstate[(size_t)2 * kApproxKMax + c];
    it_r = std::max(it_r, hstate[(size_t)kApproxKMax + c]);
    it_c = std::max(it_c, hstate[(size_t)3 * kApproxKMax + c]);
    rel_r = std::max(rel_r, hrel[(size_t)c]);
    rel_c = std::max(rel_c, hrel[(size_t)KP + c]);
    for (int d : {dr, dc})
      if (d != 1) worst = std::max(worst, d == 0 ? 1 : d);  // 1: not converged
  }
  cpca_status s = CPCA_OK;
  if (worst == 3) s = CPCA_ENAN;
  else if (worst == 2) s = CPCA_ENOTSPD;
  else if (worst == 1 || !svd_ok) s = CPCA_ENOCONV;
  finish_info(s, it_r, it_c, rel_r, rel_c);
  if (s == CPCA_ENAN) return fail(s, "approx_decode: NaN/Inf in the upsampling CG");
  if (s == CPCA_ENOTSPD) return fail(s, "approx_decode: upsampling CG breakdown (p^T A p <= 0)");
  if (s == CPCA_ENOCONV)
    return fail(s, svd_ok ? "approx_decode: upsampling CG reached max_iter"
                          : "approx_decode: Jacobi SVD did not converge");
  return CPCA_OK;
}


template <typename T>
cpca_status run_cluster(cpca_handle h, const T* Xt, int64_t rho_r, int64_t rho_c,
                        const int32_t* om_c, int64_t n, const cpca_csr* Lc, int32_t k,
                        const int32_t* init, int32_t km_max_iter, double tol, int32_t max_iter,
                        int32_t* labels_out, double* C_out, int32_t* sample_labels_out,
                        cpca_cluster_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  HIPCHK(hipStreamSynchronize(h->stream));  // inputs may still be in flight
  HostCsr hLc;
  STCHK(fetch_csr("Lc", Lc, hLc));
  std::vector<int32_t> wc, seeds;
  STCHK(fetch_indices("omega_c", om_c, rho_c, n, wc));
  STCHK(fetch_indices("init", init, k, rho_c, seeds));
  const SideHost sc = side_tables(hLc, wc);
  const int KP = pow2_at_least(k);
  const int d = (int)rho_r, N = (int)rho_c;
  double *P = nullptr, *Cen = nullptr, *R = nullptr, *dinv = nullptr;
  int *lab = nullptr, *chg = nullptr, *inv = nullptr, *dseeds = nullptr;
  UpSide A, B;
  auto layout = [&](Arena& a) {
    P = a.take<double>((size_t)N * d);
    Cen = a.take<double>((size_t)k * d);
    lab = a.take<int>((size_t)N);
    chg = a.take<int>(1);
    dseeds = a.take<int>((size_t)k);
    R = a.take<double>((size_t)N * KP);
    inv = a.take<int>((size_t)n);
    dinv = a.take<double>((size_t)n);
    const size_t NV = (size_t)n * KP;
    A.c = (int)n;
    A.nb = (int)std::max<int64_t>(1, std::min<int64_t>(kUpMaxBlocks, ((int64_t)n * KP + kThreads - 1) / kThreads));
    A.x = a.take<double>(NV);
    A.r = a.take<double>(NV);
    A.z = a.take<double>(NV);
    A.p = a.take<double>(NV);
    A.q = a.take<double>(NV);
    A.S = a.take<double>(NV);
    A.pa = a.take<double>((size_t)A.nb * KP);
    A.pb = a.take<double>((size_t)A.nb * 2 * KP);
    A.scal = a.take<double>(6 * kApproxKMax);
    A.state = a.take<int>(2 * kApproxKMax);
  };
  {
    Arena a;
    layout(a);
    STCHK(ensure_ws(h, a.off));
  }
  Arena ar;
  ar.base = h->ws;
  layout(ar);
  hipStream_t st = h->stream;
  HIPCHK(hipMemcpyAsync(inv, sc.inv.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(dinv, sc.dinv.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(dseeds, seeds.data(), sizeof(int) * k, hipMemcpyHostToDevice, st));

  // ---- 1. k-means on the columns of X~ (Lloyd, from the given seeds)
  k_km_points<T><<<vec_grid((size_t)N * d), kThreads, 0, st>>>(P, Xt, d, N);
  LAUNCHCHK();
  k_km_seed<<<vec_grid((size_t)std::max(k * d, N)), kThreads, 0, st>>>(Cen, P, dseeds, k, d, lab, N);
  LAUNCHCHK();
  const int ugrid = k * ((d + kThreads - 1) / kThreads);
  int km_it = 0;
  for (;;) {
    k_zero_int<<<1, 64, 0, st>>>(chg, 1);
    k_km_assign<<<N, kThreads, 0, st>>>(P, Cen, d, k, lab, chg);
    LAUNCHCHK();
    int hc = 0;
    HIPCHK(hipMemcpyAsync(&hc, chg, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hc == 0 || km_it >= km_max_iter) break;
    k_km_update<<<ugrid, kThreads, 0, st>>>(P, Cen, lab, N, d, k);
    LAUNCHCHK();
    ++km_it;
  }
  if (sample_labels_out)
    HIPCHK(hipMemcpyAsync(sample_labels_out, lab, sizeof(int) * N, hipMemcpyDeviceToDevice, st));

  // ---- 2. upsampling of the k indicator columns over L_c
  k_km_onehot<<<vec_grid((size_t)N * KP), kThreads, 0, st>>>(R, lab, N, KP);
  LAUNCHCHK();
  A.rp = Lc->rowptr;
  A.ci = Lc->colind;
  A.v = Lc->vals;
  A.inv = inv;
  A.dinv = dinv;
  A.R = R;
  std::vector<int> hstate;
  STCHK(upsample_solve(h, A, B, 1, KP, k, tol, max_iter, hstate));

  // ---- 3. max pooling
  k_max_pool<<<vec_grid((size_t)n), kThreads, 0, st>>>(A.S, (int)n, KP, k, labels_out, C_out);
  LAUNCHCHK();
  std::vector<double> hscal(6 * kApproxKMax);
  HIPCHK(hipMemcpyAsync(hscal.data(), A.scal, sizeof(double) * hscal.size(), hipMemcpyDeviceToHost, st));
  STCHK(read_states(h, A, B, 1, hstate));
  int it_max = 0, worst = 0;
  double rel = 0.0;
  for (int c = 0; c < k; ++c) {
    const int dc = hstate[(size_t)c];
    it_max = std::max(it_max, hstate[(size_t)kApproxKMax + c]);
    const double bb = hscal[(size_t)2 * kApproxKMax + c];
    const double rr = hscal[(size_t)kApproxKMax + c];
    if (bb > 0.0) rel = std::max(rel, std::sqrt(rr / bb));
    if (dc != 1) worst = std::max(worst, dc == 0 ? 1 : dc);
  }
  cpca_status s = CPCA_OK;
  if (worst == 3) s = CPCA_ENAN;
  else if (worst == 2) s = CPCA_ENOTSPD;
  else if (worst == 1) s = CPCA_ENOCONV;
  if (info) {
    info->kmeans_iters = km_it;
    info->cg_iters = it_max;
    info->status = (int32_t)s;
    info->reserved = 0;
    info->rel_residual = rel;
    info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (s == CPCA_ENAN) return fail(s, "cluster_decode: NaN/Inf in the upsampling CG");
  if (s == CPCA_ENOTSPD) return fail(s, "cluster_decode: upsampling CG breakdown (p^T A p <= 0)");
  if (s == CPCA_ENOCONV) return fail(s, "cluster_decode: upsampling CG reached max_iter");
  return CPCA_OK;
}

}  // namespace

extern "C" cpca_status cpca_cluster_decode(cpca_handle h, cpca_mode mode, const void* Xtil,
                                           int64_t rho_r, int64_t rho_c, const int32_t* omega_c,
                                           int64_t n, const cpca_csr* Lc, int32_t k,
                                           const int32_t* init, int32_t kmeans_max_iter,
                                           double tol, int32_t max_iter, int32_t* labels_out,
                                           double* C_out, int32_t* sample_labels_out,
                                           cpca_cluster_info* info) {
  TraceRange trace_("cpca_cluster_decode");
  clear_error();
  STCHK(check_cluster_args(mode, rho_r, rho_c, omega_c, n, Lc, k, init, kmeans_max_iter, tol,
                           max_iter));
  if (!Xtil || !labels_out) return fail(CPCA_EINVAL, "cluster_decode: null data pointer");
  if (!h) return fail(CPCA_EINVAL, "null handle");
  if (mode == CPCA_FP64)
    return run_cluster<double>(h, static_cast<const double*>(Xtil), rho_r, rho_c, omega_c, n, Lc,
                               k, init, kmeans_max_iter, tol, max_iter, labels_out, C_out,
                               sample_labels_out, info);
  return run_cluster<float>(h, static_cast<const float*>(Xtil), rho_r, rho_c, omega_c, n, Lc, k,
                            init, kmeans_max_iter, tol, max_iter, labels_out, C_out,
                            sample_labels_out, info);
}

extern "C" cpca_status cpca_approx_decode(cpca_handle h, cpca_mode mode, const void* Xtil,
                                          int64_t rho_r, int64_t rho_c, const int32_t* omega_r,
                                          const int32_t* omega_c, int64_t p, int64_t n,
                                          const cpca_csr* Lr, const cpca_csr* Lc, double delta,
                                          double sigma_ratio, int32_t k_max, double tol,
                                          int32_t max_iter, void* X_out, double* sigma_out,
                                          cpca_approx_info* info) {
  TraceRange trace_("cpca_approx_decode");
  clear_error();
  STCHK(check_approx_args(mode, rho_r, rho_c, omega_r, omega_c, p, n, Lr, Lc, delta, sigma_ratio,
                          k_max, tol, max_iter));
  if (!Xtil || !X_out) return fail(CPCA_EINVAL, "approx_decode: null data pointer");
  if (!h) return fail(CPCA_EINVAL, "null handle");
  if (mode == CPCA_FP64)
    return run_approx<double>(h, static_cast<const double*>(Xtil), rho_r, rho_c, omega_r, omega_c,
                              p, n, Lr, Lc, delta, sigma_ratio, k_max, tol, max_iter,
                              static_cast<double*>(X_out), sigma_out, info);
  return run_approx<float>(h, static_cast<const float*>(Xtil), rho_r, rho_c, omega_r, omega_c, p,
                           n, Lr, Lc, delta, sigma_ratio, k_max, tol, max_iter,
                           static_cast<float*>(X_out), sigma_out, info);
}

// Approximate decoders 2 and 3 (appendix): one graph side, full data Y.
namespace {
cpca_status check_one_side_args(const char* who, cpca_mode mode, int64_t rho_r, int64_t rho_c,
                                const int32_t* omega, int64_t rho, int64_t dim, int64_t p,
                                int64_t n, const cpca_csr* L, const void* Y, double ratio,
                                int32_t k_max, double tol, int32_t max_iter) {
  cpca_status st;
  const std::string w(who);
  if ((st = check_mode(mode))) return st;
  if ((st = check_dims("X", p, n))) return st;
  if ((unsigned long long)p * (unsigned long long)n > (1ull << 40))
    return fail(CPCA_EINVAL, w + ": p * n too large");
  if ((st = check_dims("Xtil", rho_r, rho_c))) return st;
  if (rho_r > p || rho_c > n) return fail(CPCA_EINVAL, w + ": more samples than rows/columns");
  if (rho > dim) return fail(CPCA_EINVAL, w + ": more samples than graph nodes");
  if (!omega) return fail(CPCA_EINVAL, w + ": null index set");
  if ((st = check_csr_shape("L", L, dim))) return st;
  if (!Y) return fail(CPCA_EINVAL, w + ": null Y");
  if (!std::isfinite(ratio) || ratio < 0 || ratio > 1)
    return fail(CPCA_EINVAL, w + ": sigma_ratio must be in [0, 1]");
  if (k_max < 1 || k_max > 16) return fail(CPCA_EINVAL, w + ": k_max must be in [1, 16]");
  if (!std::isfinite(tol) || !(tol > 0)) return fail(CPCA_EINVAL, w + ": tol must be > 0");
  if (max_iter < 0) return fail(CPCA_EINVAL, w + ": max_iter < 0");
  return CPCA_OK;
}
}  // namespace

extern "C" cpca_status cpca_approx_decode2(cpca_handle h, cpca_mode mode, const void* Xtil,
                                           int64_t rho_r, int64_t rho_c, const int32_t* omega_r,
                                           int64_t p, int64_t n, const cpca_csr* Lr,
                                           const void* Y, double sigma_ratio, int32_t k_max,
                                           double tol, int32_t max_iter, void* X_out,
                                           double* sigma_out, cpca_approx_info* info) {
  TraceRange trace_("cpca_approx_decode2");
  clear_error();
  STCHK(check_one_side_args("approx_decode2", mode, rho_r, rho_c, omega_r, rho_r, p, p, n, Lr, Y,
                            sigma_ratio, k_max, tol, max_iter));
  if (!Xtil || !X_out) return fail(CPCA_EINVAL, "approx_decode2: null data pointer");
  if (!h) return fail(CPCA_EINVAL, "null handle");
  if (mode == CPCA_FP64)
    return run_approx<double>(h, static_cast<const double*>(Xtil), rho_r, rho_c, omega_r, nullptr,
                              p, n, Lr, nullptr, 0.0, sigma_ratio, k_max, tol, max_iter,
                              static_cast<double*>(X_out), sigma_out, info, 1,
                              static_cast<const double*>(Y));
  return run_approx<float>(h, static_cast<const float*>(Xtil), rho_r, rho_c, omega_r, nullptr, p,
                           n, Lr, nullptr, 0.0, sigma_ratio, k_max, tol, max_iter,
                           static_cast<float*>(X_out), sigma_out, info, 1,
                           static_cast<const float*>(Y));
}

extern "C" cpca_status cpca_approx_decode3(cpca_handle h, cpca_mode mode, const void* Xtil,
                                           int64_t rho_r, int64_t rho_c, const int32_t* omega_c,
                                           int64_t p, int64_t n, const cpca_csr* Lc,
                                           const void* Y, double sigma_ratio, int32_t k_max,
                                           double tol, int32_t max_iter, void* X_out,
                                           double* sigma_out, cpca_approx_info* info) {
  TraceRange trace_("cpca_approx_decode3");
  clear_error();
  STCHK(check_one_side_args("approx_decode3", mode, rho_r, rho_c, omega_c, rho_c, n, p, n, Lc, Y,
                            sigma_ratio, k_max, tol, max_iter));
  if (!Xtil || !X_out) return fail(CPCA_EINVAL, "approx_decode3: null data pointer");
  if (!h) return fail(CPCA_EINVAL, "null handle");
  if (mode == CPCA_FP64)
    return run_approx<double>(h, static_cast<const double*>(Xtil), rho_r, rho_c, nullptr, omega_c,
                              p, n, nullptr, Lc, 0.0, sigma_ratio, k_max, tol, max_iter,
                              static_cast<double*>(X_out), sigma_out, info, 2,
                              static_cast<const double*>(Y));
  return run_approx<float>(h, static_cast<const float*>(Xtil), rho_r, rho_c, nullptr, omega_c, p,
                           n, nullptr, Lc, 0.0, sigma_ratio, k_max, tol, max_iter,
                           static_cast<float*>(X_out), sigma_out, info, 2,
                           static_cast<const float*>(Y));
}

// Kron reduction of a Laplacian onto the sampled nodes (Section IV-A).
namespace {
cpca_status run_kron(cpca_handle h, const cpca_csr* L, const int32_t* omega, int64_t rho,
                     double tol, int32_t max_iter, double* out, cpca_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  HIPCHK(hipStreamSynchronize(h->stream));
  HostCsr hL;
  STCHK(fetch_csr("L", L, hL));
  std::vector<int32_t> w;
  STCHK(fetch_indices("omega", omega, rho, L->n, w));
  const SideHost sh = side_tables(hL, w);
  const int c = (int)L->n;
  const int KP = std::min(kApproxKMax, pow2_at_least((int)rho));
  int *inv = nullptr;
  double *dinv = nullptr, *R = nullptr;
  UpSide A;
  A.c = c;
  A.nb = (int)std::max<int64_t>(1, std::min<int64_t>(kUpMaxBlocks, ((int64_t)c * KP + kThreads - 1) / kThreads));
  auto layout = [&](Arena& a) {
    inv = a.take<int>((size_t)c);
    dinv = a.take<double>((size_t)c);
    R = a.take<double>((size_t)rho * KP);
    const size_t N = (size_t)c * KP;
    A.x = a.take<double>(N);
    A.r = a.take<double>(N);
    A.z = a.take<double>(N);
    A.p = a.take<double>(N);
    A.q = a.take<double>(N);
    A.S = a.take<double>(N);
    A.pa = a.take<double>((size_t)A.nb * KP);
    A.pb = a.take<double>((size_t)A.nb * 2 * KP);
    A.scal = a.take<double>(6 * kApproxKMax);
    A.state = a.take<int>(2 * kApproxKMax);
  };
  {
    Arena a;
    layout(a);
    STCHK(ensure_ws(h, a.off));
  }
  Arena ar;
  ar.base = h->ws;
  layout(ar);
  hipStream_t st = h->stream;
  HIPCHK(hipMemcpyAsync(inv, sh.inv.data(), sizeof(int) * c, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(dinv, sh.dinv.data(), sizeof(double) * c, hipMemcpyHostToDevice, st));
  A.rp = L->rowptr;
  A.ci = L->colind;
  A.v = L->vals;
  A.inv = inv;
  A.dinv = dinv;
  A.R = R;
  int it_max = 0, worst = 0;
  double rel_max = 0.0;
  std::vector<double> hscal(6 * kApproxKMax);
  for (int col0 = 0; col0 < (int)rho; col0 += KP) {
    const int kb = std::min(KP, (int)rho - col0);
    k_kron_rhs<<<(int)(((size_t)rho * KP + kThreads - 1) / kThreads), kThreads, 0, st>>>(R, (int)rho, KP, col0, kb);
    LAUNCHCHK();
    std::vector<int> hs;
    STCHK(upsample_solve(h, A, A, 1, KP, kb, tol, max_iter, hs));
    k_kron_rows<<<(int)(((size_t)rho * KP + kThreads - 1) / kThreads), kThreads, 0, st>>>(
        A, omega, (int)rho, KP, col0, kb, out);
    LAUNCHCHK();
    STCHK(read_states(h, A, A, 1, hs));
    HIPCHK(hipMemcpyAsync(hscal.data(), A.scal, sizeof(double) * 6 * kApproxKMax,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int j = 0; j < kb; ++j) {
      const int d = hs[(size_t)j];
      it_max = std::max(it_max, hs[(size_t)kApproxKMax + j]);
      const double bb = hscal[(size_t)2 * kApproxKMax + j], rr = hscal[(size_t)kApproxKMax + j];
      if (bb > 0.0) rel_max = std::max(rel_max, std::sqrt(rr / bb));
      if (d != 1) worst = std::max(worst, d == 0 ? 1 : d);
    }
  }
  k_kron_sym<<<(int)(((size_t)rho * rho + kThreads - 1) / kThreads), kThreads, 0, st>>>(out, (int)rho);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));
  cpca_status s = CPCA_OK;
  if (worst == 3) s = fail(CPCA_ENAN, "kron_reduce: NaN/Inf in the CG");
  else if (worst == 2) s = fail(CPCA_ENOTSPD, "kron_reduce: CG breakdown (p^T A p <= 0)");
  else if (worst == 1) s = fail(CPCA_ENOCONV, "kron_reduce: CG reached max_iter");
  fill_info(info, s, it_max, 0, rel_max, 0.0, t0);
  return s;
}
}  // namespace

extern "C" cpca_status cpca_kron_reduce(cpca_handle h, const cpca_csr* L, const int32_t* omega,
                                        int64_t rho, double tol, int32_t max_iter,
                                        double* Lred_out, cpca_info* info) {
  TraceRange trace_("cpca_kron_reduce");
  clear_error();
  if (!L || !omega || !Lred_out) return fail(CPCA_EINVAL, "kron_reduce: null argument");
  if (L->n < 1 || L->n > INT32_MAX) return fail(CPCA_EINVAL, "kron_reduce: order out of range");
  STCHK(check_csr_shape("L", L, L->n));
  if (rho < 1 || rho > L->n) return fail(CPCA_EINVAL, "kron_reduce: rho must be in [1, n]");
  if (rho > 65536) return fail(CPCA_EINVAL, "kron_reduce: rho above 65536 (dense output)");
  if (!std::isfinite(tol) || !(tol > 0)) return fail(CPCA_EINVAL, "kron_reduce: tol must be > 0");
  if (max_iter < 0) return fail(CPCA_EINVAL, "kron_reduce: max_iter < 0");
  if (!h) return fail(CPCA_EINVAL, "null handle");
  return run_kron(h, L, omega, rho, tol, max_iter, Lred_out, info);
}
