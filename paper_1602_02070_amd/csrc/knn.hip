// K-nearest-neighbour Gaussian-kernel graphs and their Laplacians on the GPU
// (Section II: each point is joined to its K nearest neighbours in Euclidean
// distance, W_ij = exp(-||y_i - y_j||^2 / sigma^2) on the union of the
// directed relations, L = D - W or D^{-1/2} (D - W) D^{-1/2}; Section VII-A:
// K = 10, sigma from the mean K-NN distance).
//
//   cpca_knn_graph   points (N x d, FP64, device) -> CSR Laplacian
//
// Stages, all on the handle's stream:
//  1. k_sqnorm: ||y_i||^2.
//  2. k_knn_tiles: every workgroup takes 128 queries and one segment of the
//     points, which it sweeps in tiles of 256 (128 for K > 12). The Gram tile
//     <y_q, y_c> comes from FP64 MFMA (v_mfma_f64_16x16x4f64, the coordinates
//     staged through LDS in chunks of 16), the squared distance is
//     ||y_q||^2 + ||y_c||^2 - 2 <y_q, y_c>, and four threads per query keep
//     the CAP smallest (distance, index) pairs of their quarter of each
//     64-wide slab in registers. The four lists are merged by (distance,
//     index) and written per (query, segment). The segments exist only to
//     give every compute unit the same number of workgroups; a workgroup's
//     list is the exact CAP smallest of its segment, so the merged result
//     does not depend on how many segments there are.
//     k_knn_merge: per query, the segment lists are merged into the CAP
//     smallest, and those CAP >= K + 4 candidates are re-ranked by their
//     squared distance recomputed directly (sum over coordinates of squared
//     differences, in coordinate order, without contraction): the expanded
//     form only selects candidates, the order and the distances are the
//     direct ones.
//  3. k_knn_sigma: partial sums of the K-NN distances (deterministic order).
//  4. k_knn_extra: each directed relation i -> j whose reverse j -> i is not
//     a relation adds one entry to row j (the union); counted with integer
//     atomics (the count does not depend on their order).
//  5. k_knn_rowptr: row lengths 1 + K + extra, exclusive scan, one workgroup.
//  6. k_knn_fill: row i gets its diagonal, its K neighbours and its extra
//     entries (those in an atomically claimed slot order), then one thread
//     per row sorts the row by column, turns distances into weights and sums
//     the degree in column order (deterministic).
//  7. k_knn_values: Laplacian values from weights and degrees.
#include "common.hpp"

namespace {

constexpr int kQT = 128;        // queries per workgroup (16 per wave)
constexpr int kKnnThreads = 512;
constexpr int kSlab = 64;       // candidates per selection slab
constexpr int kDK = 16;         // coordinates per staged chunk
constexpr int kDKP = kDK + 1;   // LDS row stride of the staged chunks (doubles)
constexpr int kDS = 32;         // candidates per distance slab (selection pass)
constexpr int kDTP = kDS + 1;   // LDS row stride of the distance slab
constexpr int kMaxSeg = 8;      // most candidate segments per query block

typedef double d4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kThreads)
k_sqnorm(const double* __restrict__ Y, int N, int d, double* __restrict__ sq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double* y = Y + (size_t)i * d;
  double s = 0.0;
  for (int k = 0; k < d; ++k) s += y[k] * y[k];
  sq[i] = s;
}

// Squared distance of points a and b summed over coordinates in order,
// each term and sum rounded separately (the order a plain loop takes).
__device__ double direct_d2(const double* __restrict__ Y, int d, int a, int b) {
  const double* ya = Y + (size_t)a * d;
  const double* yb = Y + (size_t)b * d;
  double s = 0.0;
  for (int k = 0; k < d; ++k) {
    const double t = __dsub_rn(ya[k], yb[k]);
    s = __dadd_rn(s, __dmul_rn(t, t));
  }
  return s;
}

// Inserts (x, c) into the ascending list (vd, vi) of CAP entries; an equal
// key goes after the entries already there (they came from lower indices).
template <int CAP>
__device__ __forceinline__ void list_insert(double (&vd)[CAP], int (&vi)[CAP], double x, int c) {
  bool placed = false;
#pragma unroll
  for (int k = CAP - 1; k >= 1; --k) {
    const bool shift = vd[k - 1] > x;
    const bool put = !placed && !shift;
    const double nd = shift ? vd[k - 1] : (put ? x : vd[k]);
    const int ni = shift ? vi[k - 1] : (put ? c : vi[k]);
    placed = placed || put;
    vd[k] = nd;
    vi[k] = ni;
  }
  if (!placed) {
    vd[0] = x;
    vi[0] = c;
  }
}

// (d, i) < (e, j) in the lexicographic order.
__device__ __forceinline__ bool lex_less(double d, int i, double e, int j) {
  return d < e || (d == e && i < j);
}

// Inserts (x, c) into a list ascending by (distance, index); the caller has
// checked that it beats the last entry.
template <int CAP>
__device__ __forceinline__ void lex_insert(double (&vd)[CAP], int (&vi)[CAP], double x, int c) {
  bool placed = false;
#pragma unroll
  for (int k = CAP - 1; k >= 1; --k) {
    const bool shift = lex_less(x, c, vd[k - 1], vi[k - 1]);
    const bool put = !placed && !shift;
    const double nd = shift ? vd[k - 1] : (put ? x : vd[k]);
    const int ni = shift ? vi[k - 1] : (put ? c : vi[k]);
    placed = placed || put;
    vd[k] = nd;
    vi[k] = ni;
  }
  if (!placed) {
    vd[0] = x;
    vi[0] = c;
  }
}

// NS slabs of 64 candidates per tile: 4 with CAP = 16; 2 with CAP = 32, whose
// longer lists leave registers for only half the accumulators.
template <int CAP, int NS>
__global__ void __launch_bounds__(kKnnThreads)
k_knn_tiles(const double* __restrict__ Y, const double* __restrict__ sq, int N, int d, int nqb,
            int tiles_per_seg, int nseg, int* __restrict__ seg_idx, double* __restrict__ seg_d2) {
  constexpr int kCT = kSlab * NS;  // candidates per tile
  static_assert(kCT % kQT == 0, "the candidate tile is staged in rows of kQT");
  // staged chunks, double-buffered: chunk i is computed from one buffer while
  // chunk i + 1 is stored into the other, one barrier per chunk
  __shared__ double Qs[2][kQT * kDKP];
  __shared__ double Cs[2][kCT * kDKP];
  __shared__ double Ds[kQT * kDTP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  // workgroups of one segment are consecutive, so the workgroups in flight
  // sweep the same candidate tiles
  const int qb = blockIdx.x % nqb, seg = blockIdx.x / nqb;
  const int q0 = qb * kQT;
  const long long cb = (long long)seg * tiles_per_seg * kCT;
  const int cbeg = (int)(cb < N ? cb : N);
  const int cend = (int)(cb + (long long)tiles_per_seg * kCT < N ? cb + (long long)tiles_per_seg * kCT : N);
  // selection role: query qs of the tile, candidate quarter sub of a slab
  const int qs = tid >> 2, sub = tid & 3;
  const int qglob = q0 + qs;
  double vd[CAP];
  int vi[CAP];
#pragma unroll
  for (int k = 0; k < CAP; ++k) {
    vd[k] = __builtin_inf();
    vi[k] = 0x7fffffff;
  }
  const int d4pad = (d + 3) & ~3;
  // squared norms of the 4 query rows this lane holds in the MFMA output:
  // row (lane / 16) + 4 v of the wave's 16-row block
  double sqq[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int q = q0 + 16 * wid + (lane >> 4) + 4 * v;
    sqq[v] = q < N ? sq[q] : 0.0;
  }
  // (candidate tile, coordinate chunk) steps in order; the next step's
  // coordinates are loaded into registers before the current step's MFMAs,
  // so their global-memory latency overlaps the matrix work. Thread t stages
  // row t / 4 of the query chunk and rows t / 4 + 128 j of the candidate
  // chunk, coordinates 4 (t % 4) .. 4 (t % 4) + 3.
  // A row outside the range (queries past N, candidates past the segment)
  // is read from row 0 instead: its Gram entries are never used (those
  // distances are set to infinity, those queries are not written).
  // Coordinates past d must be zero, since they would enter every dot
  // product: only the last chunk checks them.
  constexpr int CG = kCT / kQT;
  const int r_st = tid >> 2, cc_st = (tid & 3) * 4;
  double qr[4], cr[CG][4];
  const double* qrow = Y + (size_t)(q0 + r_st < N ? q0 + r_st : 0) * d + cc_st;
  const double* crow[CG];
  auto set_rows = [&](int c0) {
#pragma unroll
    for (int j = 0; j < CG; ++j) {
      const int cg = c0 + r_st + kQT * j;
      crow[j] = Y + (size_t)(cg < cend ? cg : 0) * d + cc_st;
    }
  };
  auto load_chunk = [&](int k0) {
    if (k0 + kDK <= d) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        qr[u] = qrow[k0 + u];
#pragma unroll
        for (int j = 0; j < CG; ++j) cr[j][u] = crow[j][k0 + u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool in = k0 + cc_st + u < d;
        qr[u] = in ? qrow[k0 + u] : 0.0;
#pragma unroll
        for (int j = 0; j < CG; ++j) cr[j][u] = in ? crow[j][k0 + u] : 0.0;
      }
    }
  };
  d4 acc[4 * NS];
#pragma unroll
  for (int t = 0; t < 4 * NS; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      Qs[buf][r_st * kDKP + cc_st + u] = qr[u];
#pragma unroll
      for (int j = 0; j < CG; ++j) Cs[buf][(r_st + kQT * j) * kDKP + cc_st + u] = cr[j][u];
    }
  };
  // the chunk after (c, k): the next 16 coordinates, or the next tile
  auto advance = [&](int c, int k, int& nc, int& nk) {
    nk = k + kDK;
    nc = c;
    if (nk >= d4pad) {
      nk = 0;
      nc = c + kCT;
    }
  };
  int c0 = cbeg, k0 = 0, cur = 0, nc0 = cend, nk0 = 0;
  if (c0 < cend) {
    set_rows(c0);
    load_chunk(0);
    store_chunk(0);
    advance(c0, k0, nc0, nk0);
    if (nc0 < cend) {
      if (nc0 != c0) set_rows(nc0);
      load_chunk(nk0);
    }
  }
  __syncthreads();
  while (c0 < cend) {
    // buffer cur holds chunk (c0, k0); the registers hold chunk (nc0, nk0)
    // A: row lane % 16, k = lane / 16 of the 16 x 4 block; B likewise
    const double* qa = &Qs[cur][(16 * wid + (lane & 15)) * kDKP + (lane >> 4)];
    const double* cb = &Cs[cur][(lane & 15) * kDKP + (lane >> 4)];
    auto kstep = [&](int s) {
      const double a = qa[4 * s];
#pragma unroll
      for (int t = 0; t < 4 * NS; ++t) {
        const double b = cb[16 * t * kDKP + 4 * s];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
      }
    };
    // (not unrolled: the hoisted operand reads of four steps would not fit
    // in the registers next to the accumulators)
    const int ksteps = min(kDK, d4pad - k0) >> 2;
#pragma unroll 1
    for (int s = 0; s < ksteps; ++s) kstep(s);
    // the other buffer was last read by the previous chunk, before the
    // barrier every wave has passed since
    if (nc0 < cend) store_chunk(cur ^ 1);
    __syncthreads();
    if (nk0 == 0) {
      // tile complete: slab by slab, the approximate squared distances go to
      // the distance slab (output row (lane / 16) + 4 v, column lane % 16 of
      // each 16 x 16 block) and are scanned by the selection threads
#pragma unroll
      for (int sl = 0; sl < kCT / kDS; ++sl) {
#pragma unroll
        for (int t2 = 0; t2 < kDS / 16; ++t2) {
          const int t = (kDS / 16) * sl + t2;
          const int cl = 16 * t2 + (lane & 15);
          const int c = c0 + kDS * sl + cl;
          const double sqc = c < cend ? sq[c] : 0.0;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ql = 16 * wid + (lane >> 4) + 4 * v;
            const int q = q0 + ql;
            double dv = sqq[v] + sqc - 2.0 * acc[t][v];
            if (c >= cend || c == q) dv = __builtin_inf();
            Ds[ql * kDTP + cl] = dv;
          }
          acc[t] = d4{0.0, 0.0, 0.0, 0.0};
        }
        __syncthreads();
        // selection: this thread's kDS / 4 candidates of the slab, in
        // increasing index
#pragma unroll
        for (int m = 0; m < kDS / 4; ++m) {
          const int cl = (kDS / 4) * sub + m;
          const double x = Ds[qs * kDTP + cl];
          if (x < vd[CAP - 1]) list_insert<CAP>(vd, vi, x, c0 + kDS * sl + cl);
        }
        __syncthreads();
      }
    }
    c0 = nc0;
    k0 = nk0;
    cur ^= 1;
    if (c0 < cend) {
      advance(c0, k0, nc0, nk0);
      if (nc0 < cend) {
        if (nc0 != c0) set_rows(nc0);
        load_chunk(nk0);
      }
    }
  }
  // merge the four quarter lists of each query (lanes 4 qs .. 4 qs + 3 of
  // the wave) into the first one by (approximate distance, index)
  double bd[CAP];
  int bi[CAP];
#pragma unroll
  for (int k = 0; k < CAP; ++k) {
    bd[k] = vd[k];
    bi[k] = vi[k];
  }
  const int base_lane = lane & ~3;
#pragma unroll
  for (int src = 1; src < 4; ++src) {
#pragma unroll
    for (int k = 0; k < CAP; ++k) {
      const double x = __shfl(vd[k], base_lane + src, 64);
      const int c = __shfl(vi[k], base_lane + src, 64);
      if (sub == 0 && c != 0x7fffffff && lex_less(x, c, bd[CAP - 1], bi[CAP - 1]))
        lex_insert<CAP>(bd, bi, x, c);
    }
  }
  if (sub == 0 && qglob < N) {
    const size_t o = ((size_t)qglob * nseg + seg) * CAP;
#pragma unroll
    for (int k = 0; k < CAP; ++k) {
      seg_idx[o + k] = bi[k];
      seg_d2[o + k] = bd[k];
    }
  }
}

// One thread per query: the nseg segment lists (each ascending by
// (approximate distance, index)) are merged into the CAP smallest, which are
// re-ranked by the directly computed squared distance; the first K go out.
template <int CAP>
__global__ void __launch_bounds__(kThreads)
k_knn_merge(const double* __restrict__ Y, int N, int d, int K, int nseg,
            const int* __restrict__ seg_idx, const double* __restrict__ seg_d2,
            int* __restrict__ out_idx, double* __restrict__ out_d2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N) return;
  double bd[CAP];
  int bi[CAP];
  const size_t o0 = (size_t)q * nseg * CAP;
#pragma unroll
  for (int k = 0; k < CAP; ++k) {
    bd[k] = seg_d2[o0 + k];
    bi[k] = seg_idx[o0 + k];
  }
  for (int sg = 1; sg < nseg; ++sg) {
    const size_t o = o0 + (size_t)sg * CAP;
    for (int k = 0; k < CAP; ++k) {
      const double x = seg_d2[o + k];
      const int c = seg_idx[o + k];
      // the list is ascending: once an entry does not make it, none after it does
      if (c == 0x7fffffff || !lex_less(x, c, bd[CAP - 1], bi[CAP - 1])) break;
      lex_insert<CAP>(bd, bi, x, c);
    }
  }
  // re-rank by the directly computed squared distance
  for (int k = 0; k < CAP; ++k) bd[k] = bi[k] < N ? direct_d2(Y, d, q, bi[k]) : __builtin_inf();
  for (int a = 1; a < CAP; ++a) {
    const double x = bd[a];
    const int c = bi[a];
    int pos = a;
    while (pos > 0 && lex_less(x, c, bd[pos - 1], bi[pos - 1])) {
      bd[pos] = bd[pos - 1];
      bi[pos] = bi[pos - 1];
      --pos;
    }
    bd[pos] = x;
    bi[pos] = c;
  }
  for (int k = 0; k < K; ++k) {
    out_idx[(size_t)q * K + k] = bi[k];
    out_d2[(size_t)q * K + k] = bd[k];
  }
}

// Partial sums of sqrt(d2) over the N K relations (one per workgroup).
__global__ void __launch_bounds__(kThreads)
k_knn_sigma(const double* __restrict__ d2, size_t NK, double* __restrict__ part) {
  double acc[1] = {0.0};
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < NK;
       e += (size_t)gridDim.x * blockDim.x)
    acc[0] += sqrt(d2[e]);
  block_partials<1>(acc, part);
}

// sigma = total / (N K) in one workgroup; out[0] = sigma.
__global__ void __launch_bounds__(kThreads)
k_knn_sigma_final(const double* __restrict__ part, int nb, double count, double* __restrict__ out) {
  double t[1];
  sum_partials<1>(part, nb, t);
  if (threadIdx.x == 0) out[0] = t[0] / count;
}

__device__ __forceinline__ bool is_relation(const int* __restrict__ idx, int K, int from, int to) {
  const int* r = idx + (size_t)from * K;
  for (int k = 0; k < K; ++k)
    if (r[k] == to) return true;
  return false;
}

// extra[j] += 1 for every relation i -> j without its reverse.
__global__ void __launch_bounds__(kThreads)
k_knn_extra(const int* __restrict__ idx, int N, int K, int* __restrict__ extra) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)N * K) return;
  const int i = (int)(e / K);
  const int j = idx[e];
  if (j < 0 || j >= N) return;  // no neighbour (non-finite input; rejected before this)
  if (!is_relation(idx, K, j, i)) atomicAdd(&extra[j], 1);
}

// rowptr[i] = sum_{k < i} (1 + K + extra[k]) in one workgroup; rowptr[N] = nnz.
__global__ void __launch_bounds__(1024)
k_knn_rowptr(const int* __restrict__ extra, int N, int K, int* __restrict__ rowptr) {
  __shared__ long long tot[1024];
  const int T = blockDim.x;
  const int per = (N + T - 1) / T;
  const int b = threadIdx.x * per, e = min(N, b + per);
  long long s = 0;
  for (int i = b; i < e; ++i) s += 1 + K + extra[i];
  tot[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long run = 0;
    for (int t = 0; t < T; ++t) {
      const long long v = tot[t];
      tot[t] = run;
      run += v;
    }
  }
  __syncthreads();
  long long run = tot[threadIdx.x];
  for (int i = b; i < e; ++i) {
    rowptr[i] = (int)run;
    run += 1 + K + extra[i];
  }
  if (threadIdx.x == T - 1) rowptr[N] = (int)run;
}

// Row i: diagonal, its K relations, then (claimed through fillpos) the
// reverse entries; colind/vals hold column and squared distance for now.
__global__ void __launch_bounds__(kThreads)
k_knn_scatter(const int* __restrict__ idx, const double* __restrict__ d2, int N, int K,
              const int* __restrict__ rowptr, int* __restrict__ fillpos, int* __restrict__ colind,
              double* __restrict__ vals) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)N * K) return;
  const int i = (int)(e / K);
  const int k = (int)(e % K);
  const int j = idx[e];
  if (j < 0 || j >= N) return;
  const int base = rowptr[i];
  if (k == 0) {
    colind[base] = i;
    vals[base] = 0.0;
  }
  colind[base + 1 + k] = j;
  vals[base + 1 + k] = d2[e];
  if (!is_relation(idx, K, j, i)) {
    const int slot = atomicAdd(&fillpos[j], 1);
    const int pos = rowptr[j] + 1 + K + slot;
    colind[pos] = i;
    vals[pos] = d2[e];
  }
}

// One thread per row: sort by column, weights exp(-d2 / sigma^2) on the
// off-diagonal entries (the diagonal slot keeps 0), degree in column order.
__global__ void __launch_bounds__(kThreads)
k_knn_rows(int N, const int* __restrict__ rowptr, int* __restrict__ colind,
           double* __restrict__ vals, const double* __restrict__ sigma, double* __restrict__ deg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int b = rowptr[i], e = rowptr[i + 1];
  for (int a = b + 1; a < e; ++a) {
    const int c = colind[a];
    const double v = vals[a];
    int pos = a;
    while (pos > b && colind[pos - 1] > c) {
      colind[pos] = colind[pos - 1];
      vals[pos] = vals[pos - 1];
      --pos;
    }
    colind[pos] = c;
    vals[pos] = v;
  }
  const double s2 = sigma[0] * sigma[0];
  double dg = 0.0;
  for (int a = b; a < e; ++a) {
    if (colind[a] == i) continue;
    const double w = exp(-vals[a] / s2);
    vals[a] = w;
    dg += w;
  }
  deg[i] = dg;
}

// Laplacian values: combinatorial (diag = degree, off-diagonal -w) or
// normalised (diag = 1, off-diagonal -w / sqrt(deg_i deg_j)).
__global__ void __launch_bounds__(kThreads)
k_knn_values(int N, const int* __restrict__ rowptr, const int* __restrict__ colind,
             double* __restrict__ vals, const double* __restrict__ deg, int normalized) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int a = rowptr[i]; a < rowptr[i + 1]; ++a) {
    const int j = colind[a];
    if (j == i)
      vals[a] = normalized ? 1.0 : deg[i];
    else
      vals[a] = normalized ? -vals[a] / sqrt(deg[i] * deg[j]) : -vals[a];
  }
}

// Number of candidate segments per query block: the one (at most kMaxSeg,
// each segment at least 4 tiles) that fills the last round of workgroups
// best, one resident workgroup per compute unit; ties go to fewer segments.
int knn_segments(int nqb, int ntiles, int ncu) {
  int best = 1;
  double best_eff = 0.0;
  for (int s = 1; s <= kMaxSeg; ++s) {
    if (s > 1 && (ntiles + s - 1) / s < 4) break;
    const long long wg = (long long)nqb * s;
    const long long rounds = (wg + ncu - 1) / ncu;
    const double eff = (double)wg / (double)(rounds * ncu);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = s;
    }
  }
  return best;
}

template <int CAP, int NS>
hipError_t launch_tiles(hipStream_t s, const double* Y, const double* sq, int N, int d, int nqb,
                        int tps, int nseg, int* seg_idx, double* seg_d2) {
  k_knn_tiles<CAP, NS><<<nqb * nseg, kKnnThreads, 0, s>>>(Y, sq, N, d, nqb, tps, nseg, seg_idx, seg_d2);
  return hipGetLastError();
}

template <int CAP>
hipError_t launch_merge(hipStream_t s, const double* Y, int N, int d, int K, int nseg,
                        const int* seg_idx, const double* seg_d2, int* idx, double* d2) {
  k_knn_merge<CAP><<<(N + kThreads - 1) / kThreads, kThreads, 0, s>>>(Y, N, d, K, nseg, seg_idx,
                                                                      seg_d2, idx, d2);
  return hipGetLastError();
}

}  // namespace

extern "C" cpca_status cpca_knn_graph(cpca_handle h, const double* points, int64_t N, int64_t d,
                                      int32_t K, int32_t normalized, int32_t* rowptr_out,
                                      int32_t* colind_out, double* vals_out, int64_t nnz_cap,
                                      int64_t* nnz_out, double* sigma_out, int32_t* knn_out,
                                      cpca_info* info) {
  TraceRange trace_("cpca_knn_graph");
  clear_error();
  const auto t0 = std::chrono::steady_clock::now();
  if (!points || !rowptr_out || !colind_out || !vals_out || !nnz_out || !sigma_out)
    return fail(CPCA_EINVAL, "knn_graph: null argument");
  if (N < 2 || N > (1 << 28)) return fail(CPCA_EINVAL, "knn_graph: N must be in [2, 2^28]");
  if (d < 1 || d > (1 << 20)) return fail(CPCA_EINVAL, "knn_graph: d must be in [1, 2^20]");
  if (K < 1 || K > 28 || K >= N) return fail(CPCA_EINVAL, "knn_graph: K must be in [1, min(28, N - 1)]");
  if (normalized != 0 && normalized != 1) return fail(CPCA_EINVAL, "knn_graph: normalized must be 0 or 1");
  const long long need = (long long)N * (2LL * K + 1);
  if (need > INT32_MAX) return fail(CPCA_EINVAL, "knn_graph: N (2K + 1) exceeds the int32 CSR range");
  if (nnz_cap < need) return fail(CPCA_EINVAL, "knn_graph: nnz_cap must be at least N (2K + 1)");
  if (!h) return fail(CPCA_EINVAL, "null handle");
  HIPCHK(hipStreamSynchronize(h->stream));
  const int n = (int)N, dd = (int)d;
  const size_t NK = (size_t)N * K;
  const int nb = 256;
  const int cap = K <= 12 ? 16 : 32;
  int ncu = 0;
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
  const int nqb = (n + kQT - 1) / kQT;
  const int ct = cap == 16 ? 4 * kSlab : 2 * kSlab;  // candidates per tile
  const int ntiles = (n + ct - 1) / ct;
  const int nseg = knn_segments(nqb, ntiles, std::max(1, ncu));
  const int tps = (ntiles + nseg - 1) / nseg;
  double *sq = nullptr, *d2 = nullptr, *part = nullptr, *deg = nullptr, *sd2 = nullptr;
  int *idx = nullptr, *extra = nullptr, *fill = nullptr, *sidx = nullptr;
  auto layout = [&](Arena& a) {
    sd2 = a.take<double>((size_t)N * nseg * cap);
    sidx = a.take<int>((size_t)N * nseg * cap);
    sq = a.take<double>((size_t)N);
    d2 = a.take<double>(NK);
    idx = a.take<int>(NK);
    extra = a.take<int>((size_t)N);
    fill = a.take<int>((size_t)N);
    deg = a.take<double>((size_t)N);
    part = a.take<double>(nb + 8);
  };
  {
    Arena a;
    layout(a);
    STCHK(ensure_ws(h, a.off));
  }
  Arena a;
  a.base = h->ws;
  layout(a);
  double* sig = results_ptr(h) + 16;
  const int g1 = (n + kThreads - 1) / kThreads;
  k_sqnorm<<<g1, kThreads, 0, h->stream>>>(points, n, dd, sq);
  LAUNCHCHK();
  STCHK(prof_begin(h, FAM_OTHER));
  hipError_t e = cap == 16 ? launch_tiles<16, 4>(h->stream, points, sq, n, dd, nqb, tps, nseg, sidx, sd2)
                           : launch_tiles<32, 2>(h->stream, points, sq, n, dd, nqb, tps, nseg, sidx, sd2);
  if (e != hipSuccess) return fail(CPCA_EHIP, std::string("launch: ") + hipGetErrorString(e));
  STCHK(prof_end(h));
  e = cap == 16 ? launch_merge<16>(h->stream, points, n, dd, K, nseg, sidx, sd2, idx, d2)
                : launch_merge<32>(h->stream, points, n, dd, K, nseg, sidx, sd2, idx, d2);
  if (e != hipSuccess) return fail(CPCA_EHIP, std::string("launch: ") + hipGetErrorString(e));
  k_knn_sigma<<<nb, kThreads, 0, h->stream>>>(d2, NK, part);
  LAUNCHCHK();
  k_knn_sigma_final<<<1, kThreads, 0, h->stream>>>(part, nb, (double)NK, sig);
  LAUNCHCHK();
  // sigma decides whether a Gaussian kernel exists: check it before any
  // output is written
  STCHK(read_fixed(h));
  const double sigma = host_results(h)[16];
  if (!std::isfinite(sigma)) return fail(CPCA_ENAN, "knn_graph: NaN or Inf in the points");
  if (!(sigma > 0)) return fail(CPCA_EINVAL, "knn_graph: every neighbour distance is zero (sigma = 0)");
  k_fill<int><<<vec_grid((size_t)2 * N), kThreads, 0, h->stream>>>(extra, 0, (size_t)N);
  LAUNCHCHK();
  k_fill<int><<<vec_grid((size_t)N), kThreads, 0, h->stream>>>(fill, 0, (size_t)N);
  LAUNCHCHK();
  const int gk = (int)((NK + kThreads - 1) / kThreads);
  k_knn_extra<<<gk, kThreads, 0, h->stream>>>(idx, n, K, extra);
  LAUNCHCHK();
  k_knn_rowptr<<<1, 1024, 0, h->stream>>>(extra, n, K, rowptr_out);
  LAUNCHCHK();
  k_knn_scatter<<<gk, kThreads, 0, h->stream>>>(idx, d2, n, K, rowptr_out, fill, colind_out, vals_out);
  LAUNCHCHK();
  k_knn_rows<<<g1, kThreads, 0, h->stream>>>(n, rowptr_out, colind_out, vals_out, sig, deg);
  LAUNCHCHK();
  k_knn_values<<<g1, kThreads, 0, h->stream>>>(n, rowptr_out, colind_out, vals_out, deg, normalized);
  LAUNCHCHK();
  if (knn_out)
    HIPCHK(hipMemcpyAsync(knn_out, idx, NK * sizeof(int), hipMemcpyDeviceToDevice, h->stream));
  int last = 0;
  HIPCHK(hipMemcpyAsync(&last, rowptr_out + N, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  STCHK(read_fixed(h));
  STCHK(prof_collect(h));
  *sigma_out = sigma;
  *nnz_out = last;
  fill_info(info, CPCA_OK, 0, 0, 0.0, 0.0, t0);
  return CPCA_OK;
}
