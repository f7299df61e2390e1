// Two-level preconditioner for the alternate decoder's CG (not in the paper;
// the paper solves the normal equations of its decoder, Section V-B, by
// conjugate gradients, and any SPD preconditioner reaches the same unique
// solution).
//
// Coarse space: Z = U (x) V with U the 0/1 indicator of row aggregates
// (breadth-first groups of neighbouring L_r nodes) and V the indicator of
// column ranges of kPcCols consecutive columns; a coarse vector is a
// kr x kc matrix C and Z C = U C V^T is constant on every (aggregate, range)
// tile. The preconditioner is the additive two-level one
//
//     M^-1 r = Z E^-1 Z^T r + D^-1 r,   E = Z^T A Z,   D = diag(A),
//
// with Z^T r the tile sums of r. For A(X) = (m_r m_c^T) o X + g_r L_r X +
// g_c X L_c the coarse operator acting on C is
//
//     E(C) = diag(s_r) C diag(s_c) + g_r (U^T L_r U) C diag(w_c)
//          + g_c diag(w_r) C (V^T L_c V),
//
// with s the sampled counts and w the sizes of the aggregates and ranges. E
// (K = kr kc unknowns) is assembled and inverted on the device once per
// operator and (g_r, g_c).
//
// The vector kernels map one workgroup to one row aggregate and a group of
// column ranges that one wave covers in a row (4 ranges, 1 KiB of a row, in
// FP32; 2 in FP64), split over `split` workgroups along the rows; each
// writes one partial per range, so the tile sums need no atomics, and each
// lane adds the coarse value of its own range.
#pragma once

#include "kernels.hpp"

namespace cpca {

constexpr int kPcCols = 64;          // columns per coarse column range
constexpr int kPcMaxCoarse = 4096;   // target number of coarse unknowns
constexpr int kPcMinAgg = 16;        // smallest row-aggregate size aimed at

struct PcDev {
  const int32_t* rows;   // row indices grouped by row aggregate (ascending within one)
  const int32_t* rptr;   // row aggregate a owns rows[rptr[a] .. rptr[a + 1])
  const double* ldr;     // (L_r)_ii, p values
  const double* ldc;     // (L_c)_jj, n values
  const uint8_t* mr;     // row mask, p bytes
  const uint8_t* mc;     // column mask, n bytes
  const float* Einv;     // K x K inverse of the coarse operator, row-major (FP32: a
                         // preconditioner needs no more)
  double* tp;            // per vector workgroup: rg range sums of r, <r, r>, <r, D^-1 r>
  double* W;             // K tile sums of r (Z^T r), from tp
  double* C;             // K coarse coefficients E^-1 W
  double* cpart;         // per coarse workgroup: <W, C>
  double gr, gc;
  double omega;          // weight of the Jacobi part: M^-1 = Z E^-1 Z^T + omega D^-1
  int kr, kc, K;
  int p, n;
  int rg;                // ranges per group: 4 (FP32) or 2 (FP64)
  int ng;                // range groups, ceil(kc / rg)
  int split;             // workgroups per (aggregate, group)
};

// Vector workgroups of a solve in element type T.
template <typename T>
constexpr int pc_rg() { return kWave * (16 / (int)sizeof(T)) / kPcCols; }
static_assert(kWave * 2 % kPcCols == 0 && kPcCols % 4 == 0,
              "a wave's row segment must hold whole column ranges in FP32 and FP64");
__host__ __device__ inline int pc_nwg(const PcDev& pc) { return pc.kr * pc.ng * pc.split; }

// Tile sum W_k of coarse unknown k = a kc + b from the partials.
__device__ __forceinline__ double pc_w(const PcDev& pc, int k) {
  const int a = k / pc.kc, b = k - a * pc.kc;
  const int g = b / pc.rg, q = b - g * pc.rg;
  const size_t base = ((size_t)a * pc.ng + g) * pc.split;
  double s = 0.0;
  for (int t = 0; t < pc.split; ++t) s += pc.tp[(base + t) * (pc.rg + 2) + q];
  return s;
}

// Rows of a coarse workgroup (one wave per row of E^-1).
constexpr int kPcCoarseRows = kThreads / kWave;

// The Jacobi part of the preconditioner for one lane's VEC consecutive
// columns j0.. : omega D^-1 with D(i, j) = m_r(i) m_c(j) + g_r (L_r)_ii +
// g_c (L_c)_jj, the diagonal of A (every D^-1 below stands for omega D^-1).
// It is formed in T (FP32: the hardware reciprocal), since a preconditioner
// only has to be the same fixed positive diagonal in every application of a
// solve. The column parts are read once per thread, the row parts once per
// row segment. A zero diagonal (an isolated, unsampled entry: A is singular
// there) gives 0, the pseudo-inverse.
template <typename T>
struct PcJacobi {
  static constexpr int VEC = 16 / (int)sizeof(T);
  T cp[VEC];
  uint32_t mc[VEC];
  __device__ PcJacobi(const PcDev& pc, int j0) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const bool in = j0 + v < pc.n;
      cp[v] = in ? (T)(pc.gc * pc.ldc[j0 + v]) : T(0);
      mc[v] = in ? pc.mc[j0 + v] : 0u;
    }
  }
  __device__ __forceinline__ void row(const PcDev& pc, int i, T (&dinv)[VEC]) const {
    const T rp = (T)(pc.gr * pc.ldr[i]);
    const T om = (T)pc.omega;
    const uint32_t m = pc.mr[i];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const T d = (T)(m & mc[v]) + rp + cp[v];
      if constexpr (sizeof(T) == 4)
        dinv[v] = d > T(0) ? om * __builtin_amdgcn_rcpf(d) : T(0);
      else
        dinv[v] = d > T(0) ? om / d : T(0);
    }
  }
};

// This thread's place in the vector kernels: workgroup -> (aggregate a,
// range group g, row split s); lane -> range q of the group and the first
// of its VEC columns, j0. The coarse unknown of the lane is a kc + g rg + q
// (valid when that range exists).
template <typename T>
struct PcLoc {
  int a, g, s, q, j0, k;
  bool valid;
  __device__ explicit PcLoc(const PcDev& pc) {
    constexpr int VEC = 16 / (int)sizeof(T);
    constexpr int RG = pc_rg<T>();
    const int wg = blockIdx.x;
    s = wg % pc.split;
    const int ag = wg / pc.split;
    a = ag / pc.ng;
    g = ag - a * pc.ng;
    const int lane = threadIdx.x & (kWave - 1);
    q = lane * VEC / kPcCols;
    j0 = g * RG * kPcCols + lane * VEC;
    valid = g * RG + q < pc.kc;
    k = a * pc.kc + g * RG + q;
  }
};

// Walks this workgroup's rows of its aggregate, one row segment (a wave's
// rg ranges, VEC consecutive columns per lane) per wave at a time:
// f(i, j0, e0, full) with e0 = i n + j0; full: all VEC columns exist and
// 16-byte vector access is allowed (n a multiple of VEC), else the caller
// handles the columns j0 + v < n one by one.
template <typename T, class F>
__device__ __forceinline__ void pc_walk(const PcDev& pc, const PcLoc<T>& L, F&& f) {
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int WPG = kThreads / kWave;
  if (L.j0 >= pc.n) return;
  const bool full = (pc.n % VEC) == 0;
  const int w = threadIdx.x / kWave;
  const int r0 = pc.rptr[L.a], r1 = pc.rptr[L.a + 1];
  const int step = WPG * pc.split;
  // two row segments per wave and step, so two loads per lane are in flight
  int k = r0 + L.s * WPG + w;
  for (; k + step < r1; k += 2 * step) {
    const int i = pc.rows[k], i2 = pc.rows[k + step];
    f(i, L.j0, (size_t)i * pc.n + L.j0, full);
    f(i2, L.j0, (size_t)i2 * pc.n + L.j0, full);
  }
  if (k < r1) {
    const int i = pc.rows[k];
    f(i, L.j0, (size_t)i * pc.n + L.j0, full);
  }
}

// The partials of a vector workgroup: the lane's range sum in slot q, then
// <r, r> and <r, D^-1 r>.
template <typename T>
__device__ __forceinline__ void pc_partials(const PcDev& pc, int q, double wsum, double rr,
                                            double rz) {
  constexpr int RG = pc_rg<T>();
  double acc[RG + 2];
#pragma unroll
  for (int k = 0; k < RG; ++k) acc[k] = k == q ? wsum : 0.0;
  acc[RG] = rr;
  acc[RG + 1] = rz;
  block_partials<RG + 2>(acc, pc.tp);
}

// Start of a preconditioned solve (and of every segment after a residual
// replacement): tile sums W of r and the partials <r, r>, <r, D^-1 r>.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_pcg_start(const T* __restrict__ r, PcDev pc, const CgScal* sc) {
  if (sc->done != 0 || sc->conv_it != 0) return;
  constexpr int VEC = 16 / (int)sizeof(T);
  double acc[3] = {0.0, 0.0, 0.0};
  auto add = [&](T rv, T dv) {
    acc[0] += (double)rv;
    acc[1] += (double)rv * (double)rv;
    acc[2] += (double)rv * (double)(dv * rv);
  };
  const PcLoc<T> L(pc);
  const PcJacobi<T> J(pc, L.j0);
  pc_walk<T>(pc, L, [&](int i, int j0, size_t e0, bool full) {
    T dv[VEC];
    J.row(pc, i, dv);
    if (full) {
      T rv[VEC];
      vld<T, VEC>(r + e0, rv);
#pragma unroll
      for (int v = 0; v < VEC; ++v) add(rv[v], dv[v]);
    } else {
      for (int v = 0; v < VEC && j0 + v < pc.n; ++v) add(r[e0 + v], dv[v]);
    }
  });
  pc_partials<T>(pc, L.q, acc[0], acc[1], acc[2]);
}

// r -= alpha q with alpha = rho / <p, q> (rho = <r, z> of this iteration,
// <p, q> from the product's partials); tile sums W of the new r and the
// partials <r, r>, <r, D^-1 r>. Breakdown (<p, q> <= 0) or NaN ends the solve.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_pcg_update(T* __restrict__ r, const T* __restrict__ q, CgScal* sc, int it,
             const double* __restrict__ part_pq, int nb_pq, PcDev pc) {
  if (sc->done != 0 || sc->conv_it != 0) return;
  constexpr int VEC = 16 / (int)sizeof(T);
  double t[1];
  sum_partials<1>(part_pq, nb_pq, t);
  const double pq = t[0];
  const double rho = sc->rho[it & 1];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (bad(pq) || !(pq > 0.0)) {
    if (lead) {
      sc->pq = pq;
      sc->iter = it;
      sc->done = bad(pq) ? 3 : 2;
    }
    return;
  }
  const double alpha_d = rho / pq;
  if (lead) {
    sc->pq = pq;
    sc->alpha = alpha_d;
  }
  const T alpha = (T)alpha_d;
  double acc[3] = {0.0, 0.0, 0.0};
  auto add = [&](T rv, T dv) {
    acc[0] += (double)rv;
    acc[1] += (double)rv * (double)rv;
    acc[2] += (double)rv * (double)(dv * rv);
  };
  const PcLoc<T> L(pc);
  const PcJacobi<T> J(pc, L.j0);
  pc_walk<T>(pc, L, [&](int i, int j0, size_t e0, bool full) {
    T dv[VEC];
    J.row(pc, i, dv);
    if (full) {
      T rv[VEC], qv[VEC];
      vld<T, VEC>(r + e0, rv);
      vld<T, VEC>(q + e0, qv);
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        rv[v] -= alpha * qv[v];
        add(rv[v], dv[v]);
      }
      vst<T, VEC>(r + e0, rv);
    } else {
      for (int v = 0; v < VEC && j0 + v < pc.n; ++v) {
        const T rn = r[e0 + v] - alpha * q[e0 + v];
        r[e0 + v] = rn;
        add(rn, dv[v]);
      }
    }
  });
  pc_partials<T>(pc, L.q, acc[0], acc[1], acc[2]);
}

// W = Z^T r from the vector workgroups' partials (one thread per coarse
// unknown; `it` < 0: the start of a solve or segment).
__global__ void __launch_bounds__(kThreads)
k_pcg_wsum(PcDev pc, const CgScal* sc, int it) {
  if (sc->done != 0) return;
  if (it < 0 ? sc->conv_it != 0 : sc->conv_it != 0 && sc->conv_it <= it) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < pc.K) pc.W[k] = pc_w(pc, k);
}

// C = E^-1 W, one wave per row; partials of <W, C> per workgroup. `it` < 0:
// the start of a solve or segment.
__global__ void __launch_bounds__(kThreads)
k_pcg_coarse(PcDev pc, const CgScal* sc, int it) {
  if (sc->done != 0) return;
  if (it < 0 ? sc->conv_it != 0 : sc->conv_it != 0 && sc->conv_it <= it) return;
  __shared__ double red[kPcCoarseRows];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int row = blockIdx.x * kPcCoarseRows + w;
  double wc = 0.0;
  if (row < pc.K) {
    const float* e = pc.Einv + (size_t)row * pc.K;
    double s = 0.0;
    const double* W = pc.W;
    if ((pc.K & 3) == 0) {  // rows 16-byte aligned: four values per lane and load
      for (int k = 4 * lane; k < pc.K; k += 4 * kWave) {
        const float4 v = *reinterpret_cast<const float4*>(e + k);
        s += (double)v.x * W[k] + (double)v.y * W[k + 1] + (double)v.z * W[k + 2] +
             (double)v.w * W[k + 3];
      }
    } else {
      for (int k = lane; k < pc.K; k += kWave) s += (double)e[k] * W[k];
    }
    s = wave_sum(s);
    if (lane == 0) pc.C[row] = s;
    wc = s * W[row];
  }
  if (lane == 0) red[w] = wc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int k = 0; k < kPcCoarseRows; ++k) tot += red[k];
    pc.cpart[blockIdx.x] = tot;
  }
}

// One workgroup: rho_new = <W, C> + <r, D^-1 r> = <r, M^-1 r> and <r, r>
// from the partials. it < 0 (start): rho[0] = rho_new. Else beta = rho_new /
// rho, the convergence stamp (<r, r> <= thr: conv_it = it + 1) and, in an FP32
// segment of a residual-replacement solve, the divergence test.
__global__ void __launch_bounds__(1024)
k_pcg_scalars(PcDev pc, CgScal* sc, int it, int ncw) {
  if (sc->done != 0) return;
  if (it < 0 ? sc->conv_it != 0 : sc->conv_it != 0 && sc->conv_it <= it) return;
  __shared__ double red[3][1024 / kWave];
  double a[3] = {0.0, 0.0, 0.0};
  const int nwg = pc_nwg(pc);
  for (int k = threadIdx.x; k < nwg; k += blockDim.x) {
    a[0] += pc.tp[(size_t)k * (pc.rg + 2) + pc.rg];
    a[1] += pc.tp[(size_t)k * (pc.rg + 2) + pc.rg + 1];
  }
  for (int k = threadIdx.x; k < ncw; k += blockDim.x) a[2] += pc.cpart[k];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double s = wave_sum(a[c]);
    if (lane == 0) red[c][w] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) tot[c] += red[c][k];
  const double rr = tot[0], rho_new = tot[2] + tot[1];
  if (it < 0) {
    if (bad(rho_new) || bad(rr)) {
      sc->done = 3;
      return;
    }
    sc->rho[0] = rho_new;
    sc->rho[1] = rho_new;
    return;
  }
  if (bad(rr) || bad(rho_new)) {
    sc->iter = it + 1;
    sc->done = 3;
    return;
  }
  if (sc->aux > 0.0 && rr > kDiverge * sc->aux) {
    sc->iter = it + 1;
    sc->done = 4;
    return;
  }
  sc->beta = rho_new / sc->rho[it & 1];
  sc->rho[(it + 1) & 1] = rho_new;
  sc->rr[(it + 1) & 1] = rr;
  sc->iter = it + 1;
  if (rr <= sc->thr) sc->conv_it = it + 1;
}

// x += alpha p; p = z + beta p with z = C(tile) + D^-1 r. The converging
// iteration still runs in full (see CgScal::conv_it).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_pcg_pupdate(T* __restrict__ x, T* __restrict__ p, const T* __restrict__ r, CgScal* sc, int it,
              PcDev pc) {
  if (sc->done != 0) return;
  if (sc->conv_it != 0 && sc->conv_it <= it) return;
  constexpr int VEC = 16 / (int)sizeof(T);
  const T alpha = (T)sc->alpha, beta = (T)sc->beta;
  const PcLoc<T> L(pc);
  const PcJacobi<T> J(pc, L.j0);
  const T c = L.valid ? (T)pc.C[L.k] : T(0);
  pc_walk<T>(pc, L, [&](int i, int j0, size_t e0, bool full) {
    T dv[VEC];
    J.row(pc, i, dv);
    if (full) {
      T xv[VEC], pv[VEC], rv[VEC];
      vld<T, VEC>(x + e0, xv);
      vld<T, VEC>(p + e0, pv);
      vld<T, VEC>(r + e0, rv);
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        xv[v] += alpha * pv[v];
        pv[v] = c + dv[v] * rv[v] + beta * pv[v];
      }
      vst<T, VEC>(x + e0, xv);
      vst<T, VEC>(p + e0, pv);
    } else {
      for (int v = 0; v < VEC && j0 + v < pc.n; ++v) {
        const size_t e = e0 + v;
        const T pv = p[e];
        x[e] += alpha * pv;
        p[e] = c + dv[v] * r[e] + beta * pv;
      }
    }
  });
}

// p = z = C(tile) + D^-1 r (start of a solve, or of a segment that does not
// keep its direction).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_pcg_setp(T* __restrict__ p, const T* __restrict__ r, const CgScal* sc, PcDev pc) {
  if (sc->done != 0 || sc->conv_it != 0) return;
  const PcLoc<T> L(pc);
  const PcJacobi<T> J(pc, L.j0);
  const T c = L.valid ? (T)pc.C[L.k] : T(0);
  pc_walk<T>(pc, L, [&](int i, int j0, size_t e0, bool) {
    T dv[PcJacobi<T>::VEC];
    J.row(pc, i, dv);
    for (int v = 0; v < 16 / (int)sizeof(T) && j0 + v < pc.n; ++v)
      p[e0 + v] = c + dv[v] * r[e0 + v];
  });
}

// ------------------------------------------------- coarse operator set-up
struct PcCoarseDev {
  const double* Lra;   // kr x kr: U^T L_r U
  const double* Lca;   // kc x kc: V^T L_c V
  const double* sr;    // sampled rows per aggregate
  const double* scn;   // sampled columns per range
  const double* wr;    // rows per aggregate
  const double* wc;    // columns per range
  int kr, kc, K;
};

// E (K x K) from the aggregated operators.
__global__ void __launch_bounds__(kThreads)
k_pc_assemble(PcCoarseDev cd, double gr, double gc, double* __restrict__ E) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)cd.K * cd.K) return;
  const int I = (int)(e / cd.K), J = (int)(e % cd.K);
  const int a = I / cd.kc, b = I % cd.kc, a2 = J / cd.kc, b2 = J % cd.kc;
  double v = 0.0;
  if (b == b2) v += gr * cd.Lra[(size_t)a * cd.kr + a2] * cd.wc[b];
  if (a == a2) v += gc * cd.wr[a] * cd.Lca[(size_t)b * cd.kc + b2];
  if (I == J) v += cd.sr[a] * cd.scn[b];
  E[e] = v;
}

// Blocked Gauss-Jordan inversion in place (E is symmetric positive
// definite: no pivoting). Block step kb, with bb = min(kGjB, K - kb) pivots:
// the block column Ccol = A(:, kb..) and block row Rrow = A(kb.., :) are
// saved (k_gj_save); one workgroup inverts the diagonal block D (k_gj_diag);
// T' = D^-1 Rrow outside the block and D^-1 inside it (k_gj_trow); then
//   rows of the block:      A(kb + l, j) = T'(l, j)
//   other rows, block cols: A(i, j) = -(Ccol T')(i, j)
//   other rows and cols:    A(i, j) -= (Ccol T')(i, j)
// (k_gj_update, 64 x 64 tiles, each thread 4 x 4 outputs). This is the
// scalar step A -= A(:, k) A(k, :) / A(k, k) applied to kGjB pivots at once.
constexpr int kGjB = 32;
constexpr int kGjT = 64;   // output tile of k_gj_update

__global__ void __launch_bounds__(kThreads)
k_gj_save(const double* __restrict__ A, int K, int kb, int bb, double* __restrict__ Ccol,
          double* __restrict__ Rrow) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)K * kGjB) return;
  const int i = (int)(e / kGjB), l = (int)(e % kGjB);
  Ccol[e] = l < bb ? A[(size_t)i * K + kb + l] : 0.0;                  // K x kGjB
  Rrow[(size_t)l * K + i] = l < bb ? A[(size_t)(kb + l) * K + i] : 0.0;  // kGjB x K
}

// One workgroup: D^-1 of the bb x bb diagonal block (from Rrow) by scalar
// Gauss-Jordan in LDS; a non-positive pivot sets *bad.
__global__ void __launch_bounds__(kThreads)
k_gj_diag(const double* __restrict__ Rrow, int K, int kb, int bb, double* __restrict__ Dinv,
          int* __restrict__ bad) {
  __shared__ double D[kGjB][kGjB + 1];
  __shared__ double col[kGjB], row[kGjB];
  for (int e = threadIdx.x; e < kGjB * kGjB; e += blockDim.x) {
    const int l = e / kGjB, m = e % kGjB;
    D[l][m] = (l < bb && m < bb) ? Rrow[(size_t)l * K + kb + m] : (l == m ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int k = 0; k < bb; ++k) {
    if (threadIdx.x < kGjB) {
      col[threadIdx.x] = D[threadIdx.x][k];
      row[threadIdx.x] = D[k][threadIdx.x];
    }
    __syncthreads();
    const double piv = row[k];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) *bad = 1;
      return;  // uniform: every thread read the same pivot
    }
    const double pinv = 1.0 / piv;
    for (int e = threadIdx.x; e < kGjB * kGjB; e += blockDim.x) {
      const int l = e / kGjB, m = e % kGjB;
      double v;
      if (l == k && m == k) v = pinv;
      else if (l == k) v = row[m] * pinv;
      else if (m == k) v = -col[l] * pinv;
      else v = D[l][m] - col[l] * row[m] * pinv;
      D[l][m] = v;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kGjB * kGjB; e += blockDim.x) {
    const int l = e / kGjB, m = e % kGjB;
    Dinv[e] = (l < bb && m < bb) ? D[l][m] : 0.0;
  }
}

// T'(l, j) = (D^-1 Rrow)(l, j) for columns outside the block, D^-1(l, j - kb)
// inside it (kGjB x K).
__global__ void __launch_bounds__(kThreads)
k_gj_trow(const double* __restrict__ Rrow, const double* __restrict__ Dinv, int K, int kb,
          int bb, double* __restrict__ T) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)K * kGjB) return;
  const int l = (int)(e / K), j = (int)(e % K);
  double v = 0.0;
  if (l < bb) {
    if (j >= kb && j < kb + bb) {
      v = Dinv[l * kGjB + (j - kb)];
    } else {
      for (int m = 0; m < bb; ++m) v += Dinv[l * kGjB + m] * Rrow[(size_t)m * K + j];
    }
  }
  T[e] = v;
}

__global__ void __launch_bounds__(kThreads)
k_gj_update(double* __restrict__ A, int K, int kb, int bb, const double* __restrict__ Ccol,
            const double* __restrict__ T, const int* __restrict__ bad) {
  __shared__ double Cs[kGjT][kGjB + 1];
  __shared__ double Ts[kGjB][kGjT + 1];
  if (*bad) return;
  const int ntj = (K + kGjT - 1) / kGjT;
  const int i0 = (blockIdx.x / ntj) * kGjT, j0 = (blockIdx.x % ntj) * kGjT;
  for (int e = threadIdx.x; e < kGjT * kGjB; e += blockDim.x) {
    const int r = e / kGjB, l = e % kGjB;
    Cs[r][l] = i0 + r < K ? Ccol[(size_t)(i0 + r) * kGjB + l] : 0.0;
    const int l2 = e / kGjT, c = e % kGjT;
    Ts[l2][c] = j0 + c < K ? T[(size_t)l2 * K + j0 + c] : 0.0;
  }
  __syncthreads();
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int l = 0; l < kGjB; ++l) {
    double ca[4], tb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) ca[a] = Cs[ty * 4 + a][l];
#pragma unroll
    for (int b = 0; b < 4; ++b) tb[b] = Ts[l][tx * 4 + b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += ca[a] * tb[b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + ty * 4 + a;
    if (i >= K) continue;
    const bool irow = i >= kb && i < kb + bb;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + tx * 4 + b;
      if (j >= K) continue;
      const size_t e = (size_t)i * K + j;
      if (irow) {
        A[e] = Ts[i - kb][tx * 4 + b];
      } else {
        const bool jcol = j >= kb && j < kb + bb;
        A[e] = (jcol ? 0.0 : A[e]) - acc[a][b];
      }
    }
  }
}

// B = (A + A^T) / 2 rounded to FP32 (the inverse the iterations use).
__global__ void __launch_bounds__(kThreads)
k_symmetrize_f32(const double* __restrict__ A, int K, float* __restrict__ B) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)K * K) return;
  const int i = (int)(e / K), j = (int)(e % K);
  B[e] = (float)(0.5 * (A[e] + A[(size_t)j * K + i]));
}

}  // namespace cpca
