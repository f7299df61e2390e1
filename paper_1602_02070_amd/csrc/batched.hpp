// Batched solves: many independent (instance, gamma) tasks of uneven sizes
// advance together. Every launch covers all tasks; a workgroup finds its task
// through a block -> task table and works on that task's slice of the grid.
// A task whose solve has finished makes its workgroups return at once, so a
// captured chunk of iterations can be replayed until every task is done.
//
// All task matrices use a padded row stride ld (a multiple of 16 bytes /
// sizeof(T)); padding columns and padded mask entries are zero, so the
// vector code paths of the single-problem kernels apply unchanged.
#pragma once

#include "kernels.hpp"

namespace cpca {

// Device view of one task. Operator images (graphs, masks) belong to the
// task's instance and are shared by all gammas of that instance.
struct BTask {
  int p, n, ld;           // operand shape, row stride
  int rho_r, rho_c, ldt;  // sampled shape and its row stride (FISTA)
  double gr, gc;          // gammas (FISTA and decoder)
  double lam;             // FISTA step 1 / beta' (0: no graph term)
  // decoder operator images
  CsrDev<double> Lr64;
  SellDev<double> Lc64;
  CsrDev<float> Lr32;
  SellDev<float> Lc32;
  const uint8_t* mr;      // p
  const uint8_t* mc;      // ld (zero-padded)
  // FISTA operator image (sampled graphs, zero masks)
  CsrDev<double> Lrt;
  SellDev<double> Lct;
  const uint8_t* zmr;     // rho_r zeros
  const uint8_t* zmc;     // ldt zeros
  const int* om_r;        // sampling sets (device, from the caller)
  const int* om_c;
  // FISTA state (FP64, rho_r x ldt)
  const double* Y;        // padded Y~ of the instance
  double* S;
  double* Za;
  double* Zb;
  // decoder state (p x ld)
  double* B64;
  double* X64;
  double* r64;
  double* p64;
  double* q64;
  float* B32;
  float* x32;
  float* r32;
  float* p32;
  float* q32;
  CgScal* sc;
  double inner_rel2;      // residual replacement: segment stop, relative to ||round(R)||^2
  double floor2;          // residual replacement: segments need not go below this ||r||^2
  int active;             // refinement: 0 once the task has converged
  int keep_p;             // residual pass keeps the search direction (a replacement)
  int reset_p;            // P_P_FROM_R: restart the direction, p = r
  int pad0;
  // grid slices
  int ablk0, aper, anrb;  // decoder fused product: blocks [ablk0, ablk0 + 8 aper)
  int fblk0, fper, fnrb;  // FISTA fused product
  int vblk0, nvblk;       // vector kernels (p * ld elements)
};

enum BKind { B_CG32 = 0, B_CG64 = 1, B_RES = 2, B_FISTA = 3, B_RESNORM = 4 };

// One fused-product launch over all tasks. KIND selects operand, operator
// image and epilogue.
template <typename T, int R, bool LDS, int VEC, int KIND>
__global__ void __launch_bounds__(kThreads)
k_apply_batched(const BTask* __restrict__ tasks, const int* __restrict__ blk_task,
                double* partials, double fista_c, int par) {
  const int b = blockIdx.x;
  const BTask& tk = tasks[blk_task[b]];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* panel = reinterpret_cast<T*>(smem_raw);
  const bool fista = KIND == B_FISTA;
  const int blk0 = fista ? tk.fblk0 : tk.ablk0;
  const int per = fista ? tk.fper : tk.aper;
  const int nrb = fista ? tk.fnrb : tk.anrb;
  const int rows_total = fista ? tk.rho_r : tk.p;
  const int ncols = fista ? tk.rho_c : tk.n;
  const int ld = fista ? tk.ldt : tk.ld;
  const int local = b - blk0;
  const int rb = (local & 7) * per + (local >> 3);
  const int i0 = rb * R;
  const int rows = rb < nrb ? min(R, rows_total - i0) : 0;
  double acc[2] = {0.0, 0.0};
  if constexpr (KIND == B_CG32) {
    EpiCg<float> epi;
    epi.Q = tk.q32;
    epi.gr = (float)tk.gr;
    epi.gc = (float)tk.gc;
    epi.partials = partials;
    epi.sc = tk.sc;
    if (epi.prologue()) return;
    if (rows > 0)
      apply_rows<float, R, LDS, VEC, 0>(tk.p32, ld, ncols, tk.Lr32, tk.Lc32, BandDev<float>{}, tk.mr, tk.mc, i0, rows,
                                     epi, acc, reinterpret_cast<float*>(panel));
    double a1[1] = {acc[0]};
    block_partials<1>(a1, partials);
  } else if constexpr (KIND == B_CG64) {
    EpiCg<double> epi;
    epi.Q = tk.q64;
    epi.gr = tk.gr;
    epi.gc = tk.gc;
    epi.partials = partials;
    epi.sc = tk.sc;
    if (epi.prologue()) return;
    if (rows > 0)
      apply_rows<double, R, LDS, VEC, 0>(tk.p64, ld, ncols, tk.Lr64, tk.Lc64, BandDev<double>{}, tk.mr, tk.mc, i0, rows,
                                      epi, acc, reinterpret_cast<double*>(panel));
    double a1[1] = {acc[0]};
    block_partials<1>(a1, partials);
  } else if constexpr (KIND == B_RES) {
    // FP64 residual, rounded into the FP32 solve: r (and p, unless this is a
    // replacement that keeps the direction); x32 is cleared
    if (!tk.active) return;
    EpiResidual<double, float> epi{tk.B64, tk.r32, tk.keep_p ? nullptr : tk.p32, tk.x32, tk.gr,
                                   tk.gc, partials};
    if (rows > 0)
      apply_rows<double, R, LDS, VEC, 0>(tk.X64, ld, ncols, tk.Lr64, tk.Lc64, BandDev<double>{}, tk.mr, tk.mc, i0, rows,
                                      epi, acc, reinterpret_cast<double*>(panel));
    block_partials<2>(acc, partials);
  } else if constexpr (KIND == B_RESNORM) {
    EpiResNorm<double> epi{tk.B64, tk.gr, tk.gc, partials};
    if (rows > 0)
      apply_rows<double, R, LDS, VEC, 0>(tk.X64, ld, ncols, tk.Lr64, tk.Lc64, BandDev<double>{}, tk.mr, tk.mc, i0, rows,
                                      epi, acc, reinterpret_cast<double*>(panel));
    double a1[1] = {acc[0]};
    block_partials<1>(a1, partials);
  } else {
    // FISTA step on the sampled matrix: Z ping-pongs between Za and Zb
    if (tk.lam == 0.0 || rows == 0) return;
    const double* Zin = par ? tk.Zb : tk.Za;
    double* Zout = par ? tk.Za : tk.Zb;
    EpiFista<false> epi{tk.Y, tk.S, Zout, 2.0 * tk.gr, 2.0 * tk.gc, tk.lam, fista_c, 0.0,
                        nullptr, 0, nullptr, 0, nullptr};
    apply_rows<double, R, LDS, VEC, 0>(Zin, ld, ncols, tk.Lrt, tk.Lct, BandDev<double>{}, tk.zmr, tk.zmc, i0, rows,
                                    epi, acc, reinterpret_cast<double*>(panel));
  }
}

template <typename T>
struct BVec;
template <> struct BVec<float> {
  __device__ static float* x(const BTask& t) { return t.x32; }
  __device__ static float* r(const BTask& t) { return t.r32; }
  __device__ static float* p(const BTask& t) { return t.p32; }
  __device__ static float* q(const BTask& t) { return t.q32; }
  __device__ static const float* B(const BTask& t) { return t.B32; }
};
template <> struct BVec<double> {
  __device__ static double* x(const BTask& t) { return t.X64; }
  __device__ static double* r(const BTask& t) { return t.r64; }
  __device__ static double* p(const BTask& t) { return t.p64; }
  __device__ static double* q(const BTask& t) { return t.q64; }
  __device__ static const double* B(const BTask& t) { return t.B64; }
};

// x += alpha p; r -= alpha q for every running task (alpha from the apply
// partials of the task's own slice of the previous launch).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_update_batched(const BTask* __restrict__ tasks, const int* __restrict__ vblk_task,
                 const double* __restrict__ part_pq, double* __restrict__ part_rr, int parity) {
  const BTask& tk = tasks[vblk_task[blockIdx.x]];
  CgScal* sc = tk.sc;
  if (sc->done != 0) return;
  const bool lead = blockIdx.x == tk.vblk0 && threadIdx.x == 0;
  // Convergence of the previous iteration is decided here, from the <r, r>
  // that every workgroup reads alike: the p-update of that iteration has run
  // in full, so p stays a valid direction for a residual replacement (the
  // product launched in between is wasted, once per segment).
  const double rr = sc->rr[parity];
  if (rr <= sc->thr) {
    if (lead) sc->done = 1;
    return;
  }
  double t[1];
  sum_partials<1>(part_pq + tk.ablk0, 8 * tk.aper, t);
  const double pq = t[0];
  if (bad(pq) || !(pq > 0.0)) {
    if (lead) {
      sc->pq = pq;
      sc->done = bad(pq) ? 3 : 2;
    }
    return;
  }
  const double alpha_d = rr / pq;
  if (lead) {
    sc->pq = pq;
    sc->alpha = alpha_d;
    sc->iter += 1;
  }
  const T alpha = (T)alpha_d;
  T* x = BVec<T>::x(tk);
  T* r = BVec<T>::r(tk);
  const T* p = BVec<T>::p(tk);
  const T* q = BVec<T>::q(tk);
  constexpr int W = V16<T>::W;
  const size_t nv = (size_t)tk.p * tk.ld / W;  // ld is a multiple of W
  const size_t stride = (size_t)tk.nvblk * blockDim.x;
  double acc[1] = {0.0};
  for (size_t v = (size_t)(blockIdx.x - tk.vblk0) * blockDim.x + threadIdx.x; v < nv; v += stride) {
    T xv[W], rv[W], pv[W], qv[W];
    vld<T, W>(x + v * W, xv);
    vld<T, W>(r + v * W, rv);
    vld<T, W>(p + v * W, pv);
    vld<T, W>(q + v * W, qv);
#pragma unroll
    for (int k = 0; k < W; ++k) {
      xv[k] += alpha * pv[k];
      rv[k] -= alpha * qv[k];
      acc[0] += (double)rv[k] * (double)rv[k];
    }
    vst<T, W>(x + v * W, xv);
    vst<T, W>(r + v * W, rv);
  }
  block_partials<1>(acc, part_rr);
}

// beta = rr_new / rr; p = r + beta p; convergence test, per task.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_pupdate_batched(const BTask* __restrict__ tasks, const int* __restrict__ vblk_task,
                  const double* __restrict__ part_rr, int parity) {
  const BTask& tk = tasks[vblk_task[blockIdx.x]];
  CgScal* sc = tk.sc;
  if (sc->done != 0) return;
  double t[1];
  sum_partials<1>(part_rr + tk.vblk0, tk.nvblk, t);
  const double rr_new = t[0];
  const double rr = sc->rr[parity];
  const bool lead = blockIdx.x == tk.vblk0 && threadIdx.x == 0;
  if (bad(rr_new)) {
    if (lead) sc->done = 3;
    return;
  }
  if (sc->aux > 0.0 && rr_new > kDiverge * sc->aux) {  // see k_cg_pupdate
    if (lead) sc->done = 4;
    return;
  }
  const double beta_d = rr_new / rr;
  if (lead) {
    sc->rr[parity ^ 1] = rr_new;
    sc->beta = beta_d;
  }
  const T beta = (T)beta_d;
  T* p = BVec<T>::p(tk);
  const T* r = BVec<T>::r(tk);
  constexpr int W = V16<T>::W;
  const size_t nv = (size_t)tk.p * tk.ld / W;
  const size_t stride = (size_t)tk.nvblk * blockDim.x;
  for (size_t v = (size_t)(blockIdx.x - tk.vblk0) * blockDim.x + threadIdx.x; v < nv; v += stride) {
    T pv[W], rv[W];
    vld<T, W>(p + v * W, pv);
    vld<T, W>(r + v * W, rv);
#pragma unroll
    for (int k = 0; k < W; ++k) pv[k] = rv[k] + beta * pv[k];
    vst<T, W>(p + v * W, pv);
  }
}

// Per-task start of CG from zero: x = 0, r = p = B, q = 0; partials of
// <B, B>. q is cleared over the whole padded extent: the FP64 product (2
// columns per thread) writes q only up to n rounded to 2, while the vector
// kernels run over p * ld with ld = n rounded to 4; cleared, the padding of
// q (and so of r, p and x) stays zero.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_init_zero_batched(const BTask* __restrict__ tasks, const int* __restrict__ vblk_task,
                    double* part) {
  const BTask& tk = tasks[vblk_task[blockIdx.x]];
  T* x = BVec<T>::x(tk);
  T* r = BVec<T>::r(tk);
  T* p = BVec<T>::p(tk);
  T* q = BVec<T>::q(tk);
  const T* B = BVec<T>::B(tk);
  const size_t N = (size_t)tk.p * tk.ld;
  const size_t stride = (size_t)tk.nvblk * blockDim.x;
  double acc[1] = {0.0};
  for (size_t e = (size_t)(blockIdx.x - tk.vblk0) * blockDim.x + threadIdx.x; e < N; e += stride) {
    const T bv = B[e];
    x[e] = T(0);
    r[e] = bv;
    p[e] = bv;
    q[e] = T(0);
    acc[0] += (double)bv * (double)bv;
  }
  block_partials<1>(acc, part);
}

// One workgroup per task: arm the CG scalars from that task's partials.
//   FROM_APPLY = false: partials of a vector kernel (NV = 1, rr = total),
//                threshold thr_rel2 * bb;
//   FROM_APPLY = true : partials of the FP64 residual (NV = 2), threshold
//                max(tk.inner_rel2 * ||round(R)||^2, tk.floor2). Inactive
//                tasks are marked done.
template <bool FROM_APPLY>
__global__ void __launch_bounds__(kThreads)
k_arm_batched(const BTask* __restrict__ tasks, const double* part, double thr_rel2) {
  const BTask& tk = tasks[blockIdx.x];
  CgScal* sc = tk.sc;
  if (FROM_APPLY) {
    if (!tk.active) {
      if (threadIdx.x == 0) {
        sc->conv_it = 0;
        sc->done = 1;
      }
      return;
    }
    double t[2];
    sum_partials<2>(part + 2 * (size_t)tk.ablk0, 8 * tk.aper, t);
    if (threadIdx.x == 0) {
      sc->res2 = t[0];
      sc->aux = t[1];
      sc->rr[0] = sc->rr[1] = t[1];
      sc->thr = fmax(tk.inner_rel2 * t[1], tk.floor2);
      sc->iter = 0;
      sc->conv_it = 0;
      sc->done = (bad(t[0]) || bad(t[1])) ? 3 : (t[1] <= sc->thr ? 1 : 0);
    }
  } else {
    double t[1];
    sum_partials<1>(part + tk.vblk0, tk.nvblk, t);
    if (threadIdx.x == 0) {
      sc->rr[0] = sc->rr[1] = t[0];
      sc->aux = 0.0;
      sc->thr = thr_rel2 * sc->bb;
      sc->iter = 0;
      sc->conv_it = 0;
      sc->done = bad(t[0]) ? 3 : (t[0] <= sc->thr ? 1 : 0);
    }
  }
}

// Per task: ||B64||^2 into sc->bb (one workgroup per task).
__global__ void __launch_bounds__(kThreads)
k_bnorm_batched(const BTask* __restrict__ tasks) {
  const BTask& tk = tasks[blockIdx.x];
  const size_t N = (size_t)tk.p * tk.ld;
  double acc = 0.0;
  for (size_t e = threadIdx.x; e < N; e += blockDim.x) acc += tk.B64[e] * tk.B64[e];
  __shared__ double red[kMaxWaves];
  acc = wave_sum(acc);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) s += red[w];
    tk.sc->bb = s;
  }
}

// Per task: sum of the apply partials (NV values) into out[t * NV + k].
template <int NV>
__global__ void __launch_bounds__(kThreads)
k_apply_sum_batched(const BTask* __restrict__ tasks, const double* part, double* out) {
  const BTask& tk = tasks[blockIdx.x];
  double t[NV];
  sum_partials<NV>(part + NV * (size_t)tk.ablk0, 8 * tk.aper, t);
  if (threadIdx.x < NV) out[blockIdx.x * NV + threadIdx.x] = t[threadIdx.x];
}

// Element-wise per-task passes over p x ld (grid: vector blocks).
// P_ZERO_32 clears the FP32 CG vectors over the whole padded extent: the
// FP64 residual epilogue (2 columns per thread) only writes up to n rounded
// to 2, while the FP32 kernels (4 columns per thread) read up to n rounded
// to 4.
enum BPass { P_ACCUM = 0, P_B32 = 1, P_X64_FROM_32 = 2, P_ZERO_X64 = 3, P_ZERO_B64 = 4,
             P_ZERO_32 = 5, P_P_FROM_R = 6 };
template <int PASS>
__global__ void __launch_bounds__(kThreads)
k_pass_batched(const BTask* __restrict__ tasks, const int* __restrict__ vblk_task) {
  const BTask& tk = tasks[vblk_task[blockIdx.x]];
  if (PASS == P_ACCUM && !tk.active) return;
  if (PASS == P_ACCUM && tk.sc->done >= 2) return;  // failed FP32 segment: X64 kept
  if (PASS == P_P_FROM_R && !(tk.active && tk.reset_p)) return;
  const size_t N = (size_t)tk.p * tk.ld;
  const size_t stride = (size_t)tk.nvblk * blockDim.x;
  for (size_t e = (size_t)(blockIdx.x - tk.vblk0) * blockDim.x + threadIdx.x; e < N; e += stride) {
    if (PASS == P_ACCUM) tk.X64[e] += (double)tk.x32[e];
    if (PASS == P_B32) tk.B32[e] = (float)tk.B64[e];
    if (PASS == P_X64_FROM_32) tk.X64[e] = (double)tk.x32[e];
    if (PASS == P_ZERO_X64) tk.X64[e] = 0.0;
    if (PASS == P_ZERO_B64) tk.B64[e] = 0.0;
    if (PASS == P_ZERO_32) tk.x32[e] = tk.r32[e] = tk.p32[e] = tk.q32[e] = 0.f;
    if (PASS == P_P_FROM_R) tk.p32[e] = tk.r32[e];
  }
}

// B64[omega_r[a], omega_c[b]] = X~[a, b] rounded to the mode's type
// (grid: vector blocks, the task's slice strides over its samples).
template <typename TM>
__global__ void __launch_bounds__(kThreads)
k_scatter_batched(const BTask* __restrict__ tasks, const int* __restrict__ vblk_task) {
  const BTask& tk = tasks[vblk_task[blockIdx.x]];
  const size_t N = (size_t)tk.rho_r * tk.rho_c;
  const size_t stride = (size_t)tk.nvblk * blockDim.x;
  for (size_t e = (size_t)(blockIdx.x - tk.vblk0) * blockDim.x + threadIdx.x; e < N; e += stride) {
    const int a = (int)(e / tk.rho_c);
    const int c = (int)(e - (size_t)a * tk.rho_c);
    tk.B64[(size_t)tk.om_r[a] * tk.ld + tk.om_c[c]] = (double)(TM)tk.S[(size_t)a * tk.ldt + c];
  }
}

// FISTA set-up per task: S = Za = Y, Zb = 0 (grid: vector blocks).
__global__ void __launch_bounds__(kThreads)
k_fista_init_batched(const BTask* __restrict__ tasks, const int* __restrict__ vblk_task) {
  const BTask& tk = tasks[vblk_task[blockIdx.x]];
  const size_t N = (size_t)tk.rho_r * tk.ldt;
  const size_t stride = (size_t)tk.nvblk * blockDim.x;
  for (size_t e = (size_t)(blockIdx.x - tk.vblk0) * blockDim.x + threadIdx.x; e < N; e += stride) {
    tk.S[e] = tk.Y[e];
    tk.Za[e] = tk.Y[e];
    tk.Zb[e] = 0.0;
  }
}

// Copies out of the padded layouts into the caller's dense outputs.
template <typename TO>
__global__ void __launch_bounds__(kThreads)
k_copy_out(TO* __restrict__ out, const double* __restrict__ in, int rows, int cols, int ld) {
  const size_t N = (size_t)rows * cols;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const int i = (int)(e / cols);
    const int j = (int)(e - (size_t)i * cols);
    out[e] = (TO)in[(size_t)i * ld + j];
  }
}

// Converts a dense rows x cols input into a zero-padded FP64 layout.
template <typename TI>
__global__ void __launch_bounds__(kThreads)
k_copy_in(double* __restrict__ out, const TI* __restrict__ in, int rows, int cols, int ld) {
  const size_t N = (size_t)rows * ld;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const int i = (int)(e / ld);
    const int j = (int)(e - (size_t)i * ld);
    out[e] = j < cols ? (double)in[(size_t)i * cols + j] : 0.0;
  }
}

}  // namespace cpca
