// Device kernels of the CPCA solvers for gfx950 (CDNA4, wave64).
//
// The central kernel is the fused two-sided sparse product
//     out(i, j) = mask(i, j) X(i, j) + a_r (L_r X)(i, j) + a_c (X L_c)(i, j)
// which is the gradient of the graph term of FRPCAG (Section IV.B) and the
// operator of the alternate decoder's normal equations (Section V.B). One
// workgroup owns R consecutive rows of X and sweeps all n columns, VEC
// consecutive columns per thread (16-byte accesses):
//   * L_r X streams the neighbour rows of X with coalesced vector loads; the
//     CSR entries of row i are uniform across the workgroup;
//   * X L_c gathers from the R rows of X (staged in LDS, or read through the
//     L1 when LDS staging is off); L_c is held as sliced ELL with one slice
//     per wavefront (64 * VEC columns), so its index/value loads are 16-byte
//     vector loads and every lane of a wave runs the same trip count;
//   * the row-block index is remapped so that each XCD owns a contiguous
//     range of rows and neighbour rows are shared through its L2.
// What happens to out(i, j) is decided by an epilogue functor (CG apply,
// FISTA step, residual, objective, adjoint dot products).
//
// Reductions use no atomics and no fences: every workgroup writes its FP64
// partial sums, and the kernel that needs the total (the next kernel on the
// stream) sums the partials itself, in a fixed order, redundantly in every
// workgroup. Results are therefore bitwise reproducible, and scalars such as
// the CG step lengths never leave the device.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "panels.hpp"

namespace cpca {

constexpr int kWave = 64;
constexpr int kThreads = 256;  // threads per workgroup for all kernels
constexpr int kMaxWaves = kThreads / kWave;

template <typename T>
struct CsrDev {
  const int* rp;
  const int* ci;
  const T* v;
};

// Sliced ELL with slice height H = 64 * VEC: slice s covers columns
// [H s, H s + H); its entries start at sp[s], width w_s = (sp[s+1]-sp[s]) / H,
// entry e of column j sits at sp[s] + H e + (j - H s). Padding entries carry
// value 0 and a valid column index.
template <typename T>
struct SellDev {
  const int* sp;
  const int* ci;
  const T* v;
};

// Device-resident scalars of one CG solve (FP64). rr is double-buffered by
// iteration parity: iteration `it` reads rr[it & 1] and the p-update writes
// rr[(it + 1) & 1], so no workgroup reads a value another workgroup of the
// same kernel is writing.
struct CgScal {
  double rr[2];
  double thr;     // stop when rr <= thr
  double alpha;
  double beta;
  double pq;      // last <p, A p>
  double res2;    // last FP64 residual norm^2 (refinement)
  double aux;     // last rounded-residual norm^2 (refinement)
  double bb;      // ||rhs||^2
  int iter;       // iterations completed
  int done;       // 0 running, 1 converged, 2 breakdown, 3 NaN/Inf, 4 diverged
  // Convergence detected by the p-update of iteration `it` is recorded as
  // conv_it = it + 1 (-1: converged when armed). The p-update of the
  // converging iteration still runs in full, so the direction stays valid
  // for a residual replacement; later iterations see conv_it and skip.
  int conv_it;
  int pad0;
  double rho[2];  // preconditioned CG: <r, M^-1 r>, double-buffered like rr
};

// Device-resident scalars of one FISTA run.
struct FistaScal {
  double dz2;     // ||Z+ - Z||^2 of the step that stopped the run
  double z2;
  double obj_l1;  // objective pieces
  double obj_g;
  int iter;       // iteration that met the stopping test (0: none)
  int done;       // 0 running, 1 stopped by eps, 3 NaN/Inf
};

__device__ __forceinline__ bool bad(double x) { return !(x == x) || x - x != 0.0; }

// Growth of the recursive <r, r> over its armed value that marks an FP32
// segment of a residual-replacement solve as diverged.
constexpr double kDiverge = 1e6;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Writes the workgroup's NV partial sums to partials[blockIdx.x * NV + k].
template <int NV>
__device__ void block_partials(const double (&v)[NV], double* partials) {
  __shared__ double red[NV][kMaxWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[k][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) s += red[threadIdx.x][w];
    partials[(size_t)blockIdx.x * NV + threadIdx.x] = s;
  }
}

// Sums nb * NV partials written by a previous kernel, in a fixed order.
// Every thread of the workgroup receives the same totals.
template <int NV>
__device__ void sum_partials(const double* partials, int nb, double (&tot)[NV]) {
  __shared__ double red[NV][kMaxWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partials[(size_t)b * NV + k];
    s = wave_sum(s);
    if (lane == 0) red[k][wid] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) s += red[k][w];
    tot[k] = s;
  }
  __syncthreads();
}

// ------------------------------------------------------------ vector access
template <typename T, int VEC> struct VecT;
template <> struct VecT<float, 1> { using type = float; };
template <> struct VecT<float, 2> { using type = float2; };
template <> struct VecT<float, 4> { using type = float4; };
template <> struct VecT<double, 1> { using type = double; };
template <> struct VecT<double, 2> { using type = double2; };
template <> struct VecT<int, 1> { using type = int; };
template <> struct VecT<int, 2> { using type = int2; };
template <> struct VecT<int, 4> { using type = int4; };

template <typename T, int VEC>
__device__ __forceinline__ void vld(const T* __restrict__ p, T (&v)[VEC]) {
  using V = typename VecT<T, VEC>::type;
  const V t = *reinterpret_cast<const V*>(p);
  if constexpr (VEC == 1) {
    v[0] = t;
  } else if constexpr (VEC == 2) {
    v[0] = t.x; v[1] = t.y;
  } else {
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  }
}

template <typename T, int VEC>
__device__ __forceinline__ void vst(T* __restrict__ p, const T (&v)[VEC]) {
  using V = typename VecT<T, VEC>::type;
  V t;
  if constexpr (VEC == 1) {
    t = v[0];
  } else if constexpr (VEC == 2) {
    t.x = v[0]; t.y = v[1];
  } else {
    t.x = v[0]; t.y = v[1]; t.z = v[2]; t.w = v[3];
  }
  *reinterpret_cast<V*>(p) = t;
}

// ---------------------------------------------------------------------------
// Epilogues of the fused two-sided product. Each one provides
//   NV                    number of FP64 partial sums it produces
//   prologue()            called by the whole workgroup first; returns true to
//                         skip the launch (converged solve); may sum partials
//                         of the previous kernel
//   apply<VEC>(i, idx, x, mx, accr, accc, acc)
//                         VEC consecutive outputs of row i starting at flat
//                         index idx: x = X, mx = mask o X, accr = (L_r X),
//                         accc = (X L_c); acc receives the partial sums
//   partials              where the workgroup partials go (may be null)
// ---------------------------------------------------------------------------

// Q = A(P), partial <P, Q> (plain operator application).
template <typename T>
struct EpiApply {
  static constexpr int NV = 1;
  T* Q;
  T gr, gc;
  double* partials;
  __device__ bool prologue() const { return false; }
  template <int VEC>
  __device__ void apply(int, size_t idx, const T (&x)[VEC], const T (&mx)[VEC],
                        const T (&accr)[VEC], const T (&accc)[VEC], double* acc) const {
    T out[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      out[v] = mx[v] + gr * accr[v] + gc * accc[v];
      acc[0] += (double)x[v] * (double)out[v];
    }
    vst<T, VEC>(Q + idx, out);
  }
};

// CG: q = A(p) and the partials of <p, q>; skipped once the solve is done.
template <typename T>
struct EpiCg : EpiApply<T> {
  const CgScal* sc;
  __device__ bool prologue() const { return sc->done != 0 || sc->conv_it != 0; }
};

// Residual R = B - A(X) computed in T, stored rounded to TO into r_out and,
// if given, p_out (initial residual and direction of a CG solve; a residual
// replacement keeps the direction and passes null); x_out (the CG iterate),
// if given, is cleared. Partials: ||R||^2 and ||round(R)||^2.
template <typename T, typename TO>
struct EpiResidual {
  static constexpr int NV = 2;
  const T* B;
  TO* r_out;
  TO* p_out;
  TO* x_out;
  T gr, gc;
  double* partials;
  __device__ bool prologue() const { return false; }
  template <int VEC>
  __device__ void apply(int, size_t idx, const T (&)[VEC], const T (&mx)[VEC],
                        const T (&accr)[VEC], const T (&accc)[VEC], double* acc) const {
    T b[VEC];
    vld<T, VEC>(B + idx, b);
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const T R = b[v] - (mx[v] + gr * accr[v] + gc * accc[v]);
      const TO Rt = (TO)R;
      r_out[idx + v] = Rt;
      if (p_out) p_out[idx + v] = Rt;
      if (x_out) x_out[idx + v] = TO(0);
      acc[0] += (double)R * (double)R;
      acc[1] += (double)Rt * (double)Rt;
    }
  }
};

// Partials of ||B - A(X)||^2.
template <typename T>
struct EpiResNorm {
  static constexpr int NV = 1;
  const T* B;
  T gr, gc;
  double* partials;
  __device__ bool prologue() const { return false; }
  template <int VEC>
  __device__ void apply(int, size_t idx, const T (&)[VEC], const T (&mx)[VEC],
                        const T (&accr)[VEC], const T (&accc)[VEC], double* acc) const {
    T b[VEC];
    vld<T, VEC>(B + idx, b);
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const double R = (double)b[v] - (double)(mx[v] + gr * accr[v] + gc * accc[v]);
      acc[0] += R * R;
    }
  }
};

// One FISTA iteration (Algorithm 1) on the FP64 state:
//   G  = Z - lam * grad g(Z),  grad g = 2 (gc Z L_c + gr L_r Z)
//   S  = Y + sgn(G - Y) max(|G - Y| - lam, 0)
//   Z+ = S + c (S - S_prev),   c = (t_j - 1) / t_{j+1}
// S overwrites S_prev in place (same element, same thread); Z+ goes to a
// second buffer because neighbouring rows of Z are still being read.
// With REDUCE, iteration j also produces the partials of ||Z+ - Z||^2 and
// ||Z||^2, and iteration j + 1 evaluates the stopping test of iteration j in
// its prologue (partial buffers alternate with the parity of j).
template <bool REDUCE>
struct EpiFista {
  static constexpr int NV = 2;
  const double* Y;
  double* S;
  double* Zn;
  double two_gr, two_gc, lam, c, eps;
  FistaScal* fs;
  int j;                       // iteration index (1-based)
  const double* prev_partials; // partials of iteration j - 1 (REDUCE, j > 1)
  int prev_nb;
  double* partials;
  __device__ bool prologue() const {
    if (fs->done != 0) return true;
    if (!REDUCE || j == 1) return false;
    double tot[2];
    sum_partials<2>(prev_partials, prev_nb, tot);
    const bool stop = bad(tot[0]) || bad(tot[1]) || tot[0] < eps * tot[1];
    if (stop && blockIdx.x == 0 && threadIdx.x == 0) {
      fs->dz2 = tot[0];
      fs->z2 = tot[1];
      fs->iter = j - 1;
      fs->done = (bad(tot[0]) || bad(tot[1])) ? 3 : 1;
    }
    return stop;
  }
  template <int VEC>
  __device__ void apply(int, size_t idx, const double (&z)[VEC], const double (&)[VEC],
                        const double (&accr)[VEC], const double (&accc)[VEC],
                        double* acc) const {
    double y[VEC], sp[VEC], s[VEC], zn[VEC];
    vld<double, VEC>(Y + idx, y);
    vld<double, VEC>(S + idx, sp);
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const double g = z[v] - lam * (two_gr * accr[v] + two_gc * accc[v]);
      const double d = g - y[v];
      const double mag = fabs(d) - lam;
      s[v] = mag > 0.0 ? y[v] + copysign(mag, d) : y[v];
      zn[v] = s[v] + c * (s[v] - sp[v]);
      if (REDUCE) {
        const double dz = zn[v] - z[v];
        acc[0] += dz * dz;
        acc[1] += z[v] * z[v];
      }
    }
    vst<double, VEC>(S + idx, s);
    vst<double, VEC>(Zn + idx, zn);
  }
};

// FRPCAG objective pieces at X: ||Y - X||_1 and <X, gc X L_c + gr L_r X>.
struct EpiObjective {
  static constexpr int NV = 2;
  const double* Y;
  double gr, gc;
  double* partials;
  __device__ bool prologue() const { return false; }
  template <int VEC>
  __device__ void apply(int, size_t idx, const double (&x)[VEC], const double (&)[VEC],
                        const double (&accr)[VEC], const double (&accc)[VEC],
                        double* acc) const {
    double y[VEC];
    vld<double, VEC>(Y + idx, y);
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      acc[0] += fabs(y[v] - x[v]);
      acc[1] += x[v] * (gr * accr[v] + gc * accc[v]);
    }
  }
};

// Adjoint dot products <Lam, L_r X> and <Lam, X L_c>.
template <typename T>
struct EpiDot2 {
  static constexpr int NV = 2;
  const T* Lam;
  double* partials;
  __device__ bool prologue() const { return false; }
  template <int VEC>
  __device__ void apply(int, size_t idx, const T (&)[VEC], const T (&)[VEC],
                        const T (&accr)[VEC], const T (&accc)[VEC], double* acc) const {
    T l[VEC];
    vld<T, VEC>(Lam + idx, l);
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      acc[0] += (double)l[v] * (double)accr[v];
      acc[1] += (double)l[v] * (double)accc[v];
    }
  }
};

// Diagonals of L_c within half-bandwidth BW, stored diagonal-major:
// v[(d + BW) * ldb + j] = L_c[j, j + d] (zero where there is no edge), for
// d in [-BW, BW]; bit d + BW of `nonempty` is set when diagonal d holds an
// entry. Entries farther from the diagonal stay in the sliced-ELL remainder.
template <typename T>
struct BandDev {
  const T* v;
  int ldb;
  unsigned long long nonempty;
};

// ---------------------------------------------------------------------------
// The fused two-sided product on rows [i0, i0 + rows) of a p x n operand
// stored with row stride ld (ld >= n rounded up to VEC; padding columns hold
// zeros and the masks are padded with zeros, so padding outputs are zero).
// VEC consecutive columns per thread, kThreads * VEC columns per pass.
//   LDS = true : the R rows live in LDS (R * pitch * sizeof(T) bytes, with
//                pitch = ld + 2 * band_pad<BW, VEC>).
//   LDS = false: X L_c gathers from global memory (through the L1).
//   BW > 0     : L_c entries within BW of the diagonal come from BandDev; each
//                thread loads its window of 2 BW + VEC consecutive row values
//                with aligned 16-byte LDS reads (conflict-free) and applies
//                the diagonals from registers. Requires LDS and VEC = 16 / T.
// Shared by the single-problem kernel and the batched (task-table) kernel.
// ---------------------------------------------------------------------------
template <int BW, int VEC>
constexpr int band_pad() {
  return BW == 0 ? 0 : (BW + VEC - 1) / VEC * VEC;
}

template <int BW, int VEC>
constexpr int band_pitch_pad() {
  return 2 * band_pad<BW, VEC>();
}

template <typename T, int R, bool LDS, int VEC, int BW, class Epi>
__device__ __forceinline__ void apply_rows(const T* __restrict__ X, int ld, int n,
                                           const CsrDev<T>& Lr, const SellDev<T>& Lc,
                                           const BandDev<T>& Lb,
                                           const uint8_t* __restrict__ mr,
                                           const uint8_t* __restrict__ mc, int i0, int rows,
                                           const Epi& epi, double* acc, T* panel) {
  static_assert(BW == 0 || LDS, "the band path reads its windows from LDS");
  constexpr int H = kWave * VEC;         // SELL slice height
  constexpr int CPB = kThreads * VEC;    // columns per pass
  constexpr int PAD = band_pad<BW, VEC>();
  const int pitch = ld + 2 * PAD;        // LDS row pitch
  if (LDS) {
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      if (rr < rows) {
        const T* src = X + (size_t)(i0 + rr) * ld;
        T* dst = panel + rr * pitch + PAD;
        for (int c = threadIdx.x * VEC; c < n; c += CPB) {
          T t[VEC];
          vld<T, VEC>(src + c, t);
          vst<T, VEC>(dst + c, t);
        }
        if (PAD > 0) {
          // zero the band padding on both sides and the columns past n
          for (int c = threadIdx.x; c < PAD; c += kThreads) {
            dst[c - PAD] = T(0);
            dst[ld + c] = T(0);
          }
          for (int c = n + threadIdx.x; c < ld; c += kThreads) dst[c] = T(0);
        }
      }
    }
    __syncthreads();
  }
  for (int c0 = threadIdx.x * VEC; c0 < n; c0 += CPB) {
    // X L_c: columns c0 .. c0 + VEC - 1 of L_c (= rows, L_c symmetric),
    // shared by the R rows of the block
    T accc[R][VEC];
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
      for (int v = 0; v < VEC; ++v) accc[rr][v] = T(0);
    T xw[R][VEC];  // own values (filled from the band windows when BW > 0)
    if constexpr (BW > 0) {
      constexpr int WIN = 2 * PAD + VEC;
      T win[R][WIN];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        if (rr < rows) {
          const T* base = panel + rr * pitch + c0;  // = row column c0 - PAD
#pragma unroll
          for (int q = 0; q < WIN; q += VEC) {
            T t[VEC];
            vld<T, VEC>(base + q, t);
#pragma unroll
            for (int v = 0; v < VEC; ++v) win[rr][q + v] = t[v];
          }
#pragma unroll
          for (int v = 0; v < VEC; ++v) xw[rr][v] = win[rr][PAD + v];
        }
      }
#pragma unroll
      for (int d = -BW; d <= BW; ++d) {
        if (!((Lb.nonempty >> (d + BW)) & 1ull)) continue;
        T vv[VEC];
        vld<T, VEC>(Lb.v + (size_t)(d + BW) * Lb.ldb + c0, vv);
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int v = 0; v < VEC; ++v) accc[rr][v] += vv[v] * win[rr][PAD + v + d];
      }
    }
    {
      // sliced-ELL part (all of L_c when BW = 0, the far entries otherwise)
      const int s = c0 / H;
      const int beg = Lc.sp[s];
      const int w = (Lc.sp[s + 1] - beg) / H;
      const int off = beg + (c0 - s * H);
#pragma unroll 2
      for (int e = 0; e < w; ++e) {
        int kk[VEC];
        T vv[VEC];
        vld<int, VEC>(Lc.ci + off + e * H, kk);
        vld<T, VEC>(Lc.v + off + e * H, vv);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          if (rr < rows) {
            const T* rowp = LDS ? panel + rr * pitch + PAD : X + (size_t)(i0 + rr) * ld;
#pragma unroll
            for (int v = 0; v < VEC; ++v) accc[rr][v] += vv[v] * rowp[kk[v]];
          }
        }
      }
    }
    uint8_t mcv[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) mcv[v] = mc[c0 + v];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      if (rr < rows) {
        const int i = i0 + rr;
        // L_r X: row i of L_r, neighbour rows of X, coalesced over columns
        T accr[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) accr[v] = T(0);
        const int e0 = Lr.rp[i];
        const int e1 = Lr.rp[i + 1];
#pragma unroll 4
        for (int e = e0; e < e1; ++e) {
          const T w = Lr.v[e];
          T xv[VEC];
          vld<T, VEC>(X + (size_t)Lr.ci[e] * ld + c0, xv);
#pragma unroll
          for (int v = 0; v < VEC; ++v) accr[v] += w * xv[v];
        }
        const size_t idx = (size_t)i * ld + c0;
        T x[VEC], mx[VEC];
        if constexpr (BW > 0) {
#pragma unroll
          for (int v = 0; v < VEC; ++v) x[v] = xw[rr][v];
        } else if (LDS) {
          vld<T, VEC>(panel + rr * pitch + c0, x);
        } else {
          vld<T, VEC>(X + idx, x);
        }
        const uint8_t mri = mr[i];
#pragma unroll
        for (int v = 0; v < VEC; ++v) mx[v] = (mri & mcv[v]) ? x[v] : T(0);
        epi.template apply<VEC>(i, idx, x, mx, accr, accc[rr], acc);
      }
    }
  }
}

// Single problem: R rows per workgroup, all n columns (row stride n).
// Grid: 8 * per workgroups; workgroup b handles row block (b % 8) * per + b / 8
// so that each XCD (workgroups are dealt to XCDs round-robin) owns `per`
// consecutive row blocks. Workgroups past the last row block only write
// zero partials.
template <typename T, int R, bool LDS, int VEC, int BW, class Epi>
__global__ void __launch_bounds__(kThreads)
k_apply2(const T* __restrict__ X, int p, int n, CsrDev<T> Lr, SellDev<T> Lc, BandDev<T> Lb,
         const uint8_t* __restrict__ mr, const uint8_t* __restrict__ mc, int nrb, int per,
         Epi epi) {
  if (epi.prologue()) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double acc[Epi::NV];
#pragma unroll
  for (int k = 0; k < Epi::NV; ++k) acc[k] = 0.0;
  const int b = blockIdx.x;
  const int rb = (b & 7) * per + (b >> 3);
  if (rb < nrb) {
    const int i0 = rb * R;
    apply_rows<T, R, LDS, VEC, BW, Epi>(X, n, n, Lr, Lc, Lb, mr, mc, i0, min(R, p - i0), epi,
                                        acc, reinterpret_cast<T*>(smem_raw));
  }
  if (epi.partials) block_partials<Epi::NV>(acc, epi.partials);
}

// ---------------------------------------------------------------------------
// Column-strip variant for a banded L_c (BW > 0). A workgroup of kStripThreads
// threads owns the strip of columns [s * CW, s * CW + CW), CW = kStripThreads *
// VEC, and walks RB consecutive rows. The band diagonals of its columns stay
// in registers for all RB rows; each row's strip segment plus a halo of PAD
// columns on both sides is staged in LDS (double-buffered, one barrier per
// row) and every thread reads its window of 2 PAD + VEC values with aligned
// 16-byte LDS loads. Entries of L_c farther than BW from the diagonal (the
// sliced-ELL remainder) are gathered from global memory.
// Grid: 8 * cpx * nstrips workgroups. XCD x (workgroups are dealt to XCDs
// round-robin) owns row chunks [x * cpx, (x + 1) * cpx) and sweeps them strip
// by strip, so the neighbour rows of L_r X are reused from its L2.
// Requires n % VEC == 0 (row stride n).
// ---------------------------------------------------------------------------
constexpr int kStripThreads = 128;

template <typename T, int VEC, int BW, int RB, class Epi>
__global__ void __launch_bounds__(kStripThreads)
k_apply_strip(const T* __restrict__ X, int p, int n, CsrDev<T> Lr, SellDev<T> Lc, BandDev<T> Lb,
              const uint8_t* __restrict__ mr, const uint8_t* __restrict__ mc, int nchunks,
              int cpx, Epi epi) {
  if (epi.prologue()) return;
  constexpr int PAD = band_pad<BW, VEC>();
  constexpr int CW = kStripThreads * VEC;
  constexpr int SEG = CW + 2 * PAD;   // staged values per row
  constexpr int WIN = 2 * PAD + VEC;  // window per thread
  constexpr int H = kWave * VEC;      // SELL slice height
  __shared__ __align__(16) T seg[2][SEG];
  double acc[Epi::NV];
#pragma unroll
  for (int k = 0; k < Epi::NV; ++k) acc[k] = 0.0;

  const int b = blockIdx.x;
  const int x = b & 7;
  const int l = b >> 3;
  const int strip = l / cpx;
  const int chunk = x * cpx + (l - strip * cpx);
  const int cs = strip * CW;
  if (chunk < nchunks && cs < n) {
    const int i0 = chunk * RB;
    const int i1 = min(p, i0 + RB);
    const int c0 = cs + threadIdx.x * VEC;
    const bool ok = c0 < n;
    // band diagonals of this thread's columns (zero for empty diagonals)
    T vb[2 * BW + 1][VEC];
#pragma unroll
    for (int d = 0; d <= 2 * BW; ++d) {
      if (ok && ((Lb.nonempty >> d) & 1ull)) {
        vld<T, VEC>(Lb.v + (size_t)d * Lb.ldb + c0, vb[d]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) vb[d][v] = T(0);
      }
    }
    uint8_t mcv[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) mcv[v] = ok ? mc[c0 + v] : 0;
    // sliced-ELL remainder of these columns
    int sbeg = 0, sw = 0;
    if (ok) {
      const int s = c0 / H;
      sbeg = Lc.sp[s] + (c0 - s * H);
      sw = (Lc.sp[s + 1] - Lc.sp[s]) / H;
    }
    // stage the first row
    auto stage = [&](int i, T* dst) {
      const T* src = X + (size_t)i * n;
      if (ok) {
        T t[VEC];
        vld<T, VEC>(src + c0, t);
        vst<T, VEC>(dst + PAD + threadIdx.x * VEC, t);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) dst[PAD + threadIdx.x * VEC + v] = T(0);
      }
      if (threadIdx.x < PAD) {
        const int cl = cs - PAD + (int)threadIdx.x;  // left halo
        dst[threadIdx.x] = cl >= 0 ? src[cl] : T(0);
        const int cr = cs + CW + (int)threadIdx.x;   // right halo
        dst[PAD + CW + threadIdx.x] = cr < n ? src[cr] : T(0);
      }
    };
    stage(i0, seg[0]);
    __syncthreads();
    for (int i = i0; i < i1; ++i) {
      const int buf = (i - i0) & 1;
      if (i + 1 < i1) stage(i + 1, seg[buf ^ 1]);
      // window of this thread: columns c0 - PAD .. c0 + VEC + PAD - 1
      T win[WIN];
#pragma unroll
      for (int q = 0; q < WIN; q += VEC) {
        T t[VEC];
        vld<T, VEC>(&seg[buf][threadIdx.x * VEC + q], t);
#pragma unroll
        for (int v = 0; v < VEC; ++v) win[q + v] = t[v];
      }
      if (ok) {
        T accc[VEC], accr[VEC], xv[VEC], mx[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) accc[v] = T(0);
#pragma unroll
        for (int d = -BW; d <= BW; ++d)
#pragma unroll
          for (int v = 0; v < VEC; ++v) accc[v] += vb[d + BW][v] * win[PAD + v + d];
        const T* rowp = X + (size_t)i * n;
        for (int e = 0; e < sw; ++e) {
          int kk[VEC];
          T vv[VEC];
          vld<int, VEC>(Lc.ci + sbeg + e * H, kk);
          vld<T, VEC>(Lc.v + sbeg + e * H, vv);
#pragma unroll
          for (int v = 0; v < VEC; ++v) accc[v] += vv[v] * rowp[kk[v]];
        }
#pragma unroll
        for (int v = 0; v < VEC; ++v) accr[v] = T(0);
        const int e0 = Lr.rp[i];
        const int e1 = Lr.rp[i + 1];
#pragma unroll 4
        for (int e = e0; e < e1; ++e) {
          const T w = Lr.v[e];
          T t[VEC];
          vld<T, VEC>(X + (size_t)Lr.ci[e] * n + c0, t);
#pragma unroll
          for (int v = 0; v < VEC; ++v) accr[v] += w * t[v];
        }
        const uint8_t mri = mr[i];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          xv[v] = win[PAD + v];
          mx[v] = (mri & mcv[v]) ? xv[v] : T(0);
        }
        epi.template apply<VEC>(i, (size_t)i * n + c0, xv, mx, accr, accc, acc);
      }
      __syncthreads();
    }
  }
  if (epi.partials) block_partials<Epi::NV>(acc, epi.partials);
}

// ---------------------------------------------------------------------------
// Row-panel gather variant for a banded L_c (BW > 0) and any L_r whose rows
// hold at most kPanelK off-diagonal entries.
//
// The rows of L_r are grouped on the host into panels of at most kPanelRows
// rows whose L_r neighbourhoods overlap (greedy growth on the graph of L_r);
// the union U of a panel's neighbour rows (itself included) has at most
// PanelUnion<T> rows. A workgroup owns one column strip of W = 16 * VEC
// columns and G consecutive panels. Per panel it copies into LDS the strip
// segment of every row of U that is not already there from an earlier panel
// of the group (each row into the slot the host assigned it), plus a halo of
// PAD columns on both sides of the panel's own rows, so each row of X is read
// about (staged rows) / p times instead of once per L_r entry, and computes
// the panel's rows entirely from LDS: L_r X from the staged union rows (slot
// offsets precomputed on the host), X L_c from the band diagonals held in
// registers and the row's window. In k_apply_panel the next panel's global
// loads are issued into registers before the current panel is computed, so
// HBM traffic overlaps the LDS work.
// Thread t serves row slot t / 16 (16 rows in flight) and columns
// c0 = s * W + (t % 16) * VEC of strip s.
// Grid: 8 * gpx * nstrips workgroups, gpx = ceil(ceil(npan / G) / 8); XCD x
// takes panel groups [x * gpx, (x + 1) * gpx) of every strip, so panels that
// share union rows run on the same XCD (one L2).
// ---------------------------------------------------------------------------
// (layout constants kPanel*, PanelUnion: panels.hpp)

// Gather entries of a panel row handled under one loop-bound test.
constexpr int kGatherChunk = 4;

// Lane E of every 16-lane row of the wave, broadcast to the whole row (DPP
// row_newbcast): a register-only move.
template <int E>
__device__ __forceinline__ uint32_t row_bcast(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + E, 0xf, 0xf, false);
}
template <int E>
__device__ __forceinline__ float row_bcast_t(float v) {
  return __builtin_bit_cast(float, row_bcast<E>(__builtin_bit_cast(uint32_t, v)));
}
template <int E>
__device__ __forceinline__ double row_bcast_t(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = row_bcast<E>((uint32_t)u), hi = row_bcast<E>((uint32_t)(u >> 32));
  return __builtin_bit_cast(double, lo | (hi << 32));
}
// f(integral_constant<int, E>) for E = B .. N - 1, in order.
template <int B, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < N) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, N>(f);
  }
}

template <typename T>
struct PanelDev {
  const int* u_off;        // npan + 1 offsets into u
  const int* u;            // per panel and LDS slot: the union row to stage into the slot,
                           // -1 where the slot keeps what it holds
  const int* r_off;        // npan + 1 offsets into the per-row arrays
  const int* rows;         // output rows, panel by panel
  const uint16_t* eidx;    // [row][kPanelK] LDS byte offset (slot x 256) of each off-diagonal
                           // entry; the row's own slot with value 0 beyond the row's count
  const T* ew;             // [row][kPanelK] its value
  const int4* meta;        // [row] {row, own slot | count << 16, row mask, group count}:
                           // group count = the largest count of the 4 rows one wave computes
  const T* diag;           // [row] diagonal entry of L_r
  int npan;
};

// PF: the next panel's global loads are issued into registers before the
// current panel is computed (more registers, two waves per SIMD); without PF
// each panel is loaded right before it is staged, so those registers are
// free during the computation and the kernel fits three waves per SIMD,
// whose interleaving hides the load latency instead.
template <typename T, int BW, class Epi, bool PF>
__device__ __forceinline__ void panel_body(const T* __restrict__ X, int p, int n,
                                           const PanelDev<T>& pd, const SellDev<T>& Lc,
                                           const BandDev<T>& Lb, const uint8_t* __restrict__ mc,
                                           int G, int ngroups, int gpx, const Epi& epi) {
  if (epi.prologue()) return;
  constexpr int VEC = 16 / sizeof(T);
  constexpr int LN = kPanelLanes;
  constexpr int NS = kThreads / LN;              // row slots
  constexpr int W = LN * VEC;                    // strip width
  constexpr int PAD = band_pad<BW, VEC>();
  constexpr int RM = kPanelRows;
  constexpr int UM = PanelUnion<T>::value;
  constexpr int KR = kPanelK;
  constexpr int SM = UM / NS;                    // union rows staged per thread
  constexpr int HV = 2 * PAD / VEC;              // halo vectors per panel row
  constexpr int HM = (RM * HV + kThreads - 1) / kThreads;
  constexpr int EV = RM * KR / VEC;              // weight vectors per panel
  constexpr int EM = (EV + kThreads - 1) / kThreads;
  constexpr int H = kWave * VEC;                 // SELL slice height
  static_assert(BW > 0 && UM % NS == 0 && UM / NS <= 32 && KR % 8 == 0 && RM * KR == 4 * kThreads, "panel shape");
  static_assert(KR == LN, "one table entry per lane of a row slot");
  static_assert(W * sizeof(T) == kPanelRowBytes && UM * kPanelRowBytes <= 65536, "offset table");
  __shared__ __align__(16) T su[UM * W];
  __shared__ __align__(16) T shl[RM * PAD];
  __shared__ __align__(16) T shr[RM * PAD];
  __shared__ __align__(16) uint16_t sidx[RM * KR];
  __shared__ __align__(16) T swt[RM * KR];
  __shared__ __align__(16) T sdg[RM];
  __shared__ __align__(16) int4 smeta[RM];
  __shared__ int soff[2][kPanelGroupMax + 1];
  double acc[Epi::NV];
#pragma unroll
  for (int k = 0; k < Epi::NV; ++k) acc[k] = 0.0;
  const int t = threadIdx.x;
  const int b = blockIdx.x, x = b & 7, l = b >> 3;
  const int s = l / gpx, g = x * gpx + (l - s * gpx);
  const int nstrips = (n + W - 1) / W;
  if (g < ngroups && s < nstrips) {
    const int cs = s * W, ls = t % LN, rs = t / LN;
    const int c0 = cs + ls * VEC;
    const bool ok = c0 < n;
    const int k0 = g * G, np = min(pd.npan, k0 + G) - k0;
    if (t <= np) {
      soff[0][t] = pd.u_off[k0 + t];
      soff[1][t] = pd.r_off[k0 + t];
    }
    T vb[2 * BW + 1][VEC];
#pragma unroll
    for (int d = 0; d <= 2 * BW; ++d) {
      if (ok && ((Lb.nonempty >> d) & 1ull)) {
        vld<T, VEC>(Lb.v + (size_t)d * Lb.ldb + c0, vb[d]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) vb[d][v] = T(0);
      }
    }
    uint8_t mcv[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) mcv[v] = ok ? mc[c0 + v] : 0;
    int sbeg = 0, sw = 0;  // sliced-ELL remainder of these columns
    if (ok) {
      const int sl = c0 / H;
      sbeg = Lc.sp[sl] + (c0 - sl * H);
      sw = (Lc.sp[sl + 1] - Lc.sp[sl]) / H;
    }
    __syncthreads();
    // Prefetch state: union row indices (next panel but one), staged values
    // and panel tables (next panel).
    int ridx[SM], hrow[HM];
    uint32_t pmask = 0;  // bit m: slot rs + NS * m is overwritten by the rows in flight
    auto load_idx = [&](int kk) {
      const int u0 = soff[0][kk], nu = soff[0][kk + 1] - u0;
      const int r0 = soff[1][kk], nr = soff[1][kk + 1] - r0;
#pragma unroll
      for (int m = 0; m < SM; ++m) {
        const int u = rs + NS * m;
        ridx[m] = u < nu ? pd.u[u0 + u] : -1;
      }
#pragma unroll
      for (int m = 0; m < HM; ++m) {
        const int r = (t + m * kThreads) / HV;
        hrow[m] = r < nr ? pd.rows[r0 + r] : -1;
      }
    };
    T px[SM][VEC], ph[HM][VEC], pw[EM][VEC], pdg = T(0);
    uint2 pi;
    int4 pm;
    auto load_data = [&](int kk) {
      const int r0 = soff[1][kk], nr = soff[1][kk + 1] - r0;
#pragma unroll
      for (int m = 0; m < SM; ++m) {
        pmask = (m == 0 ? 0u : pmask) | (ridx[m] >= 0 ? 1u << m : 0u);
        if (ridx[m] >= 0 && ok) {
          vld<T, VEC>(X + (size_t)ridx[m] * n + c0, px[m]);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v) px[m][v] = T(0);
        }
      }
#pragma unroll
      for (int m = 0; m < HM; ++m) {
        const int hq = (t + m * kThreads) % HV;
        const int c = hq < HV / 2 ? cs - PAD + hq * VEC : cs + W + (hq - HV / 2) * VEC;
        if (hrow[m] >= 0 && c >= 0 && c + VEC <= n) {
          vld<T, VEC>(X + (size_t)hrow[m] * n + c, ph[m]);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v) ph[m][v] = T(0);
        }
      }
      pi = make_uint2(0u, 0u);
      if (t / 4 < nr) pi = *reinterpret_cast<const uint2*>(pd.eidx + (size_t)r0 * KR + t * 4);
#pragma unroll
      for (int m = 0; m < EM; ++m) {
        const int it = t + m * kThreads;
        if (it < EV && (it * VEC) / KR < nr) {
          vld<T, VEC>(pd.ew + (size_t)r0 * KR + (size_t)it * VEC, pw[m]);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v) pw[m][v] = T(0);
        }
      }
      pm = make_int4(0, 0, 0, 0);
      pdg = T(0);
      if (t < nr) {
        pm = pd.meta[r0 + t];
        pdg = pd.diag[r0 + t];
      }
    };
    if constexpr (PF) {
      load_idx(0);
      load_data(0);
      if (np > 1) load_idx(1);
    }
    for (int kk = 0; kk < np; ++kk) {
      const int nr = soff[1][kk + 1] - soff[1][kk];
      if constexpr (!PF) {
        load_idx(kk);
        load_data(kk);
      }
      __syncthreads();  // the previous panel's LDS reads are done
      // rows still resident from an earlier panel of the group keep their
      // slots; the new ones overwrite slots that this panel does not read
#pragma unroll
      for (int m = 0; m < SM; ++m)
        if (pmask >> m & 1u) vst<T, VEC>(&su[(rs + NS * m) * W + ls * VEC], px[m]);
#pragma unroll
      for (int m = 0; m < HM; ++m) {
        const int it = t + m * kThreads;
        const int r = it / HV, hq = it % HV;
        if (r < RM) {
          T* dst = hq < HV / 2 ? &shl[r * PAD + hq * VEC] : &shr[r * PAD + (hq - HV / 2) * VEC];
          vst<T, VEC>(dst, ph[m]);
        }
      }
      *reinterpret_cast<uint2*>(&sidx[t * 4]) = pi;
#pragma unroll
      for (int m = 0; m < EM; ++m) {
        const int it = t + m * kThreads;
        if (it < EV) vst<T, VEC>(&swt[it * VEC], pw[m]);
      }
      if (t < RM) {
        smeta[t] = pm;
        sdg[t] = pdg;
      }
      __syncthreads();
      if constexpr (PF) {
        if (kk + 1 < np) {
          load_data(kk + 1);
          if (kk + 2 < np) load_idx(kk + 2);
        }
      }
      {
        // every lane takes part (lanes past n compute on zeros and store
        // nothing), so the row broadcasts below always read active lanes
        const char* sub = reinterpret_cast<const char*>(su) + ls * VEC * sizeof(T);
        for (int j = rs; j < nr; j += NS) {
          const int4 mt = smeta[j];
          const int row = mt.x, ctr = mt.y & 0xffff;
          const uint8_t mri = (uint8_t)mt.z;
          // entries beyond a row's own count (up to its wave's largest) have
          // value 0 and the row's own slot, so the loop bound is wave-uniform
          const int cnt = __builtin_amdgcn_readfirstlane(mt.w);
          T win[2 * PAD + VEC];
#pragma unroll
          for (int q = 0; q < 2 * PAD + VEC; q += VEC) {
            const int c = ls * VEC - PAD + q;
            const T* ptr = c < 0 ? &shl[j * PAD + c + PAD]
                                 : (c >= W ? &shr[j * PAD + c - W] : &su[ctr * W + c]);
            T w4[VEC];
            vld<T, VEC>(ptr, w4);
#pragma unroll
            for (int v = 0; v < VEC; ++v) win[q + v] = w4[v];
          }
          T xv[VEC], mx[VEC], accr[VEC], accc[VEC];
          const T dg = sdg[j];
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            xv[v] = win[PAD + v];
            accr[v] = dg * xv[v];
            accc[v] = T(0);
            mx[v] = (mri & mcv[v]) ? xv[v] : T(0);
          }
          // lane ls of the row slot holds entry ls of the row's offset and
          // weight tables (one small LDS read per lane); entry e reaches the
          // 16 lanes of the slot, which form one DPP row, by a row broadcast.
          // Entries go in chunks of kGatherChunk under one wave-uniform test:
          // the chunk's LDS reads are all issued before the first is used,
          // so their latencies overlap (entries past the row's count in the
          // last chunk are padding: weight 0 on the row's own slot).
          const uint32_t il = sidx[j * KR + ls];
          const T wl = swt[j * KR + ls];
          static_for<0, KR / kGatherChunk>([&](auto cc) {
            constexpr int e0 = decltype(cc)::value * kGatherChunk;
            if (e0 < cnt) {
              T w[kGatherChunk];
              T u4[kGatherChunk][VEC];
              static_for<0, kGatherChunk>([&](auto ec) {
                constexpr int e = e0 + decltype(ec)::value;
                const uint32_t off = row_bcast<e>(il);
                w[decltype(ec)::value] = row_bcast_t<e>(wl);
                vld<T, VEC>(reinterpret_cast<const T*>(sub + off), u4[decltype(ec)::value]);
              });
#pragma unroll
              for (int q = 0; q < kGatherChunk; ++q)
#pragma unroll
                for (int v = 0; v < VEC; ++v) accr[v] += w[q] * u4[q][v];
            }
          });
#pragma unroll
          for (int d = 0; d <= 2 * BW; ++d)
#pragma unroll
            for (int v = 0; v < VEC; ++v) accc[v] += vb[d][v] * win[PAD + v + d - BW];
          const T* rowp = X + (size_t)row * n;
          for (int e = 0; e < sw; ++e) {
            int kk2[VEC];
            T vv[VEC];
            vld<int, VEC>(Lc.ci + sbeg + e * H, kk2);
            vld<T, VEC>(Lc.v + sbeg + e * H, vv);
#pragma unroll
            for (int v = 0; v < VEC; ++v) accc[v] += vv[v] * rowp[kk2[v]];
          }
          if (ok) epi.template apply<VEC>(row, (size_t)row * n + c0, xv, mx, accr, accc, acc);
        }
      }
    }
  }
  if (epi.partials) block_partials<Epi::NV>(acc, epi.partials);
}

template <typename T, int BW, class Epi>
__global__ void __launch_bounds__(kThreads)
k_apply_panel(const T* __restrict__ X, int p, int n, PanelDev<T> pd, SellDev<T> Lc, BandDev<T> Lb,
              const uint8_t* __restrict__ mc, int G, int ngroups, int gpx, Epi epi) {
  panel_body<T, BW, Epi, true>(X, p, n, pd, Lc, Lb, mc, G, ngroups, gpx, epi);
}

template <typename T, int BW, class Epi>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
k_apply_panel_lo(const T* __restrict__ X, int p, int n, PanelDev<T> pd, SellDev<T> Lc,
                 BandDev<T> Lb, const uint8_t* __restrict__ mc, int G, int ngroups, int gpx,
                 Epi epi) {
  panel_body<T, BW, Epi, false>(X, p, n, pd, Lc, Lb, mc, G, ngroups, gpx, epi);
}

// ---------------------------------------------------------------------------
// CG vector kernels (grid-stride over 16-byte vectors; N % VEC tail scalar).
// ---------------------------------------------------------------------------
template <typename T> struct V16 { static constexpr int W = 16 / sizeof(T); };

// r -= alpha q; partials of <r, r>. alpha = rr / <p, q> is formed here from
// the apply kernel's partials and kept in sc->alpha; the matching x update
// happens in k_cg_pupdate, which reads p anyway (12 + 20 bytes per entry and
// element size 4 instead of 24 + 12).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cg_update(T* __restrict__ r, const T* __restrict__ q, size_t N, CgScal* sc, int it,
            const double* __restrict__ part_pq, int nb_pq, double* __restrict__ part_rr) {
  if (sc->done != 0 || sc->conv_it != 0) return;
  double t[1];
  sum_partials<1>(part_pq, nb_pq, t);
  const double pq = t[0];
  const double rr = sc->rr[it & 1];
  if (bad(pq) || !(pq > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->pq = pq;
      sc->iter = it;
      sc->done = bad(pq) ? 3 : 2;
    }
    return;
  }
  const double alpha_d = rr / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->pq = pq;
    sc->alpha = alpha_d;
  }
  const T alpha = (T)alpha_d;
  constexpr int W = V16<T>::W;
  double acc[1] = {0.0};
  const size_t nv = N / W;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += stride) {
    T rv[W], qv[W];
    vld<T, W>(r + v * W, rv);
    vld<T, W>(q + v * W, qv);
#pragma unroll
    for (int k = 0; k < W; ++k) {
      rv[k] -= alpha * qv[k];
      acc[0] += (double)rv[k] * (double)rv[k];
    }
    vst<T, W>(r + v * W, rv);
  }
  for (size_t e = nv * W + (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const T rn = r[e] - alpha * q[e];
    r[e] = rn;
    acc[0] += (double)rn * (double)rn;
  }
  block_partials<1>(acc, part_rr);
}

// x += alpha p (the step of this iteration, alpha from k_cg_update); then
// beta = rr_new / rr, p = r + beta p; convergence test rr_new <= thr.
// The converging iteration updates x and p as well (see CgScal::conv_it).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cg_pupdate(T* __restrict__ x, T* __restrict__ p, const T* __restrict__ r, size_t N, CgScal* sc,
             int it, const double* __restrict__ part_rr, int nb_rr) {
  if (sc->done != 0) return;
  if (sc->conv_it != 0 && sc->conv_it <= it) return;
  double t[1];
  sum_partials<1>(part_rr, nb_rr, t);
  const double rr_new = t[0];
  const double rr = sc->rr[it & 1];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (bad(rr_new)) {
    if (lead) {
      sc->iter = it + 1;
      sc->done = 3;
    }
    return;
  }
  // An FP32 segment of a residual-replacement solve whose recursive residual
  // has grown far beyond the one it started from is abandoned (the FP64
  // iterate is untouched; the driver restarts from it).
  if (sc->aux > 0.0 && rr_new > kDiverge * sc->aux) {
    if (lead) {
      sc->iter = it + 1;
      sc->done = 4;
    }
    return;
  }
  const double beta_d = rr_new / rr;
  const T alpha = (T)sc->alpha;  // not written in this kernel
  if (lead) {
    sc->rr[(it + 1) & 1] = rr_new;
    sc->beta = beta_d;
    sc->iter = it + 1;
    if (rr_new <= sc->thr) sc->conv_it = it + 1;
  }
  const T beta = (T)beta_d;
  constexpr int W = V16<T>::W;
  const size_t nv = N / W;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += stride) {
    T xv[W], pv[W], rv[W];
    vld<T, W>(x + v * W, xv);
    vld<T, W>(p + v * W, pv);
    vld<T, W>(r + v * W, rv);
#pragma unroll
    for (int k = 0; k < W; ++k) {
      xv[k] += alpha * pv[k];
      pv[k] = rv[k] + beta * pv[k];
    }
    vst<T, W>(x + v * W, xv);
    vst<T, W>(p + v * W, pv);
  }
  for (size_t e = nv * W + (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    x[e] += alpha * p[e];
    p[e] = r[e] + beta * p[e];
  }
}

// Start of a CG solve from x = 0: x = 0, r = p = B; partials of <B, B>.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cg_init_zero(T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
               const T* __restrict__ B, size_t N, double* part) {
  double acc[1] = {0.0};
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const T b = B[e];
    x[e] = T(0);
    r[e] = b;
    p[e] = b;
    acc[0] += (double)b * (double)b;
  }
  block_partials<1>(acc, part);
}

// Arms the CG scalars from partials (one workgroup):
//   NV = 1: rr = total (start from zero), threshold thr_abs;
//   NV = 2: residual start, res2 = total[0], rr = aux = total[1],
//           threshold thr_abs if >= 0 else rel_tol2 * rr.
template <int NV>
__global__ void __launch_bounds__(kThreads)
k_cg_arm(CgScal* sc, const double* part, int nb, double thr_abs, double rel_tol2) {
  double t[NV];
  sum_partials<NV>(part, nb, t);
  if (threadIdx.x != 0) return;
  const double rr = t[NV - 1];
  const double thr = thr_abs >= 0.0 ? thr_abs : rel_tol2 * rr;
  if constexpr (NV == 2) {
    sc->res2 = t[0];
    sc->aux = t[1];
  } else {
    sc->aux = 0.0;  // no divergence test outside residual replacement
  }
  sc->rr[0] = rr;
  sc->rr[1] = rr;
  sc->thr = thr;
  sc->iter = 0;
  sc->alpha = 0.0;
  sc->beta = 0.0;
  sc->done = (bad(t[0]) || bad(rr)) ? 3 : 0;
  sc->conv_it = (sc->done == 0 && rr <= thr) ? -1 : 0;
}

// Raises the stop threshold of an armed CG solve to at least thr.
static __global__ void k_cg_set_thr(CgScal* sc, double thr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (sc->thr < thr) sc->thr = thr;
    if (sc->done == 0 && sc->conv_it == 0 && sc->rr[0] <= sc->thr) sc->conv_it = -1;
  }
}

// out[k] = sum of the partials (one workgroup).
template <int NV>
__global__ void __launch_bounds__(kThreads)
k_sum_partials(const double* part, int nb, double* out) {
  double t[NV];
  sum_partials<NV>(part, nb, t);
  if (threadIdx.x < NV) out[threadIdx.x] = t[threadIdx.x];
}

// Partials of ||a||^2.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_norm2(const T* __restrict__ a, size_t N, double* part) {
  double acc[1] = {0.0};
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const double v = (double)a[e];
    acc[0] += v * v;
  }
  block_partials<1>(acc, part);
}

// X64 += d (refinement update).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_accumulate(double* __restrict__ X, const T* __restrict__ d, size_t N) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride)
    X[e] += (double)d[e];
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kThreads)
k_convert(TO* __restrict__ out, const TI* __restrict__ in, size_t N) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride)
    out[e] = (TO)in[e];
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fill(T* __restrict__ out, T v, size_t N) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) out[e] = v;
}

// B[omega_r[a], omega_c[b]] = Xtil[a, b] (B cleared beforehand).
template <typename TI, typename TO>
__global__ void __launch_bounds__(kThreads)
k_scatter(TO* __restrict__ B, int n, const TI* __restrict__ Xtil, int rho_r, int rho_c,
          const int* __restrict__ om_r, const int* __restrict__ om_c) {
  const size_t N = (size_t)rho_r * rho_c;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const int a = (int)(e / rho_c);
    const int b = (int)(e - (size_t)a * rho_c);
    B[(size_t)om_r[a] * n + om_c[b]] = (TO)Xtil[e];
  }
}

// out[a, b] = Lam[omega_r[a], omega_c[b]].
template <typename TI, typename TO>
__global__ void __launch_bounds__(kThreads)
k_gather(TO* __restrict__ out, const TI* __restrict__ Lam, int n, int rho_r, int rho_c,
         const int* __restrict__ om_r, const int* __restrict__ om_c) {
  const size_t N = (size_t)rho_r * rho_c;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const int a = (int)(e / rho_c);
    const int b = (int)(e - (size_t)a * rho_c);
    out[e] = (TO)Lam[(size_t)om_r[a] * n + om_c[b]];
  }
}

}  // namespace cpca
