// Device kernels of the CPCA solvers for gfx950 (CDNA4, wave64).
//
// The central kernel is the fused two-sided sparse product
//     out(i, j) = mask(i, j) X(i, j) + a_r (L_r X)(i, j) + a_c (X L_c)(i, j)
// which is the gradient of the graph term of FRPCAG (Section IV.B) and the
// operator of the alternate decoder's normal equations (Section V.B). One
// workgroup owns R consecutive rows of X and sweeps all n columns:
//   * the R rows are staged in LDS, so the X L_c term gathers its operands
//     from LDS;
//   * L_c is held in a sliced ELL layout (SELL, one slice per 64 columns =
//     one wavefront), so its index/value loads are coalesced and all lanes of
//     a wave run the same trip count;
//   * the L_r X term streams neighbour rows of X straight from memory with
//     coalesced column accesses (row i's CSR entries are wave-uniform);
//   * the row-block index is remapped so that each XCD owns a contiguous
//     range of rows and neighbour rows are shared through its L2.
// What happens to out(i, j) is decided by an epilogue functor (CG apply,
// FISTA step, residual, objective, adjoint dot products).
//
// Reductions are deterministic: FP64 per-thread partials, wave butterfly,
// per-block partials in global memory, and the last block to finish (found
// with an integer atomic counter) sums the block partials in a fixed order
// and runs the epilogue's finaliser (CG alpha/beta, convergence flags).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpca {

constexpr int kWave = 64;
constexpr int kSlice = 64;        // SELL slice height (columns per slice)
constexpr int kThreads = 256;     // threads per workgroup for all kernels
constexpr int kMaxWaves = kThreads / kWave;

template <typename T>
struct CsrDev {
  const int* rp;
  const int* ci;
  const T* v;
};

// Sliced ELL: slice s covers columns [64 s, 64 s + 64); its entries start at
// sp[s], width w_s = (sp[s+1] - sp[s]) / 64, entry e of column j sits at
// sp[s] + 64 e + (j & 63). Padding entries carry value 0 and index j.
template <typename T>
struct SellDev {
  const int* sp;
  const int* ci;
  const T* v;
};

// Device-resident scalars of one CG solve (FP64).
struct CgScal {
  double rr;      // current <r, r>
  double thr;     // stop when rr <= thr
  double alpha;
  double beta;
  double pq;      // last <p, A p>
  double bb;      // ||rhs||^2
  double res2;    // last FP64 residual norm^2 (refinement)
  double aux;     // last rounded-residual norm^2 (refinement)
  int iter;       // iterations completed
  int done;       // 0 running, 1 converged, 2 breakdown, 3 NaN/Inf
  int pad0, pad1;
};

// Device-resident scalars of one FISTA run.
struct FistaScal {
  double dz2;     // ||Z+ - Z||^2 of the last reduced step
  double z2;      // ||Z||^2 of the last reduced step
  double obj_l1;  // objective pieces
  double obj_g;
  int iter;
  int done;       // 0 running, 1 stopped by eps, 3 NaN/Inf
  int pad0, pad1;
};

struct RedSlot {
  double* partials;   // gridDim.x * NV doubles
  unsigned* counter;  // zero between launches
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Deterministic grid reduction of NV FP64 values. Every thread of every
// block must call it. Returns true in all threads of the block that finished
// last; `tot` then holds the grid totals (in every thread of that block).
template <int NV>
__device__ bool grid_reduce(double (&v)[NV], RedSlot slot, double (&tot)[NV]) {
  __shared__ double red[NV][kMaxWaves];
  __shared__ int is_last;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[k][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[k][w];
      slot.partials[(size_t)blockIdx.x * NV + k] = s;
    }
    __threadfence();
    const unsigned prev = atomicAdd(slot.counter, 1u);
    is_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x)
      s += load_agent(&slot.partials[(size_t)b * NV + k]);
    s = wave_sum(s);
    if (lane == 0) red[k][wid] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[k][w];
    tot[k] = s;
  }
  if (threadIdx.x == 0)
    __hip_atomic_store(slot.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

__device__ __forceinline__ bool bad(double x) { return !(x == x) || x - x != 0.0; }

// ---------------------------------------------------------------------------
// Epilogues of the fused two-sided product. Each one provides
//   NV                      number of FP64 reduction values
//   skip()                  device-side early exit (converged solves)
//   operator()(i, j, idx, x, mx, accr, accc, acc)
//                           x = X(i,j), mx = mask(i,j) * X(i,j),
//                           accr = (L_r X)(i,j), accc = (X L_c)(i,j)
//   finalize(tot)           runs once, in the last block, threads see tot
// ---------------------------------------------------------------------------

// Q = A(P), <P, Q> -> *pq (plain operator application).
template <typename T>
struct EpiApply {
  static constexpr int NV = 1;
  T* Q;
  T gr, gc;
  double* pq;
  __device__ bool skip() const { return false; }
  __device__ void operator()(int, int, size_t idx, T x, T mx, T accr, T accc,
                             double* acc) const {
    const T out = mx + gr * accr + gc * accc;
    Q[idx] = out;
    acc[0] += (double)x * (double)out;
  }
  __device__ void finalize(const double* tot) const {
    if (threadIdx.x == 0 && pq) *pq = tot[0];
  }
};

// CG: q = A(p), alpha = rr / <p, q>.
template <typename T>
struct EpiCg {
  static constexpr int NV = 1;
  T* Q;
  T gr, gc;
  CgScal* sc;
  __device__ bool skip() const { return sc->done != 0; }
  __device__ void operator()(int, int, size_t idx, T x, T mx, T accr, T accc,
                             double* acc) const {
    const T out = mx + gr * accr + gc * accc;
    Q[idx] = out;
    acc[0] += (double)x * (double)out;
  }
  __device__ void finalize(const double* tot) const {
    if (threadIdx.x != 0) return;
    const double pq = tot[0];
    sc->pq = pq;
    if (bad(pq)) {
      sc->done = 3;
    } else if (!(pq > 0.0)) {
      sc->done = 2;
    } else {
      sc->alpha = sc->rr / pq;
    }
  }
};

// Residual R = B - A(X) computed in T, stored rounded to TO into r_out and
// p_out (initial residual and direction of a CG solve); x_out (the CG
// iterate), if given, is cleared. Totals: ||R||^2 and ||round(R)||^2 (FP64).
// The finaliser arms the CG scalars: rr = ||round(R)||^2 and the stop
// threshold thr_abs, or rel_tol2 * rr when thr_abs < 0.
template <typename T, typename TO>
struct EpiResidual {
  static constexpr int NV = 2;
  const T* B;
  TO* r_out;
  TO* p_out;
  TO* x_out;
  T gr, gc;
  CgScal* sc;
  double thr_abs;
  double rel_tol2;
  __device__ bool skip() const { return false; }
  __device__ void operator()(int, int, size_t idx, T, T mx, T accr, T accc,
                             double* acc) const {
    const T R = B[idx] - (mx + gr * accr + gc * accc);
    const TO Rt = (TO)R;
    r_out[idx] = Rt;
    p_out[idx] = Rt;
    if (x_out) x_out[idx] = TO(0);
    acc[0] += (double)R * (double)R;
    acc[1] += (double)Rt * (double)Rt;
  }
  __device__ void finalize(const double* tot) const {
    if (threadIdx.x != 0) return;
    sc->res2 = tot[0];
    sc->aux = tot[1];
    sc->rr = tot[1];
    sc->thr = thr_abs >= 0.0 ? thr_abs : rel_tol2 * tot[1];
    sc->iter = 0;
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->done = (bad(tot[0]) || bad(tot[1])) ? 3 : (tot[1] <= sc->thr ? 1 : 0);
  }
};

// Residual norm only: ||B - A(X)||^2, X of any storage type, FP64 arithmetic.
template <typename T>
struct EpiResNorm {
  static constexpr int NV = 1;
  const T* B;
  double gr, gc;
  double* out;
  __device__ bool skip() const { return false; }
  __device__ void operator()(int, int, size_t idx, T, T mx, T accr, T accc,
                             double* acc) const {
    const double R = (double)B[idx] - ((double)mx + gr * (double)accr + gc * (double)accc);
    acc[0] += R * R;
  }
  __device__ void finalize(const double* tot) const {
    if (threadIdx.x == 0) *out = tot[0];
  }
};

// One FISTA iteration (Algorithm 1) on the FP64 state:
//   G  = Z - lam * grad g(Z),  grad g = 2 (gc Z L_c + gr L_r Z)
//   S  = Y + sgn(G - Y) max(|G - Y| - lam, 0)
//   Z+ = S + c (S - S_prev),   c = (t_j - 1) / t_{j+1}
// S overwrites S_prev in place (same element, same thread); Z+ goes to a
// second buffer because neighbouring rows of Z are still being read.
template <bool REDUCE>
struct EpiFista {
  static constexpr int NV = 2;
  const double* Y;
  double* S;
  double* Zn;
  double two_gr, two_gc, lam, c, eps;
  FistaScal* fs;
  __device__ bool skip() const { return fs->done != 0; }
  __device__ void operator()(int, int, size_t idx, double z, double, double accr,
                             double accc, double* acc) const {
    const double g = z - lam * (two_gr * accr + two_gc * accc);
    const double y = Y[idx];
    const double d = g - y;
    const double mag = fabs(d) - lam;
    const double s = mag > 0.0 ? y + copysign(mag, d) : y;
    const double sp = S[idx];
    const double zn = s + c * (s - sp);
    S[idx] = s;
    Zn[idx] = zn;
    if (REDUCE) {
      const double dz = zn - z;
      acc[0] += dz * dz;
      acc[1] += z * z;
    }
  }
  __device__ void finalize(const double* tot) const {
    if (threadIdx.x != 0) return;
    fs->dz2 = tot[0];
    fs->z2 = tot[1];
    fs->iter += 1;
    if (bad(tot[0]) || bad(tot[1]))
      fs->done = 3;
    else if (tot[0] < eps * tot[1])
      fs->done = 1;
  }
};

// FRPCAG objective at X: ||Y - X||_1 + <X, gc X L_c + gr L_r X>.
struct EpiObjective {
  static constexpr int NV = 2;
  const double* Y;
  double gr, gc;
  FistaScal* fs;
  __device__ bool skip() const { return false; }
  __device__ void operator()(int, int, size_t idx, double x, double, double accr,
                             double accc, double* acc) const {
    acc[0] += fabs(Y[idx] - x);
    acc[1] += x * (gr * accr + gc * accc);
  }
  __device__ void finalize(const double* tot) const {
    if (threadIdx.x != 0) return;
    fs->obj_l1 = tot[0];
    fs->obj_g = tot[1];
  }
};

// Adjoint dot products <Lam, L_r X> and <Lam, X L_c>.
template <typename T>
struct EpiDot2 {
  static constexpr int NV = 2;
  const T* Lam;
  double* out;  // 2 doubles
  __device__ bool skip() const { return false; }
  __device__ void operator()(int, int, size_t idx, T, T, T accr, T accc,
                             double* acc) const {
    const double l = (double)Lam[idx];
    acc[0] += l * (double)accr;
    acc[1] += l * (double)accc;
  }
  __device__ void finalize(const double* tot) const {
    if (threadIdx.x != 0) return;
    out[0] = tot[0];
    out[1] = tot[1];
  }
};

// ---------------------------------------------------------------------------
// The fused two-sided product. R rows per workgroup, all n columns.
//   LDS = true : the R rows live in LDS (R * n * sizeof(T) bytes).
//   LDS = false: X L_c gathers from global memory (very wide rows).
// Grid: 8 * per blocks; block b handles row block (b % 8) * per + b / 8, so
// that each XCD (blocks are dealt to XCDs round-robin) owns `per`
// consecutive row blocks. Blocks past the last row block only join the
// reduction.
// ---------------------------------------------------------------------------
template <typename T, int R, bool LDS, class Epi>
__global__ void __launch_bounds__(kThreads)
k_apply2(const T* __restrict__ X, int p, int n, CsrDev<T> Lr, SellDev<T> Lc,
         const uint8_t* __restrict__ mr, const uint8_t* __restrict__ mc,
         int nrb, int per, Epi epi, RedSlot slot) {
  if (epi.skip()) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* panel = reinterpret_cast<T*>(smem_raw);
  double acc[Epi::NV];
#pragma unroll
  for (int k = 0; k < Epi::NV; ++k) acc[k] = 0.0;

  const int b = blockIdx.x;
  const int rb = (b & 7) * per + (b >> 3);
  if (rb < nrb) {
    const int i0 = rb * R;
    const int rows = min(R, p - i0);
    if (LDS) {
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        if (rr < rows) {
          const T* src = X + (size_t)(i0 + rr) * n;
          for (int j = threadIdx.x; j < n; j += blockDim.x) panel[rr * n + j] = src[j];
        }
      }
      __syncthreads();
    }
    for (int jb = 0; jb < n; jb += blockDim.x) {
      const int j = jb + threadIdx.x;
      if (j >= n) continue;
      // X L_c: column j of L_c (= row j, L_c symmetric), shared by the R rows
      T accc[R];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) accc[rr] = T(0);
      {
        const int s = j >> 6;
        const int beg = Lc.sp[s];
        const int w = (Lc.sp[s + 1] - beg) >> 6;
        const int* ci = Lc.ci + beg + (j & 63);
        const T* cv = Lc.v + beg + (j & 63);
#pragma unroll 4
        for (int e = 0; e < w; ++e) {
          const int k = ci[e * kSlice];
          const T v = cv[e * kSlice];
#pragma unroll
          for (int rr = 0; rr < R; ++rr) {
            if (rr < rows) {
              const T xv = LDS ? panel[rr * n + k] : X[(size_t)(i0 + rr) * n + k];
              accc[rr] += v * xv;
            }
          }
        }
      }
      const uint8_t mcj = mc[j];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        if (rr < rows) {
          const int i = i0 + rr;
          // L_r X: row i of L_r, neighbour rows of X, coalesced over j
          T accr = T(0);
          const int e0 = Lr.rp[i];
          const int e1 = Lr.rp[i + 1];
#pragma unroll 4
          for (int e = e0; e < e1; ++e) accr += Lr.v[e] * X[(size_t)Lr.ci[e] * n + j];
          const size_t idx = (size_t)i * n + j;
          const T x = LDS ? panel[rr * n + j] : X[idx];
          const T mx = (mr[i] & mcj) ? x : T(0);
          epi(i, j, idx, x, mx, accr, accc[rr], acc);
        }
      }
    }
  }
  double tot[Epi::NV];
  if (grid_reduce<Epi::NV>(acc, slot, tot)) epi.finalize(tot);
}

// ---------------------------------------------------------------------------
// CG vector kernels (grid-stride, 16-byte vector accesses where aligned).
// ---------------------------------------------------------------------------
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int W = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int W = 2; };

template <typename T>
__device__ __forceinline__ void vload(const T* p, T (&v)[Vec16<T>::W]) {
  using V = typename Vec16<T>::type;
  const V t = *reinterpret_cast<const V*>(p);
  if constexpr (Vec16<T>::W == 4) { v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w; }
  else { v[0] = t.x; v[1] = t.y; }
}
template <typename T>
__device__ __forceinline__ void vstore(T* p, const T (&v)[Vec16<T>::W]) {
  using V = typename Vec16<T>::type;
  V t;
  if constexpr (Vec16<T>::W == 4) { t.x = v[0]; t.y = v[1]; t.z = v[2]; t.w = v[3]; }
  else { t.x = v[0]; t.y = v[1]; }
  *reinterpret_cast<V*>(p) = t;
}

// x += alpha p; r -= alpha q; rr_new = <r, r>; beta = rr_new / rr.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cg_update(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
            const T* __restrict__ q, size_t N, CgScal* sc, RedSlot slot) {
  if (sc->done != 0) return;
  const T alpha = (T)sc->alpha;
  constexpr int W = Vec16<T>::W;
  double acc[1] = {0.0};
  const size_t nv = N / W;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += stride) {
    T xv[W], rv[W], pv[W], qv[W];
    vload(x + v * W, xv);
    vload(r + v * W, rv);
    vload(p + v * W, pv);
    vload(q + v * W, qv);
#pragma unroll
    for (int k = 0; k < W; ++k) {
      xv[k] += alpha * pv[k];
      rv[k] -= alpha * qv[k];
      acc[0] += (double)rv[k] * (double)rv[k];
    }
    vstore(x + v * W, xv);
    vstore(r + v * W, rv);
  }
  for (size_t e = nv * W + (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    x[e] += alpha * p[e];
    const T rn = r[e] - alpha * q[e];
    r[e] = rn;
    acc[0] += (double)rn * (double)rn;
  }
  double tot[1];
  if (grid_reduce<1>(acc, slot, tot) && threadIdx.x == 0) {
    const double rr_new = tot[0];
    sc->iter += 1;
    if (bad(rr_new)) {
      sc->done = 3;
    } else {
      sc->beta = rr_new / sc->rr;
      sc->rr = rr_new;
      if (rr_new <= sc->thr) sc->done = 1;
    }
  }
}

// p = r + beta p.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cg_pupdate(T* __restrict__ p, const T* __restrict__ r, size_t N, const CgScal* sc) {
  if (sc->done != 0) return;
  const T beta = (T)sc->beta;
  constexpr int W = Vec16<T>::W;
  const size_t nv = N / W;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += stride) {
    T pv[W], rv[W];
    vload(p + v * W, pv);
    vload(r + v * W, rv);
#pragma unroll
    for (int k = 0; k < W; ++k) pv[k] = rv[k] + beta * pv[k];
    vstore(p + v * W, pv);
  }
  for (size_t e = nv * W + (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride)
    p[e] = r[e] + beta * p[e];
}

// Start of a CG solve from x = 0: x = 0, r = p = B, rr = <B, B>.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cg_init_zero(T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
               const T* __restrict__ B, size_t N, CgScal* sc, double thr_abs,
               RedSlot slot) {
  double acc[1] = {0.0};
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const T b = B[e];
    x[e] = T(0);
    r[e] = b;
    p[e] = b;
    acc[0] += (double)b * (double)b;
  }
  double tot[1];
  if (grid_reduce<1>(acc, slot, tot) && threadIdx.x == 0) {
    sc->rr = tot[0];
    sc->thr = thr_abs;
    sc->iter = 0;
    sc->alpha = sc->beta = 0.0;
    sc->done = bad(tot[0]) ? 3 : (tot[0] == 0.0 ? 1 : 0);
  }
}

// Squared norm of a vector into *out (FP64).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_norm2(const T* __restrict__ a, size_t N, double* out, RedSlot slot) {
  double acc[1] = {0.0};
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
    const double v = (double)a[e];
    acc[0] += v * v;
  }
  double tot[1];
  if (grid_reduce<1>(acc, slot, tot) && threadIdx.x == 0) *out = tot[0];
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
