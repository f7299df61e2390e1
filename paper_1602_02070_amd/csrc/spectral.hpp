// Largest eigenvalue of a graph Laplacian on the device, for the FISTA step
// of FRPCAG (Section IV.B: the step is the inverse of
// 2 gamma_c ||L_c||_2 + 2 gamma_r ||L_r||_2, and for a symmetric PSD
// Laplacian the spectral norm is its largest eigenvalue).
//
// FP64 power iteration in one workgroup: w = L v, theta = <v, w> (v of unit
// norm), residual ||w - theta v||, v = w / ||w||. It stops when the residual
// is at most tol * theta (then an eigenvalue lies within tol * theta of
// theta) or after max_it products. The start vector is a fixed
// pseudo-random positive vector, so the result does not depend on the call.
// The paper does not say how the norm is obtained; this estimate is not
// part of the parity contract (parity runs pass the exact value).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpca {

constexpr int kPowThreads = 1024;

__device__ __forceinline__ double pow_block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kPowThreads / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// out[0] = theta, out[1] = final residual norm, out[2] = products run.
// (A template, so that every translation unit may instantiate it.)
template <int NT = kPowThreads>
__global__ void __launch_bounds__(NT)
k_power_lmax(const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ val,
             int n, double* __restrict__ v, double* __restrict__ w, int max_it, double tol,
             double* __restrict__ out) {
  __shared__ double red[kPowThreads / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kPowThreads) {
    // 32-bit integer hash of the index -> [0.5, 1.5)
    uint32_t x = (uint32_t)i * 2654435761u + 0x9e3779b9u;
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    const double a = 0.5 + (double)(x >> 8) * (1.0 / 16777216.0);
    v[i] = a;
    s += a * a;
  }
  s = pow_block_sum(s, red);
  double inv = 1.0 / sqrt(s);
  for (int i = threadIdx.x; i < n; i += kPowThreads) v[i] *= inv;
  __syncthreads();
  double theta = 0.0, res = 0.0;
  int it = 0;
  while (it < max_it) {
    double vw = 0.0, ww = 0.0;
    for (int i = threadIdx.x; i < n; i += kPowThreads) {
      double acc = 0.0;
      for (int e = rp[i]; e < rp[i + 1]; ++e) acc += val[e] * v[ci[e]];
      w[i] = acc;
      vw += v[i] * acc;
      ww += acc * acc;
    }
    ++it;
    theta = pow_block_sum(vw, red);
    ww = pow_block_sum(ww, red);
    double rr = 0.0;
    for (int i = threadIdx.x; i < n; i += kPowThreads) {
      const double d = w[i] - theta * v[i];
      rr += d * d;
    }
    res = sqrt(pow_block_sum(rr, red));
    if (!(ww > 0.0) || res <= tol * theta) break;
    inv = 1.0 / sqrt(ww);
    for (int i = threadIdx.x; i < n; i += kPowThreads) v[i] = w[i] * inv;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = theta;
    out[1] = res;
    out[2] = (double)it;
  }
}

}  // namespace cpca

// ------------------------------------------------------------------ host side
// (included after common.hpp: uses the handle, its workspace and scalars)
#ifdef CPCA_SPECTRAL_HOST
namespace {

constexpr double kLmaxTol = 1e-9;     // residual / theta at which the iteration stops
constexpr int kLmaxMaxIt = 50000;     // products at most

// Largest eigenvalue of the caller's CSR (already validated on the host by
// fetch_csr, so every column index is in range). Uses the front of the
// handle's workspace; call it before a driver lays out its own arena.
cpca_status device_lmax(cpca_handle h, const cpca_csr* L, double tol, int max_it, double* lmax,
                        double* resid, int* its) {
  const int n = (int)L->n;
  STCHK(ensure_ws(h, align_up((size_t)n * sizeof(double), 256) * 2 + 256));
  double* v = reinterpret_cast<double*>(h->ws);
  double* w = v + align_up((size_t)n * sizeof(double), 256) / sizeof(double);
  k_power_lmax<><<<1, kPowThreads, 0, h->stream>>>(L->rowptr, L->colind, L->vals, n, v, w, max_it,
                                                 tol, results_ptr(h) + 8);
  LAUNCHCHK();
  STCHK(read_fixed(h));
  const double* r = host_results(h) + 8;
  if (!std::isfinite(r[0]) || !std::isfinite(r[1])) return fail(CPCA_ENAN, "lmax: NaN or Inf");
  *lmax = r[0];
  if (resid) *resid = r[1];
  if (its) *its = (int)r[2];
  return CPCA_OK;
}

}  // namespace
#endif
