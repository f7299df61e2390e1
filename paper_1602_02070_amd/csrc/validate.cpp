// Host-side argument checks of the C ABI. Pure C++: no HIP calls, so the
// checks can run (and be tested) on machines without a GPU.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "cpca.h"
#include "validate.hpp"

namespace cpca {

static thread_local std::string g_last_error;

cpca_status fail(cpca_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

void clear_error() { g_last_error.clear(); }

const char* last_error() { return g_last_error.c_str(); }

cpca_status check_csr_host(const char* name, int64_t n, int64_t nnz,
                           const int32_t* rowptr, const int32_t* colind,
                           const double* vals) {
  char buf[256];
  if (n < 1 || n > INT32_MAX) {
    std::snprintf(buf, sizeof buf, "%s: order n=%lld out of range", name, (long long)n);
    return fail(CPCA_EINVAL, buf);
  }
  if (nnz < 0 || nnz > INT32_MAX) {
    std::snprintf(buf, sizeof buf, "%s: nnz=%lld out of range", name, (long long)nnz);
    return fail(CPCA_EINVAL, buf);
  }
  if (!rowptr || (nnz > 0 && !colind)) {
    std::snprintf(buf, sizeof buf, "%s: null CSR array", name);
    return fail(CPCA_EINVAL, buf);
  }
  if (rowptr[0] != 0 || rowptr[n] != nnz) {
    std::snprintf(buf, sizeof buf, "%s: rowptr[0]=%d, rowptr[n]=%d, expected 0 and nnz=%lld",
                  name, rowptr[0], rowptr[n], (long long)nnz);
    return fail(CPCA_EINVAL, buf);
  }
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) {
      std::snprintf(buf, sizeof buf, "%s: rowptr decreases at row %lld", name, (long long)i);
      return fail(CPCA_EINVAL, buf);
    }
  }
  for (int64_t e = 0; e < nnz; ++e) {
    if (colind[e] < 0 || colind[e] >= n) {
      std::snprintf(buf, sizeof buf, "%s: column index %d at entry %lld out of [0, %lld)", name,
                    colind[e], (long long)e, (long long)n);
      return fail(CPCA_EINVAL, buf);
    }
  }
  if (vals) {
    for (int64_t e = 0; e < nnz; ++e) {
      if (!std::isfinite(vals[e])) {
        std::snprintf(buf, sizeof buf, "%s: non-finite value at entry %lld", name, (long long)e);
        return fail(CPCA_EINVAL, buf);
      }
    }
  }
  return CPCA_OK;
}

cpca_status check_index_set_host(const char* name, int64_t count, int64_t dim,
                                 const int32_t* idx, std::vector<uint8_t>* mask_out) {
  char buf[256];
  if (count < 0 || count > dim) {
    std::snprintf(buf, sizeof buf, "%s: %lld indices for dimension %lld", name,
                  (long long)count, (long long)dim);
    return fail(CPCA_EINVAL, buf);
  }
  if (count > 0 && !idx) {
    std::snprintf(buf, sizeof buf, "%s: null index array", name);
    return fail(CPCA_EINVAL, buf);
  }
  std::vector<uint8_t> mask((size_t)dim, 0);
  for (int64_t a = 0; a < count; ++a) {
    const int64_t v = idx[a];
    if (v < 0 || v >= dim) {
      std::snprintf(buf, sizeof buf, "%s: index %lld at position %lld out of [0, %lld)", name,
                    (long long)v, (long long)a, (long long)dim);
      return fail(CPCA_EINVAL, buf);
    }
    if (mask[(size_t)v]) {
      std::snprintf(buf, sizeof buf, "%s: index %lld repeated (position %lld)", name,
                    (long long)v, (long long)a);
      return fail(CPCA_EINVAL, buf);
    }
    mask[(size_t)v] = 1;
  }
  if (mask_out) mask_out->swap(mask);
  return CPCA_OK;
}

cpca_status check_gamma(const char* name, double g) {
  if (!std::isfinite(g) || g < 0.0) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "%s=%g must be finite and >= 0", name, g);
    return fail(CPCA_EINVAL, buf);
  }
  return CPCA_OK;
}

cpca_status check_mode(cpca_mode mode) {
  if (mode != CPCA_FP64 && mode != CPCA_FP32 && mode != CPCA_FP32_IR)
    return fail(CPCA_EINVAL, "unknown mode");
  return CPCA_OK;
}

cpca_status check_dims(const char* what, int64_t rows, int64_t cols) {
  if (rows < 1 || cols < 1 || rows > INT32_MAX || cols > INT32_MAX) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s: size %lld x %lld out of range", what, (long long)rows,
                  (long long)cols);
    return fail(CPCA_EINVAL, buf);
  }
  return CPCA_OK;
}

cpca_status check_csr_shape(const char* name, const cpca_csr* A, int64_t order) {
  if (!A) return fail(CPCA_EINVAL, std::string(name) + ": null CSR descriptor");
  if (A->n != order) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s: order %lld, expected %lld", name, (long long)A->n,
                  (long long)order);
    return fail(CPCA_EINVAL, buf);
  }
  if (A->nnz < 0 || A->nnz > INT32_MAX)
    return fail(CPCA_EINVAL, std::string(name) + ": nnz out of range");
  if (!A->rowptr || (A->nnz > 0 && (!A->colind || !A->vals)))
    return fail(CPCA_EINVAL, std::string(name) + ": null CSR array");
  return CPCA_OK;
}

cpca_status check_frpcag_args(cpca_mode mode, const void* Ytil, int64_t rho_r, int64_t rho_c,
                              const cpca_csr* Lr, const cpca_csr* Lc, double gr, double gc,
                              double lmax_r, double lmax_c, int32_t max_iter, double eps,
                              const void* out) {
  cpca_status st;
  if ((st = check_mode(mode))) return st;
  if ((st = check_dims("Ytil", rho_r, rho_c))) return st;
  if (!Ytil || !out) return fail(CPCA_EINVAL, "frpcag: null data pointer");
  if ((st = check_csr_shape("Lr_til", Lr, rho_r))) return st;
  if ((st = check_csr_shape("Lc_til", Lc, rho_c))) return st;
  if ((st = check_gamma("gamma_r", gr))) return st;
  if ((st = check_gamma("gamma_c", gc))) return st;
  // lmax <= 0 asks the library to estimate the norm (device power iteration)
  if (!std::isfinite(lmax_r) || !std::isfinite(lmax_c))
    return fail(CPCA_EINVAL, "frpcag: lmax must be finite");
  if (max_iter < 0) return fail(CPCA_EINVAL, "frpcag: max_iter < 0");
  if (!std::isfinite(eps) || eps < 0) return fail(CPCA_EINVAL, "frpcag: eps must be finite and >= 0");
  return CPCA_OK;
}

cpca_status check_decode_args(cpca_mode mode, int64_t rho_r, int64_t rho_c,
                              const int32_t* om_r, const int32_t* om_c, int64_t p, int64_t n,
                              const cpca_csr* Lr, const cpca_csr* Lc, double gr, double gc,
                              double tol, int32_t max_iter) {
  cpca_status st;
  if ((st = check_mode(mode))) return st;
  if ((st = check_dims("X", p, n))) return st;
  if ((unsigned long long)p * (unsigned long long)n > (1ull << 40))
    return fail(CPCA_EINVAL, "decode: p * n too large");
  if ((st = check_dims("Xtil", rho_r, rho_c))) return st;
  if (rho_r > p || rho_c > n) return fail(CPCA_EINVAL, "decode: more samples than rows/columns");
  if (!om_r || !om_c) return fail(CPCA_EINVAL, "decode: null index set");
  if ((st = check_csr_shape("Lr", Lr, p))) return st;
  if ((st = check_csr_shape("Lc", Lc, n))) return st;
  if ((st = check_gamma("gamma_r", gr))) return st;
  if ((st = check_gamma("gamma_c", gc))) return st;
  if (!std::isfinite(tol) || !(tol > 0)) return fail(CPCA_EINVAL, "decode: tol must be > 0");
  if (max_iter < 1) return fail(CPCA_EINVAL, "decode: max_iter < 1");
  return CPCA_OK;
}

cpca_status check_approx_args(cpca_mode mode, int64_t rho_r, int64_t rho_c,
                              const int32_t* om_r, const int32_t* om_c, int64_t p, int64_t n,
                              const cpca_csr* Lr, const cpca_csr* Lc, double delta,
                              double ratio, int32_t k_max, double tol, int32_t max_iter) {
  cpca_status st;
  if ((st = check_mode(mode))) return st;
  if ((st = check_dims("X", p, n))) return st;
  if ((unsigned long long)p * (unsigned long long)n > (1ull << 40))
    return fail(CPCA_EINVAL, "approx_decode: p * n too large");
  if ((st = check_dims("Xtil", rho_r, rho_c))) return st;
  if (rho_r > p || rho_c > n)
    return fail(CPCA_EINVAL, "approx_decode: more samples than rows/columns");
  if (!om_r || !om_c) return fail(CPCA_EINVAL, "approx_decode: null index set");
  if ((st = check_csr_shape("Lr", Lr, p))) return st;
  if ((st = check_csr_shape("Lc", Lc, n))) return st;
  if (!std::isfinite(delta) || delta < 0 || !(delta < 1))
    return fail(CPCA_EINVAL, "approx_decode: delta must be in [0, 1)");
  if (!std::isfinite(ratio) || ratio < 0 || ratio > 1)
    return fail(CPCA_EINVAL, "approx_decode: sigma_ratio must be in [0, 1]");
  if (k_max < 1 || k_max > 64) return fail(CPCA_EINVAL, "approx_decode: k_max must be in [1, 64]");
  if (!std::isfinite(tol) || !(tol > 0)) return fail(CPCA_EINVAL, "approx_decode: tol must be > 0");
  if (max_iter < 0) return fail(CPCA_EINVAL, "approx_decode: max_iter < 0");
  return CPCA_OK;
}

cpca_status check_cluster_args(cpca_mode mode, int64_t rho_r, int64_t rho_c,
                               const int32_t* om_c, int64_t n, const cpca_csr* Lc, int32_t k,
                               const int32_t* init, int32_t km_max_iter, double tol,
                               int32_t max_iter) {
  cpca_status st;
  if ((st = check_mode(mode))) return st;
  if ((st = check_dims("Xtil", rho_r, rho_c))) return st;
  if (n < 1 || n > INT32_MAX) return fail(CPCA_EINVAL, "cluster_decode: n out of range");
  if (rho_c > n) return fail(CPCA_EINVAL, "cluster_decode: more samples than columns");
  if ((unsigned long long)rho_r * (unsigned long long)rho_c > (1ull << 34))
    return fail(CPCA_EINVAL, "cluster_decode: Xtil too large");
  if (!om_c) return fail(CPCA_EINVAL, "cluster_decode: null index set");
  if ((st = check_csr_shape("Lc", Lc, n))) return st;
  if (k < 1 || k > 64 || k > rho_c)
    return fail(CPCA_EINVAL, "cluster_decode: k must be in [1, 64] and <= rho_c");
  if (!init) return fail(CPCA_EINVAL, "cluster_decode: null init");
  if (km_max_iter < 0) return fail(CPCA_EINVAL, "cluster_decode: kmeans_max_iter < 0");
  if (!std::isfinite(tol) || !(tol > 0)) return fail(CPCA_EINVAL, "cluster_decode: tol must be > 0");
  if (max_iter < 0) return fail(CPCA_EINVAL, "cluster_decode: max_iter < 0");
  return CPCA_OK;
}

}  // namespace cpca

extern "C" cpca_status cpca_check_csr_host(int64_t n, int64_t nnz, const int32_t* rowptr,
                                           const int32_t* colind, const double* vals) {
  cpca::clear_error();
  return cpca::check_csr_host("csr", n, nnz, rowptr, colind, vals);
}

extern "C" cpca_status cpca_check_index_set_host(int64_t count, int64_t dim, const int32_t* idx) {
  cpca::clear_error();
  if (dim < 1 || dim > INT32_MAX) return cpca::fail(CPCA_EINVAL, "index set: dimension out of range");
  return cpca::check_index_set_host("index set", count, dim, idx, nullptr);
}

extern "C" const char* cpca_last_error(void) { return cpca::last_error(); }

extern "C" const char* cpca_version(void) { return "0.1.0"; }
