// Host-side argument checks (no HIP dependency).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "cpca.h"

namespace cpca {

cpca_status fail(cpca_status st, const std::string& msg);
void clear_error();
const char* last_error();

cpca_status check_csr_host(const char* name, int64_t n, int64_t nnz, const int32_t* rowptr,
                           const int32_t* colind, const double* vals);
cpca_status check_index_set_host(const char* name, int64_t count, int64_t dim,
                                 const int32_t* idx, std::vector<uint8_t>* mask_out);
cpca_status check_gamma(const char* name, double g);
cpca_status check_mode(cpca_mode mode);
cpca_status check_dims(const char* what, int64_t rows, int64_t cols);
cpca_status check_csr_shape(const char* name, const cpca_csr* A, int64_t order);
cpca_status check_frpcag_args(cpca_mode mode, const void* Ytil, int64_t rho_r, int64_t rho_c,
                              const cpca_csr* Lr, const cpca_csr* Lc, double gr, double gc,
                              double lmax_r, double lmax_c, int32_t max_iter, double eps,
                              const void* out);
cpca_status check_decode_args(cpca_mode mode, int64_t rho_r, int64_t rho_c,
                              const int32_t* om_r, const int32_t* om_c, int64_t p, int64_t n,
                              const cpca_csr* Lr, const cpca_csr* Lc, double gr, double gc,
                              double tol, int32_t max_iter);
cpca_status check_approx_args(cpca_mode mode, int64_t rho_r, int64_t rho_c,
                              const int32_t* om_r, const int32_t* om_c, int64_t p, int64_t n,
                              const cpca_csr* Lr, const cpca_csr* Lc, double delta,
                              double ratio, int32_t k_max, double tol, int32_t max_iter);
cpca_status check_cluster_args(cpca_mode mode, int64_t rho_r, int64_t rho_c,
                               const int32_t* om_c, int64_t n, const cpca_csr* Lc, int32_t k,
                               const int32_t* init, int32_t km_max_iter, double tol,
                               int32_t max_iter);

}  // namespace cpca
