// Host-side fuzz driver for the library's argument checks (test helper,
// built with the address and undefined-behaviour sanitizers by
// tests/test_host_sanitizers.py). It feeds check_csr_host and
// check_index_set_host valid inputs and inputs broken in one place each
// (row pointers out of order or out of range, column indices out of range,
// non-finite values, repeated or out-of-range indices) and checks the
// verdicts; the sanitizers catch any out-of-bounds access or undefined
// arithmetic on the way. Prints "ok <cases>" on success.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "validate.hpp"

using namespace cpca;

static int g_cases = 0;

static void expect(bool cond, const char* what, int seed) {
  ++g_cases;
  if (!cond) {
    std::fprintf(stderr, "check verdict wrong: %s (seed %d): %s\n", what, seed, last_error());
    std::exit(2);
  }
}

int main() {
  for (int seed = 0; seed < 400; ++seed) {
    std::mt19937 rng(seed);
    const int n = 1 + (int)(rng() % 60);
    std::vector<int32_t> rp(n + 1, 0), ci;
    std::vector<double> v;
    for (int i = 0; i < n; ++i) {
      const int deg = (int)(rng() % 6);
      for (int e = 0; e < deg; ++e) {
        ci.push_back((int32_t)(rng() % n));
        v.push_back(std::ldexp((double)(rng() % 1000) - 500.0, -7));
      }
      rp[i + 1] = (int32_t)ci.size();
    }
    const int64_t nnz = (int64_t)ci.size();
    expect(check_csr_host("L", n, nnz, rp.data(), ci.data(), v.data()) == CPCA_OK, "valid csr", seed);
    if (nnz > 0) {
      const size_t k = rng() % (size_t)nnz;
      std::vector<int32_t> c2 = ci;
      c2[k] = (seed & 1) ? n : -1;
      expect(check_csr_host("L", n, nnz, rp.data(), c2.data(), v.data()) == CPCA_EINVAL,
             "column index out of range", seed);
      std::vector<double> v2 = v;
      v2[k] = (seed & 2) ? std::numeric_limits<double>::quiet_NaN()
                         : std::numeric_limits<double>::infinity();
      expect(check_csr_host("L", n, nnz, rp.data(), ci.data(), v2.data()) == CPCA_EINVAL,
             "non-finite value", seed);
    }
    if (n > 1 && rp[n] > 0) {
      std::vector<int32_t> r2 = rp;
      const int i = 1 + (int)(rng() % (n - 1));
      r2[i] = rp[n] + 1 + (int32_t)(rng() % 3);       // beyond nnz, and out of order
      expect(check_csr_host("L", n, nnz, r2.data(), ci.data(), v.data()) == CPCA_EINVAL,
             "row pointer out of order", seed);
    }
    {
      std::vector<int32_t> r3 = rp;
      r3[0] = 1;
      expect(check_csr_host("L", n, nnz, r3.data(), ci.data(), v.data()) == CPCA_EINVAL,
             "rowptr[0] != 0", seed);
    }
    // index sets
    const int dim = n;
    const int cnt = (int)(rng() % (dim + 1));
    std::vector<int32_t> perm(dim);
    for (int i = 0; i < dim; ++i) perm[i] = i;
    std::shuffle(perm.begin(), perm.end(), rng);
    std::vector<int32_t> idx(perm.begin(), perm.begin() + cnt);
    std::vector<uint8_t> mask;
    expect(check_index_set_host("omega", cnt, dim, idx.data(), &mask) == CPCA_OK, "valid index set", seed);
    int on = 0;
    for (uint8_t m : mask) on += m;
    expect(on == cnt && (int)mask.size() == dim, "mask of a valid index set", seed);
    if (cnt >= 2) {
      std::vector<int32_t> d2 = idx;
      d2[cnt - 1] = d2[0];
      expect(check_index_set_host("omega", cnt, dim, d2.data(), &mask) == CPCA_EINVAL,
             "repeated index", seed);
    }
    if (cnt >= 1) {
      std::vector<int32_t> d3 = idx;
      d3[rng() % cnt] = (seed & 1) ? dim : -3;
      expect(check_index_set_host("omega", cnt, dim, d3.data(), nullptr) == CPCA_EINVAL,
             "index out of range", seed);
    }
  }
  std::printf("ok %d\n", g_cases);
  return 0;
}
