// Host replay of the row-panel kernel's use of its tables (test helper).
//
// Reads a CSR matrix L (binary: int64 n, int64 nnz, int32 rp[n + 1],
// int32 ci[nnz], double v[nnz]), a row mask (uint8 m[n]) and a vector x
// (double x[n]); builds the panel tables with the library's own builder for
// a union bound umax given on the command line; then walks the panels as the
// kernel does: per group of G = panel_group(npan) panels the LDS slots start
// as NaN, each panel first stages the rows its table names into their slots,
// then computes y[row] = diag x[row] + sum of its entries over the staged
// slots. Writes y (double[n]) to the output file and prints one line of
// statistics. Exits non-zero, naming the check, when a table is malformed:
// a row's own slot not holding the row, an offset outside the slots or not
// a slot boundary, a row computed twice or never, a panel above kPanelRows
// rows, a group count below a row's count.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <vector>

#include "panels.hpp"

using namespace cpca;

static void fail(const char* what, long a, long b) {
  std::fprintf(stderr, "panel table check failed: %s (%ld, %ld)\n", what, a, b);
  std::exit(2);
}

int main(int argc, char** argv) {
  if (argc != 4) {
    std::fprintf(stderr, "usage: panel_sim <input> <output> <umax>\n");
    return 1;
  }
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 1;
  HostCsr L;
  bool ok = std::fread(&L.n, 8, 1, f) == 1 && std::fread(&L.nnz, 8, 1, f) == 1;
  if (!ok) return 1;
  L.rp.resize((size_t)L.n + 1);
  L.ci.resize((size_t)L.nnz);
  L.v.resize((size_t)L.nnz);
  std::vector<uint8_t> mr((size_t)L.n);
  std::vector<double> x((size_t)L.n);
  ok = std::fread(L.rp.data(), 4, L.rp.size(), f) == L.rp.size() &&
       std::fread(L.ci.data(), 4, L.ci.size(), f) == L.ci.size() &&
       std::fread(L.v.data(), 8, L.v.size(), f) == L.v.size() &&
       std::fread(mr.data(), 1, mr.size(), f) == mr.size() &&
       std::fread(x.data(), 8, x.size(), f) == x.size();
  std::fclose(f);
  if (!ok) return 1;
  const int umax = std::atoi(argv[3]);
  HostPanels P;
  if (!build_panels(L, mr, kPanelRows, umax, P)) {
    std::printf("no_tables\n");
    return 0;
  }
  const int n = (int)L.n, G = panel_group(P.npan);
  if (P.G != G) fail("group size", P.G, G);
  if ((int)P.u_off.size() != P.npan + 1 || (int)P.r_off.size() != P.npan + 1) fail("offsets", 0, 0);
  std::vector<double> y((size_t)n, 0.0);
  std::vector<int> seen((size_t)n, 0);
  const double qnan = std::numeric_limits<double>::quiet_NaN();
  std::vector<double> lds((size_t)umax);
  int64_t staged = 0;
  int max_rows = 0;
  for (int k = 0; k < P.npan; ++k) {
    if (k % G == 0) std::fill(lds.begin(), lds.end(), qnan);
    const int u0 = P.u_off[(size_t)k], u1 = P.u_off[(size_t)k + 1];
    if (u1 - u0 != umax || u0 != k * umax) fail("staging table stride", k, u1 - u0);
    for (int s = 0; s < umax; ++s) {
      const int w = P.u[(size_t)(u0 + s)];
      if (w < -1 || w >= n) fail("staged row", k, w);
      if (w >= 0) {
        lds[(size_t)s] = x[(size_t)w];
        ++staged;
      }
    }
    const int r0 = P.r_off[(size_t)k], r1 = P.r_off[(size_t)k + 1];
    if (r1 <= r0 || r1 - r0 > kPanelRows) fail("panel rows", k, r1 - r0);
    max_rows = std::max(max_rows, r1 - r0);
    for (int j = r0; j < r1; ++j) {
      const int* m4 = &P.meta[(size_t)4 * j];
      const int row = m4[0], own = m4[1] & 0xffff, cnt = m4[1] >> 16;
      if (row != P.rows[(size_t)j] || row < 0 || row >= n) fail("meta row", j, row);
      if (seen[(size_t)row]++) fail("row computed twice", row, k);
      if (own >= umax) fail("own slot", row, own);
      // the row's own value must be resident (bitwise: it was copied)
      if (!(lds[(size_t)own] == x[(size_t)row]) && !(std::isnan(x[(size_t)row])))
        fail("own slot does not hold the row", row, own);
      if (m4[2] != (int)mr[(size_t)row]) fail("row mask", row, m4[2]);
      if (cnt > kPanelK || m4[3] < cnt || m4[3] > kPanelK) fail("entry counts", row, cnt);
      double acc = P.diag[(size_t)j] * lds[(size_t)own];
      for (int e = 0; e < kPanelK; ++e) {
        const int off = P.eidx[(size_t)j * kPanelK + e];
        if (off % kPanelRowBytes || off / kPanelRowBytes >= umax) fail("entry offset", row, off);
        const double w = P.ew[(size_t)j * kPanelK + e];
        if (e >= cnt && (w != 0.0 || off != own * kPanelRowBytes)) fail("padding entry", row, e);
        // as in the kernel, padding entries are multiplied too (0 x a
        // resident value)
        acc += w * lds[(size_t)(off / kPanelRowBytes)];
      }
      y[(size_t)row] = acc;
    }
  }
  for (int i = 0; i < n; ++i)
    if (seen[(size_t)i] != 1) fail("row never computed", i, seen[(size_t)i]);
  if (staged != P.staged) fail("staged count", (long)staged, (long)P.staged);
  f = std::fopen(argv[2], "wb");
  if (!f || std::fwrite(y.data(), 8, y.size(), f) != y.size()) return 1;
  std::fclose(f);
  std::printf("npan %d G %d staged %lld max_rows %d\n", P.npan, G, (long long)staged, max_rows);
  return 0;
}
