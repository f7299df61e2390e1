// Host-side internals shared by the single-problem drivers (engine.hip) and
// the batched driver (batched.hip): the handle, workspace, profiling, graph
// preparation (validation + device layouts) and launch helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "cpca.h"
#include "kernels.hpp"
#include "validate.hpp"

using namespace cpca;

namespace {

// apply: the CG operator application; other: residual / objective / dot launches
enum Family {
  FAM_APPLY = 0, FAM_UPDATE = 1, FAM_FISTA = 2, FAM_OTHER = 3, FAM_RANKK = 4, FAM_PUPDATE = 5,
  FAM_COARSE = 6, FAM_COUNT = 7
};

}  // namespace

namespace cpca {

// A named roctx range for the lifetime of the object: every entry point and
// its host-side phases show up as ranges in a rocprofv3 --marker-trace
// timeline (without a tool attached the calls return at once).
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace cpca

struct cpca_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;          // workspace (device)
  size_t ws_cap = 0;
  char* fixed = nullptr;       // counters + scalars (device), zeroed at creation
  void* pinned = nullptr;      // host mirror of the scalars
  int force_R = 0;             // launch-shape override (0: default, -1: autotune)
  int force_lds = -1;          // LDS override (-1: default)
  int force_band = -1;         // band path override (0: off, -1: automatic)
  int force_kernel = -1;       // banded-L_c kernel preference (-1 auto, 0 rows, 1 strip, 2 panel)
  bool debug = false;          // per-segment trace on stderr (CPCA_DEBUG=1)
  bool ir_restart = false;     // FP32_IR as restarted refinement only (CPCA_IR_MODE=restart)
  bool batch_compact = true;   // batched CG: shrink the block tables in the tail (CPCA_BATCH_COMPACT=0 off)
  std::vector<std::pair<std::string, std::pair<int, int>>> tuned;  // autotuner cache
  bool prof = false;
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  std::vector<int> ev_fam;
  std::vector<int> ev_cnt;     // launches covered by each event pair
  size_t ev_used = 0;
  bool prof_hold = false;      // per-launch events off (while a graph is captured)
  int64_t prof_n[FAM_COUNT] = {};
  double prof_ms[FAM_COUNT] = {};
  // staged operator image of the last decode on this handle, kept in its own
  // device buffer and reused while the operator's content key is unchanged
  struct DecodeCache* dcache = nullptr;
  bool dcache_on = true;       // CPCA_IMAGE_CACHE=0 turns the reuse off
};

namespace {

// Layout of the `fixed` device block.
constexpr size_t kOffCg = 256;             // CgScal[2]
constexpr size_t kOffFista = 512;          // FistaScal
static_assert(kOffCg + 2 * sizeof(CgScal) <= kOffFista, "CG scalar blocks overlap");
constexpr size_t kOffResults = 768;        // double[32]
constexpr size_t kFixedBytes = 1024;

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess) {                                                       \
      return fail(_e == hipErrorOutOfMemory ? CPCA_ENOMEM : CPCA_EHIP,            \
                  std::string(#expr) + ": " + hipGetErrorString(_e));             \
    }                                                                             \
  } while (0)

#define STCHK(expr)                   \
  do {                                \
    cpca_status _s = (expr);          \
    if (_s != CPCA_OK) return _s;     \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Two-pass bump allocator: the first pass (base == nullptr) only measures.
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

cpca_status ensure_ws(cpca_handle h, size_t bytes) {
  if (bytes <= h->ws_cap) return CPCA_OK;
  HIPCHK(hipStreamSynchronize(h->stream));
  if (h->ws) HIPCHK(hipFree(h->ws));
  h->ws = nullptr;
  h->ws_cap = 0;
  const size_t cap = align_up(bytes + bytes / 8, 1 << 20);
  HIPCHK(hipMalloc(&h->ws, cap));
  h->ws_cap = cap;
  return CPCA_OK;
}

CgScal* cg_ptr(cpca_handle h, int k = 0) { return reinterpret_cast<CgScal*>(h->fixed + kOffCg) + k; }
FistaScal* fista_ptr(cpca_handle h) { return reinterpret_cast<FistaScal*>(h->fixed + kOffFista); }
double* results_ptr(cpca_handle h) { return reinterpret_cast<double*>(h->fixed + kOffResults); }

// Copy the fixed scalar block to the pinned mirror and wait.
cpca_status read_fixed(cpca_handle h) {
  HIPCHK(hipMemcpyAsync(h->pinned, h->fixed, kFixedBytes, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return CPCA_OK;
}
const CgScal& host_cg(cpca_handle h, int k = 0) {
  return reinterpret_cast<const CgScal*>(static_cast<char*>(h->pinned) + kOffCg)[k];
}
const FistaScal& host_fista(cpca_handle h) {
  return *reinterpret_cast<const FistaScal*>(static_cast<char*>(h->pinned) + kOffFista);
}
const double* host_results(cpca_handle h) {
  return reinterpret_cast<const double*>(static_cast<char*>(h->pinned) + kOffResults);
}

// ---------------------------------------------------------------- profiling
// A timed span on `stream` that covers `count` launches of family `fam`
// (one launch, or a replayed graph of several).
cpca_status prof_span_begin(cpca_handle h, int fam, hipStream_t stream) {
  if (!h->prof) return CPCA_OK;
  if (2 * h->ev_used + 2 > h->ev.size()) {
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    h->ev.push_back(a);
    h->ev.push_back(b);
    h->ev_fam.push_back(fam);
    h->ev_cnt.push_back(1);
  }
  h->ev_fam[h->ev_used] = fam;
  HIPCHK(hipEventRecord(h->ev[2 * h->ev_used], stream));
  return CPCA_OK;
}
cpca_status prof_span_end(cpca_handle h, hipStream_t stream, int count) {
  if (!h->prof) return CPCA_OK;
  HIPCHK(hipEventRecord(h->ev[2 * h->ev_used + 1], stream));
  h->ev_cnt[h->ev_used] = count;
  ++h->ev_used;
  return CPCA_OK;
}
cpca_status prof_begin(cpca_handle h, int fam) {
  if (h->prof_hold) return CPCA_OK;
  return prof_span_begin(h, fam, h->stream);
}
cpca_status prof_end(cpca_handle h) {
  if (h->prof_hold) return CPCA_OK;
  return prof_span_end(h, h->stream, 1);
}
// Only after the stream has been synchronised.
cpca_status prof_collect(cpca_handle h) {
  if (!h->prof) return CPCA_OK;
  for (size_t k = 0; k < h->ev_used; ++k) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev[2 * k], h->ev[2 * k + 1]));
    h->prof_n[h->ev_fam[k]] += h->ev_cnt[k];
    h->prof_ms[h->ev_fam[k]] += ms;
  }
  h->ev_used = 0;
  return CPCA_OK;
}
cpca_status sync_collect(cpca_handle h) {
  HIPCHK(hipStreamSynchronize(h->stream));
  return prof_collect(h);
}

// ------------------------------------------------------------- preparation

cpca_status fetch_csr(const char* name, const cpca_csr* A, HostCsr& out) {
  out.n = A->n;
  out.nnz = A->nnz;
  out.rp.resize((size_t)A->n + 1);
  out.ci.resize((size_t)std::max<int64_t>(A->nnz, 1));
  out.v.resize((size_t)std::max<int64_t>(A->nnz, 1));
  HIPCHK(hipMemcpy(out.rp.data(), A->rowptr, sizeof(int32_t) * (A->n + 1), hipMemcpyDefault));
  if (A->nnz > 0) {
    HIPCHK(hipMemcpy(out.ci.data(), A->colind, sizeof(int32_t) * A->nnz, hipMemcpyDefault));
    HIPCHK(hipMemcpy(out.v.data(), A->vals, sizeof(double) * A->nnz, hipMemcpyDefault));
  }
  return check_csr_host(name, out.n, out.nnz, out.rp.data(), out.ci.data(), out.v.data());
}

cpca_status fetch_index_set(const char* name, const int32_t* idx, int64_t count, int64_t dim,
                            std::vector<uint8_t>& mask) {
  std::vector<int32_t> h((size_t)std::max<int64_t>(count, 1));
  if (count > 0) HIPCHK(hipMemcpy(h.data(), idx, sizeof(int32_t) * count, hipMemcpyDefault));
  return check_index_set_host(name, count, dim, h.data(), &mask);
}

// Device image of one operator (L_r CSR, L_c SELL, masks) in type T, packed
// into a single host staging buffer and copied with one transfer.
template <typename T>
struct DevGraph {
  CsrDev<T> Lr{};
  SellDev<T> Lc{};
  BandDev<T> Lb{};
  PanelDev<T> Lp{};
  const uint8_t* mr = nullptr;
  const uint8_t* mc = nullptr;
};

struct Staging {
  std::vector<char> buf;
  size_t add(const void* src, size_t bytes) {
    const size_t off = align_up(buf.size(), 256);
    buf.resize(off + bytes);
    if (bytes) std::memcpy(buf.data() + off, src, bytes);
    return off;
  }
};

template <typename T>
struct GraphImage {
  size_t o_rp, o_ci, o_v, o_sp, o_sci, o_sv, o_mr, o_mc, o_bv;
  int ldb;                      // band row stride (0: no band)
  unsigned long long nonempty;  // band diagonals holding an entry
  int npan;                     // panels of L_r rows (0: no panel tables)
  size_t o_pu_off, o_pu, o_pr_off, o_prows, o_peidx, o_pew, o_pmeta, o_pdiag;
};

// Half-bandwidth of the diagonal (band) part of L_c: the smallest of 6, 8
// and 16 that holds at least 90% of the entries, else 0 (sliced ELL only).
inline int choose_band(const HostCsr& Lc) {
  if (Lc.nnz == 0) return 0;
  int64_t in6 = 0, in8 = 0, in16 = 0;
  for (int64_t j = 0; j < Lc.n; ++j)
    for (int32_t e = Lc.rp[j]; e < Lc.rp[j + 1]; ++e) {
      const int64_t d = std::llabs((int64_t)Lc.ci[e] - j);
      in6 += d <= 6;
      in8 += d <= 8;
      in16 += d <= 16;
    }
  if (in6 * 10 >= Lc.nnz * 9) return 6;
  if (in8 * 10 >= Lc.nnz * 9) return 8;
  if (in16 * 10 >= Lc.nnz * 9) return 16;
  return 0;
}

// Stages the device image of one operator: CSR of L_r in T, L_c as band
// diagonals (|k - j| <= BW, when BW > 0) plus a sliced ELL of the remaining
// entries with slice height H, and the 0/1 masks.
template <typename T>
GraphImage<T> stage_graph(Staging& st, const HostCsr& Lr, const HostCsr& Lc,
                          const std::vector<uint8_t>& mr, const std::vector<uint8_t>& mc, int H,
                          int BW = 0, bool panels = false) {
  GraphImage<T> g{};
  g.npan = 0;
  if (BW > 0 && panels) {
    HostPanels hp;
    if (build_panels(Lr, mr, kPanelRows, PanelUnion<T>::value, hp) && hp.npan > 0) {
      g.npan = hp.npan;
      g.o_pu_off = st.add(hp.u_off.data(), sizeof(int32_t) * hp.u_off.size());
      g.o_pu = st.add(hp.u.data(), sizeof(int32_t) * hp.u.size());
      g.o_pr_off = st.add(hp.r_off.data(), sizeof(int32_t) * hp.r_off.size());
      g.o_prows = st.add(hp.rows.data(), sizeof(int32_t) * hp.rows.size());
      g.o_peidx = st.add(hp.eidx.data(), sizeof(uint16_t) * hp.eidx.size());
      std::vector<T> ew(hp.ew.begin(), hp.ew.end()), dg(hp.diag.begin(), hp.diag.end());
      g.o_pew = st.add(ew.data(), sizeof(T) * ew.size());
      g.o_pmeta = st.add(hp.meta.data(), sizeof(int32_t) * hp.meta.size());
      g.o_pdiag = st.add(dg.data(), sizeof(T) * dg.size());
    }
  }
  std::vector<T> vr(Lr.v.begin(), Lr.v.begin() + Lr.nnz);
  g.o_rp = st.add(Lr.rp.data(), sizeof(int32_t) * Lr.rp.size());
  g.o_ci = st.add(Lr.ci.data(), sizeof(int32_t) * std::max<int64_t>(Lr.nnz, 1));
  g.o_v = st.add(vr.data(), sizeof(T) * vr.size());
  const int64_t n = Lc.n;
  auto in_band = [&](int64_t j, int32_t k) { return BW > 0 && std::llabs((int64_t)k - j) <= BW; };
  // band diagonals
  g.ldb = 0;
  g.nonempty = 0;
  if (BW > 0) {
    const int vec = H / kWave;
    g.ldb = (int)((n + vec - 1) / vec * vec);
    std::vector<T> bv((size_t)(2 * BW + 1) * g.ldb, T(0));
    for (int64_t j = 0; j < n; ++j)
      for (int32_t e = Lc.rp[j]; e < Lc.rp[j + 1]; ++e)
        if (in_band(j, Lc.ci[e])) {
          const int d = (int)((int64_t)Lc.ci[e] - j);
          bv[(size_t)(d + BW) * g.ldb + j] += (T)Lc.v[e];
          g.nonempty |= 1ull << (d + BW);
        }
    g.o_bv = st.add(bv.data(), sizeof(T) * bv.size());
  }
  // sliced ELL of the remaining entries, slice height H
  const int64_t ns = (n + H - 1) / H;
  std::vector<int32_t> sp((size_t)ns + 1, 0);
  std::vector<int32_t> deg((size_t)n, 0);
  for (int64_t j = 0; j < n; ++j)
    for (int32_t e = Lc.rp[j]; e < Lc.rp[j + 1]; ++e) deg[(size_t)j] += !in_band(j, Lc.ci[e]);
  for (int64_t s = 0; s < ns; ++s) {
    int w = 0;
    for (int64_t j = s * H; j < std::min<int64_t>(n, (s + 1) * H); ++j) w = std::max(w, deg[(size_t)j]);
    sp[s + 1] = sp[s] + w * H;
  }
  std::vector<int32_t> sci((size_t)std::max(sp[ns], 1), 0);
  std::vector<T> sv((size_t)std::max(sp[ns], 1), T(0));
  for (int64_t s = 0; s < ns; ++s) {
    const int w = (sp[s + 1] - sp[s]) / H;
    for (int lane = 0; lane < H; ++lane) {
      const int64_t j = s * H + lane;
      int e_out = 0;
      if (j < n) {
        for (int32_t e = Lc.rp[j]; e < Lc.rp[j + 1]; ++e) {
          if (in_band(j, Lc.ci[e])) continue;
          const size_t pos = (size_t)sp[s] + (size_t)e_out * H + lane;
          sci[pos] = Lc.ci[e];
          sv[pos] = (T)Lc.v[e];
          ++e_out;
        }
      }
      for (; e_out < w; ++e_out) {
        const size_t pos = (size_t)sp[s] + (size_t)e_out * H + lane;
        sci[pos] = j < n ? (int32_t)j : 0;
        sv[pos] = T(0);
      }
    }
  }
  g.o_sp = st.add(sp.data(), sizeof(int32_t) * sp.size());
  g.o_sci = st.add(sci.data(), sizeof(int32_t) * sci.size());
  g.o_sv = st.add(sv.data(), sizeof(T) * sv.size());
  g.o_mr = st.add(mr.data(), mr.size());
  g.o_mc = st.add(mc.data(), mc.size());
  return g;
}

template <typename T>
DevGraph<T> bind_graph(const GraphImage<T>& g, const char* dev) {
  DevGraph<T> d;
  d.Lr.rp = reinterpret_cast<const int*>(dev + g.o_rp);
  d.Lr.ci = reinterpret_cast<const int*>(dev + g.o_ci);
  d.Lr.v = reinterpret_cast<const T*>(dev + g.o_v);
  d.Lc.sp = reinterpret_cast<const int*>(dev + g.o_sp);
  d.Lc.ci = reinterpret_cast<const int*>(dev + g.o_sci);
  d.Lc.v = reinterpret_cast<const T*>(dev + g.o_sv);
  d.mr = reinterpret_cast<const uint8_t*>(dev + g.o_mr);
  d.mc = reinterpret_cast<const uint8_t*>(dev + g.o_mc);
  d.Lb.v = g.ldb ? reinterpret_cast<const T*>(dev + g.o_bv) : nullptr;
  d.Lb.ldb = g.ldb;
  d.Lb.nonempty = g.nonempty;
  d.Lp.npan = g.npan;
  if (g.npan > 0) {
    d.Lp.u_off = reinterpret_cast<const int*>(dev + g.o_pu_off);
    d.Lp.u = reinterpret_cast<const int*>(dev + g.o_pu);
    d.Lp.r_off = reinterpret_cast<const int*>(dev + g.o_pr_off);
    d.Lp.rows = reinterpret_cast<const int*>(dev + g.o_prows);
    d.Lp.eidx = reinterpret_cast<const uint16_t*>(dev + g.o_peidx);
    d.Lp.ew = reinterpret_cast<const T*>(dev + g.o_pew);
    d.Lp.meta = reinterpret_cast<const int4*>(dev + g.o_pmeta);
    d.Lp.diag = reinterpret_cast<const T*>(dev + g.o_pdiag);
  }
  return d;
}

// ------------------------------------------------------------------ launch
struct ApplyCfg {
  int R = 1;
  bool lds = true;
  int vec = 1;  // columns per thread (16-byte accesses when > 1)
  int bw = 0;   // band half-width of L_c (0: sliced ELL only)
  bool strip = false;  // column-strip kernel (needs bw > 0 and full vectors)
  bool panel = false;  // row-panel gather kernel (needs bw > 0, full vectors, panel tables)
  bool plo = false;    // ... in its variant without cross-panel prefetch (three waves per SIMD)
  int npan = 0;        // panels in the staged image
};


constexpr int kStripRows = 16;  // rows per workgroup of the column-strip kernel

inline size_t lds_bytes(const ApplyCfg& c, int64_t ld, size_t elem) {
  const int pad = c.bw == 0 ? 0 : (c.bw + c.vec - 1) / c.vec * c.vec;
  return (size_t)c.R * (size_t)(ld + 2 * pad) * elem;
}

// Launch shape of the fused product for a p x n operand of `elem` bytes.
// Default: one row per workgroup staged in LDS (the fastest shape measured
// for banded and K-NN graphs); two rows through the L1 when a row does not
// fit in 64 KiB of LDS. `band` is the candidate band half-width of L_c
// (choose_band); it is used when the rows are staged in LDS with full
// 16-byte vectors.
ApplyCfg choose_cfg(cpca_handle h, int64_t p, int64_t n, size_t elem, int band = 0,
                    bool allow_panel = false) {
  ApplyCfg c;
  const int W = (int)(16 / elem);
  c.vec = (n % W == 0) ? W : 1;
  const size_t row_bytes = (size_t)n * elem;
  c.R = 1;
  c.lds = row_bytes <= 65536;
  if (!c.lds && p >= 4096) c.R = 2;
  if (h->force_R > 0) c.R = h->force_R;
  if (h->force_lds == 1) c.lds = (size_t)c.R * row_bytes <= 65536;
  if (h->force_lds == 0) c.lds = false;
  if (h->force_lds == -1 && h->force_R > 0) c.lds = (size_t)c.R * row_bytes <= 65536;
  c.bw = 0;
  c.strip = false;
  if (band > 0 && c.vec == W && h->force_band != 0) {
    if (h->force_R <= 0 && h->force_lds != 0 && h->force_kernel != 0) {
      // banded L_c: column strips with the diagonals held in registers, or
      // (preferred where panel tables exist) the row-panel gather kernel.
      // A 6-wide band is run by the 8-wide FP32 kernels (their two outer
      // diagonals are then empty): on the video-shaped workload they measured
      // 0.370 against 0.388 ms, both at two waves per SIMD; in FP64 the
      // 6-wide kernels keep two waves per SIMD where the 8-wide ones fit one.
      c.bw = (elem == 4 && band == 6) ? 8 : band;
      c.strip = h->force_band != 2;
      if (c.strip && allow_panel && h->force_kernel != 1) {
        c.panel = true;
        // bands up to 8 wide: the variant without cross-panel prefetch
        // (three waves per SIMD; 0.333 against 0.372 ms on the video-shaped
        // workload in FP32) unless the prefetching kernel is asked for
        c.plo = h->force_kernel != 2 && c.bw <= 8;
        c.strip = false;
      }
    }
    if (!c.strip && !c.panel && c.lds && c.R <= 4) {
      ApplyCfg t = c;
      t.bw = band;
      c.bw = lds_bytes(t, n, elem) <= 65536 ? band : 0;
    }
  }
  return c;
}

int slice_height(const ApplyCfg& c) { return kWave * c.vec; }

// Records the staged panel count; a panel shape without panel tables (a row
// of L_r too long for the table) falls back to the column-strip kernel.
inline void set_panels(ApplyCfg& c, int npan) {
  c.npan = npan;
  if (c.panel && npan == 0) {
    c.panel = false;
    c.plo = false;
    c.strip = true;
  }
}

// Workgroups of the panel kernel for npan panels of a p x n operand with
// `vec` elements per 16 bytes.
inline int panel_grid(int npan, int n, int vec) {
  const int w = kPanelLanes * vec;
  const int nstrips = (n + w - 1) / w;
  const int G = panel_group(npan);
  const int ngroups = (npan + G - 1) / G;
  return 8 * ((ngroups + 7) / 8) * nstrips;
}

int vec_grid(size_t N) {
  const size_t b = (N + kThreads - 1) / kThreads;
  return (int)std::max<size_t>(1, std::min<size_t>(b, 2048));
}

// Largest workgroup count any launch shape can use for a p x n operand
// (sizes the partial-sum buffers before the shape is known).
int max_apply_grid(int p, int n) {
  const int nchunks = (p + kStripRows - 1) / kStripRows;
  const int nstrips = (n + kStripThreads - 1) / kStripThreads;
  return std::max(8 * ((p + 7) / 8), 8 * ((nchunks + 7) / 8) * nstrips);
}

// Workgroups of one fused-product launch (= partial sums written).
int apply_grid(const ApplyCfg& cfg, int p, int n = 0) {
  if (cfg.panel) return panel_grid(cfg.npan, n, cfg.vec);
  if (cfg.strip) {
    const int cw = kStripThreads * cfg.vec;
    const int nstrips = (n + cw - 1) / cw;
    const int nchunks = (p + kStripRows - 1) / kStripRows;
    return 8 * ((nchunks + 7) / 8) * nstrips;
  }
  const int nrb = (p + cfg.R - 1) / cfg.R;
  return 8 * ((nrb + 7) / 8);
}

template <typename T, int R, bool LDS, int VEC, int BW, class Epi>
hipError_t launch_apply_t(cpca_handle h, const T* X, int p, int n, const DevGraph<T>& g,
                          const Epi& epi) {
  const int nrb = (p + R - 1) / R;
  const int per = (nrb + 7) / 8;
  constexpr int PAD = band_pad<BW, VEC>();
  const size_t shmem = LDS ? (size_t)R * (n + 2 * PAD) * sizeof(T) : 0;
  k_apply2<T, R, LDS, VEC, BW, Epi><<<dim3(8 * per), dim3(kThreads), shmem, h->stream>>>(
      X, p, n, g.Lr, g.Lc, g.Lb, g.mr, g.mc, nrb, per, epi);
  return hipGetLastError();
}

template <typename T, int BW, class Epi>
hipError_t launch_strip_t(cpca_handle h, const T* X, int p, int n, const DevGraph<T>& g,
                          const Epi& epi) {
  constexpr int W = (int)(16 / sizeof(T));
  const int cw = kStripThreads * W;
  const int nstrips = (n + cw - 1) / cw;
  const int nchunks = (p + kStripRows - 1) / kStripRows;
  const int cpx = (nchunks + 7) / 8;
  k_apply_strip<T, W, BW, kStripRows, Epi><<<dim3(8 * cpx * nstrips), dim3(kStripThreads), 0,
                                              h->stream>>>(X, p, n, g.Lr, g.Lc, g.Lb, g.mr, g.mc,
                                                           nchunks, cpx, epi);
  return hipGetLastError();
}

template <typename T, int BW, bool LO, class Epi>
hipError_t launch_panel_t(cpca_handle h, const T* X, int p, int n, const DevGraph<T>& g,
                          const Epi& epi) {
  if (g.Lp.npan <= 0) return hipErrorInvalidValue;
  constexpr int W = kPanelLanes * (int)(16 / sizeof(T));
  const int nstrips = (n + W - 1) / W;
  const int G = panel_group(g.Lp.npan);
  const int ngroups = (g.Lp.npan + G - 1) / G;
  const int gpx = (ngroups + 7) / 8;
  static_assert(8 <= kPanelGroupMax, "panel group");
  if constexpr (LO)
    k_apply_panel_lo<T, BW, Epi><<<dim3(8 * gpx * nstrips), dim3(kThreads), 0, h->stream>>>(
        X, p, n, g.Lp, g.Lc, g.Lb, g.mc, G, ngroups, gpx, epi);
  else
    k_apply_panel<T, BW, Epi><<<dim3(8 * gpx * nstrips), dim3(kThreads), 0, h->stream>>>(
        X, p, n, g.Lp, g.Lc, g.Lb, g.mc, G, ngroups, gpx, epi);
  return hipGetLastError();
}

template <typename T, int R, class Epi>
hipError_t launch_apply_r(cpca_handle h, const ApplyCfg& cfg, const T* X, int p, int n,
                          const DevGraph<T>& g, const Epi& epi) {
  constexpr int W = (int)(16 / sizeof(T));
  if (cfg.panel) {
    if (cfg.vec != W || g.Lp.npan != cfg.npan) return hipErrorInvalidValue;
    // the variant without prefetch exists for bands up to 8 wide (the
    // 16-wide band's registers alone exceed three waves per SIMD)
    if (cfg.plo && cfg.bw <= 8) {
      if (cfg.bw == 6) return launch_panel_t<T, 6, true>(h, X, p, n, g, epi);
      if (cfg.bw == 8) return launch_panel_t<T, 8, true>(h, X, p, n, g, epi);
      return hipErrorInvalidValue;
    }
    if (cfg.bw == 6) return launch_panel_t<T, 6, false>(h, X, p, n, g, epi);
    if (cfg.bw == 8) return launch_panel_t<T, 8, false>(h, X, p, n, g, epi);
    if (cfg.bw == 16) return launch_panel_t<T, 16, false>(h, X, p, n, g, epi);
    return hipErrorInvalidValue;
  }
  if (cfg.strip) {
    if (cfg.vec != W) return hipErrorInvalidValue;
    if (cfg.bw == 6) return launch_strip_t<T, 6>(h, X, p, n, g, epi);
    if (cfg.bw == 8) return launch_strip_t<T, 8>(h, X, p, n, g, epi);
    if (cfg.bw == 16) return launch_strip_t<T, 16>(h, X, p, n, g, epi);
    return hipErrorInvalidValue;
  }
  if constexpr (R <= 4) {
    if (cfg.bw == 6 && cfg.lds && cfg.vec == W) return launch_apply_t<T, R, true, W, 6>(h, X, p, n, g, epi);
    if (cfg.bw == 8 && cfg.lds && cfg.vec == W) return launch_apply_t<T, R, true, W, 8>(h, X, p, n, g, epi);
    if (cfg.bw == 16 && cfg.lds && cfg.vec == W) return launch_apply_t<T, R, true, W, 16>(h, X, p, n, g, epi);
  }
  if (cfg.bw != 0) return hipErrorInvalidValue;
  if (cfg.vec == W) {
    return cfg.lds ? launch_apply_t<T, R, true, W, 0>(h, X, p, n, g, epi)
                   : launch_apply_t<T, R, false, W, 0>(h, X, p, n, g, epi);
  }
  return cfg.lds ? launch_apply_t<T, R, true, 1, 0>(h, X, p, n, g, epi)
                 : launch_apply_t<T, R, false, 1, 0>(h, X, p, n, g, epi);
}

template <typename T, class Epi>
cpca_status launch_apply(cpca_handle h, const ApplyCfg& cfg, const T* X, int p, int n,
                         const DevGraph<T>& g, const Epi& epi, int fam) {
  STCHK(prof_begin(h, fam));
  hipError_t e;
  switch (cfg.R) {
    case 1: e = launch_apply_r<T, 1>(h, cfg, X, p, n, g, epi); break;
    case 2: e = launch_apply_r<T, 2>(h, cfg, X, p, n, g, epi); break;
    case 4: e = launch_apply_r<T, 4>(h, cfg, X, p, n, g, epi); break;
    case 8: e = launch_apply_r<T, 8>(h, cfg, X, p, n, g, epi); break;
    default: return fail(CPCA_EINVAL, "unsupported rows per workgroup");
  }
  if (e != hipSuccess) return fail(CPCA_EHIP, std::string("apply launch: ") + hipGetErrorString(e));
  return prof_end(h);
}

#define LAUNCHCHK()                                                                        \
  do {                                                                                     \
    hipError_t _e = hipGetLastError();                                                     \
    if (_e != hipSuccess) return fail(CPCA_EHIP, std::string("launch: ") + hipGetErrorString(_e)); \
  } while (0)


// ------------------------------------------------------------------ status
constexpr int kMaxOuter = 40;  // refinement steps per solve

cpca_status done_status(int done) {
  switch (done) {
    case 1: return CPCA_OK;
    case 2: return fail(CPCA_ENOTSPD, "CG breakdown: <p, A p> <= 0");
    case 3: return fail(CPCA_ENAN, "NaN or Inf in the iteration");
    default: return fail(CPCA_ENOCONV, "iteration limit reached before the tolerance");
  }
}

void fill_info(cpca_info* info, cpca_status st, int iters, int outer, double rel, double obj,
               std::chrono::steady_clock::time_point t0) {
  if (!info) return;
  info->iters = iters;
  info->outer_iters = outer;
  info->status = (int32_t)st;
  info->reserved = 0;
  info->rel_residual = rel;
  info->objective = obj;
  info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}


// --------------------------------------------------------------- autotuner
// Launch-shape autotuning of the fused product: each candidate (rows per
// workgroup, LDS staging) is timed over a few launches on the real operand
// and the fastest is kept in the handle, keyed by element type and shape.
// With CPCA_TUNE_CACHE set, choices are also appended to that file and read
// back when a handle is created.
inline std::string tune_key(const char* kind, size_t elem, int64_t p, int64_t n, int64_t nnz) {
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s:f%zu:p%lld:n%lld:z%lld", kind, elem * 8, (long long)p,
                (long long)n, (long long)nnz);
  return buf;
}

// Cached shape: rows per workgroup and a mode (0: no LDS, 1: LDS rows,
// 2: column strips, 3: row panels, 4: row panels without prefetch).
inline bool tune_lookup(cpca_handle h, const std::string& key, ApplyCfg& c) {
  for (const auto& kv : h->tuned)
    if (kv.first == key) {
      c.R = kv.second.first;
      c.lds = kv.second.second != 0;
      c.strip = kv.second.second == 2;
      c.panel = kv.second.second >= 3;
      c.plo = kv.second.second == 4;
      return true;
    }
  return false;
}

inline void tune_store(cpca_handle h, const std::string& key, const ApplyCfg& c) {
  const int mode = c.panel ? (c.plo ? 4 : 3) : (c.strip ? 2 : (c.lds ? 1 : 0));
  h->tuned.push_back({key, {c.R, mode}});
  if (const char* path = std::getenv("CPCA_TUNE_CACHE")) {
    if (FILE* f = std::fopen(path, "a")) {
      std::fprintf(f, "%s %d %d\n", key.c_str(), c.R, mode);
      std::fclose(f);
    }
  }
}

inline void tune_load_file(cpca_handle h) {
  const char* path = std::getenv("CPCA_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[200];
  int R, lds;
  while (std::fscanf(f, "%199s %d %d", key, &R, &lds) == 3) {
    if ((R == 1 || R == 2 || R == 4 || R == 8) && lds >= 0 && lds <= 4)
      h->tuned.push_back({key, {R, lds}});
  }
  std::fclose(f);
}

// Times `reps` calls of `launch(cfg)` for every candidate and returns the
// fastest. `launch` enqueues one kernel and returns a status.
template <class F>
cpca_status autotune(cpca_handle h, const std::string& key, int64_t ld, size_t elem, ApplyCfg base,
                     F launch, ApplyCfg* best) {
  if (tune_lookup(h, key, *best)) {
    best->vec = base.vec;
    best->bw = base.bw;
    best->npan = base.npan;
    if (best->bw == 0) best->strip = false;
    if (best->bw == 0 || best->npan == 0) best->panel = best->plo = false;
    if (best->panel || best->strip) best->R = 1;
    return CPCA_OK;
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best_ms = 1e30f;
  *best = base;
  // candidates: with a band image, the column-strip kernel and the row-panel
  // band kernel; otherwise rows per workgroup x LDS staging
  std::vector<ApplyCfg> cands;
  if (base.bw > 0) {
    ApplyCfg c = base;
    c.panel = false;
    c.strip = true;
    c.R = 1;
    c.lds = true;
    cands.push_back(c);
    if (base.npan > 0) {
      c.strip = false;
      c.panel = true;
      c.plo = false;
      cands.push_back(c);
      if (base.bw <= 8) {
        c.plo = true;
        cands.push_back(c);
      }
      c.panel = c.plo = false;
    }
    for (int R : {1, 2, 4}) {
      c.strip = false;
      c.R = R;
      if (lds_bytes(c, ld, elem) <= 65536) cands.push_back(c);
    }
  } else {
    for (int lds = 1; lds >= 0; --lds)
      for (int R : {1, 2, 4}) {
        ApplyCfg c = base;
        c.R = R;
        c.lds = lds != 0;
        c.strip = false;
        c.panel = false;
        if (!lds || lds_bytes(c, ld, elem) <= 65536) cands.push_back(c);
      }
  }
  cpca_status st = CPCA_OK;
  for (const ApplyCfg& c : cands) {
    if ((st = launch(c)) != CPCA_OK) break;  // warm-up
    if (hipEventRecord(e0, h->stream) != hipSuccess) {
      st = fail(CPCA_EHIP, "autotune: event record failed");
      break;
    }
    for (int k = 0; k < 3 && st == CPCA_OK; ++k) st = launch(c);
    if (st != CPCA_OK) break;
    float ms = 0.f;
    if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(CPCA_EHIP, "autotune: event timing failed");
      break;
    }
    if (ms < best_ms) {
      best_ms = ms;
      *best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == CPCA_OK) tune_store(h, key, *best);
  return st;
}

}  // namespace
