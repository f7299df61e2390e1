// Row panels of L_r for the row-panel gather kernel (k_apply_panel and
// k_apply_panel_lo): the layout constants the kernel is compiled with and the
// host code that builds its tables. Plain C++ (no HIP), so that the tables
// can be checked on the CPU.
//
// A panel is a set of at most kPanelRows rows of L_r; its union U is the set
// of rows its L_r entries reference (the panel's rows included), at most
// PanelUnion<T> rows. The product L_r X over one column strip needs, per
// panel, the strip segment of every row of U. A workgroup computes
// G = panel_group(npan) consecutive panels and keeps the staged rows in LDS
// slots between them: a row of U that is already resident from an earlier
// panel of the group is not loaded again. The builder therefore grows each
// panel along the union of the previous one, and assigns the slots.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <climits>
#include <vector>

namespace cpca {

constexpr int kPanelLanes = 16;   // lanes per row slot
constexpr int kPanelRows = 64;    // rows per panel (max)
constexpr int kPanelK = 16;       // off-diagonal L_r entries per row (max)
constexpr int kPanelGroupMax = 16;
constexpr int kPanelRowBytes = 256;  // LDS bytes of one staged union row (16 lanes x 16 bytes)
template <typename T> struct PanelUnion { static constexpr int value = sizeof(T) == 4 ? 160 : 128; };
static_assert(PanelUnion<float>::value * kPanelRowBytes <= 65536 &&
                  PanelUnion<double>::value * kPanelRowBytes <= 65536,
              "LDS offsets are 16-bit");

// CSR matrix on the host (FP64 values).
struct HostCsr {
  int64_t n = 0, nnz = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> v;
};

// Consecutive panels per workgroup of the panel kernels: the largest G <= 8
// whose panel groups fill the 8 per-XCD ranges of a strip to within 4 % (an
// empty range ends the launch early on its XCD), else 2. Fewer, longer
// workgroups load the band diagonals into registers fewer times and keep more
// union rows resident in LDS.
inline int panel_group(int npan) {
  for (int G = 8; G >= 2; --G) {
    const int ng = (npan + G - 1) / G;
    const int slots = 8 * ((ng + 7) / 8);
    if (ng >= 8 && (slots - ng) * 25 <= slots) return G;
  }
  return 2;
}

// Device tables of the panels, panel by panel (k = 0 .. npan - 1):
//   u[u_off[k] + s]              for each LDS slot s < umax (u_off[k] = k umax):
//                                the row of U_k staged into slot s when panel
//                                k starts, -1 if the slot keeps its content
//                                (a resident row of U_k, or one not needed);
//   rows[r_off[k] .. r_off[k+1]) the panel's output rows, in growth order;
//   per output row: kPanelK LDS byte offsets (slot x kPanelRowBytes) and
//   values of its off-diagonal entries (entries beyond the row's count have
//   value 0 and the row's own slot), its diagonal entry, and meta
//   {row, own slot | count << 16, row mask, group count}, where the group
//   count is the largest count of the 4 consecutive rows one wave computes.
struct HostPanels {
  int npan = 0;
  int G = 0;  // panels per workgroup the slots were assigned for
  std::vector<int32_t> u_off, u, r_off, rows, meta;  // meta: 4 ints per row
  std::vector<uint16_t> eidx;
  std::vector<double> ew, diag;
  int64_t staged = 0;  // rows staged over all panels (sum of the load lists)
};

// Phase 1: greedy growth of the panels. Panels are built in groups of Gs.
// The first panel of a group starts at the lowest row not yet assigned; a
// later one starts at the lowest unassigned row of the previous panel's union
// (falling back to the lowest unassigned row). A panel repeatedly takes,
// among the unassigned rows already in its union U, the one that adds the
// fewest rows to U that are not resident (in the previous panel's union,
// within the group), then the fewest rows to U, then the lowest index, among
// the candidates that keep |U| <= umax; it stops at rmax rows or when no
// candidate fits.
// The two counts of every candidate are kept up to date as U grows: a row
// entering U leaves the counts of the candidates in its closed neighbourhood,
// which are exactly the candidates whose closed neighbourhood holds it when
// the pattern of L_r is symmetric (as a Laplacian's is). The chosen row is
// recounted exactly before it is taken, so |U| <= umax holds for any pattern.
inline void grow_panels(const HostCsr& Lr, int rmax, int umax, int Gs,
                        std::vector<std::vector<int>>& Rs, std::vector<std::vector<int>>& Us) {
  const int p = (int)Lr.n;
  Rs.clear();
  Us.clear();
  std::vector<char> assigned((size_t)p, 0);
  std::vector<int> stamp((size_t)p, -1);  // last panel whose union holds the row
  // live candidates of the current panel with their two counts (compact, so
  // the choice scans contiguous memory), and each candidate's position there
  struct Cand {
    int nl, nu, c;
  };
  std::vector<Cand> cand;
  std::vector<int> pos((size_t)p, -1);
  std::vector<int> U, R;
  int seed = 0;
  // f(w) for w in the closed neighbourhood of v: v and its off-diagonal entries
  auto each_nb = [&](int v, auto&& f) {
    f(v);
    for (int32_t e = Lr.rp[v]; e < Lr.rp[v + 1]; ++e)
      if (Lr.ci[e] != v) f(Lr.ci[e]);
  };
  for (int k = 0;; ++k) {
    const bool first = k % Gs == 0;
    int s = -1;
    if (!first) {
      for (int w : Us.back())
        if (!assigned[(size_t)w] && (s < 0 || w < s)) s = w;
    }
    if (s < 0) {
      while (seed < p && assigned[(size_t)seed]) ++seed;
      if (seed == p) break;
      s = seed;
    }
    for (const Cand& x : cand) pos[(size_t)x.c] = -1;
    U.clear();
    R.clear();
    cand.clear();
    auto drop = [&](int c) {
      const int i = pos[(size_t)c];
      cand[(size_t)i] = cand.back();
      pos[(size_t)cand[(size_t)i].c] = i;
      cand.pop_back();
      pos[(size_t)c] = -1;
    };
    // rows v would add to U (returned), and how many of them are not resident
    auto count = [&](int v, int& nl) {
      int nu = 0;
      nl = 0;
      each_nb(v, [&](int w) {
        const int st = stamp[(size_t)w];
        if (st == k) return;
        ++nu;
        nl += first || st != k - 1;
      });
      return nu;
    };
    auto ins = [&](int w) {
      const int st = stamp[(size_t)w];
      if (st == k) return;
      const bool fresh = first || st != k - 1;
      stamp[(size_t)w] = k;
      U.push_back(w);
      each_nb(w, [&](int c) {
        const int i = pos[(size_t)c];
        if (i < 0) return;
        --cand[(size_t)i].nu;
        cand[(size_t)i].nl -= fresh;
      });
      if (!assigned[(size_t)w]) {
        Cand x;
        x.c = w;
        x.nu = count(w, x.nl);
        pos[(size_t)w] = (int)cand.size();
        cand.push_back(x);
      }
    };
    auto take = [&](int v) {
      if (pos[(size_t)v] >= 0) drop(v);
      R.push_back(v);
      assigned[(size_t)v] = 1;
      each_nb(v, ins);
    };
    take(s);
    while ((int)R.size() < rmax) {
      int best = -1, bl = INT_MAX, bu = INT_MAX;
      const int room = umax - (int)U.size();
      for (const Cand& x : cand) {
        if (x.nu > room) continue;
        if (x.nl < bl || (x.nl == bl && (x.nu < bu || (x.nu == bu && x.c < best)))) {
          bl = x.nl;
          bu = x.nu;
          best = x.c;
        }
      }
      if (best < 0) break;
      int nl;
      if (count(best, nl) > room) {
        drop(best);  // miscounted (pattern not symmetric): not a candidate
        continue;
      }
      take(best);
    }
    std::sort(U.begin(), U.end());
    Rs.push_back(R);
    Us.push_back(U);
  }
}

// Builds the panel tables of L_r (false, and no tables, when a row has more
// than kPanelK off-diagonal entries or umax is not in [kPanelK + 1, 256];
// row masks mr). Phase 1 runs with the group size that panel_group gives for
// panels of rmax - 1 rows on average. Phase 2 assigns the LDS slots for
// G = panel_group(npan), the group size the launch uses (phase 1's guess only
// affects how much is reused): per group, the slots start empty; for each panel, every row of U that
// is resident keeps its slot, and each new row takes a slot that holds no row
// of U (empty slots first, then the one whose row was used longest ago, then
// the lowest slot). |U| <= umax guarantees a slot for every new row.
inline bool build_panels(const HostCsr& Lr, const std::vector<uint8_t>& mr, int rmax, int umax,
                         HostPanels& P) {
  P = HostPanels{};
  const int64_t p64 = Lr.n;
  if (p64 <= 0 || p64 >= INT_MAX || umax > 65536 / kPanelRowBytes || umax < kPanelK + 1)
    return false;
  const int p = (int)p64;
  for (int i = 0; i < p; ++i) {
    int c = 0;
    for (int32_t e = Lr.rp[i]; e < Lr.rp[i + 1]; ++e) c += Lr.ci[e] != i;
    if (c > kPanelK) return false;
  }
  std::vector<std::vector<int>> Rs, Us;
  grow_panels(Lr, rmax, umax, panel_group((p + rmax - 2) / (rmax - 1)), Rs, Us);
  const int npan = (int)Rs.size();
  const int G = panel_group(npan);
  P.npan = npan;
  P.G = G;
  P.u_off.push_back(0);
  P.r_off.push_back(0);
  std::vector<int> rslot((size_t)p, -1), inU((size_t)p, -1);
  std::vector<int> slot_row((size_t)umax, -1), last_use((size_t)umax, -1), fr((size_t)umax);
  std::vector<int> nb((size_t)kPanelGroupMax + 2);
  P.u.reserve((size_t)npan * umax);
  P.rows.reserve((size_t)p);
  P.diag.reserve((size_t)p);
  P.meta.reserve((size_t)4 * p);
  P.eidx.reserve((size_t)kPanelK * p);
  P.ew.reserve((size_t)kPanelK * p);
  for (int k0 = 0; k0 < npan; k0 += G) {
    for (int s = 0; s < umax; ++s) {
      if (slot_row[(size_t)s] >= 0) rslot[(size_t)slot_row[(size_t)s]] = -1;
      slot_row[(size_t)s] = -1;
      last_use[(size_t)s] = -1;
    }
    for (int k = k0; k < std::min(npan, k0 + G); ++k) {
      const std::vector<int>& U = Us[(size_t)k];
      const std::vector<int>& R = Rs[(size_t)k];
      for (int w : U) inU[(size_t)w] = k;
      // free slots (holding no row of U) by last use (-1: empty, else a panel
      // k0 .. k - 1 of this group), then by index: a counting sort
      std::fill(nb.begin(), nb.end(), 0);
      auto bucket = [&](int s) { return last_use[(size_t)s] < 0 ? 0 : last_use[(size_t)s] - k0 + 1; };
      auto is_free = [&](int s) {
        return slot_row[(size_t)s] < 0 || inU[(size_t)slot_row[(size_t)s]] != k;
      };
      for (int s = 0; s < umax; ++s)
        if (is_free(s)) ++nb[(size_t)bucket(s) + 1];
      for (size_t b = 1; b < nb.size(); ++b) nb[b] += nb[b - 1];
      for (int s = 0; s < umax; ++s)
        if (is_free(s)) fr[(size_t)nb[(size_t)bucket(s)]++] = s;
      size_t f = 0;
      const size_t ub = P.u.size();
      P.u.resize(ub + (size_t)umax, -1);
      for (int w : U) {
        if (rslot[(size_t)w] >= 0) continue;
        const int s = fr[f++];
        if (slot_row[(size_t)s] >= 0) rslot[(size_t)slot_row[(size_t)s]] = -1;
        slot_row[(size_t)s] = w;
        rslot[(size_t)w] = s;
        P.u[ub + (size_t)s] = w;
        ++P.staged;
      }
      for (int w : U) last_use[(size_t)rslot[(size_t)w]] = k;
      for (int v : R) {
        const int own = rslot[(size_t)v];
        const size_t base = P.eidx.size();
        P.eidx.resize(base + kPanelK, (uint16_t)(own * kPanelRowBytes));
        P.ew.resize(base + kPanelK, 0.0);
        int c = 0;
        double dg = 0.0;
        for (int32_t e = Lr.rp[v]; e < Lr.rp[v + 1]; ++e) {
          if (Lr.ci[e] == v) {
            dg += Lr.v[e];
            continue;
          }
          P.eidx[base + c] = (uint16_t)(rslot[(size_t)Lr.ci[e]] * kPanelRowBytes);
          P.ew[base + c] = Lr.v[e];
          ++c;
        }
        P.rows.push_back(v);
        P.diag.push_back(dg);
        const int m4[4] = {v, own | (c << 16), (int)mr[(size_t)v], c};
        P.meta.insert(P.meta.end(), m4, m4 + 4);
      }
      // group count: the rows j of a panel are computed by waves in groups of
      // 4 consecutive j (j = 16 pass + 4 wave + slot); each row carries the
      // largest count of its group
      const size_t r0 = P.rows.size() - R.size();
      for (size_t g = 0; g < R.size(); g += 4) {
        int mx = 0;
        for (size_t j = g; j < std::min(R.size(), g + 4); ++j) mx = std::max(mx, P.meta[4 * (r0 + j) + 3]);
        for (size_t j = g; j < std::min(R.size(), g + 4); ++j) P.meta[4 * (r0 + j) + 3] = mx;
      }
      P.u_off.push_back((int)P.u.size());
      P.r_off.push_back((int)P.rows.size());
    }
  }
  return true;
}

}  // namespace cpca
