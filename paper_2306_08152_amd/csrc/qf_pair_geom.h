// Index maps of the two-gate pass and the two-gate environment step (one
// builder pass and one partial trace for two consecutive gate updates of a
// sweep).  Host and device share these functions; a host program checks that
// every tile geometry covers each builder entry exactly once.
//
// Bits: qubit q is bit n-1-q of a row or column index.  The union U of the
// two gates' qubits has m = 3 or 4 bit positions u[0] < ... < u[m-1]; a
// "variant" v in [0, 2^m) sets bit u[i] of an index from bit i of v.  The
// other n-m positions are the "rest"; dep_rest(x) spreads the bits of x over
// them in ascending order.
//
// Pass tile: the 2^m rows of one rest row index rq times the 2^m column
// variants of W = 2^wlog consecutive rest column indices ct*W .. ct*W+W-1,
// 4^m * W entries.  Its columns in increasing address order are indexed by
// k in [0, 2^(m+wlog)): bit j of k sets the j-th lowest "free" position
// (the m union positions and the wlog lowest rest positions).  In LDS the
// tile is [a][v][w] with one pad entry per (a, v) row: a = row variant,
// v = column variant, w = rest column offset in the tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qf {

struct Pair2Geom {
  uint32_t n, N, m, wlog, W;
  uint32_t u[4];              // union bit positions, ascending
  uint32_t rest_run_pos[5];   // rest positions as runs: position of run r
  uint32_t rest_run_len[5];   // its length; runs in ascending order
  uint32_t rest_runs;
  uint32_t free_run_pos[5];   // free positions (union + wlog lowest rest) as runs
  uint32_t free_run_len[5];
  uint32_t free_runs;
  uint32_t kv_shift[4];       // bit of k holding variant bit i
  uint32_t kw_shift[8];       // bit of k holding rest-offset bit r (r < wlog)
  uint32_t f_idx[2], s_idx[2];  // union index of gate F's / gate S's local MSB and LSB
  uint32_t o_f[2], o_s[2];      // union indices not in F (resp. S), ascending (m-2 used)
  uint32_t col_tiles;         // (N >> m) >> wlog
  uint32_t tiles_per_start;   // (N >> m) * col_tiles
  uint32_t row_stride;        // LDS entries per tile row a: 2^m * (W + 1)
  uint32_t tiles_per_wg;      // tiles each pass workgroup walks (0 = the default); set by the caller
};

// x spread over the runs (pos, len), lowest run first.
__host__ __device__ __forceinline__ uint32_t dep_runs(uint32_t x, const uint32_t* pos, const uint32_t* len,
                                                      uint32_t runs) {
  uint32_t out = 0;
  for (uint32_t r = 0; r < runs; ++r) {
    out |= (x & ((1u << len[r]) - 1u)) << pos[r];
    x >>= len[r];
  }
  return out;
}
__host__ __device__ __forceinline__ uint32_t dep_rest(const Pair2Geom& g, uint32_t x) {
  return dep_runs(x, g.rest_run_pos, g.rest_run_len, g.rest_runs);
}
__host__ __device__ __forceinline__ uint32_t dep_union(const Pair2Geom& g, uint32_t v) {
  uint32_t out = 0;
  for (uint32_t i = 0; i < g.m; ++i) out |= ((v >> i) & 1u) << g.u[i];
  return out;
}
// Column offset inside the tile of memory-order index k.
__host__ __device__ __forceinline__ uint32_t dep_free(const Pair2Geom& g, uint32_t k) {
  return dep_runs(k, g.free_run_pos, g.free_run_len, g.free_runs);
}
// (v, w) of memory-order index k, as the LDS offset v * (W + 1) + w.
__host__ __device__ __forceinline__ uint32_t lds_of_k(const Pair2Geom& g, uint32_t k) {
  uint32_t v = 0, w = 0;
  for (uint32_t i = 0; i < g.m; ++i) v |= ((k >> g.kv_shift[i]) & 1u) << i;
  for (uint32_t r = 0; r < g.wlog; ++r) w |= ((k >> g.kw_shift[r]) & 1u) << r;
  return v * (g.W + 1u) + w;
}
// Variant of gate-local index l (0..3) of a gate with union indices (i0, i1).
__host__ __device__ __forceinline__ uint32_t var_local(uint32_t l, uint32_t i0, uint32_t i1) {
  return (((l >> 1) & 1u) << i0) | ((l & 1u) << i1);
}
// Variant of the "other" bits o (m-2 of them) at union indices oi[].
__host__ __device__ __forceinline__ uint32_t var_other(uint32_t o, const uint32_t* oi, uint32_t m) {
  uint32_t v = ((o & 1u) << oi[0]);
  if (m == 4) v |= ((o >> 1) & 1u) << oi[1];
  return v;
}

// The tiles also serve one three-qubit gate on locations (l0, l1, l2), given
// as F = (l0, l1), S = (l1, l2): the union is the gate's three qubits, and
// variant v is the gate-local index (first location most significant)
// returned here.
__host__ __device__ __forceinline__ uint32_t k3_local(const Pair2Geom& g, uint32_t v) {
  return (((v >> g.f_idx[0]) & 1u) << 2) | (((v >> g.f_idx[1]) & 1u) << 1) | ((v >> g.s_idx[1]) & 1u);
}

// Host: geometry for gates F (locs f[0], f[1]) then S (s[0], s[1]) on n
// qubits with tile width 2^wlog.  Returns false when the pair does not form
// a 3- or 4-qubit union or the builder is too small for one tile.
inline bool make_pair2_geom(int n, const int32_t* f, const int32_t* s, uint32_t wlog, Pair2Geom& g) {
  g = Pair2Geom{};
  if (n < 4 || n > 16) return false;
  uint32_t bits[4] = {(uint32_t)(n - 1 - f[0]), (uint32_t)(n - 1 - f[1]), (uint32_t)(n - 1 - s[0]),
                      (uint32_t)(n - 1 - s[1])};
  uint32_t mask = 0;
  for (uint32_t b : bits) mask |= 1u << b;
  const uint32_t m = (uint32_t)__builtin_popcount(mask);
  if (m != 3 && m != 4) return false;
  if ((uint32_t)n < m + wlog) return false;
  g.n = (uint32_t)n;
  g.N = 1u << n;
  g.m = m;
  g.wlog = wlog;
  g.W = 1u << wlog;
  uint32_t k = 0;
  for (uint32_t b = 0; b < (uint32_t)n; ++b)
    if (mask & (1u << b)) g.u[k++] = b;
  auto idx = [&](uint32_t b) {
    for (uint32_t i = 0; i < m; ++i)
      if (g.u[i] == b) return i;
    return 0u;
  };
  g.f_idx[0] = idx(bits[0]);
  g.f_idx[1] = idx(bits[1]);
  g.s_idx[0] = idx(bits[2]);
  g.s_idx[1] = idx(bits[3]);
  for (int which = 0; which < 2; ++which) {
    const uint32_t* gi = which == 0 ? g.f_idx : g.s_idx;
    uint32_t* oi = which == 0 ? g.o_f : g.o_s;
    uint32_t c = 0;
    for (uint32_t i = 0; i < m; ++i)
      if (i != gi[0] && i != gi[1]) oi[c++] = i;
  }
  // rest positions as runs
  auto add_runs = [](uint32_t msk, uint32_t nbits, uint32_t* pos, uint32_t* len, uint32_t& runs) {
    runs = 0;
    for (uint32_t b = 0; b < nbits;) {
      if (!(msk & (1u << b))) {
        ++b;
        continue;
      }
      uint32_t e = b;
      while (e < nbits && (msk & (1u << e))) ++e;
      pos[runs] = b;
      len[runs] = e - b;
      ++runs;
      b = e;
    }
  };
  const uint32_t all = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
  const uint32_t rest = all & ~mask;
  add_runs(rest, (uint32_t)n, g.rest_run_pos, g.rest_run_len, g.rest_runs);
  // free positions: union + the wlog lowest rest positions
  uint32_t lowrest = 0, cnt = 0;
  for (uint32_t b = 0; b < (uint32_t)n && cnt < wlog; ++b)
    if (rest & (1u << b)) {
      lowrest |= 1u << b;
      ++cnt;
    }
  const uint32_t freem = mask | lowrest;
  add_runs(freem, (uint32_t)n, g.free_run_pos, g.free_run_len, g.free_runs);
  uint32_t j = 0, r = 0;
  for (uint32_t b = 0; b < (uint32_t)n; ++b) {
    if (!(freem & (1u << b))) continue;
    if (mask & (1u << b))
      g.kv_shift[idx(b)] = j;
    else
      g.kw_shift[r++] = j;
    ++j;
  }
  g.col_tiles = (g.N >> m) >> wlog;
  g.tiles_per_start = (g.N >> m) * g.col_tiles;
  g.row_stride = (1u << m) * (g.W + 1u);
  return true;
}

}  // namespace qf
