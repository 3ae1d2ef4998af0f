// Host check of the two-gate pass and environment index maps
// (paper_2306_08152_amd/csrc/qf_pair_geom.h, as used by k_pass2 and k_env2):
// for every qubit pair of gates forming a 3- or 4-qubit union, each tile
// shape and both builder precisions, the address-order phases of all tiles
// read and write every builder entry exactly once, each tile's LDS image
// holds entry (row variant a, column variant v, rest offset w) of that tile,
// and each gate's product phase covers every LDS entry of the tile exactly
// once with 4x4 blocks that vary only in that gate's bits; and, for a
// three-qubit gate run on the same tiles (k_pass3), that each union variant
// addresses the bits of its gate-local index.  Prints "ok" and the number of
// geometries, or the first failure.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "qf_pair_geom.h"

using namespace qf;

struct Shape {
  uint32_t wlog, upr_log, epu, active;
};

static Shape shape(bool c64, uint32_t m) {
  Shape s;
  s.wlog = (c64 ? 4u : 3u) + (m == 3 ? 2u : 0u);
  s.upr_log = m == 4 ? 7u : 8u;
  s.epu = c64 ? 2u : 1u;
  s.active = 1u << (s.wlog + 2u * (m - 2u));
  return s;
}

static int fail(const char* what, int n, const int32_t* f, const int32_t* sg) {
  std::printf("FAIL %s: n=%d F=(%d,%d) S=(%d,%d)\n", what, n, f[0], f[1], sg[0], sg[1]);
  return 1;
}

static int check(int n, const int32_t* f, const int32_t* sg, bool c64) {
  uint32_t mask = 0;
  for (int k = 0; k < 2; ++k) mask |= (1u << (n - 1 - f[k])) | (1u << (n - 1 - sg[k]));
  const uint32_t m = (uint32_t)__builtin_popcount(mask);
  const Shape sh = shape(c64, m);
  Pair2Geom g;
  if (!make_pair2_geom(n, f, sg, sh.wlog, g)) return (uint32_t)n < m + sh.wlog ? 0 : fail("geom", n, f, sg);
  const uint32_t N = g.N, W = g.W, V = 1u << m, RS = g.row_stride;
  if (RS != V * (W + 1)) return fail("row stride", n, f, sg);
  std::vector<uint8_t> seen((size_t)N * N, 0);
  std::vector<int64_t> lds(V * RS);
  const uint32_t rowstep = 256u >> sh.upr_log;
  for (uint32_t tl = 0; tl < g.tiles_per_start; ++tl) {
    const uint32_t rq = tl / g.col_tiles, ct = tl % g.col_tiles;
    const size_t origin = (size_t)dep_rest(g, rq) * N + dep_rest(g, ct << g.wlog);
    std::fill(lds.begin(), lds.end(), -1);
    for (uint32_t t = 0; t < 256; ++t) {
      const uint32_t ku = t & ((1u << sh.upr_log) - 1u), a0 = t >> sh.upr_log, k = ku * sh.epu;
      const uint32_t colk = dep_free(g, k);
      for (uint32_t jj = 0; jj < 8; ++jj) {
        const uint32_t a = a0 + jj * rowstep;
        if (a >= V) return fail("row variant range", n, f, sg);
        for (uint32_t e = 0; e < sh.epu; ++e) {
          const size_t gi = origin + (size_t)dep_union(g, a) * N + colk + e;
          if (e == 1 && dep_free(g, k + 1) != colk + 1) return fail("unit not contiguous", n, f, sg);
          if (gi >= (size_t)N * N || seen[gi]++) return fail("global coverage", n, f, sg);
          const uint32_t l = a * RS + lds_of_k(g, k + e);
          if (lds[l] != -1) return fail("lds written twice", n, f, sg);
          lds[l] = (int64_t)gi;
          // LDS entry (a, v, w) must hold row variant a, column variant v of rest offset w
          const uint32_t lv = (l % RS) / (W + 1), lw = (l % RS) % (W + 1);
          if (lw >= W) return fail("pad written", n, f, sg);
          const size_t want = (size_t)(dep_rest(g, rq) | dep_union(g, a)) * N +
                              (dep_rest(g, (ct << g.wlog) + lw) | dep_union(g, lv));
          if (want != gi) return fail("lds image", n, f, sg);
        }
      }
    }
    for (int which = 0; which < 2; ++which) {
      const uint32_t* gidx = which == 0 ? g.f_idx : g.s_idx;
      const uint32_t* oi = which == 0 ? g.o_f : g.o_s;
      const int32_t* loc = which == 0 ? f : sg;
      std::vector<uint8_t> cover(V * RS, 0);
      for (uint32_t t = 0; t < sh.active; ++t) {
        const uint32_t w = t & (W - 1u);
        const uint32_t orow = (t >> g.wlog) & ((1u << (m - 2)) - 1u), ocol = t >> (g.wlog + m - 2);
        const uint32_t vr = var_other(orow, oi, m), vc = var_other(ocol, oi, m);
        for (uint32_t i = 0; i < 4; ++i)
          for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t l = (var_local(i, gidx[0], gidx[1]) | vr) * RS + (var_local(j, gidx[0], gidx[1]) | vc) * (W + 1) + w;
            if (l >= V * RS || lds[l] < 0 || cover[l]++) return fail("phase coverage", n, f, sg);
            // the block's (i, j) entry differs from its (0, 0) entry exactly in the gate's bits:
            // local index i = 2 * bit(loc[0]) + bit(loc[1]) of the row, j of the column
            const size_t e00 = (size_t)lds[(var_local(0, gidx[0], gidx[1]) | vr) * RS + (var_local(0, gidx[0], gidx[1]) | vc) * (W + 1) + w];
            const size_t r = (size_t)lds[l] / N, c = (size_t)lds[l] % N, r0 = e00 / N, c0 = e00 % N;
            const uint32_t b0 = (uint32_t)(n - 1 - loc[0]), b1 = (uint32_t)(n - 1 - loc[1]);
            const size_t roff = (size_t)(((i >> 1) & 1u) << b0) | ((i & 1u) << b1);
            const size_t coff = (size_t)(((j >> 1) & 1u) << b0) | ((j & 1u) << b1);
            if (r != (r0 | roff) || c != (c0 | coff) || (r0 & roff) || (c0 & coff)) return fail("block shape", n, f, sg);
          }
      }
      for (uint32_t l = 0; l < V * RS; ++l)
        if ((lds[l] >= 0) != (cover[l] == 1)) return fail("phase misses an entry", n, f, sg);
    }
  }
  for (size_t i = 0; i < seen.size(); ++i)
    if (seen[i] != 1) return fail("entry not covered once", n, f, sg);
  return 0;
}

// Three-qubit gate on locations (l0, l1, l2) as the pair F = (l0, l1),
// S = (l1, l2): variant v of the union must address the bits of gate-local
// index k3_local(v) (first location most significant).
static int check3(int n, int l0, int l1, int l2) {
  const int32_t f[2] = {l0, l1}, sg[2] = {l1, l2};
  for (int c64 = 0; c64 < 2; ++c64) {
    Pair2Geom g;
    const uint32_t wlog = shape(c64 != 0, 3).wlog;
    if (!make_pair2_geom(n, f, sg, wlog, g)) {
      if ((uint32_t)n >= 3 + wlog) return fail("k3 geom", n, f, sg);
      continue;
    }
    if (g.m != 3) return fail("k3 union", n, f, sg);
    uint32_t seen = 0;
    for (uint32_t v = 0; v < 8; ++v) {
      const uint32_t l = k3_local(g, v);
      const uint32_t bits = (((l >> 2) & 1u) << (n - 1 - l0)) | (((l >> 1) & 1u) << (n - 1 - l1)) | ((l & 1u) << (n - 1 - l2));
      if (l > 7 || (seen & (1u << l)) || dep_union(g, v) != bits) return fail("k3 local index", n, f, sg);
      seen |= 1u << l;
    }
  }
  return 0;
}

int main(int argc, char** argv) {
  const int nmax = argc > 1 ? std::atoi(argv[1]) : 11;
  int count = 0;
  for (int n = 3; n <= nmax; ++n)
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b)
        for (int c = 0; c < n; ++c) {
          if (a == b || b == c || a == c) continue;
          if (check3(n, a, b, c)) return 1;
          ++count;
        }
  for (int n = 4; n <= nmax; ++n)
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b)
        for (int c = 0; c < n; ++c)
          for (int d = 0; d < n; ++d) {
            if (a == b || c == d) continue;
            const int32_t f[2] = {a, b}, sg[2] = {c, d};
            uint32_t mask = (1u << a) | (1u << b) | (1u << c) | (1u << d);
            const int m = __builtin_popcount(mask);
            if (m < 3) continue;
            // every geometry at small n; at larger n a sample of pairs
            if (n > 8 && ((a * 7 + b * 5 + c * 3 + d) % 11) != 0) continue;
            for (int c64 = 0; c64 < 2; ++c64) {
              if (check(n, f, sg, c64 != 0)) return 1;
              ++count;
            }
          }
  std::printf("ok %d\n", count);
  return 0;
}
