// Streaming kernels: builders live in HBM and every gate update is one
// LDS-staged pass over them.
//
//   k_build_init   X_s <- V^dagger (cast to the builder precision)
//   k_pass         X_s <- (A_s (x) I) X_s (B_s (x) I)   (either side optional)
//   k_env          P_s = Tr_rest X_s in FP64 over many workgroups; the last
//                  workgroup of each start finishes the sum in a fixed order
//                  and, in sweep mode, runs the FP64 gate update
//   k_cost         Tr X_s and 1 - |Tr X_s| / N in FP64
//   k_optimize     batched FP64 gate update on given environments
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "qf_device.h"
#include "qf_env_finish.h"
#include "qf_internal.h"

namespace qf {

// ------------------------------------------------------------------ helpers

template <typename R>
struct Vec16;  // 16-byte vector of builder elements
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int elems = 2;
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int elems = 1;
};

template <typename R>
__device__ __forceinline__ cx<R> to_r(cd v) {
  return cx<R>{static_cast<R>(v.re), static_cast<R>(v.im)};
}

// Load the 4x4 operand of start s (optionally conjugate-transposed) in the
// builder precision.
template <typename R>
__device__ __forceinline__ void load_operand(cx<R> m[16], const Operand& op, uint32_t s) {
  const cd* src = reinterpret_cast<const cd*>(op.ptr) + (int64_t)s * op.stride;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cd v = op.dagger ? conj(src[4 * c + r]) : src[4 * r + c];
      m[4 * r + c] = to_r<R>(v);
    }
}

__device__ __forceinline__ uint32_t ilog2u(uint32_t v) { return 31u - __builtin_clz(v); }

// ------------------------------------------------------------------ geometry

PassGeom make_pass_geom(int n, int q0, int q1, int max_tcols) {
  PassGeom g{};
  g.direct = 0;
  g.micro = 0;
  if (max_tcols == kPassDirect) {
    if (n >= 6) g.direct = 1u;
    max_tcols = pass_max_tcols(QF_C128);  // the LDS tile serves n < 6
  } else if (max_tcols == kPassMicro) {
    const int hb = (n - 1 - q0) > (n - 1 - q1) ? (n - 1 - q0) : (n - 1 - q1);
    if (n >= 9 && hb <= 2) g.micro = 1u;
    max_tcols = pass_max_tcols(QF_C128);  // the LDS tile serves other gates
  }
  g.n = (uint32_t)n;
  g.N = 1u << n;
  g.b0 = (uint32_t)(n - 1 - q0);
  g.b1 = (uint32_t)(n - 1 - q1);
  g.rlo = g.b0 < g.b1 ? g.b0 : g.b1;
  g.rhi = g.b0 < g.b1 ? g.b1 : g.b0;
  uint32_t tcols = g.N < (uint32_t)max_tcols ? g.N : (uint32_t)max_tcols;
  uint32_t tl = 0;
  while ((1u << tl) < tcols) ++tl;
  g.tcols_log = tl;
  if (g.rhi < tl) {  // both local column bits inside one contiguous segment
    g.nseg = 1;
    g.tc = tl;
    g.tb0 = g.b0;
    g.tb1 = g.b1;
    g.seg_lo = g.seg_hi = 0;
  } else if (g.rlo + 1 < tl) {  // high bit split off as two segments
    g.nseg = 2;
    g.tc = tl - 1;
    g.seg_lo = g.seg_hi = g.rhi;
    if (g.b0 == g.rhi) {
      g.tb0 = g.tc;
      g.tb1 = g.b1;
    } else {
      g.tb1 = g.tc;
      g.tb0 = g.b0;
    }
  } else {  // both bits split off: four segments, one per local column index
    g.nseg = 4;
    g.tc = tl - 2;
    g.seg_lo = g.rlo;
    g.seg_hi = g.rhi;
    g.tb0 = g.tc + 1;
    g.tb1 = g.tc;
  }
  for (uint32_t sgi = 0; sgi < 4; ++sgi) {
    if (g.nseg == 4)
      g.seg_off[sgi] = local_off(sgi, g.b0, g.b1);
    else if (g.nseg == 2)
      g.seg_off[sgi] = (sgi & 1u) << g.rhi;
    else
      g.seg_off[sgi] = 0;
  }
  g.tblo = g.tb0 < g.tb1 ? g.tb0 : g.tb1;
  g.tbhi = g.tb0 < g.tb1 ? g.tb1 : g.tb0;
  g.col_tiles = g.N >> tl;
  g.tiles_per_start = (g.N >> 2) * g.col_tiles;
  return g;
}

// ------------------------------------------------------------------ k_pass

// One tile = one row quad x TCOLS columns (4*TCOLS elements), one thread per
// 4x4 block.  A tile is loaded with 16-byte coalesced loads into LDS, every
// thread transforms its block in registers and writes it back, and the tile
// is stored with the same coalesced pattern.  The tile width TCOLS is a
// tuning choice (smaller tiles shorten the end-of-grid drain, larger ones
// cut per-workgroup overhead).
struct TileBase {
  uint32_t row, col;
  size_t start_off;
};

__device__ __forceinline__ TileBase tile_base(const PassGeom& g, uint32_t tile) {
  TileBase tb;
  const uint32_t s = tile / g.tiles_per_start;
  const uint32_t rem = tile - s * g.tiles_per_start;
  const uint32_t rq = rem / g.col_tiles;
  const uint32_t ct = rem - rq * g.col_tiles;
  tb.row = insert00(rq, g.rlo, g.rhi);
  uint32_t c = ct << g.tc;
  if (g.nseg == 2)
    c = insert0(c, g.seg_hi);
  else if (g.nseg == 4)
    c = insert00(c, g.seg_lo, g.seg_hi);
  tb.col = c;
  tb.start_off = (size_t)s * g.N * g.N;
  return tb;
}

// Global element offset of element e (row-major 4 x TCOLS) of a tile.
__device__ __forceinline__ size_t tile_elem(const PassGeom& g, const TileBase& tb, uint32_t e) {
  const uint32_t i = e >> g.tcols_log;
  const uint32_t tcol = e & ((1u << g.tcols_log) - 1u);
  const uint32_t seg = tcol >> g.tc;
  const uint32_t segoff =
      (g.nseg == 4) ? local_off(seg, g.b0, g.b1) : ((g.nseg == 2) ? (seg << g.seg_hi) : 0u);
  const size_t row = tb.row + local_off(i, g.b0, g.b1);
  const size_t col = tb.col + segoff + (tcol & ((1u << g.tc) - 1u));
  return tb.start_off + row * g.N + col;
}

template <typename R, bool HA, bool HB>
__global__ __launch_bounds__(256) void k_pass(cx<R>* __restrict__ X, PassGeom g, Operand A, Operand B) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<R>* tile = reinterpret_cast<cx<R>*>(smem_raw);
  using V = typename Vec16<R>::type;
  constexpr uint32_t VE = Vec16<R>::elems;

  const uint32_t TCOLS = 1u << g.tcols_log;
  const uint32_t NT = TCOLS >> 2;
  const uint32_t t = threadIdx.x;
  const uint32_t cur = blockIdx.x;
  const uint32_t s = cur / g.tiles_per_start;
  const TileBase tb = tile_base(g, cur);
  const uint32_t nvec = (4u << g.tcols_log) / VE;

  for (uint32_t v = t; v < nvec; v += NT) {
    const uint32_t e = v * VE;
    *reinterpret_cast<V*>(tile + e) = *reinterpret_cast<const V*>(X + tile_elem(g, tb, e));
  }
  cx<R> a[16], b[16];
  if (HA) load_operand<R>(a, A, s);
  if (HB) load_operand<R>(b, B, s);
  __syncthreads();
  {
    const uint32_t cb = insert00(t, g.tblo, g.tbhi);
    uint32_t col[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) col[j] = cb + local_off(j, g.tb0, g.tb1);
    cx<R> x[16];
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i)
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) x[4 * i + j] = tile[i * TCOLS + col[j]];
    if (HA) {  // x <- A x
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cx<R> r[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          cx<R> acc = mk<R>(0, 0);
#pragma unroll
          for (int k = 0; k < 4; ++k) cmac(acc, a[4 * i + k], x[4 * k + j]);
          r[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) x[4 * i + j] = r[i];
      }
    }
    if (HB) {  // x <- x B
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        cx<R> r[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cx<R> acc = mk<R>(0, 0);
#pragma unroll
          for (int l = 0; l < 4; ++l) cmac(acc, x[4 * i + l], b[4 * l + j]);
          r[j] = acc;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) x[4 * i + j] = r[j];
      }
    }
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i)
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) tile[i * TCOLS + col[j]] = x[4 * i + j];
  }
  __syncthreads();
  for (uint32_t v = t; v < nvec; v += NT) {
    const uint32_t e = v * VE;
    *reinterpret_cast<V*>(X + tile_elem(g, tb, e)) = *reinterpret_cast<const V*>(tile + e);
  }
}

// ------------------------------------------------------------ k_pass_block
//
// Register-direct form of the same pass for n >= 6, where a start owns a
// whole number of 256-thread workgroups (so the start index, and with it the
// operands, are uniform per workgroup and sit in scalar registers).  One 4x4
// block per thread and no LDS: every thread loads its 16 entries straight
// from HBM, which keeps many more bytes in flight per CU than an LDS-staged
// tile can (LDS capacity bounds the staged form).  Consecutive threads take
// consecutive block columns, so a wavefront's 64 loads of one block entry
// cover long runs of columns, unless both gate bits are among the lowest
// column bits (then they stride by 2..8 elements and the LDS-staged tile is
// faster).  The runtime's tuner picks between the forms per (precision, n,
// gate class).

template <typename R, bool HA, bool HB>
__device__ __forceinline__ void pass_block_body(cx<R>* __restrict__ X, const PassGeom& g, uint32_t wg_per_start,
                                                const Operand& A, const Operand& B, uint32_t wg) {
  const uint32_t N = g.N;
  const uint32_t s = wg / wg_per_start;
  const uint32_t blk = (wg - s * wg_per_start) * 256u + threadIdx.x;
  const uint32_t rq = blk >> (g.n - 2), cq = blk & ((N >> 2) - 1u);
  const uint32_t rb = insert00(rq, g.rlo, g.rhi), cb = insert00(cq, g.rlo, g.rhi);
  uint32_t off[4];
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) off[i] = local_off(i, g.b0, g.b1);
  cx<R>* base = X + (size_t)s * N * N;
  cx<R> a[16], b[16];
  if (HA) load_operand_uniform<R>(a, A, s);
  if (HB) load_operand_uniform<R>(b, B, s);
  cx<R> x[16];
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i)
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) x[4 * i + j] = base[(rb + off[i]) * N + cb + off[j]];
  if (HA) {  // x <- A x
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cx<R> r[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        cx<R> acc = mk<R>(0, 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) cmac(acc, a[4 * i + k], x[4 * k + j]);
        r[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) x[4 * i + j] = r[i];
    }
  }
  if (HB) {  // x <- x B
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      cx<R> r[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cx<R> acc = mk<R>(0, 0);
#pragma unroll
        for (int l = 0; l < 4; ++l) cmac(acc, x[4 * i + l], b[4 * l + j]);
        r[j] = acc;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) x[4 * i + j] = r[j];
    }
  }
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i)
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) base[(rb + off[i]) * N + cb + off[j]] = x[4 * i + j];
}

template <typename R, bool HA, bool HB>
__global__ __launch_bounds__(256) void k_pass_block(cx<R>* __restrict__ X, PassGeom g, uint32_t wg_per_start,
                                                    Operand A, Operand B) {
  pass_block_body<R, HA, HB>(X, g, wg_per_start, A, B, blockIdx.x);
}

// ------------------------------------------------------------ k_pass_micro
//
// Register form of the pass for complex64 gates whose two column bits are
// both among the three lowest (the class where the block-per-thread form's
// loads stride by 2..8 elements): n >= 9.  The 8 columns that share the
// high column bits form a micro-tile holding two 4x4 blocks of the gate (the
// third low bit picks the block).  A wavefront covers 512 consecutive
// columns (4 KiB) of each of a block row-group's four rows with 16 B loads:
// load k of a row puts columns 128k + 2l, 128k + 2l + 1 in lane l, so every
// load instruction reads 1 KiB contiguously and the four lanes of a quad hold
// one micro-tile's row.  The left product (rows) is lane-local; each entry of
// the right product (columns) takes its four operands from the quad by DPP
// quad_perm moves, whose patterns follow from the gate's bits at compile
// time.  Each output is the block-per-thread form's sum, term by term, so
// all forms give bitwise the same builder.

// Column (0..7) of the micro-tile holding gate-local index l in the block of
// column c; the gate's column bits are B0 (high local bit) and B1.
__host__ __device__ constexpr int mt_col(int B0, int B1, int c, int l) {
  return (((l >> 1) & 1) << B0) | ((l & 1) << B1) | (c & (1 << (3 - B0 - B1)));
}
// quad_perm selector: lane q reads the lane holding operand l of its column 2q + h.
__host__ __device__ constexpr int mt_pat(int B0, int B1, int h, int l) {
  return (mt_col(B0, B1, h, l) >> 1) | ((mt_col(B0, B1, 2 + h, l) >> 1) << 2) |
         ((mt_col(B0, B1, 4 + h, l) >> 1) << 4) | ((mt_col(B0, B1, 6 + h, l) >> 1) << 6);
}
// Which of the source lane's two columns it is (the same for every lane).
__host__ __device__ constexpr int mt_slot(int B0, int B1, int h, int l) { return mt_col(B0, B1, h, l) & 1; }
__host__ __device__ constexpr bool mt_slot_uniform(int B0, int B1) {
  for (int h = 0; h < 2; ++h)
    for (int l = 0; l < 4; ++l)
      for (int q = 0; q < 4; ++q)
        if ((mt_col(B0, B1, 2 * q + h, l) & 1) != mt_slot(B0, B1, h, l)) return false;
  return true;
}

template <int CTRL>
__device__ __forceinline__ cf dpp_cf(cf v) {
  return cf{__int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.re), CTRL, 0xF, 0xF, false)),
            __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.im), CTRL, 0xF, 0xF, false))};
}
template <int B0, int B1, int H, int L>
__device__ __forceinline__ cf mt_operand(const cf x[2]) {
  constexpr int P = mt_pat(B0, B1, H, L);
  constexpr int SL = mt_slot(B0, B1, H, L);
  if constexpr (P == 0xE4) return x[SL];  // [0,1,2,3]: the lane's own column
  else return dpp_cf<P>(x[SL]);
}
// Right product of one micro-tile row: z[h] = sum_l x(column of l) b[l][j_h].
template <int B0, int B1>
__device__ __forceinline__ void mt_right(const cf x[2], const cf bc[2][4], cf z[2]) {
  const cf o00 = mt_operand<B0, B1, 0, 0>(x), o01 = mt_operand<B0, B1, 0, 1>(x);
  const cf o02 = mt_operand<B0, B1, 0, 2>(x), o03 = mt_operand<B0, B1, 0, 3>(x);
  const cf o10 = mt_operand<B0, B1, 1, 0>(x), o11 = mt_operand<B0, B1, 1, 1>(x);
  const cf o12 = mt_operand<B0, B1, 1, 2>(x), o13 = mt_operand<B0, B1, 1, 3>(x);
  cf a0 = mk(0.f, 0.f), a1 = mk(0.f, 0.f);
  cmac(a0, o00, bc[0][0]);
  cmac(a0, o01, bc[0][1]);
  cmac(a0, o02, bc[0][2]);
  cmac(a0, o03, bc[0][3]);
  cmac(a1, o10, bc[1][0]);
  cmac(a1, o11, bc[1][1]);
  cmac(a1, o12, bc[1][2]);
  cmac(a1, o13, bc[1][3]);
  z[0] = a0;
  z[1] = a1;
}

template <int B0, int B1, bool HA, bool HB>
__device__ __forceinline__ void pass_micro_body(cf* __restrict__ X, uint32_t n, uint32_t wg_per_start,
                                                const Operand& A, const Operand& B, uint32_t wg) {
  static_assert(B0 != B1 && B0 >= 0 && B0 <= 2 && B1 >= 0 && B1 <= 2, "both gate bits among the three lowest");
  static_assert(mt_slot_uniform(B0, B1), "operand slots must not depend on the lane");
  constexpr uint32_t LO = B0 < B1 ? B0 : B1, HI = B0 < B1 ? B1 : B0;
  const uint32_t N = 1u << n;
  const uint32_t s = wg / wg_per_start;
  const uint32_t w = (wg - s * wg_per_start) * 4u + (threadIdx.x >> 6);  // wavefront within the start
  const uint32_t W = N >> 9;                                                      // 512-column spans per row
  const uint32_t rgi = w / W, span = w - rgi * W;
  const uint32_t rb = insert00(rgi, LO, HI);
  const uint32_t lane = threadIdx.x & 63u, q = lane & 3u;
  cf* base = X + (size_t)s * N * N + (size_t)span * 512u + 2u * lane;
  cf a[16], b[16];
  if (HA) load_operand_uniform<float>(a, A, s);
  if (HB) load_operand_uniform<float>(b, B, s);
  // x[i][k][h]: row rb + off(i), column 128k + 2 lane + h of the span
  cf x[4][4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const size_t row = rb + (uint32_t)mt_col(B0, B1, 0, i);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 v = *reinterpret_cast<const float4*>(base + row * N + 128u * k);
      x[i][k][0] = mk(v.x, v.y);
      x[i][k][1] = mk(v.z, v.w);
    }
  }
  if (HA) {  // x <- A x, lane-local
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        cf r[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          cf acc = mk(0.f, 0.f);
#pragma unroll
          for (int j = 0; j < 4; ++j) cmac(acc, a[4 * i + j], x[j][k][h]);
          r[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i][k][h] = r[i];
      }
  }
  if (HB) {  // x <- x B, operands from the quad
    // bc[h][l] = B[l][j] for the gate-local index j of this lane's column 2q + h
    cf bc[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t c = 2u * q + (uint32_t)h;
      const uint32_t j = (((c >> B0) & 1u) << 1) | ((c >> B1) & 1u);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        cf v = b[4 * l];
#pragma unroll
        for (int jj = 1; jj < 4; ++jj) v = sel(j == (uint32_t)jj, b[4 * l + jj], v);
        bc[h][l] = v;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        cf z[2];
        mt_right<B0, B1>(x[i][k], bc, z);
        x[i][k][0] = z[0];
        x[i][k][1] = z[1];
      }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const size_t row = rb + (uint32_t)mt_col(B0, B1, 0, i);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      *reinterpret_cast<float4*>(base + row * N + 128u * k) =
          make_float4(x[i][k][0].re, x[i][k][0].im, x[i][k][1].re, x[i][k][1].im);
  }
}

template <int B0, int B1, bool HA, bool HB>
__global__ __launch_bounds__(256) void k_pass_micro(cf* __restrict__ X, uint32_t n, uint32_t wg_per_start,
                                                    Operand A, Operand B) {
  pass_micro_body<B0, B1, HA, HB>(X, n, wg_per_start, A, B, blockIdx.x);
}

// A launch, with the kernel's own start / stop timestamps when asked for.
template <int B0, int B1, bool HA, bool HB>
static hipError_t launch_pass_micro_t(hipStream_t st, cf* x, int S, const PassGeom& g, Operand A, Operand B,
                                      KernelEvents ev) {
  const uint32_t wgps = g.N * g.N / 8192u;  // (N/4 row groups) x (N/512 spans) wavefronts, 4 per workgroup
  return launch_k(k_pass_micro<B0, B1, HA, HB>, dim3((uint32_t)S * wgps), dim3(256), 0u, st, ev, x, g.n, wgps, A,
                  B);
}
template <bool HA, bool HB>
static hipError_t launch_pass_micro(hipStream_t st, cf* x, int S, const PassGeom& g, Operand A, Operand B,
                                    KernelEvents ev) {
  switch (g.b0 * 3 + g.b1) {
    case 0 * 3 + 1: return launch_pass_micro_t<0, 1, HA, HB>(st, x, S, g, A, B, ev);
    case 0 * 3 + 2: return launch_pass_micro_t<0, 2, HA, HB>(st, x, S, g, A, B, ev);
    case 1 * 3 + 0: return launch_pass_micro_t<1, 0, HA, HB>(st, x, S, g, A, B, ev);
    case 1 * 3 + 2: return launch_pass_micro_t<1, 2, HA, HB>(st, x, S, g, A, B, ev);
    case 2 * 3 + 0: return launch_pass_micro_t<2, 0, HA, HB>(st, x, S, g, A, B, ev);
    case 2 * 3 + 1: return launch_pass_micro_t<2, 1, HA, HB>(st, x, S, g, A, B, ev);
    default: return hipErrorInvalidValue;
  }
}

template <typename R, bool HA, bool HB>
static hipError_t launch_pass_direct(hipStream_t st, cx<R>* x, int S, const PassGeom& g, Operand A, Operand B,
                                     KernelEvents ev) {
  const uint32_t wgps = g.N * g.N / 4096u;  // N^2/16 blocks, 256 per workgroup
  // The kernel uses no LDS; the 40 KiB it reserves caps it at 4 workgroups
  // (16 waves) per CU, which keeps its bandwidth and was measured to let the
  // concurrent stream groups' environment steps interleave with it better
  // (start-sweeps/s +7 to +10 % at n = 10 with 16 starts in 3-4 groups).
  constexpr size_t kPassBlockLds = 40 * 1024;
  return launch_k(k_pass_block<R, HA, HB>, dim3((uint32_t)S * wgps), dim3(256), (uint32_t)kPassBlockLds, st, ev, x,
                  g, wgps, A, B);
}

template <typename R, bool HA, bool HB>
static hipError_t launch_pass_v(hipStream_t st, cx<R>* x, uint32_t total, const PassGeom& g, Operand A,
                                Operand B, KernelEvents ev) {
  const uint32_t TCOLS = 1u << g.tcols_log;
  const size_t lds = 4u * TCOLS * sizeof(cx<R>);
  return launch_k(k_pass<R, HA, HB>, dim3(total), dim3(TCOLS >> 2), (uint32_t)lds, st, ev, x, g, A, B);
}

// Default tile width before (or without) tuning: 32 KiB of LDS per tile.
int pass_max_tcols(int precision) { return precision == QF_C64 ? 1024 : 512; }

template <typename R>
static hipError_t launch_pass_t(hipStream_t st, void* X, int S, const PassGeom& g, Operand A,
                                Operand B, KernelEvents ev) {
  const uint32_t total = (uint32_t)S * g.tiles_per_start;
  cx<R>* x = reinterpret_cast<cx<R>*>(X);
  if (g.micro && (reinterpret_cast<uintptr_t>(X) & 15u) == 0) {  // 16 B loads; else the LDS tile below
    if constexpr (sizeof(R) == 4) {
      if (A.ptr && B.ptr) return launch_pass_micro<true, true>(st, x, S, g, A, B, ev);
      if (A.ptr) return launch_pass_micro<true, false>(st, x, S, g, A, B, ev);
      if (B.ptr) return launch_pass_micro<false, true>(st, x, S, g, A, B, ev);
      return hipSuccess;
    } else {
      return hipErrorInvalidValue;  // complex64 only
    }
  }
  if (g.direct) {
    if (A.ptr && B.ptr) return launch_pass_direct<R, true, true>(st, x, S, g, A, B, ev);
    if (A.ptr) return launch_pass_direct<R, true, false>(st, x, S, g, A, B, ev);
    if (B.ptr) return launch_pass_direct<R, false, true>(st, x, S, g, A, B, ev);
    return hipSuccess;
  }
  if (A.ptr && B.ptr) return launch_pass_v<R, true, true>(st, x, total, g, A, B, ev);
  if (A.ptr) return launch_pass_v<R, true, false>(st, x, total, g, A, B, ev);
  if (B.ptr) return launch_pass_v<R, false, true>(st, x, total, g, A, B, ev);
  return hipSuccess;
}

hipError_t launch_pass(hipStream_t st, int precision, void* X, int S, const PassGeom& g, Operand A,
                       Operand B, KernelEvents ev) {
  if (precision == QF_C64) return launch_pass_t<float>(st, X, S, g, A, B, ev);
  return launch_pass_t<double>(st, X, S, g, A, B, ev);
}

// k_env: 256 threads = 16 (i,j) pairs x 16 rest lanes; one workgroup covers
// at most kEnvRestsPerWG rests (so n <= 14 fits one workgroup per start).
// A thread keeps eight loads in flight, so a workgroup takes in
// kEnvRestsPerRound rests per round of loads.
constexpr uint32_t kEnvThreads = 256;
constexpr uint32_t kEnvRestsPerWG = 4096;
constexpr uint32_t kEnvRestsPerRound = 128;
// Workgroups of all starts of one launch that the spread aims for: enough to
// put every start's rests on many CUs when starts are few.
constexpr uint32_t kEnvSpreadTarget = 256;

// ------------------------------------------------------------------ k_build_init

template <typename R>
__global__ __launch_bounds__(256) void k_build_init(const cd* __restrict__ V, cx<R>* __restrict__ X,
                                                    uint32_t N, uint32_t S) {
  __shared__ cd tile[32][33];
  const uint32_t tilesx = (N + 31) / 32;
  const uint32_t bx = blockIdx.x % tilesx, by = blockIdx.x / tilesx;
  const uint32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // read V rows by*32.., cols bx*32..
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    const uint32_t r = by * 32 + ty + 8 * k, c = bx * 32 + tx;
    if (r < N && c < N) tile[ty + 8 * k][tx] = V[(size_t)r * N + c];
  }
  __syncthreads();
  // X[c][r] = conj(V[r][c])
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    const uint32_t xr = bx * 32 + ty + 8 * k, xc = by * 32 + tx;
    if (xr < N && xc < N) {
      const cx<R> v = to_r<R>(conj(tile[tx][ty + 8 * k]));
      for (uint32_t s = 0; s < S; ++s) X[((size_t)s * N + xr) * N + xc] = v;
    }
  }
}

hipError_t launch_build_init(hipStream_t st, int precision, const void* V, void* X, int n, int S) {
  const uint32_t N = 1u << n;
  const uint32_t tiles = (N + 31) / 32;
  const dim3 grid(tiles * tiles), block(256);
  if (precision == QF_C64)
    hipLaunchKernelGGL(k_build_init<float>, grid, block, 0, st, reinterpret_cast<const cd*>(V),
                       reinterpret_cast<cf*>(X), N, (uint32_t)S);
  else
    hipLaunchKernelGGL(k_build_init<double>, grid, block, 0, st, reinterpret_cast<const cd*>(V),
                       reinterpret_cast<cd*>(X), N, (uint32_t)S);
  return hipGetLastError();
}

// ------------------------------------------------------------------ k_env

// Grid: S x nwg workgroups of kEnvThreads threads.  Thread t sums entry (i,j) = t%16
// over its rests (eight loads in flight at a time); the workgroup reduces to
// 16 FP64 sums in a fixed tree.  With nwg > 1 (n >= 15) each workgroup writes
// its 16 partials and the last one to arrive (device-scope counter) adds them
// in workgroup order.
template <typename R>
__device__ __forceinline__ void env_body(const cx<R>* __restrict__ X, const EnvDev& d, uint32_t wg) {
  __shared__ cd red[kEnvThreads];
  __shared__ cd u_sh[16], y_sh[16];
  __shared__ int last, frz;
  const uint32_t t = threadIdx.x;
  const uint32_t s = wg / d.nwg;
  const uint32_t w = wg - s * d.nwg;
  // Gate update: fetch the old gate, the frozen flag and the warm start now,
  // so their latency hides under the partial trace (the reduction's
  // barriers publish them).
  if (d.a.do_update && t < 16)
    u_sh[t] = reinterpret_cast<const cd*>(d.a.gates)[(int64_t)s * d.a.gstride + 16 * (int64_t)d.a.gidx + t];
  if (t == 16) frz = (d.a.do_update && d.a.frozen && d.a.frozen[s]) ? 1 : 0;
  if (t >= 32 && t < 48) ywarm_fetch(d.a, s, t - 32, y_sh);
  const uint32_t ij = t & 15u, i = ij >> 2, j = ij & 3u;
  const uint32_t ro = local_off(i, d.b0, d.b1), co = local_off(j, d.b0, d.b1);
  const cx<R>* Xs = X + (size_t)s * d.N * d.N;
  const uint32_t r_begin = w * d.rests_per_wg;
  const uint32_t r_end = min(d.nrest, r_begin + d.rests_per_wg);
  constexpr uint32_t kLanes = kEnvThreads / 16;
  cd acc = mk(0.0, 0.0);
  for (uint32_t r0 = r_begin + (t >> 4); r0 < r_end; r0 += 8 * kLanes) {
    cx<R> v[8];
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
      const uint32_t rest = r0 + k * kLanes;
      v[k] = mk<R>(0, 0);
      if (rest < r_end) {
        const uint32_t base = insert00(rest, d.rlo, d.rhi);
        v[k] = Xs[(size_t)(base + ro) * d.N + (base + co)];
      }
    }
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) acc = acc + mk((double)v[k].re, (double)v[k].im);
  }
  red[t] = acc;
  __syncthreads();
  for (uint32_t stride = kEnvThreads / 2; stride >= 16; stride >>= 1) {
    if (t < stride) red[t] = red[t] + red[t + stride];
    __syncthreads();
  }
  if (d.nwg == 1) {
    env_finish(d, s, red, u_sh, frz != 0, t, nullptr, y_sh);
    return;
  }
  cd* part = reinterpret_cast<cd*>(d.a.partials) + ((size_t)s * d.nwg + w) * 16;
  if (t < 16) {
    part[t] = red[t];
    __threadfence();
  }
  __syncthreads();
  if (t == 0) {
    const int old =
        __hip_atomic_fetch_add(&d.a.counters[s], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (old == (int)d.nwg - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (t < 16) {
    const cd* ps = reinterpret_cast<const cd*>(d.a.partials) + (size_t)s * d.nwg * 16;
    cd sum = mk(0.0, 0.0);
    for (uint32_t k = 0; k < d.nwg; ++k) {
      const double* q = reinterpret_cast<const double*>(&ps[k * 16 + t]);
      const double re = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const double im = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sum = sum + mk(re, im);
    }
    red[t] = sum;
  }
  __syncthreads();
  if (t == 0) __hip_atomic_store(&d.a.counters[s], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  env_finish(d, s, red, u_sh, frz != 0, t, nullptr, y_sh);
}

template <typename R>
__global__ __launch_bounds__(kEnvThreads) void k_env(const cx<R>* __restrict__ X, EnvDev d) {
  __builtin_amdgcn_s_setprio(3);  // as in k_fused: beside other groups' passes
  env_body<R>(X, d, blockIdx.x);
}

uint32_t env_min_workgroups(int n) {
  const uint32_t nrest = (1u << n) >> 2;
  return (nrest + kEnvRestsPerWG - 1) / kEnvRestsPerWG;
}

// Up to two rounds of loads stay in one workgroup per start (the last-arrival
// hand-off would cost more than the round it saves); beyond that the rests
// are spread so that each workgroup needs one round, as long as the launch
// stays within kEnvSpreadTarget workgroups (never below the minimum).
uint32_t env_workgroups(int n, int S) {
  const uint32_t nrest = (1u << n) >> 2;
  const uint32_t base = env_min_workgroups(n);
  if (nrest <= 2u * kEnvRestsPerRound) return base;
  const uint32_t one_round = (nrest + kEnvRestsPerRound - 1) / kEnvRestsPerRound;
  const uint32_t cap = S >= (int)kEnvSpreadTarget ? 1u : kEnvSpreadTarget / (uint32_t)(S < 1 ? 1 : S);
  const uint32_t spread = one_round < cap ? one_round : cap;
  return spread > base ? spread : base;
}

static EnvDev make_env_dev(const EnvArgs& a) {
  EnvDev d{};
  d.a = a;
  d.N = 1u << a.n;
  d.nrest = d.N >> 2;
  d.b0 = (uint32_t)(a.n - 1 - a.q0);
  d.b1 = (uint32_t)(a.n - 1 - a.q1);
  d.rlo = d.b0 < d.b1 ? d.b0 : d.b1;
  d.rhi = d.b0 < d.b1 ? d.b1 : d.b0;
  d.nwg = a.nwg > 0 ? (uint32_t)a.nwg : env_workgroups(a.n, a.S);
  d.rests_per_wg = (d.nrest + d.nwg - 1) / d.nwg;
  return d;
}

hipError_t launch_env(hipStream_t st, int precision, const void* X, const EnvArgs& a, KernelEvents ev) {
  const EnvDev d = make_env_dev(a);
  if (d.nwg < env_min_workgroups(a.n) || d.rests_per_wg > kEnvRestsPerWG) return hipErrorInvalidValue;
  if (d.nwg > 1 && (!a.partials || !a.counters)) return hipErrorInvalidValue;
  const dim3 grid((uint32_t)a.S * d.nwg), block(kEnvThreads);
  if (precision == QF_C64) return launch_k(k_env<float>, grid, block, 0u, st, ev, reinterpret_cast<const cf*>(X), d);
  return launch_k(k_env<double>, grid, block, 0u, st, ev, reinterpret_cast<const cd*>(X), d);
}

// ------------------------------------------------------------ k_fused
//
// One launch carrying the environment step (partial trace + FP64 update) of
// one group of starts and the two-sided pass of another group.  The two touch
// disjoint builders and gates, so their workgroups run side by side: the
// latency-bound environment workgroups (first in the grid, so dispatched
// first) sit under the HBM-bound pass, on one stream and without a
// cross-stream event.  The pass is the register-direct or the micro-tile
// form; the environment needs one workgroup per start (n <= 14).  The
// environment's waves raise their issue priority: they share SIMDs with pass
// waves that mostly wait on memory, and the launch lasts as long as its
// slower part.
template <typename R, int FORM, int B0, int B1>
__global__ __launch_bounds__(256) void k_fused(const cx<R>* Xe, EnvDev ed, uint32_t n_env, cx<R>* Xp, PassGeom g,
                                               uint32_t wgps, Operand A, Operand B) {
  if (blockIdx.x < n_env) {
    __builtin_amdgcn_s_setprio(3);
    env_body<R>(Xe, ed, blockIdx.x);
    return;
  }
  const uint32_t wg = blockIdx.x - n_env;
  if constexpr (FORM == 1 && sizeof(R) == 4)
    pass_micro_body<B0, B1, true, true>(Xp, g.n, wgps, A, B, wg);
  else
    pass_block_body<R, true, true>(Xp, g, wgps, A, B, wg);
}

bool fused_supported(int precision, int n, const PassGeom& g) {
  if (env_min_workgroups(n) != 1) return false;
  if (g.micro) return precision == QF_C64;
  return g.direct != 0;
}

template <typename R, int FORM, int B0, int B1>
static hipError_t launch_fused_t(hipStream_t st, const void* Xe, const EnvDev& d, uint32_t n_env, void* Xp, int Sp,
                                 const PassGeom& g, uint32_t wgps, Operand A, Operand B) {
  const dim3 grid(n_env + (uint32_t)Sp * wgps), block(256);
  hipLaunchKernelGGL((k_fused<R, FORM, B0, B1>), grid, block, 0, st, reinterpret_cast<const cx<R>*>(Xe), d, n_env,
                     reinterpret_cast<cx<R>*>(Xp), g, wgps, A, B);
  return hipGetLastError();
}

hipError_t launch_fused(hipStream_t st, int precision, const void* Xe, const EnvArgs& ea, void* Xp, int Sp,
                        const PassGeom& g, Operand A, Operand B) {
  EnvArgs one = ea;
  one.nwg = 1;  // the fused launch keeps each start's environment in one workgroup
  const EnvDev d = make_env_dev(one);
  if (d.rests_per_wg > kEnvRestsPerWG || !ea.do_update || !A.ptr || !B.ptr) return hipErrorInvalidValue;
  const uint32_t n_env = (uint32_t)ea.S;
  if (g.micro) {
    if (precision != QF_C64 || (reinterpret_cast<uintptr_t>(Xp) & 15u) != 0) return hipErrorInvalidValue;
    const uint32_t wgps = g.N * g.N / 8192u;
    switch (g.b0 * 3 + g.b1) {
      case 0 * 3 + 1: return launch_fused_t<float, 1, 0, 1>(st, Xe, d, n_env, Xp, Sp, g, wgps, A, B);
      case 0 * 3 + 2: return launch_fused_t<float, 1, 0, 2>(st, Xe, d, n_env, Xp, Sp, g, wgps, A, B);
      case 1 * 3 + 0: return launch_fused_t<float, 1, 1, 0>(st, Xe, d, n_env, Xp, Sp, g, wgps, A, B);
      case 1 * 3 + 2: return launch_fused_t<float, 1, 1, 2>(st, Xe, d, n_env, Xp, Sp, g, wgps, A, B);
      case 2 * 3 + 0: return launch_fused_t<float, 1, 2, 0>(st, Xe, d, n_env, Xp, Sp, g, wgps, A, B);
      case 2 * 3 + 1: return launch_fused_t<float, 1, 2, 1>(st, Xe, d, n_env, Xp, Sp, g, wgps, A, B);
      default: return hipErrorInvalidValue;
    }
  }
  if (!g.direct) return hipErrorInvalidValue;
  const uint32_t wgps = g.N * g.N / 4096u;
  if (precision == QF_C64) return launch_fused_t<float, 0, 0, 0>(st, Xe, d, n_env, Xp, Sp, g, wgps, A, B);
  return launch_fused_t<double, 0, 0, 0>(st, Xe, d, n_env, Xp, Sp, g, wgps, A, B);
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

hipError_t launch_fill_i32(hipStream_t st, int32_t* p, int32_t v, uint32_t count) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((count + 255) / 256), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}

// ------------------------------------------------------------------ k_cost

template <typename R>
__global__ __launch_bounds__(256) void k_cost(const cx<R>* __restrict__ X, uint32_t N, double* cost,
                                              double* trace) {
  __shared__ cd red[256];
  const uint32_t t = threadIdx.x, s = blockIdx.x;
  const cx<R>* Xs = X + (size_t)s * N * N;
  cd acc = mk(0.0, 0.0);
  for (uint32_t r0 = 0; r0 < N; r0 += 256u * 8u) {
    cx<R> v[8];
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
      const uint32_t r = r0 + t + 256u * k;
      v[k] = r < N ? Xs[(size_t)r * N + r] : mk<R>(0, 0);  // scalar-pair load, no array select
    }
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) acc = acc + mk((double)v[k].re, (double)v[k].im);
  }
  red[t] = acc;
  __syncthreads();
  for (uint32_t stride = 128; stride >= 1; stride >>= 1) {
    if (t < stride) red[t] = red[t] + red[t + stride];
    __syncthreads();
  }
  if (t == 0) {
    const cd tr = red[0];
    if (trace) {
      trace[2 * s] = tr.re;
      trace[2 * s + 1] = tr.im;
    }
    cost[s] = 1.0 - sqrt(norm2(tr)) / (double)N;
  }
}

hipError_t launch_cost(hipStream_t st, int precision, const void* X, int n, int S, double* cost,
                       double* trace) {
  const uint32_t N = 1u << n;
  if (precision == QF_C64)
    hipLaunchKernelGGL(k_cost<float>, dim3(S), dim3(256), 0, st, reinterpret_cast<const cf*>(X), N,
                       cost, trace);
  else
    hipLaunchKernelGGL(k_cost<double>, dim3(S), dim3(256), 0, st, reinterpret_cast<const cd*>(X), N,
                       cost, trace);
  return hipGetLastError();
}

// ------------------------------------------------------------------ k_optimize

// Sixteen lanes (one hex) per environment: lane i owns entry
// (hex_row(i), i & 3).
__global__ __launch_bounds__(64) void k_optimize(int count, const cd* __restrict__ env,
                                                 const cd* __restrict__ uold, double beta,
                                                 cd* __restrict__ unew) {
  __shared__ cd xch[64];  // the update's lane exchange, 16 entries per hex of the block
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = gt >> 4, i = gt & 15;
  if (s >= count) return;  // whole hexes leave together
  const int r = hex_row(i), c = i & 3;
  const cd* u = uold + 16 * (size_t)s;
  cd un;
  optimize_gate_f64_hex(env[16 * (size_t)s + 4 * r + c], u[4 * c + r], u[4 * r + c], r, c, beta, un,
                        xch + 16 * (threadIdx.x >> 4));
  unew[16 * (size_t)s + 4 * r + c] = un;
}

hipError_t launch_optimize(hipStream_t st, int count, const double* env, const double* uold,
                           double beta, double* unew) {
  const int threads = 64;
  const long long lanes = 16ll * count;
  hipLaunchKernelGGL(k_optimize, dim3((unsigned)((lanes + threads - 1) / threads)), dim3(threads), 0, st,
                     count, reinterpret_cast<const cd*>(env), reinterpret_cast<const cd*>(uold), beta,
                     reinterpret_cast<cd*>(unew));
  return hipGetLastError();
}

}  // namespace qf
