// Two consecutive gate updates of a sweep (Alg. 1, TwoSidedSweep) with one
// partial trace and one pass over the builder.
//
// Let F be updated first and S second, U the union of their qubits (3 or 4
// qubits) and X the builder before F's update.  In the first half of a
// sweep F's update is X' = (u_F^dagger (x) I) X (u_F' (x) I); every operator
// on U commutes with the partial trace over the qubits outside U, so with
// T = Tr_{rest U} X (a 2^|U| x 2^|U| matrix):
//   P_F = Tr_{U \ F} T                                 (F's partial trace)
//   P_S = Tr_{U \ S} [(u_F^dagger)_U T (u_F')_U]       (S's, after F's update)
// (second half: (u_F')_U T (u_F^dagger)_U).  So one gather of T gives both
// environments, the two FP64 updates run back to back, and the builder takes
// both updates in one pass: X'' = (A_S A_F (x) I) X (B_F B_S (x) I), applied
// block by block as F's two-sided 4x4 update followed by S's.  Every update
// sees the environment it sees in Alg. 1; only the summation order differs.
//
//   k_env2   T in FP64 (gathered by several workgroups per start, whose
//            partial sums the last to arrive adds in a fixed order), then
//            F's and S's gate updates
//   k_pass2  the pass: LDS tiles of 2^|U| rows x 2^|U| W columns, loaded and
//            stored in address order, F's then S's 4x4 block updates on the
//            tile in LDS (complex64 on the matrix cores); each workgroup
//            walks several tiles with the next tile's loads in flight under
//            the current tile's products
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qf_device.h"
#include "qf_env_finish.h"
#include "qf_internal.h"
#include "qf_pair_geom.h"

namespace qf {

// ------------------------------------------------------------------ k_pass2

// Tile shape per (builder precision, union size M): 4^M W entries, 32 KiB of
// builder data plus one pad entry per (row, column variant) of LDS; memory
// phases move 16-byte units (two complex64 entries or one complex128), 8 per
// thread; in a product phase a thread owns one 4x4 block of the gate.
template <typename R, int M>
struct Pair2Cfg {
  static constexpr uint32_t kWlog = (sizeof(R) == 4 ? 4u : 3u) + (M == 3 ? 2u : 0u);
  static constexpr uint32_t kW = 1u << kWlog;
  static constexpr uint32_t kEpu = sizeof(R) == 4 ? 2u : 1u;   // entries per 16-byte unit
  static constexpr uint32_t kUprLog = M == 4 ? 7u : 8u;         // units per tile row, log2
  static constexpr uint32_t kRowStep = 256u >> kUprLog;        // rows between a thread's units
  static constexpr uint32_t kRowStride = (1u << M) * (kW + 1u);
  static constexpr uint32_t kLds = (1u << M) * kRowStride;     // entries
  static constexpr uint32_t kActive = 1u << (kWlog + 2u * (M - 2u));  // threads owning a block
};
static_assert(Pair2Cfg<float, 4>::kActive == 256 && Pair2Cfg<float, 3>::kActive == 256, "one block per thread");
static_assert(Pair2Cfg<double, 4>::kActive == 128 && Pair2Cfg<double, 3>::kActive == 128, "one block per thread");
static_assert((1u << 4) * (1u << Pair2Cfg<float, 4>::kUprLog) == 2048u, "8 units per thread");
static_assert((1u << 3) * (1u << Pair2Cfg<float, 3>::kUprLog) == 2048u, "8 units per thread");

uint32_t pair2_wlog(int precision, int m) {
  if (precision == QF_C64) return m == 4 ? Pair2Cfg<float, 4>::kWlog : Pair2Cfg<float, 3>::kWlog;
  return m == 4 ? Pair2Cfg<double, 4>::kWlog : Pair2Cfg<double, 3>::kWlog;
}

// One gate's two-sided 4x4 block update on the LDS tile: x <- A x B for the
// block of thread t (rows and columns varying in the gate's two union
// indices gi, the other union bits and the rest column offset fixed by t).
template <typename R, int M>
__device__ __forceinline__ void pair2_phase(cx<R>* tile, const Pair2Geom& g, const uint32_t gi[2],
                                            const uint32_t oi[2], const cx<R>* __restrict__ a,
                                            const cx<R>* __restrict__ b, uint32_t t) {
  using C = Pair2Cfg<R, M>;
  // Recomputed in every phase rather than kept across the tile loop: the
  // sixteen LDS addresses would otherwise be hoisted out of it and spilled.
  __asm__ volatile("" : "+v"(t));
  const uint32_t w = t & (C::kW - 1u);
  const uint32_t orow = (t >> C::kWlog) & ((1u << (M - 2)) - 1u);
  const uint32_t ocol = t >> (C::kWlog + M - 2);
  const uint32_t vr = var_other(orow, oi, M), vc = var_other(ocol, oi, M);
  uint32_t ar[4], ac[4];
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) {
    ar[i] = (var_local(i, gi[0], gi[1]) | vr) * C::kRowStride;
    ac[i] = (var_local(i, gi[0], gi[1]) | vc) * (C::kW + 1u) + w;
  }
  cx<R> x[16];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) x[4 * i + j] = tile[ar[i] + ac[j]];
#pragma unroll
  for (int j = 0; j < 4; ++j) {  // x <- A x
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
  __asm__ volatile("" ::: "memory");  // B's scalar loads after A's products: half the registers
#pragma unroll
  for (int i = 0; i < 4; ++i) {  // x <- x B
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
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) tile[ar[i] + ac[j]] = x[4 * i + j];
}

typedef float v4f __attribute__((ext_vector_type(4)));

// complex64 two-sided 4x4 block update x <- A x B on the matrix cores, x in
// registers (entry (i, j) in x[4 i + j]), every lane of the wavefront owning
// a block.  v_mfma_f32_4x4x1f32 runs sixteen independent 4 x 4 x 1 products
// per wavefront: in block b = lane / 4, lane 4 b + r supplies row r of the
// 4 x 1 left factor, lane 4 b + c column c of the 1 x 4 right factor, and
// lane 4 b + c receives column c of the 4 x 4 result (entry i in
// accumulator i).  So every lane's own 4-vector is one column: with lane
// (lane % 4 = q) supplying row q of the gate matrix, four k-steps give M v
// for each lane's vector v.  Real and imaginary parts take two accumulators
// (Re y = Re M Re v - Im M Im v, Im y = Re M Im v + Im M Re v: sixteen
// products per vector).  The block update is four such products for A x
// (the block's columns) and four for x B = (B^T x^T)^T (its rows): the same
// arithmetic as the vector form at twice its rate, off the vector ALUs.
__device__ __forceinline__ void block_update_mfma(cf (&x)[16], const cf* __restrict__ a, const cf* __restrict__ b,
                                                  uint32_t t) {
  const uint32_t q = t & 3u;
  float mr[4], mi[4], mn[4];
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {  // row q of A
    const cf v = a[4u * q + k];
    mr[k] = v.re;
    mi[k] = v.im;
    mn[k] = -v.im;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    v4f yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      yr = __builtin_amdgcn_mfma_f32_4x4x1f32(mr[k], x[4 * k + j].re, yr, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f32_4x4x1f32(mr[k], x[4 * k + j].im, yi, 0, 0, 0);
      yr = __builtin_amdgcn_mfma_f32_4x4x1f32(mn[k], x[4 * k + j].im, yr, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f32_4x4x1f32(mi[k], x[4 * k + j].re, yi, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) x[4 * i + j] = cf{yr[i], yi[i]};
  }
  __asm__ volatile("" ::: "memory");  // B's loads after A's products: fewer live registers
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {  // row q of B^T
    const cf v = b[4u * k + q];
    mr[k] = v.re;
    mi[k] = v.im;
    mn[k] = -v.im;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v4f yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      yr = __builtin_amdgcn_mfma_f32_4x4x1f32(mr[l], x[4 * i + l].re, yr, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f32_4x4x1f32(mr[l], x[4 * i + l].im, yi, 0, 0, 0);
      yr = __builtin_amdgcn_mfma_f32_4x4x1f32(mn[l], x[4 * i + l].im, yr, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f32_4x4x1f32(mi[l], x[4 * i + l].re, yi, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) x[4 * i + j] = cf{yr[j], yi[j]};
  }
}

// complex64 form of pair2_phase: the block from the LDS tile, its update on
// the matrix cores (every thread of the workgroup owns a block), and back.
template <int M>
__device__ __forceinline__ void pair2_phase_mfma(cf* tile, const Pair2Geom& g, const uint32_t gi[2],
                                                 const uint32_t oi[2], const cf* __restrict__ a,
                                                 const cf* __restrict__ b, uint32_t t) {
  using C = Pair2Cfg<float, M>;
  static_assert(C::kActive == 256, "every thread owns a block");
  __asm__ volatile("" : "+v"(t));
  const uint32_t w = t & (C::kW - 1u);
  const uint32_t orow = (t >> C::kWlog) & ((1u << (M - 2)) - 1u);
  const uint32_t ocol = t >> (C::kWlog + M - 2);
  const uint32_t vr = var_other(orow, oi, M), vc = var_other(ocol, oi, M);
  uint32_t ar[4], ac[4];
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) {
    ar[i] = (var_local(i, gi[0], gi[1]) | vr) * C::kRowStride;
    ac[i] = (var_local(i, gi[0], gi[1]) | vc) * (C::kW + 1u) + w;
  }
  cf x[16];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) x[4 * i + j] = tile[ar[i] + ac[j]];
  block_update_mfma(x, a, b, t);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) tile[ar[i] + ac[j]] = x[4 * i + j];
}

// 16-byte unit of the memory phases: two complex64 entries or one complex128.
template <typename R>
struct Unit16T;
template <>
struct Unit16T<float> {
  using type = float4;
};
template <>
struct Unit16T<double> {
  using type = double2;
};

// The tile loop shared by the two-gate pass and the three-qubit pass: each
// workgroup walks tiles wg, wg + n_wg, ... < total; a tile's 16-byte units
// are loaded in address order (8 per thread) and scattered into the LDS
// image, the next tile's loads go out, P::run applies the products on the
// image, and the units are gathered and stored in address order.  P::init
// runs once before the first tile's loads (the two-gate pass stages its
// operands in LDS there); P::prep(s) runs before the barrier that publishes
// the image (the three-qubit pass's operands of start s into LDS).  Nothing
// between the next tile's loads and its scatter waits on a global load:
// vector memory loads and stores share one counter, so such a wait would
// also wait for the next tile's loads in flight.
template <typename R, int M, typename P>
__device__ __forceinline__ void tile_loop(cx<R>* __restrict__ X, const Pair2Geom& g, uint32_t total, uint32_t wg,
                                          uint32_t n_wg, cx<R>* tile, P& prod) {
  using C = Pair2Cfg<R, M>;
  using Unit16 = typename Unit16T<R>::type;
  const uint32_t t = threadIdx.x;
  const uint32_t N = g.N;
  // This thread's memory-order unit: the same column set in every row it
  // moves (rows a0, a0 + kRowStep, ...).
  const uint32_t ku = t & ((1u << C::kUprLog) - 1u);
  const uint32_t a0 = t >> C::kUprLog;
  const uint32_t k = ku * C::kEpu;
  const uint32_t colk = dep_free(g, k);
  const uint32_t lk0 = lds_of_k(g, k);
  const uint32_t lk1 = C::kEpu == 2 ? lds_of_k(g, k + 1) : 0u;
  // Row of unit jj: a0 + jj * kRowStep, whose bits split into the thread's
  // a0 (below kRowStep) and a workgroup-uniform part, so its element offset
  // is the thread's part plus a scalar.
  const uint32_t row_t = dep_union(g, a0) * N;
  uint32_t row_u[8];
#pragma unroll
  for (uint32_t jj = 0; jj < 8; ++jj) row_u[jj] = __builtin_amdgcn_readfirstlane(dep_union(g, jj * C::kRowStep) * N);

  auto tile_origin = [&](uint32_t tl, uint32_t& s, size_t& origin) {
    s = tl / g.tiles_per_start;
    const uint32_t rem = tl - s * g.tiles_per_start;
    const uint32_t rq = rem / g.col_tiles;
    const uint32_t ct = rem - rq * g.col_tiles;
    origin = (size_t)s * N * N + (size_t)dep_rest(g, rq) * N + dep_rest(g, ct << g.wlog);
  };
  Unit16 buf[8];
  auto load_tile = [&](size_t origin) {
    const Unit16* src = reinterpret_cast<const Unit16*>(X + origin + colk) + row_t / C::kEpu;
#pragma unroll
    for (uint32_t jj = 0; jj < 8; ++jj) buf[jj] = src[row_u[jj] / C::kEpu];
  };

  uint32_t tl = wg;
  if (tl >= total) return;
  prod.init(wg, n_wg, total);
  uint32_t s;
  size_t origin;
  tile_origin(tl, s, origin);
  load_tile(origin);
  while (true) {
    // scatter the tile's units into LDS
#pragma unroll
    for (uint32_t jj = 0; jj < 8; ++jj) {
      const uint32_t base = (a0 + jj * C::kRowStep) * C::kRowStride;
      if constexpr (C::kEpu == 2) {
        const float4 u = buf[jj];
        tile[base + lk0] = cx<R>{u.x, u.y};
        tile[base + lk1] = cx<R>{u.z, u.w};
      } else {
        const double2 u = buf[jj];
        tile[base + lk0] = cx<R>{u.x, u.y};
      }
    }
    prod.prep(s);
    __syncthreads();
    // next tile's loads go out now and land under this tile's products
    const uint32_t next = tl + n_wg;
    uint32_t s_next = s;
    size_t origin_next = origin;
    if (next < total) {
      tile_origin(next, s_next, origin_next);
      load_tile(origin_next);
    }
    prod.run(s);
    __syncthreads();
    // gather in address order and store
    Unit16* dst = reinterpret_cast<Unit16*>(X + origin + colk) + row_t / C::kEpu;
#pragma unroll
    for (uint32_t jj = 0; jj < 8; ++jj) {
      const uint32_t base = (a0 + jj * C::kRowStep) * C::kRowStride;
      Unit16 u;
      if constexpr (C::kEpu == 2) {
        const cx<R> lo = tile[base + lk0], hi = tile[base + lk1];
        u = Unit16{lo.re, lo.im, hi.re, hi.im};
      } else {
        const cx<R> v = tile[base + lk0];
        u = Unit16{v.re, v.im};
      }
      dst[row_u[jj] / C::kEpu] = u;
    }
    if (next >= total) break;
    __syncthreads();  // the tile's LDS is rewritten next
    tl = next;
    s = s_next;
    origin = origin_next;
  }
}

// Two-gate products.  ops: per start the four 4x4 operands A_F, B_F, A_S,
// B_S in the builder precision (64 entries, written by k_env2):
// x <- A_S A_F x B_F B_S.
constexpr uint32_t kPass2OpSlots = 8;  // tiles per workgroup whose operands are staged in LDS
template <typename R, int M>
struct Pair2Products {
  cx<R>* tile;
  const Pair2Geom& g;
  const cx<R>* __restrict__ ops;
  cx<R>* opl;     // complex64: kPass2OpSlots x 64 operand entries in LDS, one slot per tile of the workgroup
  uint32_t slot;  // slot of the current tile
  // complex64: the operands of every tile this workgroup walks, staged in LDS
  // at the start (their loads go out with the first tile's), so that the
  // products read LDS and wait on no global load, which would also wait for
  // the next tile's loads in flight
  __device__ __forceinline__ void init(uint32_t wg, uint32_t n_wg, uint32_t total) {
    if constexpr (sizeof(R) == 4) {
      for (uint32_t q = threadIdx.x; q < kPass2OpSlots * 64; q += 256) {
        const uint32_t tl = wg + (q >> 6) * n_wg;
        if (tl < total) opl[q] = ops[(size_t)(tl / g.tiles_per_start) * 64 + (q & 63u)];
      }
    }
  }
  __device__ __forceinline__ void prep(uint32_t) {}
  __device__ __forceinline__ void run(uint32_t s) {
    using C = Pair2Cfg<R, M>;
    const uint32_t t = threadIdx.x;
    if constexpr (sizeof(R) == 4) {
      const cx<R>* op = opl + 64 * slot;
      ++slot;
      pair2_phase_mfma<M>(tile, g, g.f_idx, g.o_f, op, op + 16, t);
      __syncthreads();
      pair2_phase_mfma<M>(tile, g, g.s_idx, g.o_s, op + 32, op + 48, t);
    } else {
      const cx<R>* op = ops + (size_t)__builtin_amdgcn_readfirstlane(s) * 64;
      if (t < C::kActive) pair2_phase<R, M>(tile, g, g.f_idx, g.o_f, op, op + 16, t);
      __syncthreads();
      if (t < C::kActive) pair2_phase<R, M>(tile, g, g.s_idx, g.o_s, op + 32, op + 48, t);
    }
  }
};

template <typename R, int M>
__global__ __launch_bounds__(256, 4) void k_pass2(cx<R>* __restrict__ X, Pair2Geom g, uint32_t total,
                                                  const cx<R>* __restrict__ ops) {
  __shared__ cx<R> tile[Pair2Cfg<R, M>::kLds];
  __shared__ cx<R> opl[sizeof(R) == 4 ? kPass2OpSlots * 64 : 1];
  Pair2Products<R, M> prod{tile, g, ops, opl, 0u};
  tile_loop<R, M>(X, g, total, blockIdx.x, gridDim.x, tile, prod);
}

// Tiles per workgroup of the two-gate pass (each workgroup walks this many
// tiles, the next one's loads in flight under the current one's products)
// unless the caller passes its own (the runtime tunes it per precision and
// n).
constexpr uint32_t kPass2TilesPerWG = 2;

template <typename R, int M>
static hipError_t launch_pass2_t(hipStream_t st, void* X, int S, const Pair2Geom& g, const void* ops,
                                 KernelEvents ev) {
  if (g.wlog != Pair2Cfg<R, M>::kWlog || g.m != (uint32_t)M) return hipErrorInvalidValue;
  const uint32_t total = (uint32_t)S * g.tiles_per_start;
  const uint32_t tpw = g.tiles_per_wg ? g.tiles_per_wg : kPass2TilesPerWG;
  if (sizeof(R) == 4 && tpw > kPass2OpSlots) return hipErrorInvalidValue;
  const uint32_t grid = (total + tpw - 1) / tpw;
  return launch_k(k_pass2<R, M>, dim3(grid), dim3(256), 0u, st, ev, reinterpret_cast<cx<R>*>(X), g, total,
                  reinterpret_cast<const cx<R>*>(ops));
}

hipError_t launch_pass2(hipStream_t st, int precision, void* X, int S, const Pair2Geom& g, const void* ops,
                        KernelEvents ev) {
  if (!ops || (reinterpret_cast<uintptr_t>(X) & 15u) != 0) return hipErrorInvalidValue;
  if (precision == QF_C64)
    return g.m == 4 ? launch_pass2_t<float, 4>(st, X, S, g, ops, ev) : launch_pass2_t<float, 3>(st, X, S, g, ops, ev);
  return g.m == 4 ? launch_pass2_t<double, 4>(st, X, S, g, ops, ev) : launch_pass2_t<double, 3>(st, X, S, g, ops, ev);
}

// ------------------------------------------------------------------ k_pass3
//
// One three-qubit gate's two-sided update X <- (A (x) I) X (B (x) I) on the
// same tiles (the union is the gate's three qubits: 8 row variants x 8 column
// variants x W rest columns, W = 64 for complex64 and 32 for complex128, 32
// KiB of builder data).  The operands, rounded to the builder precision and
// permuted to variant order (entry (a, b) = M[local(a)][local(b)]), go to
// LDS once per tile.  The left product takes the tile's columns (v, w) as
// vectors over the row variant, the right product its rows (a, w) as vectors
// over the column variant.

// Entry (r, k) of the real 16 x 16 form [[Mr, -Mi], [Mi, Mr]] of an 8 x 8
// complex matrix M (rows and columns 0..7 real parts, 8..15 imaginary), with
// M(a, b) = src[8 a + b], or src[8 b + a] when T.
template <bool T>
__device__ __forceinline__ float real16_of(const cf* src, uint32_t r, uint32_t k) {
  const uint32_t a = r & 7u, b = k & 7u;
  const cf m = src[T ? 8u * b + a : 8u * a + b];
  if (r < 8u) return k < 8u ? m.re : -m.im;
  return k < 8u ? m.im : m.re;
}

// complex64: y = M x for the tile's 512 vectors on v_mfma_f32_16x16x4f32,
// the real contraction [Re y; Im y] = M16 [Re x; Im x] (A operand 16 x 4:
// lane l holds row l % 16, column l / 16; B operand 4 x 16: lane l holds row
// l / 16, column l % 16; result: lane l holds rows 4 (l / 16) .. + 3 of
// column l % 16), four k-steps per 16 vectors.  Wavefront v takes vectors
// 128 v .. 128 v + 127; a vector's entries are read and written by its own
// wavefront only, so the update in place needs no barrier.  LEFT: M = A on
// the columns; otherwise M = B^T on the rows.
template <bool LEFT>
__device__ __forceinline__ void pass3_products_mfma(cf* tile, const cf* M, uint32_t t) {
  using C = Pair2Cfg<float, 3>;
  constexpr uint32_t W = C::kW, RS = C::kRowStride;
  static_assert(W == 64, "512 vectors per side");
  const uint32_t l = t & 63u, wv = t >> 6, g = l >> 4, cl = l & 15u;
  float am[4];
#pragma unroll
  for (uint32_t ks = 0; ks < 4; ++ks) am[ks] = real16_of<!LEFT>(M, cl, 4u * ks + g);
  float* tf = reinterpret_cast<float*>(tile);
#pragma unroll 2
  for (uint32_t q = 0; q < 8; ++q) {
    const uint32_t vec = (wv * 8u + q) * 16u + cl;  // 0..511
    const uint32_t hi = vec >> 6, w = vec & (W - 1u);  // LEFT: column variant; else row variant
    auto at = [&](uint32_t c) -> uint32_t {
      return LEFT ? c * RS + hi * (W + 1u) + w : hi * RS + c * (W + 1u) + w;
    };
    // k-row 4 ks + g of the vector: Re x_g, Re x_{4+g}, Im x_g, Im x_{4+g}
    const cf x0 = tile[at(g)], x1 = tile[at(4u + g)];
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(am[0], x0.re, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(am[1], x1.re, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(am[2], x0.im, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(am[3], x1.im, acc, 0, 0, 0);
#pragma unroll
    for (uint32_t v = 0; v < 4; ++v) {
      const uint32_t r = 4u * g + v;  // < 8: Re y_r, else Im y_{r-8}
      tf[2u * at(r & 7u) + (r >> 3)] = acc[v];
    }
  }
}

// complex128: vector FP64 products, one vector per thread (256 per side).
template <bool LEFT>
__device__ __forceinline__ void pass3_products_vec(cd* tile, const cd* M, uint32_t t) {
  using C = Pair2Cfg<double, 3>;
  constexpr uint32_t W = C::kW, RS = C::kRowStride;
  static_assert(W == 32, "256 vectors per side");
  const uint32_t hi = t >> 5, w = t & (W - 1u);
  auto at = [&](uint32_t c) -> uint32_t { return LEFT ? c * RS + hi * (W + 1u) + w : hi * RS + c * (W + 1u) + w; };
  cd x[8];
#pragma unroll
  for (uint32_t c = 0; c < 8; ++c) x[c] = tile[at(c)];
#pragma unroll
  for (uint32_t i = 0; i < 8; ++i) {
    cd acc = mk(0.0, 0.0);
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) cmac(acc, LEFT ? M[8 * i + k] : M[8 * k + i], x[k]);
    tile[at(i)] = acc;
  }
}

template <typename R, bool HA, bool HB>
struct Pass3Products {
  cx<R>* tile;
  cx<R>* As;
  cx<R>* Bs;
  const Pair2Geom& g;
  Operand A, B;
  uint32_t s_have;
  __device__ __forceinline__ void init(uint32_t, uint32_t, uint32_t) {}
  // operands of start s in variant order, once per start
  __device__ __forceinline__ void prep(uint32_t s) {
    if (s == s_have) return;
    s_have = s;
    const uint32_t t = threadIdx.x;
    if (t < 128) {
      const bool left = t < 64;
      const Operand& o = left ? A : B;
      if ((left && HA) || (!left && HB)) {
        const uint32_t e = t & 63u;
        const uint32_t r = k3_local(g, e >> 3), c = k3_local(g, e & 7u);
        const cd* src = reinterpret_cast<const cd*>(o.ptr) + (int64_t)s * o.stride;
        const cd v = o.dagger ? conj(src[8 * c + r]) : src[8 * r + c];
        (left ? As : Bs)[e] = cx<R>{(R)v.re, (R)v.im};
      }
    }
  }
  __device__ __forceinline__ void run(uint32_t) {
    const uint32_t t = threadIdx.x;
    if constexpr (sizeof(R) == 4) {
      if (HA) pass3_products_mfma<true>(tile, As, t);
      if (HA && HB) __syncthreads();
      if (HB) pass3_products_mfma<false>(tile, Bs, t);
    } else {
      if (HA) pass3_products_vec<true>(tile, As, t);
      if (HA && HB) __syncthreads();
      if (HB) pass3_products_vec<false>(tile, Bs, t);
    }
  }
};

template <typename R, bool HA, bool HB>
__global__ __launch_bounds__(256, 4) void k_pass3(cx<R>* __restrict__ X, Pair2Geom g, uint32_t total, Operand A,
                                                  Operand B) {
  __shared__ cx<R> tile[Pair2Cfg<R, 3>::kLds];
  __shared__ cx<R> As[64], Bs[64];
  Pass3Products<R, HA, HB> prod{tile, As, Bs, g, A, B, 0xffffffffu};
  tile_loop<R, 3>(X, g, total, blockIdx.x, gridDim.x, tile, prod);
}

// Tiles per workgroup of the three-qubit pass (n = 10, 8 starts, two-sided:
// complex64 33.2 / 27.6 / 30.1 us and complex128 54.6 / 48.4 / 45.2 us for
// 1 / 2 / 4 tiles per workgroup).
template <typename R>
constexpr uint32_t kPass3TilesPerWG = sizeof(R) == 4 ? 2u : 4u;

template <typename R>
static hipError_t launch_pass3_t(hipStream_t st, void* X, int S, const Pair2Geom& g, Operand A, Operand B) {
  if (g.wlog != Pair2Cfg<R, 3>::kWlog || g.m != 3u) return hipErrorInvalidValue;
  const uint32_t total = (uint32_t)S * g.tiles_per_start;
  const uint32_t tpw = g.tiles_per_wg ? g.tiles_per_wg : kPass3TilesPerWG<R>;
  const dim3 grid((total + tpw - 1) / tpw), block(256);
  cx<R>* x = reinterpret_cast<cx<R>*>(X);
  if (A.ptr && B.ptr) return launch_k(k_pass3<R, true, true>, grid, block, 0u, st, KernelEvents{}, x, g, total, A, B);
  if (A.ptr) return launch_k(k_pass3<R, true, false>, grid, block, 0u, st, KernelEvents{}, x, g, total, A, B);
  if (B.ptr) return launch_k(k_pass3<R, false, true>, grid, block, 0u, st, KernelEvents{}, x, g, total, A, B);
  return hipSuccess;
}

hipError_t launch_pass3(hipStream_t st, int precision, void* X, int S, const Pair2Geom& g, Operand A, Operand B) {
  if ((reinterpret_cast<uintptr_t>(X) & 15u) != 0) return hipErrorInvalidValue;
  return precision == QF_C64 ? launch_pass3_t<float>(st, X, S, g, A, B) : launch_pass3_t<double>(st, X, S, g, A, B);
}

// ------------------------------------------------------------------ k_env2

constexpr uint32_t kEnv2Threads = 256;
constexpr uint32_t kEnv2Loads = 16;  // loads in flight per thread and round

struct Env2Dev {
  Pair2Geom g;
  EnvDev dF, dS;             // per-gate update arguments (gates, kinds, u_old slots, half, beta)
  void* ops;                 // per start 64 builder-precision entries: A_F, B_F, A_S, B_S
  const int32_t* frozen;
  double* partials;          // c128, per start nwg x 4^M partial sums (nwg > 1)
  int32_t* counters;         // per start, zero before the launch; left zero
  uint32_t nrest, nwg, rests_per_wg;
};

// Workgroups per start of the gather of T.  The gather reads 4^M entries per
// rest, often one cache line each, so one workgroup per start leaves it to a
// few CUs' load bandwidth; it is spread so that a launch has about 128
// workgroups (at most 16 per start, whose partial sums the last one to
// arrive adds), and so that no workgroup needs more than four rounds of
// loads.  (n = 10, 16 starts: 2, 4, 8, 12 and 16 workgroups per start gave
// 4458, 4855, 4896, 4744 and 4581 start-sweeps/s; one 512-thread workgroup
// with the whole gather in one round, 4410.)  (Each extra workgroup costs a device-scope release, an L2
// write-back, which is why the spread stays small and why the launch that
// runs beside another group's pass keeps one workgroup per start.)
static uint32_t env2_lanes(int m) { return kEnv2Threads >> (2 * m); }
uint32_t env2_workgroups(int n, int m, int S) {
  const uint32_t lanes = env2_lanes(m);
  const uint32_t per_lane = ((1u << n) >> m) / lanes;   // rests per lane with one workgroup
  const uint32_t rounds4 = (per_lane + 4 * kEnv2Loads - 1) / (4 * kEnv2Loads);
  const uint32_t spread = std::min(16u, std::max(1u, 128u / (uint32_t)std::max(1, S)));
  return std::max(1u, std::min(per_lane, std::max(rounds4, spread)));
}
uint32_t env2_workgroups_cap(int n) {
  return std::max(std::max(env2_workgroups(n, 3, 1), env2_workgroups(n, 4, 1)), 1u);
}

template <typename R, int M>
__device__ __forceinline__ void env2_body(const cx<R>* __restrict__ X, const Env2Dev& d, uint32_t wg) {
  constexpr uint32_t E = 1u << (2 * M);  // entries of T
  constexpr uint32_t V = 1u << M;        // variants per side
  constexpr uint32_t LP = kEnv2Threads / E;
  static_assert(LP >= 1, "one thread per entry at least");
  __shared__ cd red[kEnv2Threads];
  __shared__ cd uF[16], uS[16], unF[16], unS[16], P[16], yF[16], yS[16];
  __shared__ cd Msh[16 << (M - 2)];
  __shared__ int last, frz;
  const Pair2Geom& g = d.g;
  const uint32_t t = threadIdx.x;
  const uint32_t s = wg / d.nwg;
  const uint32_t w = wg - s * d.nwg;
  const EnvArgs& aF = d.dF.a;
  const EnvArgs& aS = d.dS.a;
  // old gates and the frozen flag, fetched under the gather
  if (t < 16)
    uF[t] = reinterpret_cast<const cd*>(aF.gates)[(int64_t)s * aF.gstride + 16 * (int64_t)aF.gidx + t];
  else if (t < 32)
    uS[t - 16] = reinterpret_cast<const cd*>(aS.gates)[(int64_t)s * aS.gstride + 16 * (int64_t)aS.gidx + t - 16];
  else if (t == 32)
    frz = (d.frozen && d.frozen[s]) ? 1 : 0;
  else if (t >= 64 && t < 80)
    ywarm_fetch(aF, s, t - 64, yF);
  else if (t >= 80 && t < 96)
    ywarm_fetch(aS, s, t - 80, yS);
  // T[a][b] = sum over rests r of X[(r, a), (r, b)]
  const uint32_t e = t & (E - 1u), lane = t / E;
  const uint32_t ro = dep_union(g, e / V), co = dep_union(g, e & (V - 1u));
  const cx<R>* Xs = X + (size_t)s * g.N * g.N;
  const uint32_t r_begin = w * d.rests_per_wg;
  const uint32_t r_end = min(d.nrest, r_begin + d.rests_per_wg);
  cd acc = mk(0.0, 0.0);
  for (uint32_t r0 = r_begin + lane; r0 < r_end; r0 += kEnv2Loads * LP) {
    cx<R> v[kEnv2Loads];
#pragma unroll
    for (uint32_t kk = 0; kk < kEnv2Loads; ++kk) {
      const uint32_t rest = r0 + kk * LP;
      v[kk] = mk<R>(0, 0);
      if (rest < r_end) {
        const uint32_t base = dep_rest(g, rest);
        v[kk] = Xs[(size_t)(base | ro) * g.N + (base | co)];
      }
    }
#pragma unroll
    for (uint32_t kk = 0; kk < kEnv2Loads; ++kk) acc = acc + mk((double)v[kk].re, (double)v[kk].im);
  }
  red[t] = acc;
  __syncthreads();
  for (uint32_t stride = kEnv2Threads / 2; stride >= E; stride >>= 1) {
    if (t < stride) red[t] = red[t] + red[t + stride];
    __syncthreads();
  }
  if (d.nwg > 1) {
    // Hand-off to the last workgroup of the start: the partial sums are
    // stored, the workgroup's barrier orders them before thread 0's
    // release at device scope (one L2 write-back per workgroup), and only
    // the last to arrive acquires (one invalidate), then reads them with
    // device-scope loads.
    cd* part = reinterpret_cast<cd*>(d.partials) + ((size_t)s * d.nwg + w) * E;
    if (t < E) part[t] = red[t];
    __syncthreads();
    if (t == 0) {
      const int old = __hip_atomic_fetch_add(&d.counters[s], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      last = (old == (int)d.nwg - 1);
      if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (!last) return;
    if (t < E) {
      const cd* ps = reinterpret_cast<const cd*>(d.partials) + (size_t)s * d.nwg * E;
      cd sum = mk(0.0, 0.0);
      for (uint32_t kk = 0; kk < d.nwg; ++kk) {
        const double* q = reinterpret_cast<const double*>(&ps[kk * E + t]);
        const double re = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double im = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sum = sum + mk(re, im);
      }
      red[t] = sum;
    }
    __syncthreads();
    if (t == 0) __hip_atomic_store(&d.counters[s], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  const cd* T = red;
  // F's partial trace: P_F[i][j] = sum over the variants o of U \ F of
  // T[(F = i, o), (F = j, o)]
  if (t < 16) {
    const uint32_t i = t >> 2, j = t & 3u;
    cd sum = mk(0.0, 0.0);
    for (uint32_t o = 0; o < (1u << (M - 2)); ++o) {
      const uint32_t vo = var_other(o, g.o_f, M);
      sum = sum + T[(var_local(i, g.f_idx[0], g.f_idx[1]) | vo) * V + (var_local(j, g.f_idx[0], g.f_idx[1]) | vo)];
    }
    P[t] = sum;
  }
  __syncthreads();
  env_finish(d.dF, s, P, uF, frz != 0, t, unF, yF);
  __syncthreads();
  // S's partial trace after F's update: P_S = Tr_{U\S}[A_F T B_F] with
  // (A_F, B_F) = (u_F^dagger, u_F') in the first half, (u_F', u_F^dagger) in
  // the second (A_F acts on the row variant's F bits, B_F on the column's).
  if (t < (16u << (M - 2))) {
    const uint32_t o = t >> 4, i = (t >> 2) & 3u, j = t & 3u;
    const uint32_t vo = var_other(o, g.o_s, M);
    const uint32_t ra = var_local(i, g.s_idx[0], g.s_idx[1]) | vo;
    const uint32_t cb = var_local(j, g.s_idx[0], g.s_idx[1]) | vo;
    const uint32_t fmask = (1u << g.f_idx[0]) | (1u << g.f_idx[1]);
    const uint32_t xa = (((ra >> g.f_idx[0]) & 1u) << 1) | ((ra >> g.f_idx[1]) & 1u);  // F-local row of ra
    const uint32_t yb = (((cb >> g.f_idx[0]) & 1u) << 1) | ((cb >> g.f_idx[1]) & 1u);  // F-local column of cb
    const bool h0 = aF.half == 0;
    cd sum = mk(0.0, 0.0);
#pragma unroll
    for (uint32_t kk = 0; kk < 4; ++kk) {
      const uint32_t rk = (ra & ~fmask) | var_local(kk, g.f_idx[0], g.f_idx[1]);
      cd inner = mk(0.0, 0.0);
#pragma unroll
      for (uint32_t l = 0; l < 4; ++l) {
        const uint32_t cl = (cb & ~fmask) | var_local(l, g.f_idx[0], g.f_idx[1]);
        const cd bfl = h0 ? unF[4 * l + yb] : conj(uF[4 * yb + l]);
        cmac(inner, T[rk * V + cl], bfl);
      }
      const cd afk = h0 ? conj(uF[4 * kk + xa]) : unF[4 * xa + kk];
      cmac(sum, afk, inner);
    }
    Msh[t] = sum;
  }
  __syncthreads();
  if (t < 16) {
    cd sum = mk(0.0, 0.0);
    for (uint32_t o = 0; o < (1u << (M - 2)); ++o) sum = sum + Msh[(o << 4) | t];
    P[t] = sum;
  }
  __syncthreads();
  env_finish(d.dS, s, P, uS, frz != 0, t, unS, yS);
  __syncthreads();
  // the pass's operands: (A, B) = (u^dagger, u') per gate in the first half,
  // (u', u^dagger) in the second; x <- A_S A_F x B_F B_S
  if (t < 64) {
    const uint32_t which = t >> 4, r = (t >> 2) & 3u, c = t & 3u;
    const cd* uo = which < 2 ? uF : uS;
    const cd* un = which < 2 ? unF : unS;
    const bool dag = (which & 1u) == (aF.half == 0 ? 0u : 1u);
    const cd v = dag ? conj(uo[4 * c + r]) : un[4 * r + c];
    reinterpret_cast<cx<R>*>(d.ops)[(size_t)s * 64 + t] = cx<R>{(R)v.re, (R)v.im};
  }
}

// The environment's waves raise their issue priority: with stream groups
// they share SIMDs with other groups' pass waves, and the two FP64 updates
// are a chain of dependent instructions (measured 4450 -> 4565
// start-sweeps/s at n = 10, 16 starts).
template <typename R, int M>
__global__ __launch_bounds__(kEnv2Threads) void k_env2(const cx<R>* __restrict__ X, Env2Dev d) {
  __builtin_amdgcn_s_setprio(3);
  env2_body<R, M>(X, d, blockIdx.x);
}

static hipError_t make_env2_dev(const Env2Args& a, Env2Dev& d) {
  d = Env2Dev{};
  d.g = a.geom;
  const int M = (int)a.geom.m;
  if (M != 3 && M != 4) return hipErrorInvalidValue;
  d.dF.a = a.F;
  d.dS.a = a.S;
  d.dF.a.do_update = d.dS.a.do_update = 1;
  d.dF.a.env_out = d.dS.a.env_out = nullptr;
  d.frozen = a.frozen;
  d.ops = a.ops;
  d.partials = a.partials;
  d.counters = a.counters;
  d.nrest = a.geom.N >> M;
  d.nwg = a.nwg > 0 ? (uint32_t)a.nwg : env2_workgroups((int)a.geom.n, M, a.n_starts);
  if (d.nwg > env2_workgroups_cap((int)a.geom.n) || d.nwg > d.nrest) return hipErrorInvalidValue;
  d.rests_per_wg = (d.nrest + d.nwg - 1) / d.nwg;
  if (!a.ops || !a.counters) return hipErrorInvalidValue;
  if (d.nwg > 1 && !a.partials) return hipErrorInvalidValue;
  return hipSuccess;
}

hipError_t launch_env2(hipStream_t st, int precision, const void* X, const Env2Args& a, KernelEvents ev) {
  Env2Dev d;
  const hipError_t e = make_env2_dev(a, d);
  if (e != hipSuccess) return e;
  const dim3 grid((uint32_t)a.n_starts * d.nwg), block(kEnv2Threads);
  if (precision == QF_C64)
    return d.g.m == 4 ? launch_k(k_env2<float, 4>, grid, block, 0u, st, ev, reinterpret_cast<const cf*>(X), d)
                      : launch_k(k_env2<float, 3>, grid, block, 0u, st, ev, reinterpret_cast<const cf*>(X), d);
  return d.g.m == 4 ? launch_k(k_env2<double, 4>, grid, block, 0u, st, ev, reinterpret_cast<const cd*>(X), d)
                    : launch_k(k_env2<double, 3>, grid, block, 0u, st, ev, reinterpret_cast<const cd*>(X), d);
}

}  // namespace qf
