// Three-qubit gates: the instantiation sweep for circuits whose gates are
// 8 x 8 unitaries on three qubits (the method is stated for gates of any
// size, Sec. III; the k = 3 gate-set variant of Sec. III-A-3).
//
//   k_pass8      X <- (A (x) I) X (B (x) I) for an 8 x 8 gate: LDS tile of the
//                eight rows that differ in the gate's bits times the eight
//                column variants of up to 32 column groups; the left product
//                runs one column per thread, the right product one row per
//                thread, both on the tile.
//   k_env8       P = Tr_rest X (8 x 8, FP64 sums, one workgroup per start),
//                E = u_old^dagger P or P u_old^dagger, and the FP64 update of
//                Eq. opt_u on one wavefront (lane r + 8c = entry (r, c)).
//   k_optimize8  the same update for a batch of given environments.
#include <hip/hip_runtime.h>

#include "qf_device.h"
#include "qf_internal.h"

namespace qf {

// Offset of local index i (0..7) for a gate whose local bits, most
// significant first, sit at bit positions b[0], b[1], b[2] (Q1).
__device__ __forceinline__ uint32_t local_off8(uint32_t i, const uint32_t b[3]) {
  return (((i >> 2) & 1u) << b[0]) | (((i >> 1) & 1u) << b[1]) | ((i & 1u) << b[2]);
}
// Insert zero bits at the ascending positions s[0] < s[1] < s[2].
__device__ __forceinline__ uint32_t insert000(uint32_t v, const uint32_t s[3]) {
  return insert0(insert0(insert0(v, s[0]), s[1]), s[2]);
}

Pass8Geom make_pass8_geom(int n, const int32_t loc[3]) {
  Pass8Geom g{};
  g.n = (uint32_t)n;
  g.N = 1u << n;
  for (int t = 0; t < 3; ++t) g.b[t] = (uint32_t)(n - 1 - loc[t]);
  uint32_t s0 = g.b[0], s1 = g.b[1], s2 = g.b[2], tmp;
  if (s0 > s1) { tmp = s0; s0 = s1; s1 = tmp; }
  if (s1 > s2) { tmp = s1; s1 = s2; s2 = tmp; }
  if (s0 > s1) { tmp = s0; s0 = s1; s1 = tmp; }
  g.s[0] = s0;
  g.s[1] = s1;
  g.s[2] = s2;
  const uint32_t groups = g.N >> 3;  // column groups (base columns with the gate's bits zero)
  g.W = groups < 32u ? groups : 32u;
  g.wlog = 0;
  while ((1u << g.wlog) < g.W) ++g.wlog;
  g.col_tiles = groups >> g.wlog;
  g.tiles_per_start = groups * g.col_tiles;
  // the two-gate pass's tiles, whose union is this gate's three qubits
  const int32_t f[2] = {loc[0], loc[1]}, sg[2] = {loc[1], loc[2]};
  for (int ti = 0; ti < 2; ++ti)
    g.tg_ok[ti] = make_pair2_geom(n, f, sg, pair2_wlog(ti == 0 ? QF_C64 : QF_C128, 3), g.tg[ti]) ? 1 : 0;
  return g;
}

// ------------------------------------------------------------------ k_pass8

typedef float v4f __attribute__((ext_vector_type(4)));

// Entry (r, k) of the real 16 x 16 form [[Mr, -Mi], [Mi, Mr]] of an 8 x 8
// complex matrix M (rows and columns 0..7 real parts, 8..15 imaginary), with
// M(a, b) = src[8 a + b], or src[8 b + a] when T.
template <bool T>
__device__ __forceinline__ float real16(const cf* src, uint32_t r, uint32_t k) {
  const uint32_t a = r & 7u, b = k & 7u;
  const cf m = src[T ? 8u * b + a : 8u * a + b];
  if (r < 8u) return k < 8u ? m.re : -m.im;
  return k < 8u ? m.im : m.re;
}

// Matrix-core form of one product over a complex64 tile of W = 32 column
// groups: y = M x for the tile's 256 vectors x, in place.  LEFT: the vectors
// are the columns (j, w) and M = A (entry i of a vector is tile entry
// (i, j, w)); otherwise the rows (i, w) and M = B^T (entry j is (i, j, w)).
// Each product is the real contraction [Re y; Im y] = M16 [Re x; Im x] on
// v_mfma_f32_16x16x4f32 (A operand 16 x 4: lane l holds row l % 16, column
// l / 16; B operand 4 x 16: lane l holds row l / 16, column l % 16; result:
// lane l holds rows 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16), four
// k-steps of four.  Wavefront v takes vectors 64 v .. 64 v + 63, sixteen per
// MFMA tile; a vector's entries are read and written by its own wavefront
// only, so the update in place needs no barrier.  Sums run in the matrix
// core's order, so the result differs from the vector form's in rounding only.
template <bool LEFT>
__device__ __forceinline__ void tile_products_mfma(cf* tile, const cf* M, uint32_t t) {
  const uint32_t l = t & 63u, wv = t >> 6, g = l >> 4, cl = l & 15u;
  float am[4];
#pragma unroll
  for (uint32_t ks = 0; ks < 4; ++ks) am[ks] = real16<!LEFT>(M, cl, 4u * ks + g);
  float* tf = reinterpret_cast<float*>(tile);
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    const uint32_t vec = (wv * 4u + q) * 16u + cl;  // 0..255
    const uint32_t hi = vec >> 5, w = vec & 31u;     // LEFT: column variant j; else row i
    auto at = [&](uint32_t c) -> uint32_t { return (LEFT ? ((c * 8u + hi) << 5) : ((hi * 8u + c) << 5)) + w; };
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

// Grid: S x tiles_per_start workgroups of 256 threads.  Tile entry
// ((i * 8 + j) * W + w) holds row rb + off(i), column cb_w + off(j); the
// loads and stores run w fastest, so a wavefront touches W consecutive
// column groups of one (row, column variant).  complex64 at W = 32 (n >= 8)
// takes the pipelined form below instead.
template <typename R, bool HA, bool HB>
__global__ __launch_bounds__(256) void k_pass8(cx<R>* __restrict__ X, Pass8Geom g, Operand A, Operand B) {
  __shared__ cx<R> tile[64 * 32];
  __shared__ cx<R> As[64], Bs[64];
  const uint32_t t = threadIdx.x;
  const uint32_t s = blockIdx.x / g.tiles_per_start;
  const uint32_t rem = blockIdx.x - s * g.tiles_per_start;
  const uint32_t rgi = rem / g.col_tiles, cti = rem - rgi * g.col_tiles;
  const uint32_t rb = insert000(rgi, g.s);
  const uint32_t W = g.W, wlog = g.wlog, nel = 64u << wlog;
  cx<R>* Xs = X + (size_t)s * g.N * g.N;
  if (HA && t < 64) {
    const cd* src = reinterpret_cast<const cd*>(A.ptr) + (int64_t)s * A.stride;
    const uint32_t r = t >> 3, c = t & 7u;
    const cd v = A.dagger ? conj(src[8 * c + r]) : src[8 * r + c];
    As[t] = cx<R>{(R)v.re, (R)v.im};
  }
  if (HB && t >= 64 && t < 128) {
    const cd* src = reinterpret_cast<const cd*>(B.ptr) + (int64_t)s * B.stride;
    const uint32_t r = (t - 64) >> 3, c = (t - 64) & 7u;
    const cd v = B.dagger ? conj(src[8 * c + r]) : src[8 * r + c];
    Bs[t - 64] = cx<R>{(R)v.re, (R)v.im};
  }
  for (uint32_t e = t; e < nel; e += 256u) {
    const uint32_t w = e & (W - 1u), ij = e >> wlog, i = ij >> 3, j = ij & 7u;
    const uint32_t cb = insert000((cti << wlog) + w, g.s);
    tile[e] = Xs[(size_t)(rb + local_off8(i, g.b)) * g.N + cb + local_off8(j, g.b)];
  }
  __syncthreads();
  if (HA && t < (8u << wlog)) {  // one column (variant j of group w): x <- A x
    const uint32_t j = t >> wlog, w = t & (W - 1u);
    cx<R> x[8], y[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = tile[(((uint32_t)i * 8u + j) << wlog) + w];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      cx<R> acc = mk<R>(0, 0);
#pragma unroll
      for (int k = 0; k < 8; ++k) cmac(acc, As[8 * i + k], x[k]);
      y[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) tile[(((uint32_t)i * 8u + j) << wlog) + w] = y[i];
  }
  __syncthreads();
  if (HB && t < (8u << wlog)) {  // one row (i of group w): x <- x B
    const uint32_t i = t >> wlog, w = t & (W - 1u);
    cx<R> x[8], y[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = tile[((i * 8u + (uint32_t)j) << wlog) + w];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      cx<R> acc = mk<R>(0, 0);
#pragma unroll
      for (int l = 0; l < 8; ++l) cmac(acc, x[l], Bs[8 * l + j]);
      y[j] = acc;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) tile[((i * 8u + (uint32_t)j) << wlog) + w] = y[j];
  }
  __syncthreads();
  for (uint32_t e = t; e < nel; e += 256u) {
    const uint32_t w = e & (W - 1u), ij = e >> wlog, i = ij >> 3, j = ij & 7u;
    const uint32_t cb = insert000((cti << wlog) + w, g.s);
    Xs[(size_t)(rb + local_off8(i, g.b)) * g.N + cb + local_off8(j, g.b)] = tile[e];
  }
}

// Complex64, W = 32 (n >= 8), software-pipelined: a workgroup walks tiles
// blockIdx.x, blockIdx.x + gridDim.x, ... and issues the loads of its next
// tile (eight entries per thread, held in registers) before it multiplies
// and stores the current one, so their latency runs under that work.  Tiles
// are those of k_pass8; every entry is read and written once; the products
// run on the matrix cores.
constexpr uint32_t kPass8PipeGrid = 2048;
template <bool HA, bool HB>
__global__ __launch_bounds__(256) void k_pass8_pipe(cf* __restrict__ X, Pass8Geom g, Operand A, Operand B,
                                                    uint32_t total) {
  __shared__ cf tile[64 * 32];
  __shared__ cf As[64], Bs[64];
  const uint32_t t = threadIdx.x;
  auto entry = [&](uint32_t tl, uint32_t e) -> size_t {  // offset of tile entry e of tile tl
    const uint32_t s = tl / g.tiles_per_start;
    const uint32_t rem = tl - s * g.tiles_per_start;
    const uint32_t rgi = rem / g.col_tiles, cti = rem - rgi * g.col_tiles;
    const uint32_t w = e & 31u, ij = e >> 5, i = ij >> 3, j = ij & 7u;
    const uint32_t rb = insert000(rgi, g.s), cb = insert000((cti << 5) + w, g.s);
    return (size_t)s * g.N * g.N + (size_t)(rb + local_off8(i, g.b)) * g.N + cb + local_off8(j, g.b);
  };
  cf pre[8];
  uint32_t tl = blockIdx.x;
#pragma unroll
  for (uint32_t k = 0; k < 8; ++k) pre[k] = X[entry(tl, t + 256u * k)];
  for (; tl < total; tl += gridDim.x) {
    const uint32_t s = tl / g.tiles_per_start;
    __syncthreads();  // the previous tile's stores have read the LDS tile
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) tile[t + 256u * k] = pre[k];
    if (HA && t < 64) {
      const cd* src = reinterpret_cast<const cd*>(A.ptr) + (int64_t)s * A.stride;
      const uint32_t r = t >> 3, c = t & 7u;
      const cd v = A.dagger ? conj(src[8 * c + r]) : src[8 * r + c];
      As[t] = cf{(float)v.re, (float)v.im};
    }
    if (HB && t >= 64 && t < 128) {
      const cd* src = reinterpret_cast<const cd*>(B.ptr) + (int64_t)s * B.stride;
      const uint32_t r = (t - 64) >> 3, c = (t - 64) & 7u;
      const cd v = B.dagger ? conj(src[8 * c + r]) : src[8 * r + c];
      Bs[t - 64] = cf{(float)v.re, (float)v.im};
    }
    const uint32_t nx = tl + gridDim.x;
    if (nx < total) {
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k) pre[k] = X[entry(nx, t + 256u * k)];
    }
    __syncthreads();
    if (HA) tile_products_mfma<true>(tile, As, t);
    __syncthreads();
    if (HB) tile_products_mfma<false>(tile, Bs, t);
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) X[entry(tl, t + 256u * k)] = tile[t + 256u * k];
  }
}

template <typename R>
static hipError_t launch_pass8_t(hipStream_t st, void* X, int S, const Pass8Geom& g, Operand A, Operand B) {
  const dim3 grid((uint32_t)S * g.tiles_per_start), block(256);
  cx<R>* x = reinterpret_cast<cx<R>*>(X);
  if (A.ptr && B.ptr)
    hipLaunchKernelGGL((k_pass8<R, true, true>), grid, block, 0, st, x, g, A, B);
  else if (A.ptr)
    hipLaunchKernelGGL((k_pass8<R, true, false>), grid, block, 0, st, x, g, A, B);
  else if (B.ptr)
    hipLaunchKernelGGL((k_pass8<R, false, true>), grid, block, 0, st, x, g, A, B);
  else
    return hipSuccess;
  return hipGetLastError();
}

static hipError_t launch_pass8_pipe(hipStream_t st, void* X, int S, const Pass8Geom& g, Operand A, Operand B) {
  const uint32_t total = (uint32_t)S * g.tiles_per_start;
  const dim3 grid(total < kPass8PipeGrid ? total : kPass8PipeGrid), block(256);
  cf* x = reinterpret_cast<cf*>(X);
  if (A.ptr && B.ptr)
    hipLaunchKernelGGL((k_pass8_pipe<true, true>), grid, block, 0, st, x, g, A, B, total);
  else if (A.ptr)
    hipLaunchKernelGGL((k_pass8_pipe<true, false>), grid, block, 0, st, x, g, A, B, total);
  else if (B.ptr)
    hipLaunchKernelGGL((k_pass8_pipe<false, true>), grid, block, 0, st, x, g, A, B, total);
  else
    return hipSuccess;
  return hipGetLastError();
}

hipError_t launch_pass8(hipStream_t st, int precision, void* X, int S, const Pass8Geom& g, Operand A, Operand B) {
  // Where the two-gate pass's tiles fit (n >= 9 for complex64, n >= 8 for
  // complex128), the gate runs on them (k_pass3: address-order 16-byte
  // loads and stores, the next tile's loads under the current one's
  // products).
  const int ti = precision == QF_C64 ? 0 : 1;
  if (g.tg_ok[ti]) return launch_pass3(st, precision, X, S, g.tg[ti], A, B);
  // complex128 keeps k_pass8 also at W = 32: a pipelined form with vector
  // FP64 products (34 KiB of LDS, four workgroups per CU) was measured
  // slower, 83 against 54 us at n = 10, 8 starts.
  const bool w32 = g.W == 32u && g.wlog == 5u;  // n >= 8
  if (precision == QF_C64) {
    if (w32) return launch_pass8_pipe(st, X, S, g, A, B);
    return launch_pass8_t<float>(st, X, S, g, A, B);
  }
  return launch_pass8_t<double>(st, X, S, g, A, B);
}

// ------------------------------------------------- FP64 update, 8 x 8 (oct form)
//
// The one-sided Jacobi step of the 4 x 4 forms (jacobi_params / jacobi_apply,
// rank tolerance kRankTol2) on the 64 lanes of a wavefront: lane r + 8c holds
// entry (r, c) of M and of the accumulated rotation Y.  A sweep is seven
// rounds; in round K column c pairs with c ^ K (every pair once per sweep,
// four disjoint pairs per round, all at once on different lanes).  A column
// sum is a butterfly over the three low lane bits (rows), by DPP moves within
// each group of eight lanes, so every lane of a column gets bitwise the same
// sum; the partner column is lane ^ 8K: a DPP row rotation for K = 1, a
// swizzle within 32 lanes for K = 2, 3, a permute across the halves for K >= 4.

// lane ^ 4 within each group of eight: mirror the eight (lane ^ 7), then
// quad_perm [3,2,1,0] (lane ^ 3).
__device__ __forceinline__ double dpp_xor4(double v) { return dpp_quad<kQuadXor3>(dpp_quad<0x141>(v)); }
// lane ^ XM within each half of the wavefront (ds_swizzle bit-mask mode).
template <int XM>
__device__ __forceinline__ double swz_xor(double v) {
  constexpr int pat = 0x1F | (XM << 10);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)b, pat);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), pat);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
// lane ^ 8K (partner column of round K)
template <int K>
__device__ __forceinline__ double col_xor(double v) {
  if constexpr (K == 1) return dpp_quad<kRowRor8>(v);
  else if constexpr (K < 4) return swz_xor<8 * K>(v);
  else return __shfl_xor(v, 8 * K, 64);
}
template <int K>
__device__ __forceinline__ cd col_xor_cd(cd v) {
  return mk(col_xor<K>(v.re), col_xor<K>(v.im));
}
__device__ __forceinline__ cd shfl_cd(cd v, int src) { return mk(__shfl(v.re, src, 64), __shfl(v.im, src, 64)); }
__device__ __forceinline__ double oct_colsum(double v) {  // over the 8 rows of this lane's column
  v += dpp_quad<kQuadXor1>(v);
  v += dpp_quad<kQuadXor2>(v);
  return v + dpp_xor4(v);
}
__device__ __forceinline__ double oct_rowmax(double v) {  // over the 8 columns of this lane's row
  v = fmax(v, dpp_quad<kRowRor8>(v));
  v = fmax(v, swz_xor<16>(v));
  return fmax(v, __shfl_xor(v, 32, 64));
}
__device__ __forceinline__ double oct_wavemax(double v) {
  v = fmax(v, dpp_quad<kQuadXor1>(v));
  v = fmax(v, dpp_quad<kQuadXor2>(v));
  v = fmax(v, dpp_xor4(v));
  return oct_rowmax(v);
}

template <int K>
__device__ __forceinline__ double oct_round(cd& m, cd& y, int c) {
  const bool pside = c < (c ^ K);
  const cd mo = col_xor_cd<K>(m);
  const cd yo = col_xor_cd<K>(y);
  const cd mP = sel(pside, m, mo), mQ = sel(pside, mo, m);
  const double na = oct_colsum(nrm2x(m));
  const cd gl = cjmulx(mP, mQ);
  const cd g = mk(oct_colsum(gl.re), oct_colsum(gl.im));
  const double nb = col_xor<K>(na);
  JacobiRot j;
  if (!jacobi_params(pside ? na : nb, pside ? nb : na, g, j)) return 0.0;
  cd np, nq;
  jacobi_apply(j, mP, mQ, np, nq);
  m = sel(pside, np, nq);
  jacobi_apply(j, sel(pside, y, yo), sel(pside, yo, y), np, nq);
  y = sel(pside, np, nq);
  return j.large;
}

// Sum over the 64 lanes; bitwise the same in every lane (each level adds a
// pair of lanes that differ in one bit, so the two see the same operands).
__device__ __forceinline__ double oct_wavesum(double v) {
  v += dpp_quad<kQuadXor1>(v);
  v += dpp_quad<kQuadXor2>(v);
  v += dpp_xor4(v);
  v += dpp_quad<kRowRor8>(v);
  v += swz_xor<16>(v);
  return v + __shfl_xor(v, 32, 64);
}
// A wave-uniform lane's value (lane in an SGPR).
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// Newton form of the 8 x 8 nearest-unitary step: the unitary polar factor Q
// of M (M = Q H) by the scaled Newton iteration of the hex form (Higham 1986;
// X <- (z X + X^{-dagger} / z) / 2, z = (|X^-1|_F / |X|_F)^(1/2)) while X is
// far from unitary, and by the Newton-Schulz iteration X <- X (3 I - X^dagger
// X) / 2 once |X^dagger X - I|_F < 1/2 (Higham's hybrid; there every singular
// value s has |s^2 - 1| < 1/2, and the step maps s^2 - 1 = d to (d^3 - 3 d^2)
// / 4, quadratic convergence with two matrix products and no inverse).  X
// starts at M scaled to |X|_F^2 = 8.  Newton steps take X^-1 from
// Gauss-Jordan elimination with partial pivoting on [X | I] across the
// wavefront: in step k the pivot row p_k is the unused row of largest
// |X[r][k]|, every other row (used or not) loses its column-k component, and
// no rows are swapped, so X^-1[k][c] is entry (p_k, c) of the right half.
// The Newton-Schulz step taken at |X^dagger X - I|_F <= 1e-8 is the last
// (after it every |s - 1| is near 1e-16).  The first Newton step checks
// |M|_F^2 |M^-1|_F^2 < 1e8 (the pivoted elimination is accurate to about the
// condition number times the unit roundoff); an ill-conditioned M, a
// vanishing pivot or 16 steps without convergence return false for the
// Jacobi form.  All decisions are on wave-uniform values.  x: entry (r, c)
// of M (entries at most 1 in magnitude), lane r + 8c; q: entry (r, c) of Q.
// xs: 128 entries of LDS owned by this wavefront, through which the lanes
// exchange entries (each lane stores its own at its lane index and loads
// the ones it needs, one 16-byte load per entry instead of four lane
// permutes).  Only this wavefront touches xs, and a wavefront's LDS
// instructions execute in issue order, so loads issued after the stores see
// them and the next stores cannot overtake them; the wave barriers keep the
// compiler from moving the accesses across.
constexpr double kPolar8Cond2 = 1e8;
constexpr double kPolar8SchulzBelow = 0.25;  // |X^dagger X - I|_F^2
constexpr double kPolar8Done = 1e-16;        // |X^dagger X - I|_F^2 of the last step
constexpr int kPolar8MaxSteps = 16;

__device__ inline bool polar_newton_oct(cd x, int r, int c, cd& q, cd* xs) {
  const int grp = 8 * c;  // first lane of this lane's column group
  const int t = r + 8 * c;
  cd* bs = xs + 64;
  x = scale(x, rsqrt_nr(oct_wavesum(nrm2x(x)) * 0.125));
  bool checked = false;
  for (int step = 0; step < kPolar8MaxSteps; ++step) {
    // G = X^dagger X: G[r][c] = sum_k conj(X[k][r]) X[k][c]
    __builtin_amdgcn_wave_barrier();
    xs[t] = x;
    __builtin_amdgcn_wave_barrier();
    cd g = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 8; ++k) cmac(g, conj(xs[k + 8 * r]), xs[grp + k]);
    const double off = nrm2x(mk(g.re - (r == c ? 1.0 : 0.0), g.im));
    const double g2 = oct_wavesum(off);
    if (g2 < kPolar8SchulzBelow) {
      // X <- X H, H = (3 I - G) / 2: entry (r, c) = sum_k X[r][k] H[k][c]
      const cd h = mk((r == c ? 1.5 : 0.0) - 0.5 * g.re, -0.5 * g.im);
      bs[t] = h;
      __builtin_amdgcn_wave_barrier();
      cd y = mk(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 8; ++k) cmac(y, xs[r + 8 * k], bs[grp + k]);
      x = y;
      if (g2 <= kPolar8Done) {
        q = x;
        return true;
      }
      continue;
    }
    cd a = x, b = mk(r == c ? 1.0 : 0.0, 0.0);
    int piv[8];
    unsigned used = 0;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      __builtin_amdgcn_wave_barrier();
      xs[t] = a;
      bs[t] = b;
      __builtin_amdgcn_wave_barrier();
      const cd col = xs[r + 8 * k];  // entry (r, k) of the left half
      const double mag = ((used >> r) & 1u) ? -1.0 : nrm2x(col);
      // the largest over the eight rows (every group holds the same column),
      // then the lowest row that attains it, from group 0's ballot bits
      double mx = fmax(mag, dpp_quad<kQuadXor1>(mag));
      mx = fmax(mx, dpp_quad<kQuadXor2>(mx));
      mx = fmax(mx, dpp_xor4(mx));
      const unsigned long long hit = __ballot(mag == mx) & 0xFFull;
      if (hit == 0) {  // a non-finite column
        ok = false;
        break;
      }
      const int p = __builtin_ctzll(hit);
      const cd pv = mk(readlane_d(col.re, p), readlane_d(col.im, p));
      const double pv2 = nrm2x(pv);
      if (!(pv2 > 1e-280)) {
        ok = false;
        break;
      }
      const double ip = rcp_nr(pv2);
      const cd inv = mk(pv.re * ip, -(pv.im * ip));  // 1 / pv
      const cd pa = mulx(xs[grp + p], inv);
      const cd pb = mulx(bs[grp + p], inv);
      const bool prow = r == p;
      const cd ua = a - mulx(col, pa), ub = b - mulx(col, pb);
      a = sel(prow, pa, ua);
      b = sel(prow, pb, ub);
      used |= 1u << p;
      piv[k] = p;
    }
    if (!ok) return false;
    int pc = piv[0];  // pivot row of column c
#pragma unroll
    for (int j = 1; j < 8; ++j) pc = (c == j) ? piv[j] : pc;
    __builtin_amdgcn_wave_barrier();
    bs[t] = b;
    __builtin_amdgcn_wave_barrier();
    const cd xi = conj(bs[pc + 8 * r]);  // X^{-dagger}[r][c] = conj(X^-1[c][r])
    const double nx = oct_wavesum(nrm2x(x));
    const double nxi = oct_wavesum(nrm2x(b));
    if (!checked && !(nx * nxi < kPolar8Cond2)) return false;
    checked = true;
    // z = (nxi / nx)^(1/4) and 1 / z from hardware estimates (any positive
    // scaling keeps the limit)
    const double t = __builtin_amdgcn_rsq(nxi * __builtin_amdgcn_rcp(nx));
    const double z = __builtin_amdgcn_rsq(t), zi = t * z;
    const double hz = 0.5 * z, hzi = 0.5 * zi;
    x = mk(fma(hz, x.re, hzi * xi.re), fma(hz, x.im, hzi * xi.im));
  }
  return false;
}

// m: entry (r, c) of M (overwritten); keep: entry (r, c) of the result for a
// zero M.  Result entry (r, c) of the maximiser of Re Tr(M u); codes as the
// 4 x 4 forms (0 computed, 1 zero M, 2 non-finite M).  All 64 lanes active,
// lane = r + 8c.  The Newton form runs first; the one-sided Jacobi step where
// it declines.  y_io / warm: the warm start of the hex form's Jacobi step
// (entry (r, c) of the gate's previous rotation in, the new one out; the
// identity after a Newton update and after a zero or non-finite M).
__device__ inline int nearest_unitary_f64_oct(cd& m, cd keep, int r, int c, cd& unew, cd* xs, cd* y_io = nullptr,
                                              bool warm = false) {
  const double amax = oct_wavemax(fmax(fabs(m.re), fabs(m.im)));
  const double bad = oct_wavemax((finite_d(m.re) && finite_d(m.im)) ? 0.0 : 1.0);
  if (bad != 0.0 || !(amax >= 1e-300)) {
    if (y_io) *y_io = mk(c == r ? 1.0 : 0.0, 0.0);
    if (bad != 0.0) {
      const double nan = __builtin_nan("");
      unew = mk(nan, nan);
      return 2;
    }
    unew = keep;
    return 1;
  }
  m = scale(m, rcp_nr(amax));
  cd y = mk(c == r ? 1.0 : 0.0, 0.0);
  {
    cd q;
    if (polar_newton_oct(m, r, c, q, xs)) {
      if (y_io) *y_io = y;
      unew = conj(shfl_cd(q, c + 8 * r));  // u_new[r][c] = conj(Q[c][r])
      return 0;
    }
  }
  if (y_io && warm) {
    // M <- M Y: row r of M from lanes r + 8k, column c of Y from lanes k + 8c
    y = *y_io;
    cd acc = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 8; ++k) cmac(acc, shfl_cd(m, r + 8 * k), shfl_cd(y, k + 8 * c));
    m = acc;
  }
  for (int sweep = 0; sweep < 30; ++sweep) {
    double rel = oct_round<1>(m, y, c);
    rel = fmax(rel, oct_round<2>(m, y, c));
    rel = fmax(rel, oct_round<3>(m, y, c));
    rel = fmax(rel, oct_round<4>(m, y, c));
    rel = fmax(rel, oct_round<5>(m, y, c));
    rel = fmax(rel, oct_round<6>(m, y, c));
    rel = fmax(rel, oct_round<7>(m, y, c));
    if (!(oct_rowmax(rel) > 0.0)) break;
  }
  const double sig2 = oct_colsum(nrm2x(m));
  const double smax2 = oct_rowmax(sig2);
  const bool acc = sig2 > smax2 * kRankTol2;
  double accv[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) accv[j] = __shfl(acc ? 1.0 : 0.0, r + 8 * j, 64);
  cd x = sel(acc, scale(m, rsqrt_nr(acc ? sig2 : 1.0)), mk(0.0, 0.0));  // X[r][c]
  bool singular = false;
#pragma unroll
  for (int j = 0; j < 8; ++j) singular = singular || accv[j] == 0.0;
  if (singular) {
    // Gram-Schmidt of e_0..e_7 against the accepted columns; lane (r, c)
    // computes component r, alike for every c.  A complement of dimension
    // >= 1 leaves some e_k with squared norm >= 1/8 after projection.
    for (int j = 0; j < 8; ++j) {
      if (accv[j] == 0.0) {
        bool found = false;
        cd xj = mk(0.0, 0.0);
        for (int k = 0; k < 8; ++k) {
          cd v = mk(r == k ? 1.0 : 0.0, 0.0);
          for (int jj = 0; jj < 8; ++jj) {
            if (accv[jj] != 0.0) {
              const cd xjj = shfl_cd(x, r + 8 * jj);
              const cd pr = cjmulx(xjj, v);
              const cd d = mk(oct_colsum(pr.re), oct_colsum(pr.im));
              v = v - mulx(xjj, d);
            }
          }
          const double nv = oct_colsum(nrm2x(v));
          const bool take = !found && nv >= 0.125;
          if (take) xj = scale(v, rsqrt_nr(nv));
          found = found || take;
        }
        if (c == j) x = xj;
        accv[j] = 1.0;
      }
    }
  }
  // u_new[r][c] = sum_j Y[r][j] conj(X[c][j])
  cd a = mk(0.0, 0.0);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const cd yrj = shfl_cd(y, r + 8 * j);
    const cd xcj = shfl_cd(x, c + 8 * j);
    cmac(a, yrj, conj(xcj));
  }
  unew = a;
  if (y_io) *y_io = y;
  return 0;
}

// Lane (r, c) passes E[r][c], u_old[c][r], u_old[r][c]; receives u_new[r][c]
// for M = (1 - beta) E + beta u_old^dagger (Eq. opt_u; beta of Sec. III-A-2).
__device__ inline void optimize_gate_f64_oct(cd e, cd uold_cr, cd uold_rc, int r, int c, double beta, cd& unew,
                                             cd* xs, cd* y_io = nullptr, bool warm = false) {
  cd m = axpbyx(e, 1.0 - beta, conj(uold_cr), beta);
  nearest_unitary_f64_oct(m, uold_rc, r, c, unew, xs, y_io, warm);
}

// ------------------------------------------------------------------ k_env8

// Grid: one workgroup of kEnv8Threads per start (n <= 14).  Thread t sums
// entry (i, j) = t % 64 over the rests congruent to t / 64 mod 16 (eight
// loads in flight: at n = 10 every thread's loads are one round); the 16
// partial sums of an entry are added in a fixed tree.
constexpr uint32_t kEnv8Threads = 1024;
constexpr uint32_t kEnv8Lanes = kEnv8Threads / 64;  // rest lanes per entry
template <typename R>
__global__ __launch_bounds__(kEnv8Threads) void k_env8(const cx<R>* __restrict__ X, Pass8Geom g, Env8Args a) {
  __builtin_amdgcn_s_setprio(3);  // beside other groups' passes (stream groups)
  __shared__ cd red[kEnv8Threads];
  __shared__ cd P[64], U[64];
  __shared__ int frz;
  const uint32_t t = threadIdx.x;
  const uint32_t s = blockIdx.x;
  const cd* gsrc = reinterpret_cast<const cd*>(a.gates) + (int64_t)s * a.gstride + 64 * (int64_t)a.gidx;
  if (a.do_update && t < 64) U[t] = gsrc[t];
  if (t == 64) frz = (a.do_update && a.frozen && a.frozen[s]) ? 1 : 0;
  // the warm start (this gate's rotation of the previous sweep, same half),
  // fetched under the partial trace; lane r + 8c holds entry (r, c)
  cd* yw = a.ywarm ? reinterpret_cast<cd*>(a.ywarm) + (size_t)s * a.ywstride + 128 * (size_t)a.gidx + 64 * a.half
                   : nullptr;
  cd yv = mk(0.0, 0.0);
  if (yw && a.do_update && t < 64) yv = yw[t];
  const uint32_t ij = t & 63u, i = ij >> 3, j = ij & 7u, rl = t >> 6;
  const uint32_t ro = local_off8(i, g.b), co = local_off8(j, g.b);
  const uint32_t nrest = g.N >> 3;
  const cx<R>* Xs = X + (size_t)s * g.N * g.N;
  cd acc = mk(0.0, 0.0);
  for (uint32_t r0 = rl; r0 < nrest; r0 += 8u * kEnv8Lanes) {
    cx<R> v[8];
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
      const uint32_t rest = r0 + kEnv8Lanes * k;
      v[k] = mk<R>(0, 0);
      if (rest < nrest) {
        const uint32_t base = insert000(rest, g.s);
        v[k] = Xs[(size_t)(base + ro) * g.N + base + co];
      }
    }
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) acc = acc + mk((double)v[k].re, (double)v[k].im);
  }
  red[t] = acc;
  __syncthreads();
  for (uint32_t stride = kEnv8Threads / 2; stride >= 64; stride >>= 1) {
    if (t < stride) red[t] = red[t] + red[t + stride];
    __syncthreads();
  }
  if (t < 64) P[t] = red[t];
  __syncthreads();
  if (t >= 64) return;
  const int r = (int)(t & 7u), c = (int)(t >> 3);  // lane r + 8c
  const int rc = 8 * r + c;                          // row-major entry of this lane
  if (!a.do_update) {
    reinterpret_cast<cd*>(a.env_out)[64 * (size_t)s + t] = P[t];
    return;
  }
  // E = u_old^dagger P (first half) or P u_old^dagger (second half)
  cd e = mk(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (a.half == 0)
      cmac(e, conj(U[8 * k + r]), P[8 * k + c]);
    else
      cmac(e, P[8 * r + k], conj(U[8 * c + k]));
  }
  const cd urc = U[8 * r + c];
  cd un = urc;
  // the reduction buffer is free now: the update's lane exchanges use it
  if (!frz) optimize_gate_f64_oct(e, U[8 * c + r], urc, r, c, a.beta, un, red, yw ? &yv : nullptr, a.warm != 0);
  if (yw) yw[t] = yv;
  reinterpret_cast<cd*>(a.uold)[64 * (size_t)s + rc] = urc;
  reinterpret_cast<cd*>(a.gates)[(int64_t)s * a.gstride + 64 * (int64_t)a.gidx + rc] = un;
}

hipError_t launch_env8(hipStream_t st, int precision, const void* X, const Pass8Geom& g, const Env8Args& a) {
  if (g.n > 14) return hipErrorInvalidValue;
  const dim3 grid((uint32_t)a.S), block(kEnv8Threads);
  if (precision == QF_C64)
    hipLaunchKernelGGL(k_env8<float>, grid, block, 0, st, reinterpret_cast<const cf*>(X), g, a);
  else
    hipLaunchKernelGGL(k_env8<double>, grid, block, 0, st, reinterpret_cast<const cd*>(X), g, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ k_optimize8

// One wavefront per environment, lane r + 8c = entry (r, c).
__global__ __launch_bounds__(64) void k_optimize8(const cd* __restrict__ env, const cd* __restrict__ uold, double beta,
                                                  cd* __restrict__ unew) {
  __shared__ cd xs[128];  // the update's lane exchange
  const size_t s = blockIdx.x;
  const int t = (int)threadIdx.x, r = t & 7, c = t >> 3;
  const cd* u = uold + 64 * s;
  cd un;
  optimize_gate_f64_oct(env[64 * s + 8 * r + c], u[8 * c + r], u[8 * r + c], r, c, beta, un, xs);
  unew[64 * s + 8 * r + c] = un;
}

hipError_t launch_optimize8(hipStream_t st, int count, const double* env, const double* uold, double beta,
                            double* unew) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_optimize8, dim3((uint32_t)count), dim3(64), 0, st, reinterpret_cast<const cd*>(env),
                     reinterpret_cast<const cd*>(uold), beta, reinterpret_cast<cd*>(unew));
  return hipGetLastError();
}

}  // namespace qf
