// Device helpers for the QFactor kernels: complex arithmetic, qubit-bit
// index maps and the FP64 4x4 gate update (nearest unitary to an environment).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qf {

// ---------------------------------------------------------------- complex

template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> scale(cx<R> a, R s) { return {a.re * s, a.im * s}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <typename R>
__host__ __device__ __forceinline__ R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }
// acc += a * b
template <typename R>
__host__ __device__ __forceinline__ void cmac(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ void cmac_cj(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}

using cd = cx<double>;
using cf = cx<float>;

// c ? a : b for complex values, component-wise.  (A conditional operator on
// the struct itself is lowered to a select of addresses plus a copy, which
// sends both operands to scratch memory.)
template <typename R>
__host__ __device__ __forceinline__ cx<R> sel(bool c, cx<R> a, cx<R> b) {
  return cx<R>{c ? a.re : b.re, c ? a.im : b.im};
}

// ---------------------------------------------------------------- qubit bits

// Insert a zero bit at position p of v (bits >= p move up by one).
__host__ __device__ __forceinline__ uint32_t insert0(uint32_t v, uint32_t p) {
  return ((v >> p) << (p + 1)) | (v & ((1u << p) - 1u));
}
// Insert zero bits at positions lo < hi (positions in the result).
__host__ __device__ __forceinline__ uint32_t insert00(uint32_t v, uint32_t lo, uint32_t hi) {
  return insert0(insert0(v, lo), hi);
}
// Offset of local index i (0..3) for a gate whose local MSB sits at bit b0
// and local LSB at bit b1.
__host__ __device__ __forceinline__ uint32_t local_off(uint32_t i, uint32_t b0, uint32_t b1) {
  return (((i >> 1) & 1u) << b0) | ((i & 1u) << b1);
}

// ---------------------------------------------------------------- FP64 4x4

__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

// FP64 reciprocal and reciprocal square root for the SVD step's rotations:
// the hardware estimate refined by two Newton steps, y <- y (2 - x y) and
// y <- y (3 - x y^2) / 2, each FMA-based; about 1 ulp for normal arguments
// (the arguments here are column norms of a matrix scaled to entries <= 1).
// Far shorter dependent chains than IEEE division and square root.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// Complex products of the FP64 gate update with every fused multiply-add
// spelled out, so that each kernel that inlines the update rounds the same
// way whatever contractions the compiler would choose for it.
__device__ __forceinline__ double nrm2x(cd a) { return fma(a.re, a.re, a.im * a.im); }
__device__ __forceinline__ cd mulx(cd a, cd b) {  // a b
  return mk(fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re));
}
__device__ __forceinline__ cd cjmulx(cd a, cd b) {  // conj(a) b
  return mk(fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -(a.im * b.re)));
}
__device__ __forceinline__ cd axpbyx(cd x, double a, cd y, double b) {  // a x + b y
  return mk(fma(x.re, a, y.re * b), fma(x.im, a, y.im * b));
}

// Rank tolerance of the update: a column of the orthogonalised M whose
// squared norm is at most 1e-30 of another's (singular value ratio 1e-15,
// about 4.5 machine epsilons, numpy's matrix_rank tolerance for 4 x 4) is a
// numerically vanishing singular direction.  Such a column is round-off
// that lies in the span of the others and cannot be orthogonalised (the
// rotations would only shrink it, down to angles the float tangent cannot
// represent); it takes no rotation and is replaced at the end by the
// Gram-Schmidt completion (any completion attains the same Re Tr(M u) to
// within the neglected singular value).
constexpr double kRankTol2 = 1e-30;

// Entry (k, r) of a 4x4 row-major array for a runtime r, by a select chain
// (keeps the array in registers).
__device__ __forceinline__ cd at_kr(const cd u[16], int k, int r) {
  cd v = u[4 * k];
#pragma unroll
  for (int rr = 1; rr < 4; ++rr) v = sel(r == rr, u[4 * k + rr], v);
  return v;
}

// Entry (r, k) of a 4x4 row-major array for a runtime row r.
__device__ __forceinline__ cd at_rk(const cd u[16], int r, int k) {
  cd v = u[k];
#pragma unroll
  for (int rr = 1; rr < 4; ++rr) v = sel(r == rr, u[4 * rr + k], v);
  return v;
}

// ---------------------------------------------------------------- quad form

// The same nearest-unitary step spread over the 4 lanes of a quad (lanes
// 4k..4k+3 of a wavefront, all active): lane r owns row r of M and of the
// accumulated rotation Y.  A Jacobi sweep is three rounds of two disjoint
// column pairs ((0,1),(2,3)), ((0,2),(1,3)), ((0,3),(1,2)); each lane adds its
// row's share of the pair's column norms and inner product and a two-step
// butterfly completes the sums, so every lane holds bitwise-identical sums
// and takes identical rotation decisions.
// Lane exchange inside a quad with DPP quad_perm moves (plain VALU moves, no
// trip through the LDS crossbar).  CTRL is the quad_perm selector
// p0 | p1 << 2 | p2 << 4 | p3 << 6 (lane i of each quad reads lane p_i).
template <int CTRL>
__device__ __forceinline__ double dpp_quad(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
constexpr int kQuadXor1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);  // [1,0,3,2]
constexpr int kQuadXor2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);  // [2,3,0,1]

// Sum over the quad; every lane gets bitwise the same value (the two
// addition orders it sees are commutations of the same pairs).
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_quad<kQuadXor1>(v);
  return v + dpp_quad<kQuadXor2>(v);
}
__device__ __forceinline__ double quad_max(double v) {
  v = fmax(v, dpp_quad<kQuadXor1>(v));
  return fmax(v, dpp_quad<kQuadXor2>(v));
}
// o[c] = this value as held by lane c of the quad.
__device__ __forceinline__ void quad_gather(double v, double o[4]) {
  o[0] = dpp_quad<0x00>(v);
  o[1] = dpp_quad<0x55>(v);
  o[2] = dpp_quad<0xAA>(v);
  o[3] = dpp_quad<0xFF>(v);
}
__device__ __forceinline__ void quad_gather(cd v, cd o[4]) {
  double re[4], im[4];
  quad_gather(v.re, re);
  quad_gather(v.im, im);
#pragma unroll
  for (int c = 0; c < 4; ++c) o[c] = mk(re[c], im[c]);
}

// Jacobi rotation of columns (p, q) given the summed norms a, b and inner
// product g.  The rotation angle follows the symmetric 2x2 Schur step (Golub
// and Van Loan): with zeta = (b - a) / (2|g|), t = sign(zeta) / (|zeta| +
// sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2), s = c t, after the phase of g is
// moved onto column q.  The tangent t only steers convergence (any t gives an
// exact rotation once c and s are consistent with it), so it comes from
// single-precision hardware estimates; the phase of g and c are computed in
// FP64 (Newton-refined), so the applied rotation is unitary to FP64
// round-off.  Returns false when the pair is already orthogonal (no
// rotation); `large` is 1 for a large rotation, 0 for a small one: cosine of
// the pair and tan of the angle both below 1e-8.  A later rotation (p, r)
// moves the cosine of an orthogonalised pair (p, q) by at most about
// max(tan, cosine of (p, r)) times the cosine of (r, q), so a sweep of small
// rotations leaves every cosine below ~4e-16, the round-off threshold: no
// confirming sweep.
struct JacobiRot {
  double c, s, large;
  cd ph;  // e^{-i arg g}
};
__device__ __forceinline__ bool jacobi_params(double a, double b, cd g, JacobiRot& q) {
  const double tol2 = 1.6e-31;  // (4e-16)^2: |g| <= 4e-16 sqrt(a b) counts as orthogonal
  const double g2 = nrm2x(g);
  if (!(g2 > tol2 * (a * b))) return false;
  if (!(fmin(a, b) > kRankTol2 * fmax(a, b))) return false;  // a vanishing column
  const double rg = rsqrt_nr(g2);              // 1 / |g|
  const float zeta = (float)(0.5 * (b - a) * rg);
  const float az = fabsf(zeta);
  float tf;
  if (az < 1e18f) {
    const float q2 = fmaf(zeta, zeta, 1.0f);
    tf = __builtin_amdgcn_rcpf(az + q2 * __builtin_amdgcn_rsqf(q2));  // 1 / (|zeta| + sqrt(1 + zeta^2))
  } else {
    tf = 0.5f * __builtin_amdgcn_rcpf(az);
  }
  const double t = zeta >= 0.0f ? (double)tf : -(double)tf;
  q.c = rsqrt_nr(fma(t, t, 1.0));
  q.s = q.c * t;
  q.ph = mk(g.re * rg, -g.im * rg);
  q.large = (g2 > 1e-16 * (a * b) || fabs(t) > 1e-8) ? 1.0 : 0.0;
  return true;
}
// (xp, xq) <- (c xp - s ph xq, s xp + c ph xq): one row of the rotated pair.
__device__ __forceinline__ void jacobi_apply(const JacobiRot& q, cd xp, cd mq, cd& np, cd& nq) {
  const cd xq = mulx(q.ph, mq);
  np = axpbyx(xp, q.c, xq, -q.s);
  nq = axpbyx(xp, q.s, xq, q.c);
}

// Quad form: applies the rotation of columns (p, q) to this lane's row of M
// and Y; returns 1 for a large rotation, 0 for a small one or none.
__device__ __forceinline__ double quad_rotate(cd m[4], cd y[4], int p, int q, double a, double b, cd g) {
  JacobiRot j;
  if (!jacobi_params(a, b, g, j)) return 0.0;
  jacobi_apply(j, m[p], m[q], m[p], m[q]);
  jacobi_apply(j, y[p], y[q], y[p], y[q]);
  return j.large;
}

template <int P0, int Q0, int P1, int Q1>
__device__ __forceinline__ double quad_round(cd m[4], cd y[4]) {
  double v[8];
  v[0] = nrm2x(m[P0]);
  v[1] = nrm2x(m[Q0]);
  const cd g0 = cjmulx(m[P0], m[Q0]);
  v[2] = g0.re;
  v[3] = g0.im;
  v[4] = nrm2x(m[P1]);
  v[5] = nrm2x(m[Q1]);
  const cd g1 = cjmulx(m[P1], m[Q1]);
  v[6] = g1.re;
  v[7] = g1.im;
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = quad_sum(v[k]);
  const double r0 = quad_rotate(m, y, P0, Q0, v[0], v[1], mk(v[2], v[3]));
  const double r1 = quad_rotate(m, y, P1, Q1, v[4], v[5], mk(v[6], v[7]));
  return fmax(r0, r1);
}

// mrow: this lane's row r of M (overwritten); keep_row: row r of the result
// to return for a zero M; returns row r of the maximiser of Re Tr(M u).
// Result: 0 = computed, 1 = zero M (keep_row returned), 2 = non-finite M.
__device__ inline int nearest_unitary_f64_quad(cd mrow[4], const cd keep_row[4], int r, cd unew_row[4]) {
  double amax = 0.0, bad = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    amax = fmax(amax, fmax(fabs(mrow[j].re), fabs(mrow[j].im)));
    bad = (finite_d(mrow[j].re) && finite_d(mrow[j].im)) ? bad : 1.0;
  }
  amax = quad_max(amax);
  bad = quad_max(bad);
  if (bad != 0.0) {
    const double nan = __builtin_nan("");
#pragma unroll
    for (int j = 0; j < 4; ++j) unew_row[j] = mk(nan, nan);
    return 2;
  }
  if (!(amax >= 1e-300)) {
#pragma unroll
    for (int j = 0; j < 4; ++j) unew_row[j] = keep_row[j];
    return 1;
  }
  const double inv = rcp_nr(amax);  // any positive scale serves
#pragma unroll
  for (int j = 0; j < 4; ++j) mrow[j] = scale(mrow[j], inv);
  cd y[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) y[j] = mk(j == r ? 1.0 : 0.0, 0.0);
  // Cyclic sweeps until a sweep makes no large rotation.
  for (int sweep = 0; sweep < 30; ++sweep) {
    double rel = quad_round<0, 1, 2, 3>(mrow, y);
    rel = fmax(rel, quad_round<0, 2, 1, 3>(mrow, y));
    rel = fmax(rel, quad_round<0, 3, 1, 2>(mrow, y));
    if (!(rel > 0.0)) break;
  }
  double sig2[4], smax2 = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    sig2[j] = quad_sum(nrm2x(mrow[j]));
    smax2 = fmax(smax2, sig2[j]);
  }
  bool acc[4];
  bool singular = false;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    acc[j] = sig2[j] > smax2 * kRankTol2;
    singular = singular || !acc[j];
  }
  cd x[4];  // row r of X
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] = sel(acc[j], scale(mrow[j], rsqrt_nr(acc[j] ? sig2[j] : 1.0)), mk(0.0, 0.0));
  if (singular) {
    // A vanishing singular direction (see kRankTol2): complete X by
    // Gram-Schmidt of e_0..e_3 against the accepted columns (any completion
    // attains the same Re Tr(M u)); lane r holds component r of each vector.
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!acc[j]) {
        bool found = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          cd v = mk(r == k ? 1.0 : 0.0, 0.0);
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            if (acc[jj]) {
              const cd pr = cjmulx(x[jj], v);
              const cd d = mk(quad_sum(pr.re), quad_sum(pr.im));
              v = v - mulx(x[jj], d);
            }
          }
          const double nv = quad_sum(nrm2x(v));
          const bool take = !found && nv >= 0.25;
          if (take) x[j] = scale(v, rsqrt_nr(nv));
          found = found || take;
        }
        acc[j] = true;
      }
    }
  }
  // u_new[r][c] = sum_j Y[r][j] conj(X[c][j]); rows of X from the quad
  cd xall[4][4];  // xall[j][c] = X[c][j]
#pragma unroll
  for (int j = 0; j < 4; ++j) quad_gather(x[j], xall[j]);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cd acc = mk(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 4; ++j) cmac(acc, y[j], conj(xall[j][c]));
    unew_row[c] = acc;
  }
  return 0;
}

// Quad form of OptimizeGate (Sec. III-A-1, Eq. opt_u; beta of Sec. III-A-2).
// Lane r passes row r of E and the whole u_old (16 entries) and receives row
// r of u_new, the maximiser of Re Tr(M u) for M = (1-beta) E + beta
// u_old^dagger.  The result is Y X^dagger from the Jacobi step, unitary to
// round-off whatever the gate's history; a zero M keeps u_old exactly.
__device__ inline void optimize_gate_f64_quad(const cd e_row[4], const cd uold[16], int r, double beta,
                                              cd unew_row[4]) {
  cd m[4], keep[4];
  const double we = 1.0 - beta;  // exact 1 for beta = 0
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    m[c] = axpbyx(e_row[c], we, conj(at_kr(uold, c, r)), beta);  // + beta (u_old^dagger)[r][c]
    keep[c] = at_rk(uold, r, c);
  }
  nearest_unitary_f64_quad(m, keep, r, unew_row);
}

// ---------------------------------------------------------------- hex form
//
// The same nearest-unitary step on 16 lanes (lanes 16k..16k+15 of a
// wavefront, all active): lane i holds entry (r, c) of M and of Y, with
// c = i & 3 and r the two-bit reversal of i >> 2 (rows 0, 2, 1, 3 on the
// four quads).  A round's two disjoint column pairs run on different lanes at
// once, so a round costs one rotation's dependent chain and about half the
// instructions of the quad form.  The row placement makes a column sum
// (rotate by 8, then by 4 lanes within the row of 16) add in the order
// (r0 + r1) + (r2 + r3), the quad form's order, and every other operation is
// the quad form's expression on the same operands, so the two forms give
// bitwise-identical results.
constexpr int kQuadXor3 = 3 | (2 << 2) | (1 << 4) | (0 << 6);  // [3,2,1,0]
constexpr int kRowRor4 = 0x124;                                 // DPP row_ror:4
constexpr int kRowRor8 = 0x128;                                 // DPP row_ror:8

__host__ __device__ __forceinline__ int hex_row(int i) { return (((i >> 2) & 1) << 1) | ((i >> 3) & 1); }
__host__ __device__ __forceinline__ int hex_lane(int r, int c) { return c + 4 * ((((r & 1) << 1) | (r >> 1))); }

template <int CTRL>
__device__ __forceinline__ cd dpp_cx(cd v) {
  return mk(dpp_quad<CTRL>(v.re), dpp_quad<CTRL>(v.im));
}
// Sum over the 4 rows of this lane's column; bitwise the same in every lane.
__device__ __forceinline__ double hex_colsum(double v) {
  v += dpp_quad<kRowRor8>(v);
  return v + dpp_quad<kRowRor4>(v);
}
__device__ __forceinline__ double hex_max(double v) {
  v = quad_max(v);
  v = fmax(v, dpp_quad<kRowRor8>(v));
  return fmax(v, dpp_quad<kRowRor4>(v));
}
// Entry (r, j) of the quad's row (lane j of this quad) for a compile-time j
// after unrolling.
__device__ __forceinline__ cd quad_bcast(cd v, int j) {
  if (j == 0) return dpp_cx<0x00>(v);
  if (j == 1) return dpp_cx<0x55>(v);
  if (j == 2) return dpp_cx<0xAA>(v);
  return dpp_cx<0xFF>(v);
}

// One round: the pair (c, c ^ K) of this lane's column; XK is the quad_perm
// selector of lane ^ K.  Returns 1 for a large rotation, 0 otherwise.
template <int K, int XK>
__device__ __forceinline__ double hex_round(cd& m, cd& y, int c) {
  const bool pside = c < (c ^ K);
  const cd mo = dpp_cx<XK>(m);
  const cd yo = dpp_cx<XK>(y);
  const cd mP = sel(pside, m, mo), mQ = sel(pside, mo, m);
  const double na = hex_colsum(nrm2x(m));
  const cd gl = cjmulx(mP, mQ);
  const cd g = mk(hex_colsum(gl.re), hex_colsum(gl.im));
  const double nb = dpp_quad<XK>(na);
  JacobiRot j;
  if (!jacobi_params(pside ? na : nb, pside ? nb : na, g, j)) return 0.0;
  cd np, nq;
  jacobi_apply(j, mP, mQ, np, nq);
  m = sel(pside, np, nq);
  jacobi_apply(j, sel(pside, y, yo), sel(pside, yo, y), np, nq);
  y = sel(pside, np, nq);
  return j.large;
}

// Sum over all 16 lanes of a hex group; bitwise the same in every lane.
__device__ __forceinline__ double hex_sum(double v) { return hex_colsum(quad_sum(v)); }

// Newton form of the nearest-unitary step.  The maximiser of Re Tr(M u) over
// unitary u is Q^dagger, Q the unitary polar factor of M (M = Q H, H
// Hermitian positive semidefinite).  For a nonsingular M, Q is the limit of
// the scaled Newton iteration of Higham ("Computing the polar decomposition
// -- with applications", SIAM J. Sci. Stat. Comput. 7, 1986):
//   X_0 = M,  X_{k+1} = (z_k X_k + X_k^{-dagger} / z_k) / 2,
// with the Frobenius-norm scaling z_k = (|X_k^-1|_F / |X_k|_F)^(1/2).  Each
// step keeps the singular vectors and maps every singular value s to
// (z s + 1 / (z s)) / 2, so the iteration converges quadratically once they
// are near 1.  In the hex layout each lane forms its own cofactor C[r][c]
// (the signed determinant of the 3 x 3 minor without row r and column c):
// X^{-dagger}[r][c] = conj(C[r][c]) / conj(det X), and det X is the sum of
// X[r][c] C[r][c] over the 16 lanes divided by 4 (each row's Laplace
// expansion gives it once).  dist = |X|_F^2 + |X^-1|_F^2 - 8, the sum of
// (s - 1/s)^2 over the singular values, measures the distance from
// unitarity: steps are scaled while dist > 1e-2, and the iteration ends
// with the step taken at dist <= 1e-14 (every |s - 1| is then below 5e-8,
// and the step leaves it near 1e-15).  Every decision is taken on hex sums,
// bitwise the same in all 16 lanes.
// Cramer's rule is accurate only for a well-conditioned X (the polar
// factor's error grows like the squared condition number times the unit
// roundoff), so the form is taken only when |M|_F^2 |M^-1|_F^2 < 1e6; for
// other M, and if 10 steps have not converged, it returns false and the
// caller takes the Jacobi form.
constexpr double kPolarCond2 = 1e6;
constexpr double kPolarScaleAbove = 1e-2;
constexpr double kPolarDone = 1e-14;
constexpr int kPolarMaxSteps = 10;

// x: this lane's entry (r, c) of M, entries at most 1 in magnitude.  On
// success q is entry (r, c) of Q.  xch: 16 entries of LDS owned by this hex
// group during the call, through which its lanes exchange entries (each lane
// stores its own at index hex_lane(r, c) and loads the nine of its minor, one
// 16-byte load each instead of four lane permutes).  The 16 lanes are one
// wavefront's, whose LDS instructions execute in issue order: loads issued
// after the stores see them, and the next stores cannot overtake them; the
// wave barriers keep the compiler from moving the accesses across.
__device__ inline bool polar_newton_hex(cd x, int r, int c, cd& q, cd* xch) {
  int src[9];  // indices of the minor's entries, rows and columns ascending
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) src[3 * i + j] = hex_lane(i + (i >= r ? 1 : 0), j + (j >= c ? 1 : 0));
  const int own = hex_lane(r, c);
  const double sgn = ((r + c) & 1) ? -1.0 : 1.0;
  for (int step = 0; step < kPolarMaxSteps; ++step) {
    __builtin_amdgcn_wave_barrier();
    xch[own] = x;
    __builtin_amdgcn_wave_barrier();
    cd a[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) a[k] = xch[src[k]];
    const cd m0 = mulx(a[4], a[8]) - mulx(a[5], a[7]);
    const cd m1 = mulx(a[3], a[8]) - mulx(a[5], a[6]);
    const cd m2 = mulx(a[3], a[7]) - mulx(a[4], a[6]);
    const cd cof = scale(mulx(a[0], m0) - mulx(a[1], m1) + mulx(a[2], m2), sgn);
    const cd p = mulx(x, cof);
    const double nx = hex_sum(nrm2x(x));
    const double nc = hex_sum(nrm2x(cof));
    const cd det = mk(0.25 * hex_sum(p.re), 0.25 * hex_sum(p.im));
    const double d2 = nrm2x(det);
    if (step == 0 && !(nx * nc < kPolarCond2 * d2)) return false;  // also a zero or non-finite det
    const double inv_d2 = rcp_nr(d2);
    const double nxi = nc * inv_d2;  // |X^-1|_F^2
    const double dist = (nx + nxi) - 8.0;
    double z = 1.0, zi = 1.0;
    if (dist > kPolarScaleAbove) {
      // z = (nxi / nx)^(1/4) and 1 / z from hardware estimates: any positive
      // scaling keeps the limit, and the last steps are unscaled
      const double t = __builtin_amdgcn_rsq(nxi * __builtin_amdgcn_rcp(nx));
      z = __builtin_amdgcn_rsq(t);
      zi = t * z;
    }
    const cd w = scale(det, 0.5 * zi * inv_d2);  // conj(C) w = X^{-dagger} / (2 z)
    const double hz = 0.5 * z;
    x = mk(fma(hz, x.re, fma(cof.re, w.re, cof.im * w.im)), fma(hz, x.im, fma(cof.re, w.im, -(cof.im * w.re))));
    if (dist <= kPolarDone) {
      q = x;
      return true;
    }
  }
  return false;
}

// m: this lane's entry (r, c) of M (overwritten); keep: entry (r, c) of the
// result for a zero M; unew: entry (r, c) of the maximiser of Re Tr(M u);
// xch: the hex group's 16 LDS entries for the Newton form (overwritten).
// The Newton form above runs first; where it declines, a one-sided Jacobi
// step in the hex layout takes over, with the same results and return
// codes as nearest_unitary_f64_quad when y_io is null.
//
// Warm start (y_io non-null): y_io holds entry (r, c) of the accumulated
// rotation Y of the gate's last Jacobi update.  With warm set, the Jacobi
// step starts from that Y (M Y for M, Y for the rotation): any unitary start
// gives the same orthogonalised columns and so the same maximiser up to
// round-off, and where consecutive environments of a gate are alike M Y is
// nearly column-orthogonal already, so fewer rounds run.  The new Y is
// written back; the identity after a Newton update and for a zero or a
// non-finite M.
// Callers start cold now and then so that the round-off of Y's accumulated
// rotations stays at a few ulps.
constexpr int kWarmPeriod = 16;  // a gate's updates start cold once in this many sweeps

__device__ inline int nearest_unitary_f64_hex(cd& m, cd keep, int r, int c, cd& unew, cd* xch, cd* y_io = nullptr,
                                              bool warm = false) {
  double amax = fmax(fabs(m.re), fabs(m.im));
  double bad = (finite_d(m.re) && finite_d(m.im)) ? 0.0 : 1.0;
  amax = hex_max(amax);
  bad = hex_max(bad);
  if (bad != 0.0 || !(amax >= 1e-300)) {
    if (y_io) *y_io = mk(c == r ? 1.0 : 0.0, 0.0);  // the next warm start is a cold one
    if (bad != 0.0) {
      const double nan = __builtin_nan("");
      unew = mk(nan, nan);
      return 2;
    }
    unew = keep;
    return 1;
  }
  const double inv = rcp_nr(amax);
  m = scale(m, inv);
  cd y = mk(c == r ? 1.0 : 0.0, 0.0);
  const int base = (int)(__lane_id() & ~15u);
  {
    cd q;
    if (polar_newton_hex(m, r, c, q, xch)) {
      if (y_io) *y_io = y;
      // u_new[r][c] = conj(Q[c][r])
      const int src = base + hex_lane(c, r);
      unew = conj(mk(__shfl(q.re, src, 64), __shfl(q.im, src, 64)));
      return 0;
    }
  }
  if (y_io && warm) {
    // M <- M Y: row r of M from the quad, column c of Y from the four quads
    y = *y_io;
    cd mr[4];
    quad_gather(m, mr);
    cd acc = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int src = base + hex_lane(k, c);
      cmac(acc, mr[k], mk(__shfl(y.re, src, 64), __shfl(y.im, src, 64)));
    }
    m = acc;
  }
  for (int sweep = 0; sweep < 30; ++sweep) {
    double rel = hex_round<1, kQuadXor1>(m, y, c);
    rel = fmax(rel, hex_round<2, kQuadXor2>(m, y, c));
    rel = fmax(rel, hex_round<3, kQuadXor3>(m, y, c));
    if (!(quad_max(rel) > 0.0)) break;
  }
  const double sig2 = hex_colsum(nrm2x(m));
  const double smax2 = quad_max(sig2);
  const bool acc = sig2 > smax2 * kRankTol2;
  double accv[4];
  quad_gather(acc ? 1.0 : 0.0, accv);
  cd x = sel(acc, scale(m, rsqrt_nr(acc ? sig2 : 1.0)), mk(0.0, 0.0));  // X[r][c]
  if (accv[0] == 0.0 || accv[1] == 0.0 || accv[2] == 0.0 || accv[3] == 0.0) {
    // Gram-Schmidt completion as in the quad form, each row's component
    // computed by the four lanes of its quad alike.
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (accv[j] == 0.0) {
        bool found = false;
        cd xj = mk(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          cd v = mk(r == k ? 1.0 : 0.0, 0.0);
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            if (accv[jj] != 0.0) {
              const cd xjj = quad_bcast(x, jj);
              const cd pr = cjmulx(xjj, v);
              const cd d = mk(hex_colsum(pr.re), hex_colsum(pr.im));
              v = v - mulx(xjj, d);
            }
          }
          const double nv = hex_colsum(nrm2x(v));
          const bool take = !found && nv >= 0.25;
          if (take) xj = scale(v, rsqrt_nr(nv));
          found = found || take;
        }
        if (c == j) x = xj;
        accv[j] = 1.0;
      }
    }
  }
  // u_new[r][c] = sum_j Y[r][j] conj(X[c][j]); row r of Y from the quad, row
  // c of X from the quad that holds it.
  cd yr[4];
  quad_gather(y, yr);
  if (y_io) *y_io = y;
  cd a = mk(0.0, 0.0);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int src = base + hex_lane(c, j);
    const cd xcj = mk(__shfl(x.re, src, 64), __shfl(x.im, src, 64));
    cmac(a, yr[j], conj(xcj));
  }
  unew = a;
  return 0;
}

// Entry (r, c) of the environment E of the gate being updated, from the
// partial trace P and u_old (row-major 4 x 4 arrays readable by every lane):
// E = u_old^dagger P in the first half of a sweep, P u_old^dagger in the
// second (the removal of the old gate commutes with the partial trace); the
// quad form's sum order.
__device__ __forceinline__ cd env_entry(const cd* P, const cd* uold, int half, int r, int c) {
  cd acc = mk(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (half == 0)
      cmac(acc, conj(uold[4 * k + r]), P[4 * k + c]);
    else
      cmac(acc, P[4 * r + k], conj(uold[4 * c + k]));
  }
  return acc;
}

// Hex form of OptimizeGate (Sec. III-A-1, Eq. opt_u; beta of Sec. III-A-2):
// lane (r, c) passes E[r][c], u_old[c][r] and u_old[r][c] and receives
// u_new[r][c]; the quad form's result up to round-off (bitwise where the
// Newton form declines and y_io is null).
__device__ inline void optimize_gate_f64_hex(cd e, cd uold_cr, cd uold_rc, int r, int c, double beta, cd& unew,
                                             cd* xch, cd* y_io = nullptr, bool warm = false) {
  const double we = 1.0 - beta;  // exact 1 for beta = 0
  cd m = axpbyx(e, we, conj(uold_cr), beta);
  nearest_unitary_f64_hex(m, uold_rc, r, c, unew, xch, y_io, warm);
}

// ---------------------------------------------------------------- gate kinds
//
// Restricted gates (Sec. III-A-3, Specializing Gate Sets; the U3 + CNOT set
// of the evaluation).  Every gate is stored as a 4 x 4 matrix on its two
// locations; single-qubit kinds act on the first and are stored as g (x) I,
// the second location being only a partner qubit.  For them
// Re Tr(E (g (x) I)) = Re Tr(E2 g) with E2[a][b] = E[2a][2b] + E[2a+1][2b+1],
// and the update maximises Re Tr(M2 g), M2 = (1-beta) E2 + beta g_old^dagger:
//   U(2): g = W^dagger, W the unitary polar factor of M2.  For a 2 x 2 matrix
//         M = W P (P = diag(s1, s2) in its eigenbasis), P + s1 s2 P^-1 =
//         (s1 + s2) I, hence M + |det M| M^-dagger = (s1 + s2) W, and
//         |det M| M^-dagger = e^{i arg det M} adj(M)^dagger; W is that sum
//         divided by its Frobenius norm / sqrt 2.  A singular M (det = 0)
//         gives a rank-one M plus the orthogonal rank-one completion, which
//         attains the same maximum.
//   Rz:   g = diag(1, e^{it}), t = -arg M2[1][1]
//   GPI:  g = [[0, e^{-if}], [e^{if}, 0]], f = -arg(M2[0][1] + conj(M2[1][0]))
//   fixed: the gate is kept.
// The two-qubit Molmer-Sorensen kind MS(f1, f2) acts on both locations; with
// M = (1-beta) E + beta u_old^dagger, s = f1 + f2 and d = f1 - f2,
// Re Tr(M MS) = const + (Re(w_s e^{is}) + Re(w_d e^{id})) / sqrt 2 with
// w_s = -i M[0][3] + i conj(M[3][0]), w_d = -i M[1][2] + i conj(M[2][1]);
// s and d are independent, so e^{is} = conj(w_s) / |w_s| and likewise d.
// A zero M2 (or a zero quantity to take the argument of) keeps the gate.
enum : int { kKindU4 = 0, kKindFixed = 1, kKindU2 = 2, kKindRz = 3, kKindGpi = 4, kKindMs = 5 };

// Lane r of a quad passes row r of E and the whole u_old; receives row r of
// the new stored matrix.  Every lane computes the same 2 x 2 update.
__device__ inline void update_gate_quad(int kind, const cd e_row[4], const cd uold[16], int r, double beta,
                                        cd unew_row[4]) {
  if (kind == kKindU4) {
    optimize_gate_f64_quad(e_row, uold, r, beta, unew_row);
    return;
  }
  if (kind == kKindFixed) {
#pragma unroll
    for (int c = 0; c < 4; ++c) unew_row[c] = at_rk(uold, r, c);
    return;
  }
  cd col[4][4];  // col[j][k] = E[k][j]
#pragma unroll
  for (int j = 0; j < 4; ++j) quad_gather(e_row[j], col[j]);
  const double we = 1.0 - beta;
  if (kind == kKindMs) {
    // M[j][k] = we E[j][k] + beta conj(u_old[k][j])
    const cd m03 = scale(col[3][0], we) + scale(conj(uold[4 * 3 + 0]), beta);
    const cd m30 = scale(col[0][3], we) + scale(conj(uold[4 * 0 + 3]), beta);
    const cd m12 = scale(col[2][1], we) + scale(conj(uold[4 * 2 + 1]), beta);
    const cd m21 = scale(col[1][2], we) + scale(conj(uold[4 * 1 + 2]), beta);
    const cd mi = mk(0.0, -1.0), pi = mk(0.0, 1.0);
    const cd ws = mi * m03 + pi * conj(m30), wd = mi * m12 + pi * conj(m21);
    const bool fin = finite_d(ws.re) && finite_d(ws.im) && finite_d(wd.re) && finite_d(wd.im);
    const double as = sqrt(norm2(ws)), adn = sqrt(norm2(wd));
    if (!fin) {
      const double nan = __builtin_nan("");
#pragma unroll
      for (int c = 0; c < 4; ++c) unew_row[c] = mk(nan, nan);
      return;
    }
    if (!(as >= 1e-300) || !(adn >= 1e-300)) {
#pragma unroll
      for (int c = 0; c < 4; ++c) unew_row[c] = at_rk(uold, r, c);
      return;
    }
    const cd us = scale(conj(ws), 1.0 / as), ud = scale(conj(wd), 1.0 / adn);  // e^{is}, e^{id}
    const double h = 0.70710678118654752440;  // 1 / sqrt 2
    const cd z = mk(0.0, 0.0), dg = mk(h, 0.0);
    const cd a03 = scale(mi * conj(us), h), a30 = scale(mi * us, h);
    const cd a12 = scale(mi * conj(ud), h), a21 = scale(mi * ud, h);
    unew_row[0] = sel(r == 0, dg, sel(r == 3, a30, z));
    unew_row[1] = sel(r == 1, dg, sel(r == 2, a21, z));
    unew_row[2] = sel(r == 1, a12, sel(r == 2, dg, z));
    unew_row[3] = sel(r == 0, a03, sel(r == 3, dg, z));
    return;
  }
  cd m[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const cd e2 = col[2 * b][2 * a] + col[2 * b + 1][2 * a + 1];
      m[a][b] = scale(e2, we) + scale(conj(uold[4 * (2 * b) + 2 * a]), beta);  // + beta g_old^dagger
    }
  bool finite = true;
  double amax = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      finite = finite && finite_d(m[a][b].re) && finite_d(m[a][b].im);
      amax = fmax(amax, fmax(fabs(m[a][b].re), fabs(m[a][b].im)));
    }
  cd g[2][2];
  bool keep = false;
  if (kind == kKindU2) {
    keep = !(amax >= 1e-300);
    const double inv = keep ? 1.0 : rcp_nr(amax);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) m[a][b] = scale(m[a][b], inv);
    const cd det = m[0][0] * m[1][1] - m[0][1] * m[1][0];
    const double ad = sqrt(norm2(det));
    const cd ph = ad > 0.0 ? scale(det, 1.0 / ad) : mk(1.0, 0.0);
    // B = M + ph adj(M)^dagger, adj(M) = [[m11, -m01], [-m10, m00]]
    cd bm[2][2];
    bm[0][0] = m[0][0] + ph * conj(m[1][1]);
    bm[0][1] = m[0][1] - ph * conj(m[1][0]);
    bm[1][0] = m[1][0] - ph * conj(m[0][1]);
    bm[1][1] = m[1][1] + ph * conj(m[0][0]);
    const double nb = sqrt(0.5 * (norm2(bm[0][0]) + norm2(bm[0][1]) + norm2(bm[1][0]) + norm2(bm[1][1])));
    const double inb = 1.0 / nb;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) g[a][b] = scale(conj(bm[b][a]), inb);  // W^dagger
  } else if (kind == kKindRz) {
    const double a11 = sqrt(norm2(m[1][1]));
    keep = !(a11 >= 1e-300);
    g[0][0] = mk(1.0, 0.0);
    g[0][1] = mk(0.0, 0.0);
    g[1][0] = mk(0.0, 0.0);
    g[1][1] = keep ? mk(1.0, 0.0) : scale(conj(m[1][1]), 1.0 / a11);
  } else {  // GPI
    const cd w = m[0][1] + conj(m[1][0]);
    const double aw = sqrt(norm2(w));
    keep = !(aw >= 1e-300);
    const cd e = keep ? mk(1.0, 0.0) : scale(w, 1.0 / aw);  // e^{-if}
    g[0][0] = mk(0.0, 0.0);
    g[0][1] = e;
    g[1][0] = conj(e);
    g[1][1] = mk(0.0, 0.0);
  }
  if (!finite) {
    const double nan = __builtin_nan("");
#pragma unroll
    for (int c = 0; c < 4; ++c) unew_row[c] = mk(nan, nan);
    return;
  }
  if (keep) {
#pragma unroll
    for (int c = 0; c < 4; ++c) unew_row[c] = at_rk(uold, r, c);
    return;
  }
  // row r = (a, c) of g (x) I: entry (b, d) is g[a][b] when d = c
  const int a = r >> 1, cbit = r & 1;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const cd v = sel(a == 0, g[0][b], g[1][b]);
      unew_row[2 * b + d] = sel(d == cbit, v, mk(0.0, 0.0));
    }
}

}  // namespace qf
