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

// Nearest unitary to an environment (Sec. III-A-1): with M = X D Y^dagger,
// the maximiser of Re Tr(M u) over unitary u is u = Y X^dagger.  The SVD is a
// one-sided (Hestenes) Jacobi iteration on the columns of M: complex Jacobi
// rotations J accumulate in Yacc until the columns of M Yacc are mutually
// orthogonal, so M Yacc = X D with X's columns the normalised results and
// Y = Yacc.  Plain single-thread FP64; `m` is overwritten.
// Returns the number of Jacobi sweeps used (0 for the zero/NaN guards).
__device__ inline int nearest_unitary_f64(cd m[16], const cd uold[16], cd unew[16]) {
  double amax = 0.0;  // largest |component|, free of under/overflow
  bool ok = true;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    amax = fmax(amax, fmax(fabs(m[e].re), fabs(m[e].im)));
    ok = ok && finite_d(m[e].re) && finite_d(m[e].im);
  }
  if (!ok) {
    const double nan = __builtin_nan("");
#pragma unroll
    for (int e = 0; e < 16; ++e) unew[e] = mk(nan, nan);
    return 0;
  }
  if (!(amax >= 1e-300)) {  // zero environment: keep the gate
#pragma unroll
    for (int e = 0; e < 16; ++e) unew[e] = uold[e];
    return 0;
  }
  // The maximiser does not change under a positive scaling of M; normalise
  // so that the squared column norms below neither underflow nor overflow.
  {
    const double inv = 1.0 / amax;
#pragma unroll
    for (int e = 0; e < 16; ++e) m[e] = scale(m[e], inv);
  }
  cd y[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) y[e] = mk((e % 5 == 0) ? 1.0 : 0.0, 0.0);

  const double tol = 4.0e-16;
  int sweep = 0;
  for (; sweep < 30; ++sweep) {
    bool rotated = false;
#pragma unroll
    for (int pair = 0; pair < 6; ++pair) {
      const int p = (pair < 3) ? 0 : (pair < 5 ? 1 : 2);
      const int q = (pair < 3) ? pair + 1 : (pair < 5 ? pair - 1 : 3);
      double a = 0.0, b = 0.0;
      cd g = mk(0.0, 0.0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a += norm2(m[4 * r + p]);
        b += norm2(m[4 * r + q]);
        cmac_cj(g, m[4 * r + p], m[4 * r + q]);
      }
      const double ag = sqrt(norm2(g));
      if (!(ag > tol * sqrt(a * b))) continue;
      rotated = true;
      const double zeta = (b - a) / (2.0 * ag);
      const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      const double c = 1.0 / sqrt(1.0 + t * t);
      const double s = c * t;
      const cd ph = mk(g.re / ag, -g.im / ag);  // e^{-i arg g}
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const cd xp = m[4 * r + p], xq = ph * m[4 * r + q];
        m[4 * r + p] = scale(xp, c) - scale(xq, s);
        m[4 * r + q] = scale(xp, s) + scale(xq, c);
        const cd yp = y[4 * r + p], yq = ph * y[4 * r + q];
        y[4 * r + p] = scale(yp, c) - scale(yq, s);
        y[4 * r + q] = scale(yp, s) + scale(yq, c);
      }
    }
    if (!rotated) break;
  }
  // X = normalised columns of m; complete any exactly vanishing column.
  double sig[4];
  double smax = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double s2 = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) s2 += norm2(m[4 * r + j]);
    sig[j] = sqrt(s2);
    smax = fmax(smax, sig[j]);
  }
  bool accepted[4];
  bool any_missing = false;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    accepted[j] = sig[j] > smax * 1e-290;
    any_missing = any_missing || !accepted[j];
    if (accepted[j]) {
      const double inv = 1.0 / sig[j];
#pragma unroll
      for (int r = 0; r < 4; ++r) m[4 * r + j] = scale(m[4 * r + j], inv);
    }
  }
  if (any_missing) {
    // A singular value is exactly zero: any unit vector orthogonal to the
    // other columns completes X (that direction does not change Re Tr(M u)).
    // Gram-Schmidt of e_0..e_3 against the accepted columns; with at most
    // three accepted orthonormal columns some e_k keeps a residual >= 1/4.
    // (Fully unrolled, flag-driven: every array index is a constant.)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!accepted[j]) {
        bool found = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          cd v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = mk(r == k ? 1.0 : 0.0, 0.0);
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            if (accepted[jj]) {
              cd d = mk(0.0, 0.0);
#pragma unroll
              for (int r = 0; r < 4; ++r) cmac_cj(d, m[4 * r + jj], v[r]);
#pragma unroll
              for (int r = 0; r < 4; ++r) v[r] = v[r] - m[4 * r + jj] * d;
            }
          }
          double nv = 0.0;
#pragma unroll
          for (int r = 0; r < 4; ++r) nv += norm2(v[r]);
          const bool take = !found && nv >= 0.25;
          if (take) {
            const double inv = 1.0 / sqrt(nv);
#pragma unroll
            for (int r = 0; r < 4; ++r) m[4 * r + j] = scale(v[r], inv);
          }
          found = found || take;
        }
        accepted[j] = true;
      }
    }
  }
  // u_new = Y X^dagger
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      cd acc = mk(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < 4; ++j) cmac(acc, y[4 * r + j], conj(m[4 * c + j]));
      unew[4 * r + c] = acc;
    }
  }
  return sweep + 1;
}

// Full OptimizeGate for a general unitary: M = (1-beta) E + beta u_old^dagger,
// then the nearest unitary.  E, uold, unew: 16 entries row-major.
__device__ inline int optimize_gate_f64(const cd e[16], const cd uold[16], double beta, cd unew[16]) {
  cd m[16];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cd ud = conj(uold[4 * c + r]);
      m[4 * r + c] = (beta == 0.0) ? e[4 * r + c] : scale(e[4 * r + c], 1.0 - beta) + scale(ud, beta);
    }
  return nearest_unitary_f64(m, uold, unew);
}

}  // namespace qf
