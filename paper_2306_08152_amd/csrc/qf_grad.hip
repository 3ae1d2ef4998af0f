// Gradient kernels: the derivative of the cost with respect to every gate
// matrix (from the environments of one half-sweep with the gates held fixed)
// and the parameterised SU(4) gates exp(i H(theta)) of the gradient-based
// baseline, with their chain rule.
//
// Cost (Sec. II): Delta = 1 - |T| / N, T = Tr(V^dagger C).  Every gate enters T
// linearly, T = Tr(E_g u_g) (Sec. III), so the real gradient packed as a
// complex matrix, G_g = dDelta/dRe u_g + i dDelta/dIm u_g, is
// -(T / |T|) E_g^dagger / N.  During the first half of Alg. 1's sweep the
// builder before gate g's turn holds u_g on its output legs and
// E_g = u_g^dagger P_g with P_g = Tr_rest(builder), so G_g = -(T/|T|) P_g^dagger
// u_g / N; moving u_g to the input legs with the gate unchanged (the fused pass
// with (A, B) = (u_g^dagger, u_g)) prepares gate g-1.  One half-sweep gives all
// p environments: memory stays one builder per start, no stored slices.
#include <hip/hip_runtime.h>

#include "qf_device.h"
#include "qf_internal.h"

namespace qf {

// grad[s][g] = -(T_s / (N |T_s|)) P_g[s]^dagger u_g[s]; zero where T_s = 0.
// envP: p x S x 16, gates: S x p x 16 (gstride = p * 16), trace: S, all c128.
__global__ void k_grad_finish(const cd* __restrict__ envP, const cd* __restrict__ gates,
                              const cd* __restrict__ trace, double N, int S, int p, cd* __restrict__ grad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)S * p * 16;
  if (e >= total) return;
  const int ij = (int)(e & 15);
  const int64_t sg = e >> 4;
  const int g = (int)(sg % p), s = (int)(sg / p);
  const int i = ij >> 2, j = ij & 3;
  const cd* P = envP + ((int64_t)g * S + s) * 16;
  const cd* u = gates + ((int64_t)s * p + g) * 16;
  cd acc = mk(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 4; ++k) cmac_cj(acc, P[4 * k + i], u[4 * k + j]);
  const cd T = trace[s];
  const double a = sqrt(norm2(T));
  cd out = mk(0.0, 0.0);
  if (!(a == 0.0)) {
    const double inv = -1.0 / (N * a);
    out = scale(T * acc, inv);
  }
  grad[e] = out;
}

hipError_t launch_grad_finish(hipStream_t st, const double* envP, const double* gates, const double* trace, int n,
                              int S, int p, double* grad) {
  const int64_t total = (int64_t)S * p * 16;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL(k_grad_finish, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const cd*>(envP),
                     reinterpret_cast<const cd*>(gates), reinterpret_cast<const cd*>(trace),
                     (double)((int64_t)1 << n), S, p, reinterpret_cast<cd*>(grad));
  return hipGetLastError();
}

// ---------------------------------------------------------------- SU(4) gates
//
// exp(i H), H = sum_k theta_k P_k over the 15 non-identity Pauli products
// P_k = sigma_a (x) sigma_b, k = 4a + b - 1.  One quad per gate, lane r
// holding row r.  H = Q diag(lambda) Q^dagger comes from the one-sided Jacobi
// of the SVD step applied to B = H + c I, c = 1 + ||H||_F > spectral radius:
// B is positive definite, so its right singular vectors are eigenvectors of H
// and its singular values are lambda + c.

__device__ __forceinline__ cd pauli1(int a, int i, int j) {
  // sigma_0 = I, sigma_1 = X, sigma_2 = Y, sigma_3 = Z
  double re = 0.0, im = 0.0;
  if (a == 0) re = (i == j) ? 1.0 : 0.0;
  if (a == 1) re = (i != j) ? 1.0 : 0.0;
  if (a == 2) im = (i == j) ? 0.0 : (i == 0 ? -1.0 : 1.0);
  if (a == 3) re = (i == j) ? (i == 0 ? 1.0 : -1.0) : 0.0;
  return mk(re, im);
}

// Entry (r, c) of P_k.
__device__ __forceinline__ cd pauli2(int k, int r, int c) {
  const int a = (k + 1) >> 2, b = (k + 1) & 3;
  return pauli1(a, r >> 1, c >> 1) * pauli1(b, r & 1, c & 1);
}

// Row r of Q (q[j] = Q[r][j]) and the eigenvalues lam[j] of H, from row r of H.
__device__ inline void quad_heig(const cd hrow[4], int r, cd q[4], double lam[4]) {
  double f2 = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) f2 += norm2(hrow[j]);
  const double c = 1.0 + sqrt(quad_sum(f2));
  cd m[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    m[j] = hrow[j];
    m[j].re += (j == r) ? c : 0.0;
    q[j] = mk(j == r ? 1.0 : 0.0, 0.0);
  }
  for (int sweep = 0; sweep < 30; ++sweep) {
    double rel = quad_round<0, 1, 2, 3>(m, q);
    rel = fmax(rel, quad_round<0, 2, 1, 3>(m, q));
    rel = fmax(rel, quad_round<0, 3, 1, 2>(m, q));
    if (!(rel > 0.0)) break;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) lam[j] = sqrt(quad_sum(norm2(m[j]))) - c;
}

__device__ __forceinline__ void load_hrow(const double* th, int r, cd h[4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) h[c] = mk(0.0, 0.0);
  for (int k = 0; k < 15; ++k) {
    const double t = th[k];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cd pk = pauli2(k, r, c);
      h[c] = h[c] + scale(pk, t);
    }
  }
}

// theta: count x 15; gates: count x 16 c128 (row-major 4 x 4).
__global__ __launch_bounds__(64) void k_su4_expm(const double* __restrict__ theta, int count, cd* __restrict__ gates) {
  const int t = threadIdx.x, r = t & 3;
  const int gi = blockIdx.x * 16 + (t >> 2);
  if (gi >= count) return;  // whole quad leaves together
  cd h[4], q[4];
  double lam[4];
  load_hrow(theta + (int64_t)gi * 15, r, h);
  quad_heig(h, r, q, lam);
  cd qa[4][4];  // qa[j][k] = Q[k][j]
#pragma unroll
  for (int j = 0; j < 4; ++j) quad_gather(q[j], qa[j]);
  cd ph[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double s, c;
    sincos(lam[j], &s, &c);
    ph[j] = mk(c, s);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cd acc = mk(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 4; ++j) cmac(acc, q[j] * ph[j], conj(qa[j][c]));
    gates[(int64_t)gi * 16 + 4 * r + c] = acc;
  }
}

// Divided difference of exp at i a and i b: (e^{ia} - e^{ib}) / (i (a - b)),
// written as e^{i (a+b)/2} sin(d) / d with d = (a - b) / 2 (e^{ia} at a = b).
__device__ __forceinline__ cd exp_divdiff(double a, double b) {
  const double d = 0.5 * (a - b);
  double sc;
  if (fabs(d) < 1e-4) {
    const double d2 = d * d;
    sc = 1.0 - d2 * (1.0 / 6.0) + d2 * d2 * (1.0 / 120.0);
  } else {
    sc = sin(d) / d;
  }
  double s, c;
  sincos(0.5 * (a + b), &s, &c);
  return mk(c * sc, s * sc);
}

// Vector-Jacobian product of the map theta -> exp(i H(theta)):
// dtheta_k = Re Tr(G^dagger dU/dtheta_k).  With H = Q diag(lambda) Q^dagger,
// dU = Q (F o (Q^dagger i dH Q)) Q^dagger, F_jl = divided difference of exp at
// (i lambda_j, i lambda_l), so dtheta_k = Re Tr(Gamma^dagger i P_k) with
// Gamma = Q (conj(F) o (Q^dagger G Q)) Q^dagger.
__global__ __launch_bounds__(64) void k_su4_vjp(const double* __restrict__ theta, const cd* __restrict__ gG,
                                                int count, double* __restrict__ dtheta) {
  const int t = threadIdx.x, r = t & 3;
  const int gi = blockIdx.x * 16 + (t >> 2);
  if (gi >= count) return;
  cd h[4], q[4];
  double lam[4];
  load_hrow(theta + (int64_t)gi * 15, r, h);
  quad_heig(h, r, q, lam);
  cd qa[4][4];  // qa[j][k] = Q[k][j]
#pragma unroll
  for (int j = 0; j < 4; ++j) quad_gather(q[j], qa[j]);
  // t_r[l] = sum_b G[r][b] Q[b][l]
  cd grow[4], tr[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) grow[b] = gG[(int64_t)gi * 16 + 4 * r + b];
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    cd acc = mk(0.0, 0.0);
#pragma unroll
    for (int b = 0; b < 4; ++b) cmac(acc, grow[b], qa[l][b]);
    tr[l] = acc;
  }
  // Y = conj(F) o W, W[j][l] = sum_a conj(Q[a][j]) t_a[l]
  cd Y[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      cd pr = conj(q[j]) * tr[l];
      const cd w = mk(quad_sum(pr.re), quad_sum(pr.im));
      Y[j][l] = conj(exp_divdiff(lam[j], lam[l])) * w;
    }
  // row r of Gamma: Gamma[r][c] = sum_{j,l} Q[r][j] Y[j][l] conj(Q[c][l])
  cd grow2[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cd acc = mk(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cd inner = mk(0.0, 0.0);
#pragma unroll
      for (int l = 0; l < 4; ++l) cmac(inner, Y[j][l], conj(qa[l][c]));
      cmac(acc, q[j], inner);
    }
    grow2[c] = acc;
  }
  // dtheta_k = Re(i Tr(Gamma^dagger P_k)) = -Im sum_{r,c} conj(Gamma[r][c]) P_k[r][c]
  for (int k = 0; k < 15; ++k) {
    double im = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cd pk = pauli2(k, r, c);
      im += grow2[c].re * pk.im - grow2[c].im * pk.re;
    }
    const double tot = -quad_sum(im);
    if (r == 0) dtheta[(int64_t)gi * 15 + k] = tot;
  }
}

hipError_t launch_su4_expm(hipStream_t st, const double* theta, int count, double* gates) {
  const unsigned blocks = (unsigned)((count + 15) / 16);
  hipLaunchKernelGGL(k_su4_expm, dim3(blocks), dim3(64), 0, st, theta, count, reinterpret_cast<cd*>(gates));
  return hipGetLastError();
}

hipError_t launch_su4_vjp(hipStream_t st, const double* theta, const double* grad_gates, int count,
                          double* dtheta) {
  const unsigned blocks = (unsigned)((count + 15) / 16);
  hipLaunchKernelGGL(k_su4_vjp, dim3(blocks), dim3(64), 0, st, theta, reinterpret_cast<const cd*>(grad_gates),
                     count, dtheta);
  return hipGetLastError();
}

}  // namespace qf
