// The finishing step of an environment launch, shared by the one-gate and
// the two-gate environment kernels: from the FP64 partial trace P of one
// start (in LDS) to the environment E = u_old^dagger P (first half of a
// sweep) or P u_old^dagger (second half), the FP64 gate update of
// Sec. III-A-1 (Eq. opt_u), and the writes of u_new and u_old.
#pragma once

#include "qf_device.h"
#include "qf_internal.h"

namespace qf {

struct EnvDev {
  EnvArgs a;
  uint32_t N, nrest, b0, b1, rlo, rhi, nwg, rests_per_wg;
};

// Finish one start on the 4 lanes of a quad (lane r = row r): P (16 FP64
// complex, LDS) -> env_out and/or the gate update.
__device__ inline void env_finish_quad(const EnvDev& d, uint32_t s, const cd* P, const cd* u_sh, bool frozen,
                                       int r, cd* un_sh = nullptr) {
  const EnvArgs& a = d.a;
  if (!a.do_update) {
    if (a.env_out) {
      cd* eo = reinterpret_cast<cd*>(a.env_out) + 16 * (size_t)s;
#pragma unroll
      for (int c = 0; c < 4; ++c) eo[4 * r + c] = P[4 * r + c];
    }
    return;
  }
  cd* gp = reinterpret_cast<cd*>(a.gates) + (int64_t)s * a.gstride + 16 * (int64_t)a.gidx;
  cd uold[16];  // loaded into LDS at kernel start, under the partial trace
#pragma unroll
  for (int k = 0; k < 16; ++k) uold[k] = u_sh[k];
  // E = u_old^dagger P (half 0) or P u_old^dagger (half 1): the removal of the
  // old gate commutes with the partial trace.  Row r of E:
  cd erow[4], urow[4], unew[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cd acc = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (a.half == 0)
        cmac(acc, conj(at_kr(uold, k, r)), P[4 * k + c]);
      else
        cmac(acc, P[4 * r + k], conj(uold[4 * c + k]));
    }
    erow[c] = acc;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cd v = uold[c];
#pragma unroll
    for (int rr = 1; rr < 4; ++rr) v = sel(r == rr, uold[4 * rr + c], v);
    urow[c] = v;
  }
  if (a.env_out) {
    cd* eo = reinterpret_cast<cd*>(a.env_out) + 16 * (size_t)s;
#pragma unroll
    for (int c = 0; c < 4; ++c) eo[4 * r + c] = erow[c];
  }
  if (frozen) {
#pragma unroll
    for (int c = 0; c < 4; ++c) unew[c] = urow[c];
  } else {
    update_gate_quad(a.kind, erow, uold, r, a.beta, unew);
  }
  cd* uo = reinterpret_cast<cd*>(a.uold) + a.uold_stride * (size_t)s;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uo[4 * r + c] = urow[c];
    gp[4 * r + c] = unew[c];
    if (un_sh) un_sh[4 * r + c] = unew[c];
  }
}

// The general U(4) update on the 16 lanes of a hex (lane i = entry
// (hex_row(i), i & 3)): the Newton polar form, or the hex Jacobi form
// (bitwise the quad form's result) where that declines.
// y_sh: the warm-start rotation (row-major, LDS) when a.ywarm is set,
// fetched at kernel start by ywarm_fetch.
__device__ inline void env_finish_hex(const EnvDev& d, uint32_t s, cd* P, const cd* u_sh, bool frozen,
                                      int i, cd* un_sh = nullptr, const cd* y_sh = nullptr) {
  const EnvArgs& a = d.a;
  const int r = hex_row(i), c = i & 3;
  const cd e = env_entry(P, u_sh, a.half, r, c);
  const cd urc = u_sh[4 * r + c];
  if (a.env_out) reinterpret_cast<cd*>(a.env_out)[16 * (size_t)s + 4 * r + c] = e;
  cd unew = urc;
  cd* yp = a.ywarm ? reinterpret_cast<cd*>(a.ywarm) + a.ywstride * (size_t)s + 32 * a.gidx + 16 * a.half + 4 * r + c
                   : nullptr;
  cd yv = y_sh ? y_sh[4 * r + c] : (yp ? *yp : mk(0.0, 0.0));
  // every lane has read P (env_entry) before the update's lane exchange overwrites it
  if (!frozen) optimize_gate_f64_hex(e, u_sh[4 * c + r], urc, r, c, a.beta, unew, P, yp ? &yv : nullptr, a.warm != 0);
  if (yp) *yp = yv;
  reinterpret_cast<cd*>(a.uold)[a.uold_stride * (size_t)s + 4 * r + c] = urc;
  reinterpret_cast<cd*>(a.gates)[(int64_t)s * a.gstride + 16 * (int64_t)a.gidx + 4 * r + c] = unew;
  if (un_sh) un_sh[4 * r + c] = unew;
}

// Lane k < 16 of the caller fetches entry k of start s's warm-start
// rotation into y_sh (under the partial trace; a later barrier publishes it).
__device__ __forceinline__ void ywarm_fetch(const EnvArgs& a, uint32_t s, uint32_t k, cd* y_sh) {
  if (a.ywarm && a.do_update && a.kind == kKindU4 && k < 16)
    y_sh[k] = reinterpret_cast<const cd*>(a.ywarm)[a.ywstride * (size_t)s + 32 * a.gidx + 16 * a.half + k];
}

// The finishing step of one start by the lanes it needs.  P (LDS) is read
// first and then serves the general update's lane exchange, so it is
// overwritten.
__device__ __forceinline__ void env_finish(const EnvDev& d, uint32_t s, cd* P, const cd* u_sh, bool frozen,
                                          uint32_t t, cd* un_sh = nullptr, const cd* y_sh = nullptr) {
  if (d.a.do_update && d.a.kind == kKindU4) {
    if (t < 16) env_finish_hex(d, s, P, u_sh, frozen, (int)t, un_sh, d.a.ywarm ? y_sh : nullptr);
  } else if (t < 4) {
    env_finish_quad(d, s, P, u_sh, frozen, (int)t, un_sh);
  }
}

}  // namespace qf
