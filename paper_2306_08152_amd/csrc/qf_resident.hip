// LDS-resident QFactor: one workgroup per start holds its whole builder in
// LDS (n <= 6: 64 KiB in complex128) and runs every sweep of the
// instantiation in one cooperative launch.  After each sweep every start
// publishes its termination flags, the workgroups meet at a device-scope
// barrier (bounded spin), and each one takes the same job decision from the
// same flags, so the multistart rule of Sec. IV-A is applied in lockstep.
#include <hip/hip_runtime.h>

#include "qf_device.h"
#include "qf_internal.h"
#include "qf_termination.h"

namespace qf {

constexpr int kResThreads = 256;
constexpr long long kSpinLimit = 1ll << 25;  // bounded barrier wait (~2 s of s_sleep)

template <typename R>
struct ResLds {
  cx<R>* X;     // N x N builder
  cd* Y;        // N x N FP64 scratch builder (complex64 form only), else nullptr
  cd* red;      // 256
  cx<R>* opsR;  // 32: A then B in builder precision
  cd* opsD;     // 32: FP64 copies (FP64 rebuilds)
  int* word;    // 4 ints of workgroup-shared control
};

// X <- (A (x) I) X (B (x) I) on the LDS builder (either side optional).
template <typename R, bool HA, bool HB>
__device__ inline void lds_pass(cx<R>* X, uint32_t n, uint32_t b0, uint32_t b1, const cx<R>* A,
                                const cx<R>* B) {
  const uint32_t N = 1u << n, lo = b0 < b1 ? b0 : b1, hi = b0 < b1 ? b1 : b0;
  const uint32_t q = N >> 2, nblk = q * q;
  cx<R> a[16], b[16];
  if (HA)
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = A[k];
  if (HB)
#pragma unroll
    for (int k = 0; k < 16; ++k) b[k] = B[k];
  for (uint32_t blk = threadIdx.x; blk < nblk; blk += blockDim.x) {
    const uint32_t rq = blk / q, cq = blk - rq * q;
    const uint32_t rb = insert00(rq, lo, hi), cb = insert00(cq, lo, hi);
    uint32_t off[4];
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) off[i] = local_off(i, b0, b1);
    cx<R> x[16];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) x[4 * i + j] = X[(rb + off[i]) * N + cb + off[j]];
    if (HA) {
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
    if (HB) {
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
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) X[(rb + off[i]) * N + cb + off[j]] = x[4 * i + j];
  }
}

// Partial trace of the LDS builder over every qubit but the gate's, FP64,
// fixed summation order.  Result in red[0..15]; ends with a barrier.
template <typename R>
__device__ inline void lds_ptrace(const cx<R>* X, uint32_t n, uint32_t b0, uint32_t b1, cd* red) {
  const uint32_t N = 1u << n, lo = b0 < b1 ? b0 : b1, hi = b0 < b1 ? b1 : b0;
  const uint32_t t = threadIdx.x, ij = t & 15u;
  const uint32_t ro = local_off(ij >> 2, b0, b1), co = local_off(ij & 3u, b0, b1);
  cd acc = mk(0.0, 0.0);
  for (uint32_t rest = t >> 4; rest < (N >> 2); rest += 16) {
    const uint32_t base = insert00(rest, lo, hi);
    const cx<R> v = X[(base + ro) * N + base + co];
    acc = acc + mk((double)v.re, (double)v.im);
  }
  red[t] = acc;
  __syncthreads();
  for (uint32_t stride = 128; stride >= 16; stride >>= 1) {
    if (t < stride) red[t] = red[t] + red[t + stride];
    __syncthreads();
  }
}

// Trace in FP64 (fixed order); ends with a barrier; result in red[0].
template <typename R>
__device__ inline cd lds_trace(const cx<R>* X, uint32_t N, cd* red) {
  const uint32_t t = threadIdx.x;
  cd acc = mk(0.0, 0.0);
  for (uint32_t r = t; r < N; r += blockDim.x) acc = acc + mk((double)X[r * N + r].re, (double)X[r * N + r].im);
  red[t] = acc;
  __syncthreads();
  for (uint32_t stride = 128; stride >= 1; stride >>= 1) {
    if (t < stride) red[t] = red[t] + red[t + stride];
    __syncthreads();
  }
  const cd tr = red[0];
  __syncthreads();
  return tr;
}

// Builder <- G_p ... G_1 V^dagger in precision Q, gates from global FP64.
template <typename Q>
__device__ inline void lds_build(cx<Q>* X, const ResidentArgs& a, const cd* V, const cd* gates,
                                 cx<Q>* ops) {
  const uint32_t N = 1u << a.n;
  for (uint32_t e = threadIdx.x; e < N * N; e += blockDim.x) {
    const uint32_t r = e / N, c = e - r * N;
    const cd v = conj(V[(size_t)c * N + r]);
    X[e] = cx<Q>{(Q)v.re, (Q)v.im};
  }
  for (int g = 0; g < a.p; ++g) {
    __syncthreads();
    if (threadIdx.x < 16) {
      const cd v = gates[16 * g + threadIdx.x];
      ops[threadIdx.x] = cx<Q>{(Q)v.re, (Q)v.im};
    }
    __syncthreads();
    const uint32_t b0 = a.n - 1 - a.locs[2 * g], b1 = a.n - 1 - a.locs[2 * g + 1];
    lds_pass<Q, true, false>(X, a.n, b0, b1, ops, nullptr);
  }
  __syncthreads();
}

__device__ inline bool grid_barrier(int32_t* sync, int32_t target, int32_t* timeout_flag) {
  __threadfence();
  __hip_atomic_fetch_add(&sync[0], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  long long spins = 0;
  while (__hip_atomic_load(&sync[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (__hip_atomic_load(timeout_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (++spins > kSpinLimit) {
      __hip_atomic_store(timeout_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  __threadfence();
  return true;
}

template <typename R>
__global__ __launch_bounds__(kResThreads) void k_resident(ResidentArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint32_t n = a.n, N = 1u << n;
  const uint32_t s = blockIdx.x;
  const uint32_t t = threadIdx.x;
  const bool c64 = (sizeof(R) == 4);
  ResLds<R> L;
  unsigned char* p = smem_raw;
  L.X = reinterpret_cast<cx<R>*>(p);
  p += sizeof(cx<R>) * N * N;
  L.Y = nullptr;
  if (c64) {
    L.Y = reinterpret_cast<cd*>(p);
    p += sizeof(cd) * N * N;
  }
  L.red = reinterpret_cast<cd*>(p);
  p += sizeof(cd) * kResThreads;
  L.opsD = reinterpret_cast<cd*>(p);
  p += sizeof(cd) * 32;
  L.opsR = reinterpret_cast<cx<R>*>(p);
  p += sizeof(cx<R>) * 32;
  L.word = reinterpret_cast<int*>(p);

  const cd* V = reinterpret_cast<const cd*>(a.V);
  cd* gates = reinterpret_cast<cd*>(a.gates) + (size_t)s * a.p * 16;
  int32_t* timeout_flag = &a.out_info[4];
  const qf_options& o = a.opt;

  // FP64 cost of the current gates (fresh complex128 builder).
  auto fp64_cost = [&]() -> double {
    cd* Yb = c64 ? L.Y : reinterpret_cast<cd*>(L.X);
    lds_build<double>(Yb, a, V, gates, L.opsD);
    const cd tr = lds_trace<double>(Yb, N, L.red);
    return 1.0 - sqrt(norm2(tr)) / (double)N;
  };
  // Builder cost (its own precision, FP64 sums).
  auto builder_cost = [&]() -> double {
    const cd tr = lds_trace<R>(L.X, N, L.red);
    return 1.0 - sqrt(norm2(tr)) / (double)N;
  };
  auto rebuild = [&]() {
    if (c64) {
      // complex64 builder rounded from a fresh FP64 build
      lds_build<double>(L.Y, a, V, gates, L.opsD);
      for (uint32_t e = t; e < N * N; e += blockDim.x)
        L.X[e] = cx<R>{(R)L.Y[e].re, (R)L.Y[e].im};
      __syncthreads();
    } else {
      lds_build<R>(L.X, a, V, gates, L.opsR);
    }
  };

  rebuild();
  double c_cur = builder_cost();
  // complex64: once the cost is below recheck_below the sweeps run on the
  // FP64 builder Y (escalated), whose costs need no recheck.
  bool esc = false;
  if (c64 && c_cur < o.recheck_below) {  // the FP64 build is still in Y
    const cd tr = lds_trace<double>(L.Y, N, L.red);
    c_cur = 1.0 - sqrt(norm2(tr)) / (double)N;
    esc = true;
  }
  double* hist = a.hist + (size_t)s * a.ring;
  if (t == 0) {
    if (!isfinite(c_cur)) c_cur = __builtin_inf();
    hist[0] = c_cur;
    a.flags[s] = isfinite(c_cur) ? 0 : (kFlagNumeric | kFlagPlateau);
    a.cur_cost[s] = c_cur;
    if (a.history_out && a.history_rows > 0) a.history_out[s] = c_cur;
  }
  int32_t my_flags = isfinite(c_cur) ? 0 : (kFlagNumeric | kFlagPlateau);
  int32_t i = 0;
  int32_t decision = kContinue;
  int32_t resets = 0, rechecks = 0;
  // An empty run (max_iter <= 0) stops before the first sweep.
  if (o.max_iter <= 0) decision = kStopMaxIter;

  while (decision == kContinue) {
    ++i;
    const bool frozen = (my_flags & kFlagNumeric) != 0;
    // ---------------- TwoSidedSweep (Alg. 1 order)
    for (int step = 0; step < 2 * a.p; ++step) {
      const int half = step < a.p ? 0 : 1;
      const int g = half == 0 ? a.p - 1 - step : step - a.p;
      const uint32_t b0 = n - 1 - a.locs[2 * g], b1 = n - 1 - a.locs[2 * g + 1];
      if (c64 && esc)
        lds_ptrace<double>(L.Y, n, b0, b1, L.red);
      else
        lds_ptrace<R>(L.X, n, b0, b1, L.red);
      const int kind = a.kinds ? a.kinds[g] : kKindU4;
      if (kind == kKindU4) {
        if (t < 16) {  // general U(4) update on one hex, lane t = entry (hex_row(t), t & 3)
          const int r = hex_row((int)t), c = (int)t & 3;
          const cd ucr = gates[16 * g + 4 * c + r], urc = gates[16 * g + 4 * r + c];
          const cd e = env_entry(L.red, gates + 16 * g, half, r, c);
          cd unew = urc;
          // warm start from this gate's rotation of the previous sweep
          cd* yp = reinterpret_cast<cd*>(a.ywarm) + ((size_t)s * a.p + g) * 32 + 16 * half + 4 * r + c;
          cd yv = *yp;
          // the partial trace is read (env_entry) before the update's lane exchange overwrites it
          if (!frozen)
            optimize_gate_f64_hex(e, ucr, urc, r, c, o.beta, unew, L.red, &yv, ((i - 1) % kWarmPeriod) != 0);
          *yp = yv;
          gates[16 * g + 4 * r + c] = unew;
          const cd udc = conj(ucr);  // (u_old^dagger)[r][c]
          const cd Av = sel(half == 0, udc, unew), Bv = sel(half == 0, unew, udc);
          L.opsR[4 * r + c] = cx<R>{(R)Av.re, (R)Av.im};
          L.opsR[16 + 4 * r + c] = cx<R>{(R)Bv.re, (R)Bv.im};
          L.opsD[4 * r + c] = Av;
          L.opsD[16 + 4 * r + c] = Bv;
        }
      } else if (t < 4) {  // restricted kinds on one quad, lane r = row r
        const int r = (int)t;
        cd uold[16], erow[4], urow[4], unew[4];
#pragma unroll
        for (int k = 0; k < 16; ++k) uold[k] = gates[16 * g + k];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          cd acc = mk(0.0, 0.0);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            if (half == 0)
              cmac(acc, conj(at_kr(uold, k, r)), L.red[4 * k + c]);
            else
              cmac(acc, L.red[4 * r + k], conj(uold[4 * c + k]));
          }
          erow[c] = acc;
          cd v = uold[c];
#pragma unroll
          for (int rr = 1; rr < 4; ++rr) v = sel(r == rr, uold[4 * rr + c], v);
          urow[c] = v;
        }
        if (frozen) {
#pragma unroll
          for (int c = 0; c < 4; ++c) unew[c] = urow[c];
        } else {
          update_gate_quad(kind, erow, uold, r, o.beta, unew);
        }
        // half 0: X <- (u_old^dagger (x) I) X (u_new (x) I); half 1 mirrored.
        // Row r of u_old^dagger is conj(column r of u_old).
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          gates[16 * g + 4 * r + c] = unew[c];
          cd udc = uold[c * 4];
#pragma unroll
          for (int rr = 1; rr < 4; ++rr) udc = sel(r == rr, uold[4 * c + rr], udc);
          udc = conj(udc);
          const cd Av = sel(half == 0, udc, unew[c]), Bv = sel(half == 0, unew[c], udc);
          L.opsR[4 * r + c] = cx<R>{(R)Av.re, (R)Av.im};
          L.opsR[16 + 4 * r + c] = cx<R>{(R)Bv.re, (R)Bv.im};
          L.opsD[4 * r + c] = Av;
          L.opsD[16 + 4 * r + c] = Bv;
        }
      }
      __syncthreads();
      if (c64 && esc)
        lds_pass<double, true, true>(L.Y, n, b0, b1, L.opsD, L.opsD + 16);
      else
        lds_pass<R, true, true>(L.X, n, b0, b1, L.opsR, L.opsR + 16);
      __syncthreads();
    }
    // ---------------- cost, reset, recheck
    if (o.reset_iter > 0 && (i % o.reset_iter) == 0) {
      rebuild();
      ++resets;
    }
    double c_i;
    if (c64 && esc) {
      const cd tr = lds_trace<double>(L.Y, N, L.red);
      c_i = 1.0 - sqrt(norm2(tr)) / (double)N;
    } else {
      c_i = builder_cost();
    }
    if (c64 && !esc && c_i < o.recheck_below) {
      // FP64 cost from a fresh complex128 builder, which the sweeps use from
      // now on
      c_i = fp64_cost();
      ++rechecks;
      esc = true;
    }
    // ---------------- termination (lockstep over starts)
    if (t == 0) {
      const double c_prev = hist[(i - 1) % a.ring];
      const int32_t Lh = o.long_diff_count;
      const double c_back = (Lh > 0 && i >= Lh) ? hist[(i - Lh) % a.ring] : 0.0;
      if (!isfinite(c_i)) c_i = __builtin_inf();
      my_flags = (my_flags & kFlagNumeric) ? my_flags
                                           : start_flags_after_sweep(o, a.tol, i, my_flags, c_i, c_prev, c_back);
      if (my_flags & kFlagNumeric) c_i = __builtin_inf();
      hist[i % a.ring] = c_i;
      a.cur_cost[s] = c_i;
      if (a.history_out && i < a.history_rows) a.history_out[(size_t)i * a.S + s] = c_i;
      a.flags[(size_t)(i & 1) * a.S + s] = my_flags;
      bool ok = grid_barrier(a.sync, a.S * i, timeout_flag);
      int32_t dcs = kStopMaxIter;
      if (ok) dcs = job_decision(o, i, a.flags + (size_t)(i & 1) * a.S, a.S);
      L.word[0] = dcs;
      L.word[1] = my_flags;
    }
    __syncthreads();
    decision = L.word[0];
    my_flags = L.word[1];
    __syncthreads();
  }
  // ---------------- final FP64 cost of the returned gates
  const double cf = fp64_cost();
  if (t == 0) {
    a.final_cost[s] = (my_flags & kFlagNumeric) || !isfinite(cf) ? __builtin_inf() : cf;
    if (s == 0) {
      a.out_info[0] = i;
      a.out_info[1] = decision;
      a.out_info[2] = resets;
    }
    __hip_atomic_fetch_add(&a.out_info[3], rechecks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

size_t resident_lds_bytes(int n, int precision) {
  const size_t N = (size_t)1 << n;
  size_t b = 0;
  if (precision == QF_C64)
    b += N * N * 8 + N * N * 16 + 32 * 8;
  else
    b += N * N * 16 + 32 * 16;
  b += 16 * kResThreads + 16 * 32 + 16;
  return b;
}

hipError_t launch_resident(hipStream_t st, const ResidentArgs& a, int* ok_coresident) {
  const size_t lds = resident_lds_bytes(a.n, a.precision);
  const void* fn = a.precision == QF_C64 ? reinterpret_cast<const void*>(&k_resident<float>)
                                         : reinterpret_cast<const void*>(&k_resident<double>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, per_cu = 0, cus = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kResThreads, lds);
  if (e != hipSuccess) return e;
  *ok_coresident = (per_cu > 0 && (long long)per_cu * cus >= a.S) ? 1 : 0;
  if (!*ok_coresident) return hipSuccess;
  ResidentArgs args = a;
  void* kargs[] = {&args};
  return hipLaunchCooperativeKernel(fn, dim3(a.S), dim3(kResThreads), kargs, (unsigned)lds, st);
}

}  // namespace qf
