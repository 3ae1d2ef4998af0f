// Batched QFactor: many independent small problems (n <= 4 qubits, builders
// up to 16 x 16) in one persistent launch.
//
// One workgroup is one wavefront of 16 quads.  Each quad owns one (block,
// start) instantiation: its builder lives in LDS, lane r of the quad sums row
// r of the partial trace, the quad runs the FP64 nearest-unitary step of
// Sec. III-A-1 (one row per lane), and the lanes share the 4x4 block updates
// of the fused remove/re-apply.  The starts of one block sit in adjacent
// quads of the same wavefront and take the multistart decision of Sec. IV-A
// together after every sweep (flags exchanged through LDS).  Wavefronts take
// groups of blocks from a device-side counter until the queue is empty, so
// every wavefront reaches the exit.
#include <hip/hip_runtime.h>

#include "qf_device.h"
#include "qf_internal.h"
#include "qf_termination.h"

namespace qf {

constexpr int kBQuads = 16;     // quads per wavefront
constexpr int kBNmax = 16;      // largest builder side (n <= 4)

__device__ __forceinline__ void wave_sync() { __syncthreads(); }  // one-wave workgroup

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
  return v;
}

// Left product by a 4x4 gate (A) and right product (B) on one quad's N x N
// builder in LDS; lane r takes blocks r, r + 4, ...
template <typename R, bool HA, bool HB>
__device__ inline void quad_pass(cx<R>* X, uint32_t N, uint32_t b0, uint32_t b1, const cx<R> a[16],
                                 const cx<R> b[16], int r) {
  const uint32_t lo = b0 < b1 ? b0 : b1, hi = b0 < b1 ? b1 : b0;
  const uint32_t q = N >> 2, nblk = q * q;
  uint32_t off[4];
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) off[i] = local_off(i, b0, b1);
  for (uint32_t blk = (uint32_t)r; blk < nblk; blk += 4) {
    const uint32_t rb = insert00(blk / q, lo, hi), cb = insert00(blk % q, lo, hi);
    cx<R> x[16];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) x[4 * i + j] = X[(rb + off[i]) * N + cb + off[j]];
    if (HA) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cx<R> t[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          cx<R> acc = mk<R>(0, 0);
#pragma unroll
          for (int k = 0; k < 4; ++k) cmac(acc, a[4 * i + k], x[4 * k + j]);
          t[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) x[4 * i + j] = t[i];
      }
    }
    if (HB) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        cx<R> t[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cx<R> acc = mk<R>(0, 0);
#pragma unroll
          for (int l = 0; l < 4; ++l) cmac(acc, x[4 * i + l], b[4 * l + j]);
          t[j] = acc;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) x[4 * i + j] = t[j];
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) X[(rb + off[i]) * N + cb + off[j]] = x[4 * i + j];
  }
}

struct BatchDev {
  int n_blocks, S, B, n_groups;
  const int32_t* order;     // processing order of the blocks
  const int32_t* blk_n;     // qubits per block
  const int32_t* gate_off;  // n_blocks + 1 prefix sums of gate counts
  const int64_t* tgt_off;   // complex-entry offset of each target
  const int32_t* locs;      // total_gates x 2
  const cd* V;              // targets
  cd* gates;                // in: initial gates, out: final gates
  double tol;
  qf_options opt;
  double* hist;             // (block, start) x ring
  int ring;
  cd* scratch;              // FP64 builder per (workgroup, quad): N_max^2 each
  double* out_cost;         // (block, start)
  int32_t* out_best, *out_status, *out_sweeps;
  int32_t* queue;           // work counter (zero before launch)
  const int32_t* kinds;     // gate kinds over all gates (nullptr = all general U(4))
};

// Per-quad problem description.
struct QuadJob {
  bool valid;
  int b, s, n, p;
  uint32_t N;
  const int32_t* locs;  // this block's locations
  const cd* V;          // this block's target
  cd* g;                // this start's gates (p x 16)
  const int32_t* kinds; // this block's gate kinds (nullptr = all general U(4))
};

// Builder <- G_p ... G_1 V^dagger for one quad, in precision Q, at X
// (LDS or global).  All quads of the wavefront call it with the same
// pmax (uniform barriers); inactive quads only take part in the barriers.
template <typename Q>
__device__ inline void quad_build(cx<Q>* X, const QuadJob& jb, int r, int pmax) {
  if (jb.valid) {
    const uint32_t N = jb.N;
    for (uint32_t e = (uint32_t)r; e < N * N; e += 4) {
      const uint32_t row = e / N, col = e - row * N;
      const cd v = conj(jb.V[col * N + row]);
      X[e] = cx<Q>{(Q)v.re, (Q)v.im};
    }
  }
  for (int g = 0; g < pmax; ++g) {
    wave_sync();
    if (jb.valid && g < jb.p) {
      cx<Q> a[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const cd v = jb.g[16 * g + k];
        a[k] = cx<Q>{(Q)v.re, (Q)v.im};
      }
      const uint32_t b0 = (uint32_t)(jb.n - 1 - jb.locs[2 * g]), b1 = (uint32_t)(jb.n - 1 - jb.locs[2 * g + 1]);
      quad_pass<Q, true, false>(X, jb.N, b0, b1, a, a, r);
    }
  }
  wave_sync();
}

// 1 - |Tr X| / N for one quad (all lanes get the same value).
template <typename Q>
__device__ inline double quad_cost(const cx<Q>* X, uint32_t N, int r) {
  double re = 0.0, im = 0.0;
  for (uint32_t d = (uint32_t)r; d < N; d += 4) {
    re += (double)X[d * N + d].re;
    im += (double)X[d * N + d].im;
  }
  re = quad_sum(re);
  im = quad_sum(im);
  return 1.0 - sqrt(re * re + im * im) / (double)N;
}

template <typename R>
__global__ __launch_bounds__(64) void k_batch(BatchDev d) {
  __shared__ __align__(16) cx<R> Xs[kBQuads][kBNmax * kBNmax];
  __shared__ int flags_sh[kBQuads];
  __shared__ int grp_sh;
  const int t = threadIdx.x, q = t >> 2, r = t & 3;
  const qf_options& o = d.opt;
  cx<R>* X = Xs[q];
  cd* Y = d.scratch + ((size_t)blockIdx.x * kBQuads + q) * (kBNmax * kBNmax);
  const bool c64 = sizeof(R) == 4;

  for (;;) {
    if (t == 0) grp_sh = __hip_atomic_fetch_add(d.queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wave_sync();
    const int grp = grp_sh;
    wave_sync();
    if (grp >= d.n_groups) break;

    // ---- this quad's job
    QuadJob jb;
    const int slot = q / d.S;
    jb.s = q - slot * d.S;
    const int idx = grp * d.B + slot;
    jb.valid = (slot < d.B) && (idx < d.n_blocks);
    jb.b = jb.valid ? d.order[idx] : 0;
    jb.n = jb.valid ? d.blk_n[jb.b] : 2;
    jb.N = 1u << jb.n;
    jb.p = jb.valid ? d.gate_off[jb.b + 1] - d.gate_off[jb.b] : 0;
    jb.locs = d.locs + 2 * (size_t)d.gate_off[jb.b];
    jb.V = d.V + (jb.valid ? d.tgt_off[jb.b] : 0);
    jb.g = d.gates + ((size_t)d.gate_off[jb.b] * d.S + (size_t)jb.s * jb.p) * 16;
    jb.kinds = d.kinds ? d.kinds + d.gate_off[jb.b] : nullptr;
    const int pmax = wave_max_int(jb.p);
    double* hist = d.hist + ((size_t)jb.b * d.S + jb.s) * d.ring;

    // ---- InitCircuitTensor and initial cost
    auto rebuild = [&]() {
      if (c64) {
        quad_build<double>(reinterpret_cast<cx<double>*>(Y), jb, r, pmax);
        if (jb.valid)
          for (uint32_t e = (uint32_t)r; e < jb.N * jb.N; e += 4) X[e] = cx<R>{(R)Y[e].re, (R)Y[e].im};
        wave_sync();
      } else {
        quad_build<R>(X, jb, r, pmax);
      }
    };
    auto fp64_cost = [&]() -> double {  // fresh complex128 builder in the quad's scratch
      quad_build<double>(reinterpret_cast<cx<double>*>(Y), jb, r, pmax);
      return jb.valid ? quad_cost<double>(reinterpret_cast<cx<double>*>(Y), jb.N, r) : 0.0;
    };
    rebuild();
    double c_cur = jb.valid ? quad_cost<R>(X, jb.N, r) : 0.0;
    int32_t my_flags = 0;
    if (c64 && jb.valid && c_cur < o.recheck_below)
      c_cur = quad_cost<double>(reinterpret_cast<cx<double>*>(Y), jb.N, r);
    if (!isfinite(c_cur)) {
      c_cur = __builtin_inf();
      my_flags = kFlagNumeric | kFlagPlateau;
    }
    if (jb.valid && r == 0) hist[0] = c_cur;

    bool running = jb.valid && o.max_iter > 0;
    int32_t decision = kStopMaxIter;
    int i = 0, sweeps = 0;
    while (__any(running ? 1 : 0)) {
      ++i;
      // ---- one TwoSidedSweep (Alg. 1 order); quads of smaller blocks idle
      const int steps = 2 * wave_max_int(running ? jb.p : 0);
      for (int step = 0; step < steps; ++step) {
        const bool act = running && step < 2 * jb.p;
        const int half = (act && step >= jb.p) ? 1 : 0;
        const int g = act ? (half == 0 ? jb.p - 1 - step : step - jb.p) : 0;
        const uint32_t b0 = act ? (uint32_t)(jb.n - 1 - jb.locs[2 * g]) : 0u;
        const uint32_t b1 = act ? (uint32_t)(jb.n - 1 - jb.locs[2 * g + 1]) : 1u;
        cx<R> A[16], Bm[16];
        if (act) {
          // partial trace, row r: P[r][j] = sum_rest X[(r, rest), (j, rest)]
          const uint32_t lo = b0 < b1 ? b0 : b1, hi = b0 < b1 ? b1 : b0;
          const uint32_t ro = local_off((uint32_t)r, b0, b1);
          cd prow[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t co = local_off((uint32_t)j, b0, b1);
            double re = 0.0, im = 0.0;
            for (uint32_t rest = 0; rest < (jb.N >> 2); ++rest) {
              const uint32_t base = insert00(rest, lo, hi);
              const cx<R> v = X[(base + ro) * jb.N + base + co];
              re += (double)v.re;
              im += (double)v.im;
            }
            prow[j] = mk(re, im);
          }
          cd P[4][4];  // P[k][c], gathered over the quad
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            cd col[4];
            quad_gather(prow[c], col);
#pragma unroll
            for (int k = 0; k < 4; ++k) P[k][c] = col[k];
          }
          cd uold[16];
#pragma unroll
          for (int k = 0; k < 16; ++k) uold[k] = jb.g[16 * g + k];
          cd erow[4], unew[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            cd acc = mk(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              if (half == 0)
                cmac(acc, conj(at_kr(uold, k, r)), P[k][c]);
              else {
                cd prk = P[0][k];  // P[r][k] by a select chain
#pragma unroll
                for (int rr = 1; rr < 4; ++rr) prk = sel(r == rr, P[rr][k], prk);
                cmac(acc, prk, conj(uold[4 * c + k]));
              }
            }
            erow[c] = acc;
          }
          if (my_flags & kFlagNumeric) {
#pragma unroll
            for (int c = 0; c < 4; ++c) unew[c] = at_rk(uold, r, c);
          } else {
            update_gate_quad(jb.kinds ? jb.kinds[g] : kKindU4, erow, uold, r, o.beta, unew);
          }
#pragma unroll
          for (int c = 0; c < 4; ++c) jb.g[16 * g + 4 * r + c] = unew[c];
          // full u_new in every lane, then the pass operands
          cd un[16];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            cd col[4];
            quad_gather(unew[c], col);
#pragma unroll
            for (int k = 0; k < 4; ++k) un[4 * k + c] = col[k];
          }
#pragma unroll
          for (int i2 = 0; i2 < 4; ++i2)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const cd ud = conj(uold[4 * c + i2]);  // (u_old^dagger)[i2][c]
              const cd nv = un[4 * i2 + c];
              const cd av = sel(half == 0, ud, nv), bv = sel(half == 0, nv, ud);
              A[4 * i2 + c] = cx<R>{(R)av.re, (R)av.im};
              Bm[4 * i2 + c] = cx<R>{(R)bv.re, (R)bv.im};
            }
        }
        wave_sync();  // every lane's trace reads are done before any block is rewritten
        if (act) quad_pass<R, true, true>(X, jb.N, b0, b1, A, Bm, r);
        wave_sync();
      }
      // ---- cost, reset, recheck, per-start tests
      if (o.reset_iter > 0 && (i % o.reset_iter) == 0) rebuild();
      double c_i = running ? quad_cost<R>(X, jb.N, r) : c_cur;
      const bool need = c64 && running && c_i < o.recheck_below;
      if (__any(need ? 1 : 0)) {
        const double cf = fp64_cost();
        if (need) {
          c_i = cf;
          for (uint32_t e = (uint32_t)r; e < jb.N * jb.N; e += 4) X[e] = cx<R>{(R)Y[e].re, (R)Y[e].im};
        }
        wave_sync();
      }
      if (running) {
        const int32_t Lh = o.long_diff_count;
        const double c_prev = hist[(i - 1) % d.ring];
        const double c_back = (Lh > 0 && i >= Lh) ? hist[(i - Lh) % d.ring] : 0.0;
        if (!isfinite(c_i)) c_i = __builtin_inf();
        if (!(my_flags & kFlagNumeric)) my_flags = start_flags_after_sweep(o, d.tol, i, my_flags, c_i, c_prev, c_back);
        if (my_flags & kFlagNumeric) c_i = __builtin_inf();
        c_cur = c_i;
        if (r == 0) hist[i % d.ring] = c_i;  // other lanes read other ring slots
      }
      if (r == 0) flags_sh[q] = my_flags;
      wave_sync();
      if (running) {
        decision = job_decision(o, i, &flags_sh[slot * d.S], d.S);
        if (decision != kContinue) {
          running = false;
          sweeps = i;
        }
      }
      wave_sync();
    }
    // ---- final FP64 cost of every start, best start per block
    const double cf = fp64_cost();
    double cfin = (my_flags & kFlagNumeric) || !isfinite(cf) ? __builtin_inf() : cf;
    if (jb.valid && r == 0) d.out_cost[(size_t)jb.b * d.S + jb.s] = cfin;
    if (r == 0) flags_sh[q] = my_flags;
    wave_sync();
    if (jb.valid && jb.s == 0 && r == 0) {
      int best = 0;
      double bc = d.out_cost[(size_t)jb.b * d.S];
      bool all_numeric = (flags_sh[q] & kFlagNumeric) != 0;
      for (int k = 1; k < d.S; ++k) {
        const double ck = d.out_cost[(size_t)jb.b * d.S + k];
        all_numeric = all_numeric && (flags_sh[q + k] & kFlagNumeric);
        if (ck < bc) {
          bc = ck;
          best = k;
        }
      }
      d.out_best[jb.b] = best;
      int st = QF_MAX_ITER;
      if (all_numeric)
        st = QF_NUMERIC;
      else if (bc < d.tol)
        st = QF_CONVERGED;
      else if (decision == kStopPlateau)
        st = QF_PLATEAU;
      d.out_status[jb.b] = st;
      d.out_sweeps[jb.b] = sweeps;
    }
    wave_sync();
  }
}

size_t batch_scratch_entries(int grid) { return (size_t)grid * kBQuads * kBNmax * kBNmax; }

int batch_groups(int n_blocks, int S) {
  const int B = kBQuads / S;
  return (n_blocks + B - 1) / B;
}

int batch_grid(int precision, int n_groups) {
  int dev = 0, cus = 256, per = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const void* fn = precision == QF_C64 ? reinterpret_cast<const void*>(&k_batch<float>)
                                       : reinterpret_cast<const void*>(&k_batch<double>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 64, 0) != hipSuccess || per < 1) per = 1;
  int g = cus * per;
  if (g > kBatchMaxGrid) g = kBatchMaxGrid;
  return g < n_groups ? g : n_groups;
}

hipError_t launch_batch(hipStream_t st, int precision, int grid, const BatchArgs& a) {
  BatchDev d;
  d.n_blocks = a.n_blocks;
  d.S = a.S;
  d.B = kBQuads / a.S;
  d.n_groups = batch_groups(a.n_blocks, a.S);
  if (grid < 1 || grid > kBatchMaxGrid || grid > d.n_groups) return hipErrorInvalidValue;
  d.order = a.order;
  d.blk_n = a.blk_n;
  d.gate_off = a.gate_off;
  d.tgt_off = a.tgt_off;
  d.locs = a.locs;
  d.V = reinterpret_cast<const cd*>(a.V);
  d.gates = reinterpret_cast<cd*>(a.gates);
  d.tol = a.tol;
  d.opt = a.opt;
  d.hist = a.hist;
  d.ring = a.ring;
  d.scratch = reinterpret_cast<cd*>(a.scratch);
  d.out_cost = a.out_cost;
  d.out_best = a.out_best;
  d.out_status = a.out_status;
  d.out_sweeps = a.out_sweeps;
  d.queue = a.queue;
  d.kinds = a.kinds;
  if (precision == QF_C64)
    hipLaunchKernelGGL(k_batch<float>, dim3(grid), dim3(64), 0, st, d);
  else
    hipLaunchKernelGGL(k_batch<double>, dim3(grid), dim3(64), 0, st, d);
  return hipGetLastError();
}

}  // namespace qf
