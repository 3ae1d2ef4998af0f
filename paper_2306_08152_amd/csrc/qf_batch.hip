// Batched QFactor: many independent small problems (n <= 4 qubits, builders
// up to 16 x 16) in one persistent launch.
//
// One workgroup is four wavefronts, 16 hexes of 16 lanes.  Each hex owns one
// (block, start) instantiation: its builder lives in LDS, lane (r, c) of the
// hex (r = hex_row(i), c = i & 3 for lane i) sums entry (r, c) of the partial
// trace and holds that entry in the FP64 nearest-unitary step of
// Sec. III-A-1, and the 16 lanes share the 4x4 block updates of the fused
// remove/re-apply.  A sweep of a block is a chain of gate updates, so the
// time of the slowest blocks (the launch time) is set by the latency of one
// update: sixteen lanes per instantiation shorten it over one row per lane.
// The starts of one block sit in adjacent hexes of the same workgroup and
// take the multistart decision of Sec. IV-A together after every sweep
// (flags exchanged through LDS).  Workgroups take groups of blocks from a
// device-side counter until the queue is empty, so every workgroup reaches
// the exit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qf_device.h"
#include "qf_internal.h"
#include "qf_termination.h"

namespace qf {

constexpr int kBLanes = 16;                    // lanes per hex
constexpr int kBNmax = 16;                     // largest builder side (n <= 4)

// Left product by a 4x4 gate (A) and right product (B) on one hex's N x N
// builder; lane i takes blocks i, i + 16, ...
template <typename R, bool HA, bool HB>
__device__ inline void hex_pass(cx<R>* X, uint32_t N, uint32_t b0, uint32_t b1, const cx<R> a[16],
                                const cx<R> b[16], int i) {
  const uint32_t lo = b0 < b1 ? b0 : b1, hi = b0 < b1 ? b1 : b0;
  const uint32_t q = N >> 2, nblk = q * q;
  uint32_t off[4];
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) off[k] = local_off(k, b0, b1);
  for (uint32_t blk = (uint32_t)i; blk < nblk; blk += kBLanes) {
    const uint32_t rb = insert00(blk / q, lo, hi), cb = insert00(blk % q, lo, hi);
    cx<R> x[16];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) x[4 * k + j] = X[(rb + off[k]) * N + cb + off[j]];
    if (HA) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cx<R> t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          cx<R> acc = mk<R>(0, 0);
#pragma unroll
          for (int l = 0; l < 4; ++l) cmac(acc, a[4 * k + l], x[4 * l + j]);
          t[k] = acc;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) x[4 * k + j] = t[k];
      }
    }
    if (HB) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        cx<R> t[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cx<R> acc = mk<R>(0, 0);
#pragma unroll
          for (int l = 0; l < 4; ++l) cmac(acc, x[4 * k + l], b[4 * l + j]);
          t[j] = acc;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) x[4 * k + j] = t[j];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) X[(rb + off[k]) * N + cb + off[j]] = x[4 * k + j];
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
  cd* scratch;              // FP64 builder per (workgroup, hex): N_max^2 each
  double* out_cost;         // (block, start)
  int32_t* out_best, *out_status, *out_sweeps;
  int32_t* queue;           // work counter (zero before launch)
  const int32_t* kinds;     // gate kinds over all gates (nullptr = all general U(4))
  cd* ywarm;                // per (gate, start, half) the FP64 update's last rotation Y
};

// Per-hex problem description.
struct HexJob {
  bool valid;
  int b, s, n, p;
  uint32_t N;
  const int32_t* locs;  // this block's locations
  const cd* V;          // this block's target
  cd* g;                // this start's gates (p x 16)
  cd* y;                // this start's warm-start rotations (p x 2 x 16)
  const int32_t* kinds; // this block's gate kinds (nullptr = all general U(4))
};

// Builder <- G_p ... G_1 V^dagger for one hex, in precision Q, at X (LDS or
// global).  Every thread of the workgroup calls it with the same pmax
// (uniform barriers); inactive hexes only take part in the barriers.
template <typename Q>
__device__ inline void hex_build(cx<Q>* X, const HexJob& jb, int i, int pmax) {
  if (jb.valid) {
    const uint32_t N = jb.N;
    for (uint32_t e = (uint32_t)i; e < N * N; e += kBLanes) {
      const uint32_t row = e / N, col = e - row * N;
      const cd v = conj(jb.V[col * N + row]);
      X[e] = cx<Q>{(Q)v.re, (Q)v.im};
    }
  }
  for (int g = 0; g < pmax; ++g) {
    __syncthreads();
    if (jb.valid && g < jb.p) {
      cx<Q> a[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const cd v = jb.g[16 * g + k];
        a[k] = cx<Q>{(Q)v.re, (Q)v.im};
      }
      const uint32_t b0 = (uint32_t)(jb.n - 1 - jb.locs[2 * g]), b1 = (uint32_t)(jb.n - 1 - jb.locs[2 * g + 1]);
      hex_pass<Q, true, false>(X, jb.N, b0, b1, a, a, i);
    }
  }
  __syncthreads();
}

// 1 - |Tr X| / N for one hex; every quad of the hex forms the same sum (lane
// c adds diagonal entries c, c + 4, ..., the quad adds the four pairwise), so
// all 16 lanes get bitwise the same value.
template <typename Q>
__device__ inline double hex_cost(const cx<Q>* X, uint32_t N, int c) {
  double re = 0.0, im = 0.0;
  for (uint32_t d = (uint32_t)c; d < N; d += 4) {
    re += (double)X[d * N + d].re;
    im += (double)X[d * N + d].im;
  }
  re = quad_sum(re);
  im = quad_sum(im);
  return 1.0 - sqrt(re * re + im * im) / (double)N;
}

// Builders in complex128: a block's builder is at most 16 x 16 and lives in
// LDS, and a sweep is a chain of FP64 gate updates, so a complex64 builder
// saves nothing there and would need FP64 re-evaluations of the cost below
// recheck_below (measured: 2.18 s against 1.91 s for the 4096-block
// workload); QF_C64 requests run this kernel too.
//
// SLOTS hexes (instantiations) per workgroup: 16 (four wavefronts) or 8 (two);
// the runtime's tuner picks it, and the workgroups per CU, per number of
// starts.  Every hex computes the same sums in the same order whatever the
// choice (only the idle steps of a workgroup's shorter blocks differ), so
// the results are bitwise independent of it.
template <int SLOTS>
__global__ __launch_bounds__(SLOTS* kBLanes) void k_batch(BatchDev d) {
  using R = double;
  __shared__ __align__(16) cx<R> Xs[SLOTS][kBNmax * kBNmax];
  __shared__ cd Us[SLOTS][16];   // u_old of the gate being updated
  __shared__ cd PUs[SLOTS][16];  // its partial trace, then u_new
  __shared__ int flags_sh[SLOTS];
  __shared__ int p_sh[SLOTS];
  __shared__ int grp_sh;
  const int t = threadIdx.x, h = t / kBLanes, i = t % kBLanes;
  const int r = hex_row(i), c = i & 3;
  const qf_options& o = d.opt;
  cx<R>* X = Xs[h];
  // Fresh FP64 builder of each hex for the final costs, in global scratch.
  cd* Y = d.scratch + ((size_t)blockIdx.x * SLOTS + h) * (kBNmax * kBNmax);
  // Largest per-hex value over the workgroup (v uniform within each hex).
  auto wg_max = [&](int v) -> int {
    __syncthreads();
    if (i == 0) p_sh[h] = v;
    __syncthreads();
    int m = p_sh[0];
#pragma unroll
    for (int k = 1; k < SLOTS; ++k) m = max(m, p_sh[k]);
    return m;
  };

  for (;;) {
    __syncthreads();
    if (t == 0) grp_sh = __hip_atomic_fetch_add(d.queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int grp = grp_sh;
    if (grp >= d.n_groups) break;

    // ---- this hex's job
    HexJob jb;
    const int slot = h / d.S;
    jb.s = h - slot * d.S;
    const int idx = grp * d.B + slot;
    jb.valid = (slot < d.B) && (idx < d.n_blocks);
    jb.b = jb.valid ? d.order[idx] : 0;
    jb.n = jb.valid ? d.blk_n[jb.b] : 2;
    jb.N = 1u << jb.n;
    jb.p = jb.valid ? d.gate_off[jb.b + 1] - d.gate_off[jb.b] : 0;
    jb.locs = d.locs + 2 * (size_t)d.gate_off[jb.b];
    jb.V = d.V + (jb.valid ? d.tgt_off[jb.b] : 0);
    jb.g = d.gates + ((size_t)d.gate_off[jb.b] * d.S + (size_t)jb.s * jb.p) * 16;
    jb.y = d.ywarm + ((size_t)d.gate_off[jb.b] * d.S + (size_t)jb.s * jb.p) * 32;
    jb.kinds = d.kinds ? d.kinds + d.gate_off[jb.b] : nullptr;
    const int pmax = wg_max(jb.p);
    double* hist = d.hist + ((size_t)jb.b * d.S + jb.s) * d.ring;

    // ---- InitCircuitTensor and initial cost
    auto rebuild = [&]() { hex_build<R>(X, jb, i, pmax); };
    auto fp64_cost = [&]() -> double {  // fresh complex128 builder in the hex's scratch
      hex_build<double>(reinterpret_cast<cx<double>*>(Y), jb, i, pmax);
      return jb.valid ? hex_cost<double>(reinterpret_cast<cx<double>*>(Y), jb.N, c) : 0.0;
    };
    rebuild();
    double c_cur = jb.valid ? hex_cost<R>(X, jb.N, c) : 0.0;
    int32_t my_flags = 0;
    if (!isfinite(c_cur)) {
      c_cur = __builtin_inf();
      my_flags = kFlagNumeric | kFlagPlateau;
    }
    if (jb.valid && i == 0) hist[0] = c_cur;

    bool running = jb.valid && o.max_iter > 0;
    int32_t decision = kStopMaxIter;
    int it = 0, sweeps = 0;
    while (__syncthreads_or(running ? 1 : 0)) {
      ++it;
      // ---- one TwoSidedSweep (Alg. 1 order); hexes of smaller blocks idle
      const int steps = 2 * wg_max(running ? jb.p : 0);
      for (int step = 0; step < steps; ++step) {
        const bool act = running && step < 2 * jb.p;
        const int half = (act && step >= jb.p) ? 1 : 0;
        const int g = act ? (half == 0 ? jb.p - 1 - step : step - jb.p) : 0;
        const uint32_t b0 = act ? (uint32_t)(jb.n - 1 - jb.locs[2 * g]) : 0u;
        const uint32_t b1 = act ? (uint32_t)(jb.n - 1 - jb.locs[2 * g + 1]) : 1u;
        if (act) {
          // partial trace, entry (r, c): P[r][c] = sum_rest X[(r, rest), (c, rest)]
          const uint32_t lo = b0 < b1 ? b0 : b1, hi = b0 < b1 ? b1 : b0;
          const uint32_t ro = local_off((uint32_t)r, b0, b1), co = local_off((uint32_t)c, b0, b1);
          double re = 0.0, im = 0.0;
          for (uint32_t rest = 0; rest < (jb.N >> 2); ++rest) {
            const uint32_t base = insert00(rest, lo, hi);
            const cx<R> v = X[(base + ro) * jb.N + base + co];
            re += (double)v.re;
            im += (double)v.im;
          }
          PUs[h][4 * r + c] = mk(re, im);
          Us[h][i] = jb.g[16 * g + i];
        }
        __syncthreads();  // P and u_old in LDS; every trace read is done
        if (act) {
          const cd* U = Us[h];
          const cd* P = PUs[h];
          const int kind = jb.kinds ? jb.kinds[g] : kKindU4;
          const bool frozen = (my_flags & kFlagNumeric) != 0;
          // Every lane of the hex (one wavefront) reads P before any lane
          // overwrites it with u_new below.
          if (kind == kKindU4) {
            const cd e = env_entry(P, U, half, r, c);
            const cd urc = U[4 * r + c];
            cd un = urc;
            // warm start from this gate's rotation of the previous sweep
            // (same half); cold in the first sweep and every kWarmPeriod-th
            cd* yp = jb.y + 32 * g + 16 * half + 4 * r + c;
            cd yv = *yp;
            const bool warm = ((it - 1) % kWarmPeriod) != 0;
            // the update's lane exchange overwrites P, which every lane has read
            if (!frozen) optimize_gate_f64_hex(e, U[4 * c + r], urc, r, c, o.beta, un, PUs[h], &yv, warm);
            *yp = yv;
            PUs[h][4 * r + c] = un;
            jb.g[16 * g + 4 * r + c] = un;
          } else if (i < 4) {  // restricted kinds: the quad form on lanes 0..3, lane i = row i
            cd uold[16], erow[4], unew[4];
#pragma unroll
            for (int k = 0; k < 16; ++k) uold[k] = U[k];
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) erow[cc] = env_entry(P, U, half, i, cc);
            if (frozen) {
#pragma unroll
              for (int cc = 0; cc < 4; ++cc) unew[cc] = at_rk(uold, i, cc);
            } else {
              update_gate_quad(kind, erow, uold, i, o.beta, unew);
            }
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
              PUs[h][4 * i + cc] = unew[cc];
              jb.g[16 * g + 4 * i + cc] = unew[cc];
            }
          }
        }
        __syncthreads();  // u_new in LDS
        if (act) {
          // half 0: X <- (u_old^dagger (x) I) X (u_new (x) I); half 1 mirrored
          cx<R> A[16], Bm[16];
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const cd ud = conj(Us[h][4 * j + k]);  // (u_old^dagger)[k][j]
              const cd nv = PUs[h][4 * k + j];
              const cd av = sel(half == 0, ud, nv), bv = sel(half == 0, nv, ud);
              A[4 * k + j] = cx<R>{(R)av.re, (R)av.im};
              Bm[4 * k + j] = cx<R>{(R)bv.re, (R)bv.im};
            }
          hex_pass<R, true, true>(X, jb.N, b0, b1, A, Bm, i);
        }
        __syncthreads();  // the pass is done before the next trace and LDS reuse
      }
      // ---- cost, reset, recheck, per-start tests
      if (o.reset_iter > 0 && (it % o.reset_iter) == 0) rebuild();
      double c_i = running ? hex_cost<R>(X, jb.N, c) : c_cur;
      if (running) {
        const int32_t Lh = o.long_diff_count;
        const double c_prev = hist[(it - 1) % d.ring];
        const double c_back = (Lh > 0 && it >= Lh) ? hist[(it - Lh) % d.ring] : 0.0;
        if (!isfinite(c_i)) c_i = __builtin_inf();
        if (!(my_flags & kFlagNumeric)) my_flags = start_flags_after_sweep(o, d.tol, it, my_flags, c_i, c_prev, c_back);
        if (my_flags & kFlagNumeric) c_i = __builtin_inf();
        c_cur = c_i;
      }
      __syncthreads();  // every lane has read the ring slots it needs
      if (running && i == 0) hist[it % d.ring] = c_cur;
      if (i == 0) flags_sh[h] = my_flags;
      __syncthreads();
      if (running) {
        decision = job_decision(o, it, &flags_sh[slot * d.S], d.S);
        if (decision != kContinue) {
          running = false;
          sweeps = it;
        }
      }
    }
    // ---- final FP64 cost of every start, best start per block
    const double cf = fp64_cost();
    double cfin = (my_flags & kFlagNumeric) || !isfinite(cf) ? __builtin_inf() : cf;
    if (jb.valid && i == 0) d.out_cost[(size_t)jb.b * d.S + jb.s] = cfin;
    if (i == 0) flags_sh[h] = my_flags;
    __syncthreads();
    if (jb.valid && jb.s == 0 && i == 0) {
      int best = 0;
      double bc = d.out_cost[(size_t)jb.b * d.S];
      bool all_numeric = (flags_sh[h] & kFlagNumeric) != 0;
      for (int k = 1; k < d.S; ++k) {
        const double ck = d.out_cost[(size_t)jb.b * d.S + k];
        all_numeric = all_numeric && (flags_sh[h + k] & kFlagNumeric);
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
  }
}

int batch_groups(int n_blocks, int S, int slots) {
  const int B = slots / S;
  return (n_blocks + B - 1) / B;
}

int batch_max_grid(int slots) { return kBatchMaxHexes / slots; }

size_t batch_scratch_entries(int n_blocks, int S) {
  size_t hexes = 0;
  for (int slots : {8, 16})
    if (slots >= S)
      hexes = std::max(hexes, (size_t)std::min(batch_groups(n_blocks, S, slots), batch_max_grid(slots)) * slots);
  return hexes * kBNmax * kBNmax;
}

template <int SLOTS>
static const void* batch_fn() {
  return reinterpret_cast<const void*>(&k_batch<SLOTS>);
}

int batch_wg_per_cu_max(int slots) {
  int per = 1;
  const void* fn = slots == 8 ? batch_fn<8>() : batch_fn<16>();
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, slots * kBLanes, 0) != hipSuccess || per < 1) per = 1;
  return per;
}

int batch_grid(int slots, int wg_per_cu, int n_groups) {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int g = cus * std::max(1, wg_per_cu);
  g = std::min(g, batch_max_grid(slots));
  return std::min(g, n_groups);
}

hipError_t launch_batch(hipStream_t st, int slots, int grid, const BatchArgs& a) {
  if (slots != 8 && slots != 16) return hipErrorInvalidValue;
  if (a.S < 1 || a.S > slots) return hipErrorInvalidValue;
  BatchDev d;
  d.n_blocks = a.n_blocks;
  d.S = a.S;
  d.B = slots / a.S;
  d.n_groups = batch_groups(a.n_blocks, a.S, slots);
  if (grid < 1 || grid > batch_max_grid(slots) || grid > d.n_groups) return hipErrorInvalidValue;
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
  d.ywarm = reinterpret_cast<cd*>(a.ywarm);
  if (!d.ywarm) return hipErrorInvalidValue;
  if (slots == 8)
    hipLaunchKernelGGL(k_batch<8>, dim3(grid), dim3(8 * kBLanes), 0, st, d);
  else
    hipLaunchKernelGGL(k_batch<16>, dim3(grid), dim3(16 * kBLanes), 0, st, d);
  return hipGetLastError();
}

}  // namespace qf
