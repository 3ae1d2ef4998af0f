// Internal launch interface between the C-ABI/runtime layer and the HIP
// kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "qf_device.h"
#include "qf_pair_geom.h"
#include "qfactor.h"

namespace qf {

// Geometry of one two-sided pass X <- (A (x) I) X (B (x) I) over S builders
// for a gate whose local MSB sits at bit b0 and local LSB at bit b1 of the
// row/column index.  A workgroup owns one "row quad" (the 4 rows that differ
// only in b0/b1) times TCOLS columns: nseg segments of TC contiguous columns,
// chosen so that the 4 column variants of every block lie inside the tile.
struct PassGeom {
  uint32_t n, N;
  uint32_t b0, b1, rlo, rhi;
  uint32_t tc;         // log2 TC
  uint32_t tcols_log;  // log2 TCOLS
  uint32_t nseg;       // 1, 2 or 4
  uint32_t seg_lo, seg_hi;   // column bits split off as segments (insert order)
  uint32_t seg_off[4];       // column offset of each segment
  uint32_t tb0, tb1, tblo, tbhi;  // local bit positions inside a tile column index
  uint32_t col_tiles;        // column tiles per row quad
  uint32_t tiles_per_start;  // (N/4) * col_tiles
  uint32_t direct;           // 1: register-direct pass (no LDS tile), n >= 6 only
  uint32_t micro;            // 1: micro-tile register pass (complex64, both bits <= 2, n >= 9)
};
// Tile-width values that select the register-direct pass and the micro-tile
// register pass.
constexpr int kPassDirect = -1;
constexpr int kPassMicro = -2;

PassGeom make_pass_geom(int n, int q0, int q1, int max_tcols);

// Operand of a pass: per-start 4x4 c128 FP64 matrix (stride in complex
// entries between starts), optionally conjugate-transposed.
struct Operand {
  const double* ptr;  // interleaved c128, nullptr = identity (side skipped)
  int64_t stride;     // complex entries between consecutive starts
  int dagger;
};

// Optional timestamps of one kernel's own execution (hipExtLaunchKernel's
// start / stop events: the dispatch's begin and end, not the stream's
// position around the launch).  Both null: a plain launch.
struct KernelEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

hipError_t launch_pass(hipStream_t st, int precision, void* X, int S, const PassGeom& g, Operand A,
                       Operand B, KernelEvents ev = {});

// Three-qubit gates (qf_k3.hip).  Operands are 8 x 8 c128 per start.
struct Pass8Geom {
  uint32_t n, N;
  uint32_t b[3];             // bit positions of the gate's local bits, most significant first
  uint32_t s[3];             // the same positions in ascending order
  uint32_t W, wlog;          // column groups per tile (a power of two <= 32) and its log2
  uint32_t col_tiles, tiles_per_start;
  Pair2Geom tg[2];           // the two-gate pass's tiles for this gate (complex64, complex128)
  int tg_ok[2];              // whether those tiles fit (n >= 3 + their width's log2)
};
Pass8Geom make_pass8_geom(int n, const int32_t loc[3]);
hipError_t launch_pass8(hipStream_t st, int precision, void* X, int S, const Pass8Geom& g, Operand A, Operand B);
struct Env8Args {
  int S, half, do_update;
  double beta;
  double* gates;             // per start: gstride complex entries, gate g at 64 g
  int64_t gstride;
  int gidx;
  double* uold;              // S x 64 complex: u_old as used (for the pass)
  const int32_t* frozen;     // per start, nullptr = none
  double* env_out;           // S x 64 complex partial traces when do_update == 0
  // warm starts of the update (optional): start s at ywarm + ywstride * s
  // complex entries, gate g and half h at 128 g + 64 h, lane r + 8c holding
  // entry (r, c); warm = 0 starts cold
  double* ywarm = nullptr;
  int64_t ywstride = 0;
  int warm = 0;
};
hipError_t launch_env8(hipStream_t st, int precision, const void* X, const Pass8Geom& g, const Env8Args& a);
hipError_t launch_optimize8(hipStream_t st, int count, const double* env, const double* uold, double beta,
                            double* unew);

hipError_t launch_build_init(hipStream_t st, int precision, const void* V, void* X, int n, int S);

// Partial trace over every qubit but (q0, q1), FP64.  Optionally followed by
// the sweep's gate update for gate `gidx` (see qf_update_gate): then the
// environment is E = u_old^dagger P (half 0) or P u_old^dagger (half 1),
// u_new is written to gates[s*gstride + gidx*16], u_old is saved to uold.
struct EnvArgs {
  int n, q0, q1;
  int S;
  int do_update;   // 0: env only (env_out = P)
  int half;
  double beta;
  double* gates;   // c128, per start stride gstride complex entries
  int64_t gstride;
  int gidx;
  double* uold;    // c128, u_old of start s at uold + 2 * uold_stride * s (update mode)
  double* env_out; // c128 S x 16, optional
  const int32_t* frozen;  // optional per-start flag: nonzero keeps the gate
  double* partials;       // c128 S x nwg x 16 (needed when nwg > 1)
  int32_t* counters;      // S ints, zero before the first launch; left zero
  int kind;               // qf_gate_kind of the updated gate (update mode)
  int nwg;                // workgroups per start; 0 = env_workgroups(n, S)
  int64_t uold_stride = 16;  // complex entries between consecutive starts' u_old
  // Warm starts of the general U(4) update (update mode, optional): start
  // s at ywarm + ywstride * s complex entries, gate g and half h at
  // 32 g + 16 h from there; warm = 0 starts cold (and stores the new
  // rotation).
  double* ywarm = nullptr;
  int64_t ywstride = 0;
  int warm = 0;
};
// Workgroups per start of the partial trace: at least env_min_workgroups(n)
// (more than one for n >= 15); env_workgroups(n, S) spreads a launch of S
// starts over more of them when S is small (at most env_workgroups(n, 1)).
uint32_t env_min_workgroups(int n);
uint32_t env_workgroups(int n, int S);
// Small fill kernel (used instead of hipMemsetAsync so the enqueued work can
// be captured in a HIP graph).
hipError_t launch_fill_i32(hipStream_t st, int32_t* p, int32_t v, uint32_t count);
int pass_max_tcols(int precision);
hipError_t launch_env(hipStream_t st, int precision, const void* X, const EnvArgs& a, KernelEvents ev = {});
// One launch: the environment step `ea` (update mode) on builders Xe and the
// two-sided pass of gate geometry g on the Sp builders at Xp (disjoint data).
bool fused_supported(int precision, int n, const PassGeom& g);
hipError_t launch_fused(hipStream_t st, int precision, const void* Xe, const EnvArgs& ea, void* Xp, int Sp,
                        const PassGeom& g, Operand A, Operand B);

// Two consecutive gate updates F then S with one partial trace and one
// builder pass (qf_pair.hip).  The geometry comes from make_pair2_geom with
// wlog = pair2_wlog(precision, m).
struct Env2Args {
  Pair2Geom geom;
  int n_starts;
  EnvArgs F, S;            // per-gate update arguments: gates, gstride, gidx, half, beta, kind, uold
                           // (slot of the gate; uold_stride between starts)
  const int32_t* frozen;   // per start, nullptr = none
  double* partials;        // c128, env2_workgroups_cap(n) x 4^m sums per start (when more than one)
  int32_t* counters;       // per start, zero before the launch; left zero
  void* ops;               // out: per start the pass's operands A_F, B_F, A_S, B_S (64 entries in the
                           // builder precision)
  int nwg;                 // gather workgroups per start; 0 = env2_workgroups(n, m, n_starts).  The sums
                           // depend on it, so every launch of one instantiation passes the same value
};
uint32_t pair2_wlog(int precision, int m);
uint32_t env2_workgroups(int n, int m, int S);  // gather workgroups per start for a launch of S starts
uint32_t env2_workgroups_cap(int n);            // the most of them for any m and S (workspace sizing)
hipError_t launch_env2(hipStream_t st, int precision, const void* X, const Env2Args& a, KernelEvents ev = {});
// One three-qubit gate's two-sided pass on the two-gate pass's tiles
// (qf_pair.hip); g from make_pair2_geom with F = (l0, l1), S = (l1, l2).
hipError_t launch_pass3(hipStream_t st, int precision, void* X, int S, const Pair2Geom& g, Operand A, Operand B);
hipError_t launch_pass2(hipStream_t st, int precision, void* X, int S, const Pair2Geom& g, const void* ops,
                        KernelEvents ev = {});

hipError_t launch_cost(hipStream_t st, int precision, const void* X, int n, int S, double* cost,
                       double* trace);

hipError_t launch_optimize(hipStream_t st, int count, const double* env, const double* uold,
                           double beta, double* unew);

// LDS-resident whole instantiation (n <= 6).
struct ResidentArgs {
  int n, p, S;
  int precision;
  const double* V;        // c128 N x N
  const int32_t* locs;    // device p x 2
  double* gates;          // c128 S x p x 16 (in: init, out: final)
  double tol;
  qf_options opt;
  // per-start state (device): costs history ring, flags
  double* hist;           // S x (ring) doubles
  int32_t ring;           // ring length (>= long_diff_count + 1)
  int32_t* flags;         // 2 x S (double-buffered by sweep parity)
  double* cur_cost;       // S, last cost seen by the tests
  double* final_cost;     // S, FP64 cost of the final gates
  int32_t* sync;          // grid barrier words (zeroed by the host)
  int32_t* out_info;      // [0]=sweeps [1]=decision [2]=resets [3]=rechecks [4]=timeout
  double* history_out;    // optional (rows x S)
  int32_t history_rows;
  const int32_t* kinds;   // device, p gate kinds (nullptr = all general U(4))
  double* ywarm;          // c128 S x p x 2 x 16: warm starts of the FP64 updates
};
hipError_t launch_resident(hipStream_t st, const ResidentArgs& a, int* ok_coresident);

// Batched small problems (n <= 4), one persistent launch.
struct BatchArgs {
  int n_blocks, S;
  const int32_t* order;     // device, n_blocks
  const int32_t* blk_n;     // device, n_blocks
  const int32_t* gate_off;  // device, n_blocks + 1
  const int64_t* tgt_off;   // device, n_blocks
  const int32_t* locs;      // device, total_gates x 2
  const double* V;          // device targets (c128)
  double* gates;            // device (c128), in/out
  double tol;
  qf_options opt;
  double* hist;             // device, n_blocks x S x ring
  int ring;
  double* scratch;          // device, batch_scratch_entries(n_blocks, S) c128 entries
  double* ywarm;            // device, total_gates x S x 2 x 16 c128: the FP64 update's warm starts
  double* out_cost;         // device, n_blocks x S
  int32_t* out_best;        // device, n_blocks
  int32_t* out_status;      // device, n_blocks
  int32_t* out_sweeps;      // device, n_blocks
  int32_t* queue;           // device, 1 (zero before launch)
  const int32_t* kinds;     // device, total_gates gate kinds (nullptr = all general U(4))
};
// A workgroup of `slots` hexes (8 or 16, each one (block, start)) takes
// slots / S blocks per group of work; at most kBatchMaxHexes hexes in a
// launch, each with its own FP64 scratch.
constexpr int kBatchMaxHexes = 32768;
int batch_groups(int n_blocks, int S, int slots);
int batch_max_grid(int slots);
int batch_wg_per_cu_max(int slots);                   // occupancy limit of the kernel
int batch_grid(int slots, int wg_per_cu, int n_groups);  // workgroups to launch
size_t batch_scratch_entries(int n_blocks, int S);    // c128 scratch entries for every slots choice

// Gradient (qf_grad.hip).
hipError_t launch_grad_finish(hipStream_t st, const double* envP, const double* gates, const double* trace, int n,
                              int S, int p, double* grad);
hipError_t launch_su4_expm(hipStream_t st, const double* theta, int count, double* gates);
hipError_t launch_su4_vjp(hipStream_t st, const double* theta, const double* grad_gates, int count,
                          double* dtheta);
hipError_t launch_batch(hipStream_t st, int slots, int grid, const BatchArgs& a);
size_t resident_lds_bytes(int n, int precision);


// Read a value that is the same in every lane into a scalar register.
template <typename R>
__device__ __forceinline__ R uniform_r(R v);
template <>
__device__ __forceinline__ float uniform_r<float>(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
template <>
__device__ __forceinline__ double uniform_r<double>(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// Operand of a workgroup-uniform start s, held in scalar registers.
template <typename R>
__device__ __forceinline__ void load_operand_uniform(cx<R> m[16], const Operand& op, uint32_t s) {
  const cd* src = reinterpret_cast<const cd*>(op.ptr) + (int64_t)s * op.stride;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cd v = op.dagger ? conj(src[4 * c + r]) : src[4 * r + c];
      m[4 * r + c] = cx<R>{uniform_r<R>((R)v.re), uniform_r<R>((R)v.im)};
    }
}

// Plain launch, or one whose dispatch stamps the events of `ev`.
template <typename F, typename... Args>
inline hipError_t launch_k(F kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t st, KernelEvents ev,
                           Args... args) {
  if (ev.start || ev.stop)
    hipExtLaunchKernelGGL(kernel, grid, block, lds, st, ev.start, ev.stop, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
  return hipGetLastError();
}

}  // namespace qf
