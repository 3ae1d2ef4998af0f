// C-ABI entry points and the host runtime around the kernels: argument
// validation, workspace layout, the streaming sweep loop (Alg. 1 with the
// host-side termination test once per sweep), the complex64 FP64 recheck,
// and dispatch to the LDS-resident kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qf_internal.h"
#include "qf_termination.h"
#include "qfactor.h"

constexpr int kMaxGroups = 4;
// Default stream groups of the three-qubit sweep: one.  Two to four
// staggered groups were measured at n = 10, 8 starts and gave no overlap
// (complex64 62.5 us per gate update with one group, 64.6-65.7 with more;
// complex128 89.6-91.6 either way; with the Newton form of the 8 x 8 update,
// steady state, complex64 41.6 against 44.7-46.6, complex128 60.8 against
// 60.8-63.5): every pass fills all CUs, so another group's environment step
// cannot run beside it.
constexpr int kDefaultGroups3 = 1;

struct qf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // Streams of the context (default priority) that run the sweeps of groups
  // of starts concurrently, forked from and joined to `stream` by events.
  hipStream_t aux[kMaxGroups] = {};
  hipEvent_t fork = nullptr, join[kMaxGroups] = {}, stagger[kMaxGroups] = {};
  hipEvent_t tune[2] = {};      // timing events of the pass-form tuner
  double* pinned = nullptr;     // host read-back buffer (kPinnedCount doubles)
  void* scratch = nullptr;      // device scratch of the stand-alone step calls
  // Autotuned pass tile width per (precision, n); 0 = not tuned yet.
  int tuned_tcols[2][2][17] = {};
  // Tuned tiles per workgroup of the two-gate pass per (precision, n); 0 = not tuned yet.
  int tuned_pass2[2][17] = {};
  // Batched launch per number of starts: hexes per workgroup and workgroups
  // per CU; 0 = not tuned yet.
  int batch_cfg[17][2] = {};
  double* identity = nullptr;   // one 4x4 c128 identity (tuning operand)
  void* static_ws = nullptr;    // this device's address of `scratch` (below); null if unresolved
  std::string last_error;
};

// Workspace of qf_instantiate_noalloc: a fixed device array, one copy per
// device, held from the library's load on that device until the process
// ends.  Host code never passes `scratch` itself to a kernel or a copy (its
// host-side name is only a stand-in for the symbol); it uses the address
// hipGetSymbolAddress gives on each device, resolved once per device by
// qf_create (static_scratch_ptr).  Every call on a device shares the array.
static __device__ __align__(256) unsigned char scratch[QF_NOALLOC_WORKSPACE_BYTES];

namespace {

using namespace qf;

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int fail(qf_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return code;
}

// Device address of `scratch` on `device` (which must be current), resolved
// once per device and kept for the process's lifetime.  Null when the
// lookup fails; qf_instantiate_noalloc then reports QF_EHIP.
constexpr int kMaxDevices = 64;
void* static_scratch_ptr(int device) {
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  static bool tried[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!tried[device]) {
    tried[device] = true;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) ptr[device] = p;
  }
  return ptr[device];
}

#define QF_HIP(ctx, expr)                                                                     \
  do {                                                                                        \
    hipError_t e__ = (expr);                                                                  \
    if (e__ != hipSuccess) return fail((ctx), QF_EHIP, "%s: %s", #expr, hipGetErrorString(e__)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Everything a context allocates is allocated by qf_create: the pinned
// read-back buffer, the tuner's identity operand and the scratch of the
// stand-alone step calls, which process their builders in chunks of at most
// kScratchChunk so that the scratch has a fixed size (environment partial
// sums for kScratchSlots (builder, workgroup) pairs, arrival counters and
// u_old of one chunk).  No call allocates afterwards.
constexpr size_t kPinnedCount = 4096;
constexpr int kScratchChunk = 1024;
constexpr size_t kScratchSlots = 4096;
constexpr size_t kScratchPartials = 0;
constexpr size_t kScratchCounters = kScratchSlots * 256;
constexpr size_t kScratchUold = kScratchCounters + (size_t)kScratchChunk * 4;
constexpr size_t kScratchBytes = kScratchUold + (size_t)kScratchChunk * 256;
static_assert(kScratchSlots >= (size_t)kScratchChunk * 4 && kScratchSlots >= 256,
              "a chunk's spread environment must fit: at most max(4 per builder at n = 16, 256) slots");

size_t elem_bytes(int precision) { return precision == QF_C64 ? 8 : 16; }

bool valid_loc(int n, const int32_t* loc) {
  return loc && loc[0] >= 0 && loc[0] < n && loc[1] >= 0 && loc[1] < n && loc[0] != loc[1];
}

int resolve_mode(int n, const qf_options& o) {
  if (o.mode == QF_MODE_RESIDENT) return QF_MODE_RESIDENT;
  if (o.mode == QF_MODE_STREAMING) return QF_MODE_STREAMING;
  return n <= 6 ? QF_MODE_RESIDENT : QF_MODE_STREAMING;
}

// Workspace layout of qf_instantiate.
struct Layout {
  size_t X = 0, R = 0, gates = 0, uold = 0, partials = 0, counters = 0, costs = 0, trace = 0,
         frozen = 0, locs = 0, kinds = 0, hist = 0, flags = 0, cur = 0, fin = 0, sync = 0, info = 0, histo = 0,
         uold2 = 0, ops2 = 0, partials2 = 0, ywarm = 0;
  size_t total = 0;
  int ring = 2;
};

Layout make_layout(int n, int p, int S, const qf_options& o, int mode, int history_rows) {
  Layout L;
  const size_t N = (size_t)1 << n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  if (mode == QF_MODE_STREAMING) {
    L.X = take((size_t)S * N * N * elem_bytes(o.precision));
    if (o.precision == QF_C64) L.R = take((size_t)S * N * N * 16);
    L.partials = take((size_t)S * env_workgroups(n, 1) * 16 * 16);
    L.counters = take((size_t)S * 4);
    L.uold = take((size_t)S * 16 * 16);
    L.trace = take((size_t)S * 16);
    L.frozen = take((size_t)S * 4);
    if (o.gate_pairs == 2 || (o.gate_pairs == 1 && o.precision == QF_C64)) {
      // two-gate updates: both gates' u_old, the pass's operands, partial traces
      L.uold2 = take((size_t)S * 32 * 16);
      L.ops2 = take((size_t)S * 64 * elem_bytes(o.precision));
      const uint32_t nwg2 = env2_workgroups_cap(n);
      if (nwg2 > 1) L.partials2 = take((size_t)S * nwg2 * 256 * 16);
    }
  }
  L.gates = take((size_t)S * p * 16 * 16);
  L.ywarm = take((size_t)S * p * 2 * 16 * 16);  // warm starts of the FP64 updates, per (start, gate, half)
  L.costs = take((size_t)S * 8);
  L.locs = take((size_t)p * 2 * 4);
  L.kinds = take((size_t)p * 4);
  L.ring = std::max(2, o.long_diff_count + 1);
  if (mode == QF_MODE_RESIDENT) {
    L.hist = take((size_t)S * L.ring * 8);
    L.flags = take((size_t)2 * S * 4);
    L.cur = take((size_t)S * 8);
    L.fin = take((size_t)S * 8);
    L.sync = take(64);
    L.info = take(64);
    if (history_rows > 0) L.histo = take((size_t)history_rows * S * 8);
  }
  L.total = off;
  return L;
}

// The resident kernel records the per-sweep costs of at most this many rows
// (initial cost + sweeps) in the workspace.
constexpr int kResidentHistoryCap = 4097;
int resident_history_rows(int mode, const qf_options& o) {
  return mode == QF_MODE_RESIDENT ? std::min(o.max_iter + 1, kResidentHistoryCap) : 0;
}

int validate_options(qf_ctx* ctx, const qf_options& o) {
  if (!(o.dist_tol > 0) || !std::isfinite(o.dist_tol)) return fail(ctx, QF_EINVAL, "dist_tol must be > 0");
  if (!(o.diff_tol_a >= 0) || !(o.diff_tol_r >= 0)) return fail(ctx, QF_EINVAL, "diff_tol_a/r must be >= 0");
  if (!(o.long_diff_r >= 0)) return fail(ctx, QF_EINVAL, "long_diff_r must be >= 0");
  if (o.long_diff_count > (1 << 20)) return fail(ctx, QF_EINVAL, "long_diff_count too large");
  if (o.min_iter < 0 || o.max_iter < 0 || o.reset_iter < 0) return fail(ctx, QF_EINVAL, "iteration counts must be >= 0");
  if (!(o.beta >= 0.0 && o.beta <= 1.0)) return fail(ctx, QF_EINVAL, "beta must be in [0, 1]");
  if (o.precision != QF_C128 && o.precision != QF_C64) return fail(ctx, QF_EINVAL, "unknown precision %d", o.precision);
  if (o.gate_pairs < 0 || o.gate_pairs > 2) return fail(ctx, QF_EINVAL, "gate_pairs must be 0, 1 or 2");
  if (o.mode < QF_MODE_AUTO || o.mode > QF_MODE_STREAMING) return fail(ctx, QF_EINVAL, "unknown mode %d", o.mode);
  if (!(o.recheck_below >= 0) || !std::isfinite(o.recheck_below)) return fail(ctx, QF_EINVAL, "recheck_below must be >= 0");
  if (o.stream_groups < 0 || o.stream_groups > kMaxGroups) return fail(ctx, QF_EINVAL, "stream_groups must be in [0, 4]");
  return QF_OK;
}

int validate_problem(qf_ctx* ctx, int n, int p, const int32_t* locs, int S) {
  if (n < 2 || n > 16) return fail(ctx, QF_EINVAL, "n=%d outside [2, 16]", n);
  if (p < 1) return fail(ctx, QF_EINVAL, "n_gates must be >= 1");
  if (!locs) return fail(ctx, QF_EINVAL, "locations is NULL");
  for (int g = 0; g < p; ++g)
    if (!valid_loc(n, locs + 2 * g))
      return fail(ctx, QF_EINVAL, "gate %d: location (%d, %d) invalid for n=%d", g, locs[2 * g], locs[2 * g + 1], n);
  if (S < 1) return fail(ctx, QF_EINVAL, "n_starts must be >= 1");
  return QF_OK;
}

int validate_kinds(qf_ctx* ctx, const int32_t* kinds, int count) {
  if (!kinds) return QF_OK;
  for (int g = 0; g < count; ++g)
    if (kinds[g] < QF_KIND_U4 || kinds[g] > QF_KIND_MS)
      return fail(ctx, QF_EINVAL, "gate %d: unknown gate kind %d", g, kinds[g]);
  return QF_OK;
}


int ensure_aux_streams(qf_ctx* ctx) {
  if (ctx->aux[0]) return QF_OK;
  for (int i = 0; i < kMaxGroups; ++i) {
    // group 0 runs on the caller's stream: kMaxGroups - 1 streams of our own
    if (i + 1 < kMaxGroups) QF_HIP(ctx, hipStreamCreateWithFlags(&ctx->aux[i], hipStreamNonBlocking));
    QF_HIP(ctx, hipEventCreateWithFlags(&ctx->join[i], hipEventDisableTiming));
    QF_HIP(ctx, hipEventCreateWithFlags(&ctx->stagger[i], hipEventDisableTiming));
  }
  QF_HIP(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
  QF_HIP(ctx, hipEventCreate(&ctx->tune[0]));
  QF_HIP(ctx, hipEventCreate(&ctx->tune[1]));
  return QF_OK;
}


// Pass form of a gate: the tile width of the LDS-staged pass, kPassDirect
// for the register-direct one or kPassMicro for the micro-tile register one
// (complex64 class-1 gates at n >= 9).  Gates fall in two classes by where their two
// column bits are (class 1: both among the three lowest bits, where the
// direct form's loads stride by 2..8 elements); each (precision, class, n) is tuned once
// per context by timing every candidate on the caller's builder with identity
// operands on both sides (x * 1 + 0 * y = x exactly, so the builder is left
// bit-for-bit unchanged).  Untuned: the register-direct form for class 0 at
// n >= 6, else the 512-column LDS tile.
int pass_class(int n, int q0, int q1) {
  const int hi = std::max(n - 1 - q0, n - 1 - q1);
  return (n >= 6 && hi <= 2) ? 1 : 0;
}

int pass_tcols(qf_ctx* ctx, int precision, int n, int q0, int q1) {
  const int cls = pass_class(n, q0, q1);
  const int t = ctx->tuned_tcols[precision == QF_C64][cls][n];
  if (t) return t;
  return (n >= 6 && cls == 0) ? kPassDirect : 512;
}

int autotune_pass(qf_ctx* ctx, int precision, int n, void* X, int S) {
  const int N = 1 << n;
  const int cands64[] = {kPassDirect, kPassMicro, 256, 512, 1024}, cands128[] = {kPassDirect, 256, 512};
  const int* cands = precision == QF_C64 ? cands64 : cands128;
  const int nc = precision == QF_C64 ? 5 : 3;
  const Operand I{ctx->identity, 0, 0};
  for (int cls = 0; cls < 2; ++cls) {
    int& slot = ctx->tuned_tcols[precision == QF_C64][cls][n];
    if (slot) continue;
    if (N < 512) {
      slot = pass_max_tcols(precision);
      continue;
    }
    const int q0 = cls == 0 ? n / 2 - 1 : n - 2, q1 = q0 + 1;  // a mid-circuit pair / the two lowest bits
    hipEvent_t e0 = ctx->tune[0], e1 = ctx->tune[1];
    // Two rounds over the candidates (warm-up launch, then 4 timed launches);
    // each candidate keeps its better round.
    float t_best[5] = {1e30f, 1e30f, 1e30f, 1e30f, 1e30f};
    for (int round = 0; round < 2; ++round)
      for (int c = 0; c < nc; ++c) {
        if (cands[c] > N) continue;
        if (cands[c] == kPassMicro && (cls == 0 || n < 9)) continue;  // class-1 gates at n >= 9 only
        const PassGeom geo = make_pass_geom(n, q0, q1, cands[c]);
        hipError_t err = launch_pass(ctx->stream, precision, X, S, geo, I, I);
        if (err == hipSuccess) err = hipEventRecord(e0, ctx->stream);
        for (int r = 0; r < 4 && err == hipSuccess; ++r) err = launch_pass(ctx->stream, precision, X, S, geo, I, I);
        if (err == hipSuccess) err = hipEventRecord(e1, ctx->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err != hipSuccess) return fail(ctx, QF_EHIP, "pass autotune: %s", hipGetErrorString(err));
        t_best[c] = std::min(t_best[c], ms);
      }
    float best = 1e30f;
    int best_t = pass_max_tcols(precision);
    for (int c = 0; c < nc; ++c)
      if (t_best[c] < best) {
        best = t_best[c];
        best_t = cands[c];
      }
    slot = best_t;
  }
  return QF_OK;
}

// Tiles per workgroup of the two-gate pass, tuned once per context and
// (precision, n) by timing the candidates on the caller's builder with
// identity operands (the builder is left bit-for-bit unchanged), two rounds
// of four launches each; the geometry is the circuit's first two-gate unit.
__global__ void k_identity_ops(void* ops, int precision, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t e = i & 15u;
  const double v = ((e >> 2) == (e & 3u)) ? 1.0 : 0.0;
  if (precision == QF_C64)
    reinterpret_cast<float2*>(ops)[i] = make_float2((float)v, 0.f);
  else
    reinterpret_cast<double2*>(ops)[i] = make_double2(v, 0.0);
}

int autotune_pass2(qf_ctx* ctx, int precision, int n, void* X, int S, const Pair2Geom& g0, void* ops) {
  int& slot = ctx->tuned_pass2[precision == QF_C64][n];
  if (slot) return QF_OK;
  const uint32_t count = (uint32_t)S * 64;
  hipLaunchKernelGGL(k_identity_ops, dim3((count + 255) / 256), dim3(256), 0, ctx->stream, ops, precision, count);
  QF_HIP(ctx, hipGetLastError());
  const int cands[] = {1, 2, 4, 8};
  float t_best[4] = {1e30f, 1e30f, 1e30f, 1e30f};
  hipEvent_t e0 = ctx->tune[0], e1 = ctx->tune[1];
  for (int round = 0; round < 2; ++round)
    for (int c = 0; c < 4; ++c) {
      Pair2Geom g = g0;
      g.tiles_per_wg = (uint32_t)cands[c];
      hipError_t err = launch_pass2(ctx->stream, precision, X, S, g, ops);
      if (err == hipSuccess) err = hipEventRecord(e0, ctx->stream);
      for (int r = 0; r < 4 && err == hipSuccess; ++r) err = launch_pass2(ctx->stream, precision, X, S, g, ops);
      if (err == hipSuccess) err = hipEventRecord(e1, ctx->stream);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err != hipSuccess) return fail(ctx, QF_EHIP, "two-gate pass autotune: %s", hipGetErrorString(err));
      t_best[c] = std::min(t_best[c], ms);
    }
  int best = 0;
  for (int c = 1; c < 4; ++c)
    if (t_best[c] < t_best[best]) best = c;
  slot = cands[best];
  return QF_OK;
}

// Build X_s = G_p ... G_1 V^dagger on the device (all starts).
int build_builder(qf_ctx* ctx, int n, const void* V, int p, const int32_t* locs, const double* gates,
                  int64_t gstride, int S, int precision, void* X) {
  QF_HIP(ctx, launch_build_init(ctx->stream, precision, V, X, n, S));
  for (int g = 0; g < p; ++g) {
    const PassGeom geo = make_pass_geom(n, locs[2 * g], locs[2 * g + 1], pass_tcols(ctx, precision, n, locs[2 * g], locs[2 * g + 1]));
    Operand A{gates + 2 * 16 * (int64_t)g, gstride, 0};
    Operand B{nullptr, 0, 0};
    QF_HIP(ctx, launch_pass(ctx->stream, precision, X, S, geo, A, B));
  }
  return QF_OK;
}

__global__ void k_cast_c128_c64(const double2* __restrict__ src, float2* __restrict__ dst, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) {
    const double2 v = src[i];
    dst[i] = make_float2((float)v.x, (float)v.y);
  }
}

// dst[s][k] = src[s][idx[k]] for 4x4 c128 gates (S starts, p source gates,
// q selected); src_start0 (optional) replaces the source of start 0.
__global__ void k_gather_gates(const double2* __restrict__ src, const double2* __restrict__ src_start0,
                               int S, int p, const int32_t* __restrict__ idx, int q, double2* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)S * q * 16) return;
  const int k16 = (int)(e & 15);
  const int64_t sk = e >> 4;
  const int k = (int)(sk % q), s = (int)(sk / q);
  const double2* from = (s == 0 && src_start0) ? src_start0 + (int64_t)idx[k] * 16
                                               : src + ((int64_t)s * p + idx[k]) * 16;
  dst[e] = from[k16];
}

int cast_to_c64(qf_ctx* ctx, const void* R, void* X, size_t count) {
  const unsigned blocks = (unsigned)std::min<size_t>((count + 255) / 256, 65536);
  hipLaunchKernelGGL(k_cast_c128_c64, dim3(blocks), dim3(256), 0, ctx->stream,
                     reinterpret_cast<const double2*>(R), reinterpret_cast<float2*>(X), count);
  QF_HIP(ctx, hipGetLastError());
  return QF_OK;
}

int read_costs(qf_ctx* ctx, const double* dev, int S, std::vector<double>& out) {
  out.resize((size_t)S);
  for (size_t at = 0; at < (size_t)S; at += kPinnedCount) {  // through the fixed pinned buffer
    const size_t cnt = std::min(kPinnedCount, (size_t)S - at);
    QF_HIP(ctx, hipMemcpyAsync(ctx->pinned, dev + at, cnt * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    QF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::copy(ctx->pinned, ctx->pinned + cnt, out.begin() + (ptrdiff_t)at);
  }
  return QF_OK;
}

// Optional per-kernel timing of the streaming sweeps with HIP events: each
// timed launch carries a start / stop pair that the dispatch itself stamps
// (the kernel's execution, without the stream's dispatch gap around it);
// the pairs are summed after the per-sweep synchronisation.
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> ev;  // pairs
  std::vector<int> kind;       // 0 = pass, 1 = env, 2 = two-gate pass
  size_t used = 0;
  double pass_ms = 0, env_ms = 0, sweep_ms = 0, pass2_ms = 0;
  int pass_n = 0, env_n = 0, pass2_n = 0;
  hipEvent_t s0 = nullptr, s1 = nullptr;
  ~KernelTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
    if (s0) (void)hipEventDestroy(s0);
    if (s1) (void)hipEventDestroy(s1);
  }
  hipError_t init(size_t pairs) {
    on = true;
    ev.resize(2 * pairs, nullptr);
    kind.resize(pairs, 0);
    for (auto& e : ev) {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
    }
    hipError_t r = hipEventCreate(&s0);
    if (r != hipSuccess) return r;
    return hipEventCreate(&s1);
  }
  // the event pair for the next launch of kind k (0 = pass, 1 = env, 2 =
  // two-gate pass, which also counts as a pass), or none
  KernelEvents next(int k) {
    if (!on || used >= kind.size()) return {};
    kind[used] = k;
    const KernelEvents e{ev[2 * used], ev[2 * used + 1]};
    ++used;
    return e;
  }
  // after a stream synchronisation: fold the recorded pairs into the sums
  hipError_t collect() {
    for (size_t i = 0; i < used; ++i) {
      float ms = 0.f;
      hipError_t r = hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
      if (r != hipSuccess) return r;
      if (kind[i] == 0 || kind[i] == 2) {
        pass_ms += ms;
        ++pass_n;
        if (kind[i] == 2) {
          pass2_ms += ms;
          ++pass2_n;
        }
      } else {
        env_ms += ms;
        ++env_n;
      }
    }
    used = 0;
    return hipSuccess;
  }
};

struct RunOut {
  int32_t sweeps = 0, decision = kContinue, resets = 0, rechecks = 0;
  std::vector<double> final_costs;
  std::vector<int32_t> flags;
};

// ----------------------------------------------------------------- streaming

int run_streaming(qf_ctx* ctx, int n, const void* V, int p, const int32_t* locs, int S, double tol,
                  const qf_options& o, unsigned char* ws, const Layout& L, qf_stats* stats, RunOut& out) {
  hipStream_t st = ctx->stream;
  const int prec = o.precision;
  void* X = ws + L.X;
  void* R = prec == QF_C64 ? (void*)(ws + L.R) : nullptr;
  double* gates = reinterpret_cast<double*>(ws + L.gates);
  double* uold = reinterpret_cast<double*>(ws + L.uold);
  double* costs = reinterpret_cast<double*>(ws + L.costs);
  double* trace = reinterpret_cast<double*>(ws + L.trace);
  int32_t* frozen = reinterpret_cast<int32_t*>(ws + L.frozen);
  const int64_t gstride = (int64_t)p * 16;
  const size_t N = (size_t)1 << n;

  QF_HIP(ctx, launch_fill_i32(st, reinterpret_cast<int32_t*>(ws + L.counters), 0, (uint32_t)S));
  QF_HIP(ctx, launch_fill_i32(st, frozen, 0, (uint32_t)S));

  std::vector<PassGeom> geo(p);
  for (int g = 0; g < p; ++g) geo[g] = make_pass_geom(n, locs[2 * g], locs[2 * g + 1], pass_tcols(ctx, prec, n, locs[2 * g], locs[2 * g + 1]));

  // Update units of each half-sweep, in Alg. 1's order (g = p..1, then
  // 1..p): one gate, or two consecutive gates F then S whose updates share
  // one partial trace and one builder pass (k_env2 + k_pass2) when they span
  // 3 or 4 qubits and neither is fixed.
  struct Unit {
    int g1 = 0, g2 = -1;  // g2 < 0: a single gate
    Pair2Geom pg{};
  };
  auto pair_geom = [&](int f, int sg, Pair2Geom& pg) -> bool {
    if (o.gate_pairs == 0 || (o.gate_pairs == 1 && prec != QF_C64)) return false;
    if (o.gate_kinds && (o.gate_kinds[f] == QF_KIND_FIXED || o.gate_kinds[sg] == QF_KIND_FIXED)) return false;
    uint32_t mask = 0;
    for (int k = 0; k < 2; ++k) mask |= (1u << (n - 1 - locs[2 * f + k])) | (1u << (n - 1 - locs[2 * sg + k]));
    const int m = __builtin_popcount(mask);
    if (m != 3 && m != 4) return false;
    return make_pair2_geom(n, locs + 2 * f, locs + 2 * sg, pair2_wlog(prec, m), pg);
  };
  std::vector<Unit> units[2];
  bool any_pair = false;
  for (int half = 0; half < 2; ++half) {
    std::vector<int> order(p);
    for (int k = 0; k < p; ++k) order[k] = half == 0 ? p - 1 - k : k;
    for (int k = 0; k < p;) {
      Unit u;
      u.g1 = order[k];
      if (k + 1 < p && pair_geom(order[k], order[k + 1], u.pg)) {
        u.g2 = order[k + 1];
        any_pair = true;
        k += 2;
      } else {
        k += 1;
      }
      units[half].push_back(u);
    }
  }
  double* uold2 = reinterpret_cast<double*>(ws + L.uold2);
  unsigned char* ops2 = ws + L.ops2;
  double* partials2 = reinterpret_cast<double*>(ws + L.partials2);
  const uint32_t nwg2_stride = L.partials2 ? env2_workgroups_cap(n) : 0;

  // The starts split into G groups whose sweeps run on separate streams:
  // while one group's latency-bound environment + SVD step runs, the other
  // group's pass keeps HBM busy.  Groups share nothing but the join.  Group
  // 0 runs on the caller's stream and groups 1.. on the library's own, so
  // that four groups occupy the device's four hardware queues (a fifth
  // stream would share a queue with another and serialise behind it).
  // (Per-kernel timing runs the starts as one group so that every measured
  // kernel duration is the kernel's own, not shared with a concurrent one.)
  int G = o.stream_groups > 0 ? o.stream_groups : kMaxGroups;
  G = std::min(std::min(G, kMaxGroups), S);
  if (stats && stats->timing) G = 1;
  // Default schedule: two groups on the caller's stream, each launch carrying
  // one group's environment step beside the other group's pass (k_fused).
  const bool fused =
      o.stream_groups == 0 && !(stats && stats->timing) && S >= 2 && !any_pair && env_min_workgroups(n) == 1;
  // With two-gate updates, three staggered groups: a group's environment
  // step (two FP64 updates in a row) runs while the others' passes stream
  // (measured at n = 10, 16 starts: 1 group 3758, 2: 3828, 3: 3898, 4: 3657
  // start-sweeps/s; the pairing of one group's environment with another's
  // pass in one launch, as for single updates, gave 3830-3874).
  if (any_pair && o.stream_groups == 0 && !(stats && stats->timing)) G = std::min(3, S);
  constexpr int kFusedPairs = 2;  // pairs of groups, one stream each
  static_assert(kFusedPairs >= 1 && kFusedPairs <= kMaxGroups, "one stream per pair: the caller's and kMaxGroups - 1 own");
  const int pairs = fused ? std::min(kFusedPairs, S / 2) : 0;
  if (fused) G = 2 * pairs;
  if ((G > 1 && !fused) || pairs > 1) {
    int rc0 = ensure_aux_streams(ctx);
    if (rc0) return rc0;
  }
  struct Group {
    int s0 = 0, ns = 0;
    hipStream_t st = nullptr;
    void* X = nullptr;
    EnvArgs ea{};
  };
  Group grp[2 * kMaxGroups];
  const uint32_t nwg_stride = env_workgroups(n, 1);  // partial-sum slots per start
  for (int gi = 0; gi < G; ++gi) {
    Group& q = grp[gi];
    q.s0 = gi * S / G;
    q.ns = (gi + 1) * S / G - q.s0;
    q.st = fused ? (gi < 2 ? st : ctx->aux[gi / 2 - 1]) : (gi == 0 ? st : ctx->aux[gi - 1]);
    q.X = reinterpret_cast<unsigned char*>(X) + (size_t)q.s0 * N * N * elem_bytes(prec);
    EnvArgs& ea = q.ea;
    ea.n = n;
    ea.S = q.ns;
    ea.do_update = 1;
    ea.beta = o.beta;
    ea.gates = gates + (size_t)q.s0 * gstride * 2;
    ea.gstride = gstride;
    ea.uold = uold + (size_t)q.s0 * 32;
    ea.env_out = nullptr;
    ea.frozen = frozen + q.s0;
    ea.partials = reinterpret_cast<double*>(ws + L.partials) + (size_t)q.s0 * nwg_stride * 32;
    ea.counters = reinterpret_cast<int32_t*>(ws + L.counters) + q.s0;
    ea.nwg = (int)env_workgroups(n, q.ns);
    ea.ywstride = (int64_t)p * 32;
    ea.ywarm = reinterpret_cast<double*>(ws + L.ywarm) + (size_t)q.s0 * ea.ywstride * 2;
  }

  KernelTimer timer;
  if (stats && stats->timing) QF_HIP(ctx, timer.init((size_t)4 * p * G));

  auto update = [&](Group& q, int g, int half, hipEvent_t after_env) -> int {
    EnvArgs& ea = q.ea;
    const int kind = o.gate_kinds ? o.gate_kinds[g] : QF_KIND_U4;
    if (kind == QF_KIND_FIXED) {  // never optimised: move the gate across, no environment
      Operand ud{ea.gates + 2 * 16 * (int64_t)g, gstride, 1};
      Operand u{ea.gates + 2 * 16 * (int64_t)g, gstride, 0};
      if (after_env) QF_HIP(ctx, hipEventRecord(after_env, q.st));
      const KernelEvents te = timer.next(0);
      if (half == 0)
        QF_HIP(ctx, launch_pass(q.st, prec, q.X, q.ns, geo[g], ud, u, te));
      else
        QF_HIP(ctx, launch_pass(q.st, prec, q.X, q.ns, geo[g], u, ud, te));
      return QF_OK;
    }
    ea.kind = kind;
    ea.q0 = locs[2 * g];
    ea.q1 = locs[2 * g + 1];
    ea.half = half;
    ea.gidx = g;
    QF_HIP(ctx, launch_env(q.st, prec, q.X, ea, timer.next(1)));
    if (after_env) QF_HIP(ctx, hipEventRecord(after_env, q.st));
    Operand gnew{ea.gates + 2 * 16 * (int64_t)g, gstride, 0};
    Operand gold{ea.uold, 16, 1};
    const KernelEvents te = timer.next(0);
    if (half == 0)
      QF_HIP(ctx, launch_pass(q.st, prec, q.X, q.ns, geo[g], gold, gnew, te));
    else
      QF_HIP(ctx, launch_pass(q.st, prec, q.X, q.ns, geo[g], gnew, gold, te));
    return QF_OK;
  };
  auto env2_args = [&](Group& q, const Unit& u, int half) -> Env2Args {
    Env2Args a2{};
    a2.geom = u.pg;
    a2.n_starts = q.ns;
    for (int k = 0; k < 2; ++k) {
      EnvArgs& e = k == 0 ? a2.F : a2.S;
      const int g = k == 0 ? u.g1 : u.g2;
      e = q.ea;
      e.kind = o.gate_kinds ? o.gate_kinds[g] : QF_KIND_U4;
      e.q0 = locs[2 * g];
      e.q1 = locs[2 * g + 1];
      e.half = half;
      e.gidx = g;
      e.uold = uold2 + (size_t)q.s0 * 64 + 32 * k;
      e.uold_stride = 32;
      e.env_out = nullptr;
    }
    a2.frozen = frozen + q.s0;
    a2.partials = nwg2_stride ? partials2 + (size_t)q.s0 * nwg2_stride * 512 : nullptr;
    a2.counters = q.ea.counters;
    a2.ops = ops2 + (size_t)q.s0 * 64 * elem_bytes(prec);
    // the same gather split for every group and schedule: bitwise the same sums
    a2.nwg = (int)env2_workgroups(n, (int)u.pg.m, S);
    return a2;
  };
  auto ops_of = [&](const Group& q) -> const void* { return ops2 + (size_t)q.s0 * 64 * elem_bytes(prec); };
  auto update_unit = [&](Group& q, const Unit& u, int half, hipEvent_t after_env) -> int {
    if (u.g2 < 0) return update(q, u.g1, half, after_env);
    const Env2Args a2 = env2_args(q, u, half);
    QF_HIP(ctx, launch_env2(q.st, prec, q.X, a2, timer.next(1)));
    if (after_env) QF_HIP(ctx, hipEventRecord(after_env, q.st));
    QF_HIP(ctx, launch_pass2(q.st, prec, q.X, q.ns, u.pg, a2.ops, timer.next(2)));
    return QF_OK;
  };
  // One TwoSidedSweep of every start (Alg. 1 order), groups interleaved,
  // forked from and joined back to stream `home`.
  auto sweep_on = [&](hipStream_t home) -> int {
    if (G > 1) {
      QF_HIP(ctx, hipEventRecord(ctx->fork, home));
      for (int gi = 0; gi < G; ++gi)
        if (grp[gi].st != home) QF_HIP(ctx, hipStreamWaitEvent(grp[gi].st, ctx->fork, 0));
    }
    // Stagger: group k starts once group k-1's first environment + SVD step
    // is done, so the groups' latency-bound steps fall under each other's
    // passes instead of running in lockstep.
    int rc1;
    for (size_t k = 0; k < units[0].size(); ++k)
      for (int gi = 0; gi < G; ++gi) {
        const bool first = (k == 0);
        if (first && gi > 0) QF_HIP(ctx, hipStreamWaitEvent(grp[gi].st, ctx->stagger[gi - 1], 0));
        if ((rc1 = update_unit(grp[gi], units[0][k], 0, (first && gi + 1 < G) ? ctx->stagger[gi] : nullptr)))
          return rc1;
      }
    for (size_t k = 0; k < units[1].size(); ++k)
      for (int gi = 0; gi < G; ++gi)
        if ((rc1 = update_unit(grp[gi], units[1][k], 1, nullptr))) return rc1;
    if (G > 1) {
      for (int gi = 0; gi < G; ++gi) {
        if (grp[gi].st == home) continue;
        QF_HIP(ctx, hipEventRecord(ctx->join[gi], grp[gi].st));
        QF_HIP(ctx, hipStreamWaitEvent(home, ctx->join[gi], 0));
      }
    }
    return QF_OK;
  };
  // Fused schedule: both groups run the same sequence of steps (an
  // environment step unless the gate is fixed, then a pass); group 1 trails
  // group 0 by one step, so each launch pairs one group's environment with
  // the other's pass.  Steps that do not pair (two passes, a pass form
  // without a fused kernel) are launched alone, in order.
  struct Step {
    int u, half, env;  // unit index within units[half]; env: 1 = environment step, 0 = pass
  };
  std::vector<Step> steps;
  if (fused) {
    for (int half = 0; half < 2; ++half)
      for (int k = 0; k < (int)units[half].size(); ++k) {
        const Unit& un = units[half][k];
        const bool fx = un.g2 < 0 && o.gate_kinds && o.gate_kinds[un.g1] == QF_KIND_FIXED;
        if (!fx) steps.push_back({k, half, 1});
        steps.push_back({k, half, 0});
      }
  }
  auto unit_of = [&](const Step& k) -> const Unit& { return units[k.half][k.u]; };
  auto prep_env = [&](Group& q, const Step& k) -> EnvArgs& {
    const int g = unit_of(k).g1;
    EnvArgs& ea = q.ea;
    ea.kind = o.gate_kinds ? o.gate_kinds[g] : QF_KIND_U4;
    ea.q0 = locs[2 * g];
    ea.q1 = locs[2 * g + 1];
    ea.half = k.half;
    ea.gidx = g;
    return ea;
  };
  auto pass_ops = [&](Group& q, const Step& k, Operand& A, Operand& B) {
    const int g = unit_of(k).g1;
    const bool fx = o.gate_kinds && o.gate_kinds[g] == QF_KIND_FIXED;
    const Operand gnew{q.ea.gates + 2 * 16 * (int64_t)g, gstride, 0};
    const Operand gold = fx ? Operand{q.ea.gates + 2 * 16 * (int64_t)g, gstride, 1} : Operand{q.ea.uold, 16, 1};
    A = k.half == 0 ? gold : gnew;
    B = k.half == 0 ? gnew : gold;
  };
  auto run_alone = [&](Group& q, const Step& k) -> int {
    const Unit& un = unit_of(k);
    if (un.g2 >= 0) {
      if (k.env)
        QF_HIP(ctx, launch_env2(q.st, prec, q.X, env2_args(q, un, k.half)));
      else
        QF_HIP(ctx, launch_pass2(q.st, prec, q.X, q.ns, un.pg, ops_of(q)));
      return QF_OK;
    }
    if (k.env) {
      QF_HIP(ctx, launch_env(q.st, prec, q.X, prep_env(q, k)));
    } else {
      Operand A, B;
      pass_ops(q, k, A, B);
      QF_HIP(ctx, launch_pass(q.st, prec, q.X, q.ns, geo[un.g1], A, B));
    }
    return QF_OK;
  };
  // One pair of groups (q0 leading, q1 trailing by a step) on q0's stream;
  // advance() enqueues one launch of the pair and returns 1 when done.
  struct PairState {
    size_t i0 = 0, i1 = 0;
  };
  auto advance = [&](Group& q0, Group& q1, PairState& ps, int& rc1) -> bool {
    const size_t ns = steps.size();
    if (ps.i0 >= ns && ps.i1 >= ns) return true;
    const Step* a = ps.i0 < ns ? &steps[ps.i0] : nullptr;
    const Step* b = (ps.i1 < ns && ps.i1 < ps.i0) ? &steps[ps.i1] : nullptr;
    if (a && b && a->env != b->env) {
      Group& qe = a->env ? q0 : q1;
      Group& qp = a->env ? q1 : q0;
      const Step& ke = a->env ? *a : *b;
      const Step& kp = a->env ? *b : *a;
      const Unit& ue = unit_of(ke);
      const Unit& up = unit_of(kp);
      hipError_t e = hipErrorNotReady;  // not launched
      if (ue.g2 < 0 && up.g2 < 0 && fused_supported(prec, n, geo[up.g1])) {
        Operand A, B;
        pass_ops(qp, kp, A, B);
        e = launch_fused(q0.st, prec, qe.X, prep_env(qe, ke), qp.X, qp.ns, geo[up.g1], A, B);
      }
      if (e != hipErrorNotReady) {
        if (e != hipSuccess) {
          rc1 = fail(ctx, QF_EHIP, "fused launch: %s", hipGetErrorString(e));
          return true;
        }
        ++ps.i0;
        ++ps.i1;
        return false;
      }
    }
    if (b && (!a || ps.i1 + 1 < ps.i0 || a->env == b->env)) {
      rc1 = run_alone(q1, *b);
      ++ps.i1;
    } else {
      rc1 = run_alone(q0, *a);
      ++ps.i0;
    }
    return rc1 != QF_OK;
  };
  auto sweep_fused = [&]() -> int {
    int rc1 = QF_OK;
    if (pairs > 1) {
      QF_HIP(ctx, hipEventRecord(ctx->fork, st));
      for (int k = 1; k < pairs; ++k) QF_HIP(ctx, hipStreamWaitEvent(ctx->aux[k - 1], ctx->fork, 0));
    }
    PairState ps[kFusedPairs];
    bool done[kFusedPairs] = {};
    for (int k = pairs; k < kFusedPairs; ++k) done[k] = true;
    for (bool all = false; !all;) {  // the pairs' launches are enqueued in turn
      all = true;
      for (int k = 0; k < pairs; ++k) {
        if (!done[k]) done[k] = advance(grp[2 * k], grp[2 * k + 1], ps[k], rc1);
        if (rc1) return rc1;
        all = all && done[k];
      }
    }
    for (int k = 1; k < pairs; ++k) {
      QF_HIP(ctx, hipEventRecord(ctx->join[k], ctx->aux[k - 1]));
      QF_HIP(ctx, hipStreamWaitEvent(st, ctx->join[k], 0));
    }
    return QF_OK;
  };
  auto sweep = [&]() -> int { return fused ? sweep_fused() : sweep_on(st); };
  // FP64 costs of the current gates from a fresh complex128 builder (into
  // R for complex64, into X itself for complex128).
  auto fp64_costs = [&](std::vector<double>& c) -> int {
    void* dst = prec == QF_C64 ? R : X;
    int rc = build_builder(ctx, n, V, p, locs, gates, gstride, S, QF_C128, dst);
    if (rc) return rc;
    QF_HIP(ctx, launch_cost(st, QF_C128, dst, n, S, costs, trace));
    return read_costs(ctx, costs, S, c);
  };

  int rc = build_builder(ctx, n, V, p, locs, gates, gstride, S, prec, X);
  if (rc) return rc;
  // Tune the pass tile width on the freshly built builder (identity operands
  // leave it bit-for-bit unchanged), then lay out every gate's geometry.
  if (!ctx->tuned_tcols[prec == QF_C64][0][n] || !ctx->tuned_tcols[prec == QF_C64][1][n]) {
    if ((rc = autotune_pass(ctx, prec, n, X, S))) return rc;
    if (prec == QF_C64) {  // the FP64 rebuilds use complex128 passes
      if ((rc = build_builder(ctx, n, V, p, locs, gates, gstride, S, QF_C128, R))) return rc;
      if ((rc = autotune_pass(ctx, QF_C128, n, R, S))) return rc;
    }
  }
  for (int g = 0; g < p; ++g) geo[g] = make_pass_geom(n, locs[2 * g], locs[2 * g + 1], pass_tcols(ctx, prec, n, locs[2 * g], locs[2 * g + 1]));
  if (any_pair) {
    const Unit* first = nullptr;
    for (const Unit& u : units[0])
      if (u.g2 >= 0 && !first) first = &u;
    if (!first)
      for (const Unit& u : units[1])
        if (u.g2 >= 0 && !first) first = &u;
    if ((rc = autotune_pass2(ctx, prec, n, X, S, first->pg, ops2))) return rc;
    for (auto& hv : units)
      for (Unit& u : hv) u.pg.tiles_per_wg = (uint32_t)ctx->tuned_pass2[prec == QF_C64][n];
  }
  QF_HIP(ctx, launch_cost(st, prec, X, n, S, costs, trace));
  std::vector<double> c;
  rc = read_costs(ctx, costs, S, c);
  if (rc) return rc;

  bool any_recheck = false;
  if (prec == QF_C64)
    for (int s = 0; s < S; ++s) any_recheck = any_recheck || (c[s] < o.recheck_below);
  if (any_recheck) {
    std::vector<double> c64v = c;
    rc = fp64_costs(c);
    if (rc) return rc;
    ++out.rechecks;
    for (int s = 0; s < S; ++s)
      if (!(c64v[s] < o.recheck_below)) c[s] = c64v[s];
  }

  std::vector<std::vector<double>> hist;
  out.flags.assign(S, 0);
  for (int s = 0; s < S; ++s) {
    if (!std::isfinite(c[s])) {
      c[s] = INFINITY;
      out.flags[s] = kFlagNumeric | kFlagPlateau;
    }
  }
  hist.push_back(c);
  auto record = [&](int i, const std::vector<double>& cv) {
    if (stats && stats->cost_history && i < stats->cost_history_rows)
      for (int s = 0; s < S; ++s) stats->cost_history[(size_t)i * S + s] = cv[s];
  };
  record(0, c);
  std::vector<int32_t> frozen_host(S, 0);
  auto sync_frozen = [&]() -> int {
    bool changed = false;
    for (int s = 0; s < S; ++s) {
      const int32_t fz = (out.flags[s] & kFlagNumeric) ? 1 : 0;
      changed = changed || (fz != frozen_host[s]);
      frozen_host[s] = fz;
    }
    if (changed)
      QF_HIP(ctx, hipMemcpyAsync(frozen, frozen_host.data(), (size_t)S * 4, hipMemcpyHostToDevice, st));
    return QF_OK;
  };
  rc = sync_frozen();
  if (rc) return rc;

  int32_t i = 0;
  int32_t decision = o.max_iter <= 0 ? kStopMaxIter : kContinue;
  if (timer.on) QF_HIP(ctx, hipEventRecord(timer.s0, st));
  while (decision == kContinue) {
    ++i;
    // the FP64 updates start from their gate's previous rotation, cold in
    // the first sweep and once every kWarmPeriod sweeps
    for (int gi = 0; gi < 2 * kMaxGroups; ++gi) grp[gi].ea.warm = ((i - 1) % kWarmPeriod) != 0;
    if ((rc = sweep())) return rc;
    if (o.reset_iter > 0 && i % o.reset_iter == 0) {
      if ((rc = build_builder(ctx, n, V, p, locs, gates, gstride, S, prec, X))) return rc;
      ++out.resets;
    }
    QF_HIP(ctx, launch_cost(st, prec, X, n, S, costs, trace));
    if ((rc = read_costs(ctx, costs, S, c))) return rc;
    if (timer.on) QF_HIP(ctx, timer.collect());
    if (prec == QF_C64) {
      bool need = false;
      for (int s = 0; s < S; ++s) need = need || (!(out.flags[s] & kFlagNumeric) && c[s] < o.recheck_below);
      if (need) {
        std::vector<double> c64v = c, c64d;
        if ((rc = fp64_costs(c64d))) return rc;
        ++out.rechecks;
        for (int s = 0; s < S; ++s)
          if (c64v[s] < o.recheck_below) c[s] = c64d[s];
        if ((rc = cast_to_c64(ctx, R, X, (size_t)S * N * N))) return rc;  // refresh the builder
      }
    }
    const int32_t Lh = o.long_diff_count;
    for (int s = 0; s < S; ++s) {
      double ci = std::isfinite(c[s]) ? c[s] : INFINITY;
      if (out.flags[s] & kFlagNumeric) {
        c[s] = INFINITY;
        continue;
      }
      const double cprev = hist[i - 1][s];
      const double cback = (Lh > 0 && i >= Lh) ? hist[i - Lh][s] : 0.0;
      out.flags[s] = start_flags_after_sweep(o, tol, i, out.flags[s], ci, cprev, cback);
      c[s] = (out.flags[s] & kFlagNumeric) ? INFINITY : ci;
    }
    hist.push_back(c);
    record(i, c);
    if ((rc = sync_frozen())) return rc;
    decision = job_decision(o, i, out.flags.data(), S);
  }
  if (timer.on) {
    QF_HIP(ctx, hipEventRecord(timer.s1, st));
    QF_HIP(ctx, hipEventSynchronize(timer.s1));
    float ms = 0.f;
    QF_HIP(ctx, hipEventElapsedTime(&ms, timer.s0, timer.s1));
    stats->pass_ms = timer.pass_ms;
    stats->env_ms = timer.env_ms;
    stats->pass_launches = timer.pass_n;
    stats->env_launches = timer.env_n;
    stats->pass2_launches = timer.pass2_n;
    stats->pass2_ms = timer.pass2_ms;
    stats->sweep_ms = ms;
  }
  out.sweeps = i;
  out.decision = decision;
  rc = fp64_costs(out.final_costs);
  if (rc) return rc;
  return QF_OK;
}

// ----------------------------------------------------------------- resident

int run_resident(qf_ctx* ctx, int n, const void* V, int p, int S, double tol, const qf_options& o,
                 unsigned char* ws, const Layout& L, qf_stats* stats, int history_rows, RunOut& out) {
  hipStream_t st = ctx->stream;
  ResidentArgs a{};
  a.n = n;
  a.p = p;
  a.S = S;
  a.precision = o.precision;
  a.V = reinterpret_cast<const double*>(V);
  a.locs = reinterpret_cast<const int32_t*>(ws + L.locs);
  a.gates = reinterpret_cast<double*>(ws + L.gates);
  a.tol = tol;
  a.opt = o;
  a.hist = reinterpret_cast<double*>(ws + L.hist);
  a.ring = L.ring;
  a.flags = reinterpret_cast<int32_t*>(ws + L.flags);
  a.cur_cost = reinterpret_cast<double*>(ws + L.cur);
  a.final_cost = reinterpret_cast<double*>(ws + L.fin);
  a.sync = reinterpret_cast<int32_t*>(ws + L.sync);
  a.out_info = reinterpret_cast<int32_t*>(ws + L.info);
  a.history_out = history_rows > 0 ? reinterpret_cast<double*>(ws + L.histo) : nullptr;
  a.history_rows = history_rows;
  a.kinds = o.gate_kinds ? reinterpret_cast<const int32_t*>(ws + L.kinds) : nullptr;
  a.ywarm = reinterpret_cast<double*>(ws + L.ywarm);
  QF_HIP(ctx, launch_fill_i32(st, a.sync, 0, 16));
  QF_HIP(ctx, launch_fill_i32(st, a.out_info, 0, 16));
  int ok = 0;
  QF_HIP(ctx, launch_resident(st, a, &ok));
  if (!ok) return fail(ctx, QF_EUNSUPPORTED, "resident mode: %d starts do not fit on the device at once", S);
  int32_t info[8];
  QF_HIP(ctx, hipMemcpyAsync(info, ws + L.info, sizeof info, hipMemcpyDeviceToHost, st));
  std::vector<double> fin(S);
  std::vector<int32_t> fl(2 * (size_t)S);
  QF_HIP(ctx, hipMemcpyAsync(fin.data(), ws + L.fin, (size_t)S * 8, hipMemcpyDeviceToHost, st));
  QF_HIP(ctx, hipMemcpyAsync(fl.data(), ws + L.flags, (size_t)2 * S * 4, hipMemcpyDeviceToHost, st));
  std::vector<double> ho;
  if (history_rows > 0) {
    ho.resize((size_t)history_rows * S);
    QF_HIP(ctx, hipMemcpyAsync(ho.data(), ws + L.histo, ho.size() * 8, hipMemcpyDeviceToHost, st));
  }
  QF_HIP(ctx, hipStreamSynchronize(st));
  if (info[4]) return fail(ctx, QF_ETIMEOUT, "resident mode: device barrier wait gave up");
  out.sweeps = info[0];
  out.decision = info[1];
  out.resets = info[2];
  out.rechecks = info[3];
  out.final_costs = fin;
  out.flags.assign(fl.begin() + (size_t)(out.sweeps & 1) * S, fl.begin() + (size_t)(out.sweeps & 1) * S + S);
  if (out.sweeps == 0) out.flags.assign(S, 0);
  if (stats && stats->cost_history && history_rows > 0) {
    const int rows = std::min(std::min(history_rows, out.sweeps + 1), stats->cost_history_rows);
    if (rows > 0) std::memcpy(stats->cost_history, ho.data(), (size_t)rows * S * 8);
  }
  return QF_OK;
}

// Workspace layout of qf_instantiate_batch.
struct BatchLayout {
  size_t order = 0, blk_n = 0, gate_off = 0, tgt_off = 0, locs = 0, kinds = 0, hist = 0, scratch = 0, ywarm = 0,
         cost = 0, best = 0, status = 0, sweeps = 0, queue = 0;
  size_t total = 0;
  int ring = 2;
};

BatchLayout make_batch_layout(int n_blocks, int total_gates, int S, const qf_options& o) {
  BatchLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t nb = (size_t)n_blocks;
  L.order = take(nb * 4);
  L.blk_n = take(nb * 4);
  L.gate_off = take((nb + 1) * 4);
  L.tgt_off = take(nb * 8);
  L.locs = take((size_t)total_gates * 8);
  L.kinds = take((size_t)total_gates * 4);
  L.ring = std::max(2, o.long_diff_count + 1);
  L.hist = take(nb * S * L.ring * 8);
  L.scratch = take(batch_scratch_entries(n_blocks, S) * 16);
  L.ywarm = take((size_t)total_gates * S * 2 * 16 * 16);
  L.cost = take(nb * S * 8);
  L.best = take(nb * 4);
  L.status = take(nb * 4);
  L.sweeps = take(nb * 4);
  L.queue = take(4);
  L.total = off;
  return L;
}

int validate_batch(qf_ctx* ctx, int n_blocks, const int32_t* block_n, const int32_t* gate_offsets,
                   const int32_t* locs, int S) {
  if (n_blocks < 1) return fail(ctx, QF_EINVAL, "n_blocks must be >= 1");
  if (!block_n || !gate_offsets) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  if (S < 1 || S > 16) return fail(ctx, QF_EINVAL, "n_starts=%d outside [1, 16]", S);
  if (gate_offsets[0] != 0) return fail(ctx, QF_EINVAL, "gate_offsets[0] must be 0");
  for (int b = 0; b < n_blocks; ++b) {
    if (block_n[b] < 2 || block_n[b] > 4) return fail(ctx, QF_EINVAL, "block %d: n=%d outside [2, 4]", b, block_n[b]);
    if (gate_offsets[b + 1] <= gate_offsets[b]) return fail(ctx, QF_EINVAL, "block %d has no gates", b);
    if ((int64_t)gate_offsets[b + 1] * S * 16 > ((int64_t)1 << 31))
      return fail(ctx, QF_EINVAL, "too many gates in the batch");
  }
  if (!locs) return fail(ctx, QF_EINVAL, "locations is NULL");
  for (int b = 0; b < n_blocks; ++b)
    for (int g = gate_offsets[b]; g < gate_offsets[b + 1]; ++g)
      if (!valid_loc(block_n[b], locs + 2 * g))
        return fail(ctx, QF_EINVAL, "block %d gate %d: location (%d, %d) invalid for n=%d", b, g - gate_offsets[b],
                    locs[2 * g], locs[2 * g + 1], block_n[b]);
  return QF_OK;
}

// Workspace layout of qf_gradient.
struct GradLayout {
  size_t X = 0, partials = 0, counters = 0, envP = 0, trace = 0, total = 0;
};

GradLayout make_grad_layout(int n, int p, int S, int precision) {
  GradLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t N = (size_t)1 << n;
  L.X = take((size_t)S * N * N * elem_bytes(precision));
  L.partials = take((size_t)S * env_workgroups(n, 1) * 16 * 16);
  L.counters = take((size_t)S * 4);
  L.envP = take((size_t)p * S * 16 * 16);
  L.trace = take((size_t)S * 16);
  L.total = off;
  return L;
}

// Cost and gate gradient of S starts (gates: device S x p x 16 c128).
int run_gradient(qf_ctx* ctx, int n, const void* V, int p, const int32_t* locs, const double* gates, int S,
                 int prec, unsigned char* ws, const GradLayout& L, double* cost_out, double* grad_out) {
  hipStream_t st = ctx->stream;
  void* X = ws + L.X;
  const int64_t gstride = (int64_t)p * 16;
  double* envP = reinterpret_cast<double*>(ws + L.envP);
  double* trace = reinterpret_cast<double*>(ws + L.trace);
  int32_t* counters = reinterpret_cast<int32_t*>(ws + L.counters);
  QF_HIP(ctx, launch_fill_i32(st, counters, 0, (uint32_t)S));
  int rc = build_builder(ctx, n, V, p, locs, gates, gstride, S, prec, X);
  if (rc) return rc;
  QF_HIP(ctx, launch_cost(st, prec, X, n, S, cost_out, trace));
  EnvArgs ea{};
  ea.n = n;
  ea.S = S;
  ea.do_update = 0;
  ea.partials = reinterpret_cast<double*>(ws + L.partials);
  ea.counters = counters;
  ea.nwg = (int)env_workgroups(n, S);
  for (int g = p - 1; g >= 0; --g) {
    ea.q0 = locs[2 * g];
    ea.q1 = locs[2 * g + 1];
    ea.env_out = envP + (size_t)g * S * 32;
    QF_HIP(ctx, launch_env(st, prec, X, ea));
    if (g > 0) {  // move u_g to the input legs; the last move is not needed
      const PassGeom geo = make_pass_geom(n, locs[2 * g], locs[2 * g + 1], pass_tcols(ctx, prec, n, locs[2 * g], locs[2 * g + 1]));
      Operand ud{gates + 2 * 16 * (int64_t)g, gstride, 1};
      Operand u{gates + 2 * 16 * (int64_t)g, gstride, 0};
      QF_HIP(ctx, launch_pass(st, prec, X, S, geo, ud, u));
    }
  }
  QF_HIP(ctx, launch_grad_finish(st, envP, gates, trace, n, S, p, grad_out));
  return QF_OK;
}

// Workspace layout of qf_lbfgs: the gradient's, plus gates, gate gradients,
// trial parameters, parameter gradients and costs of every start.
struct LbfgsLayout {
  GradLayout G;
  size_t gates = 0, ggrad = 0, theta = 0, dtheta = 0, costs = 0, total = 0;
};

LbfgsLayout make_lbfgs_layout(int n, int p, int S, int precision) {
  LbfgsLayout L;
  L.G = make_grad_layout(n, p, S, precision);
  size_t off = L.G.total;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.gates = take((size_t)S * p * 256);
  L.ggrad = take((size_t)S * p * 256);
  L.theta = take((size_t)S * p * 15 * 8);
  L.dtheta = take((size_t)S * p * 15 * 8);
  L.costs = take((size_t)S * 8);
  L.total = off;
  return L;
}

}  // namespace

// =================================================================== C ABI

extern "C" {

const char* qf_strerror(int status) {
  switch (status) {
    case QF_OK: return "ok";
    case QF_EINVAL: return "invalid argument";
    case QF_EUNSUPPORTED: return "unsupported request";
    case QF_EHIP: return "HIP runtime error";
    case QF_EWORKSPACE: return "workspace missing or too small";
    case QF_ENUMERIC: return "every start produced non-finite values";
    case QF_ETIMEOUT: return "device-side wait timed out";
    default: return "unknown status";
  }
}

const char* qf_last_error(const qf_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

void qf_options_default(qf_options* o) {
  if (!o) return;
  o->dist_tol = 1e-10;
  o->diff_tol_a = 0.0;
  o->diff_tol_r = 1e-5;
  o->long_diff_count = 100;
  o->long_diff_r = 0.1;
  o->min_iter = 0;
  o->max_iter = 100000;
  o->reset_iter = 40;
  o->beta = 0.0;
  o->precision = QF_C128;
  o->mode = QF_MODE_AUTO;
  o->recheck_below = 1e-3;
  o->stream_groups = 0;
  o->gate_kinds = nullptr;
  o->gate_pairs = 1;
}

int qf_create(qf_ctx** out, int device, void* hip_stream) {
  if (!out) return QF_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return QF_EINVAL;
  qf_ctx* ctx = new (std::nothrow) qf_ctx();
  if (!ctx) return QF_EHIP;
  ctx->device = device;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  DeviceGuard dg(device);
  double id[32] = {};
  for (int k = 0; k < 4; ++k) id[2 * (5 * k)] = 1.0;
  const bool ok =
      dg.ok &&
      hipHostMalloc(reinterpret_cast<void**>(&ctx->pinned), kPinnedCount * sizeof(double), hipHostMallocDefault) ==
          hipSuccess &&
      hipMalloc(&ctx->scratch, kScratchBytes) == hipSuccess &&
      hipMalloc(reinterpret_cast<void**>(&ctx->identity), sizeof id) == hipSuccess &&
      hipMemcpy(ctx->identity, id, sizeof id, hipMemcpyHostToDevice) == hipSuccess &&
      hipMemset(ctx->scratch, 0, kScratchBytes) == hipSuccess &&  // arrival counters start at zero
      ensure_aux_streams(ctx) == QF_OK;
  if (!ok) {
    (void)qf_destroy(ctx);
    return QF_EHIP;
  }
  ctx->static_ws = static_scratch_ptr(device);  // device current (DeviceGuard)
  *out = ctx;
  return QF_OK;
}

int qf_destroy(qf_ctx* ctx) {
  if (!ctx) return QF_EINVAL;
  {
    DeviceGuard dg(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (int i = 0; i < kMaxGroups; ++i) {
      if (ctx->aux[i]) {
        (void)hipStreamSynchronize(ctx->aux[i]);
        (void)hipStreamDestroy(ctx->aux[i]);
      }
      if (ctx->join[i]) (void)hipEventDestroy(ctx->join[i]);
      if (ctx->stagger[i]) (void)hipEventDestroy(ctx->stagger[i]);
    }
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    for (hipEvent_t e : ctx->tune)
      if (e) (void)hipEventDestroy(e);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->identity) (void)hipFree(ctx->identity);
  }
  delete ctx;
  return QF_OK;
}

int qf_set_stream(qf_ctx* ctx, void* hip_stream) {
  if (!ctx) return QF_EINVAL;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return QF_OK;
}

int qf_set_pass_tile(qf_ctx* ctx, int precision, int n, int gate_class, int tile) {
  if (!ctx) return QF_EINVAL;
  if (precision != QF_C128 && precision != QF_C64) return fail(ctx, QF_EINVAL, "unknown precision");
  if (n < 2 || n > 16) return fail(ctx, QF_EINVAL, "n=%d outside [2, 16]", n);
  if (gate_class != 0 && gate_class != 1) return fail(ctx, QF_EINVAL, "gate_class must be 0 or 1");
  const bool ok = tile == 0 || tile == kPassDirect || tile == 256 || tile == 512 ||
                  ((tile == 1024 || tile == kPassMicro) && precision == QF_C64);
  if (!ok) return fail(ctx, QF_EINVAL, "tile %d not supported", tile);
  ctx->tuned_tcols[precision == QF_C64][gate_class][n] = tile;
  return QF_OK;
}

int qf_set_pass2_tiles(qf_ctx* ctx, int precision, int n, int tiles) {
  if (!ctx) return QF_EINVAL;
  if (precision != QF_C128 && precision != QF_C64) return fail(ctx, QF_EINVAL, "unknown precision");
  if (n < 4 || n > 16) return fail(ctx, QF_EINVAL, "n=%d outside [4, 16]", n);
  if (tiles != 0 && tiles != 1 && tiles != 2 && tiles != 4 && tiles != 8)
    return fail(ctx, QF_EINVAL, "tiles %d not supported", tiles);
  ctx->tuned_pass2[precision == QF_C64][n] = tiles;
  return QF_OK;
}

size_t qf_workspace_size(int n, int n_gates, int n_starts, const qf_options* opt) {
  qf_options o;
  if (opt)
    o = *opt;
  else
    qf_options_default(&o);
  if (n < 2 || n > 16 || n_gates < 1 || n_starts < 1) return 0;
  if (validate_options(nullptr, o) != QF_OK) return 0;
  const int mode = resolve_mode(n, o);
  return make_layout(n, n_gates, n_starts, o, mode, resident_history_rows(mode, o)).total;
}

int qf_build(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations,
             const void* gates, int n_starts, int precision, void* builder) {
  if (!ctx) return QF_EINVAL;
  int rc = validate_problem(ctx, n, n_gates, locations, n_starts);
  if (rc) return rc;
  if (!target || !gates || !builder) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  if (precision != QF_C128 && precision != QF_C64) return fail(ctx, QF_EINVAL, "unknown precision");
  DeviceGuard dg(ctx->device);
  return build_builder(ctx, n, target, n_gates, locations, reinterpret_cast<const double*>(gates),
                       (int64_t)n_gates * 16, n_starts, precision, builder);
}

int qf_apply_gate(qf_ctx* ctx, int n, int n_builders, void* builder, int precision, const int32_t* loc,
                  const void* gates, int side, int dagger) {
  if (!ctx) return QF_EINVAL;
  if (n < 2 || n > 16) return fail(ctx, QF_EINVAL, "n=%d outside [2, 16]", n);
  if (n_builders < 1) return fail(ctx, QF_EINVAL, "n_builders must be >= 1");
  if (!valid_loc(n, loc)) return fail(ctx, QF_EINVAL, "invalid gate location");
  if (!builder || !gates) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  if (precision != QF_C128 && precision != QF_C64) return fail(ctx, QF_EINVAL, "unknown precision");
  if (side != QF_LEFT && side != QF_RIGHT) return fail(ctx, QF_EINVAL, "side must be QF_LEFT or QF_RIGHT");
  DeviceGuard dg(ctx->device);
  const PassGeom geo = make_pass_geom(n, loc[0], loc[1], pass_tcols(ctx, precision, n, loc[0], loc[1]));
  Operand G{reinterpret_cast<const double*>(gates), 16, dagger ? 1 : 0};
  Operand none{nullptr, 0, 0};
  QF_HIP(ctx, launch_pass(ctx->stream, precision, builder, n_builders, geo, side == QF_LEFT ? G : none,
                          side == QF_LEFT ? none : G));
  return QF_OK;
}

int qf_environment(qf_ctx* ctx, int n, int n_builders, const void* builder, int precision,
                   const int32_t* loc, void* env_out) {
  if (!ctx) return QF_EINVAL;
  if (n < 2 || n > 16) return fail(ctx, QF_EINVAL, "n=%d outside [2, 16]", n);
  if (n_builders < 1) return fail(ctx, QF_EINVAL, "n_builders must be >= 1");
  if (!valid_loc(n, loc)) return fail(ctx, QF_EINVAL, "invalid gate location");
  if (!builder || !env_out) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  if (precision != QF_C128 && precision != QF_C64) return fail(ctx, QF_EINVAL, "unknown precision");
  DeviceGuard dg(ctx->device);
  unsigned char* sc = reinterpret_cast<unsigned char*>(ctx->scratch);
  const size_t bstride = ((size_t)1 << (2 * n)) * elem_bytes(precision);
  for (int c0 = 0; c0 < n_builders; c0 += kScratchChunk) {
    const int cs = std::min(kScratchChunk, n_builders - c0);
    EnvArgs ea{};
    ea.n = n;
    ea.q0 = loc[0];
    ea.q1 = loc[1];
    ea.S = cs;
    ea.nwg = (int)env_workgroups(n, cs);
    ea.do_update = 0;
    ea.env_out = reinterpret_cast<double*>(env_out) + (size_t)c0 * 32;
    ea.partials = reinterpret_cast<double*>(sc + kScratchPartials);
    ea.counters = reinterpret_cast<int32_t*>(sc + kScratchCounters);  // left zero by every launch
    QF_HIP(ctx, launch_env(ctx->stream, precision, reinterpret_cast<const unsigned char*>(builder) + c0 * bstride, ea));
  }
  return QF_OK;
}

int qf_optimize_gate(qf_ctx* ctx, int count, const void* env, const void* u_old, double beta, void* u_new) {
  if (!ctx) return QF_EINVAL;
  if (count < 1) return fail(ctx, QF_EINVAL, "count must be >= 1");
  if (!env || !u_old || !u_new) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  if (!(beta >= 0.0 && beta <= 1.0)) return fail(ctx, QF_EINVAL, "beta must be in [0, 1]");
  DeviceGuard dg(ctx->device);
  QF_HIP(ctx, launch_optimize(ctx->stream, count, reinterpret_cast<const double*>(env),
                              reinterpret_cast<const double*>(u_old), beta, reinterpret_cast<double*>(u_new)));
  return QF_OK;
}

int qf_update_gate(qf_ctx* ctx, int n, int n_builders, void* builder, int precision, const int32_t* loc,
                   int half, double beta, void* gates, void* env_out) {
  if (!ctx) return QF_EINVAL;
  if (n < 2 || n > 16) return fail(ctx, QF_EINVAL, "n=%d outside [2, 16]", n);
  if (n_builders < 1) return fail(ctx, QF_EINVAL, "n_builders must be >= 1");
  if (!valid_loc(n, loc)) return fail(ctx, QF_EINVAL, "invalid gate location");
  if (!builder || !gates) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  if (precision != QF_C128 && precision != QF_C64) return fail(ctx, QF_EINVAL, "unknown precision");
  if (half != 0 && half != 1) return fail(ctx, QF_EINVAL, "half must be 0 or 1");
  if (!(beta >= 0.0 && beta <= 1.0)) return fail(ctx, QF_EINVAL, "beta must be in [0, 1]");
  DeviceGuard dg(ctx->device);
  unsigned char* sc = reinterpret_cast<unsigned char*>(ctx->scratch);
  const size_t bstride = ((size_t)1 << (2 * n)) * elem_bytes(precision);
  const PassGeom geo = make_pass_geom(n, loc[0], loc[1], pass_tcols(ctx, precision, n, loc[0], loc[1]));
  for (int c0 = 0; c0 < n_builders; c0 += kScratchChunk) {
    const int cs = std::min(kScratchChunk, n_builders - c0);
    void* Xc = reinterpret_cast<unsigned char*>(builder) + c0 * bstride;
    EnvArgs ea{};
    ea.n = n;
    ea.q0 = loc[0];
    ea.q1 = loc[1];
    ea.S = cs;
    ea.nwg = (int)env_workgroups(n, cs);
    ea.do_update = 1;
    ea.half = half;
    ea.beta = beta;
    ea.gates = reinterpret_cast<double*>(gates) + (size_t)c0 * 32;
    ea.gstride = 16;
    ea.gidx = 0;
    ea.uold = reinterpret_cast<double*>(sc + kScratchUold);
    ea.env_out = env_out ? reinterpret_cast<double*>(env_out) + (size_t)c0 * 32 : nullptr;
    ea.partials = reinterpret_cast<double*>(sc + kScratchPartials);
    ea.counters = reinterpret_cast<int32_t*>(sc + kScratchCounters);  // left zero by every launch
    QF_HIP(ctx, launch_env(ctx->stream, precision, Xc, ea));
    Operand gnew{ea.gates, 16, 0};
    Operand gold{ea.uold, 16, 1};
    if (half == 0)
      QF_HIP(ctx, launch_pass(ctx->stream, precision, Xc, cs, geo, gold, gnew));
    else
      QF_HIP(ctx, launch_pass(ctx->stream, precision, Xc, cs, geo, gnew, gold));
  }
  return QF_OK;
}

int qf_cost(qf_ctx* ctx, int n, int n_builders, const void* builder, int precision, double* cost_out,
            void* trace_out) {
  if (!ctx) return QF_EINVAL;
  if (n < 2 || n > 16) return fail(ctx, QF_EINVAL, "n=%d outside [2, 16]", n);
  if (n_builders < 1) return fail(ctx, QF_EINVAL, "n_builders must be >= 1");
  if (!builder || !cost_out) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  if (precision != QF_C128 && precision != QF_C64) return fail(ctx, QF_EINVAL, "unknown precision");
  DeviceGuard dg(ctx->device);
  QF_HIP(ctx, launch_cost(ctx->stream, precision, builder, n, n_builders, cost_out,
                          reinterpret_cast<double*>(trace_out)));
  return QF_OK;
}

int qf_instantiate(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations,
                   const void* init_gates, int n_starts, double tol, const qf_options* opt, void* workspace,
                   size_t ws_bytes, void* out_gates, void* out_all_gates, double* out_costs, qf_stats* stats) {
  if (!ctx) return QF_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  qf_options o;
  if (opt)
    o = *opt;
  else
    qf_options_default(&o);
  if (!(tol > 0) || !std::isfinite(tol)) return fail(ctx, QF_EINVAL, "tol must be finite and > 0");
  o.dist_tol = tol;
  int rc = validate_options(ctx, o);
  if (rc) return rc;
  rc = validate_problem(ctx, n, n_gates, locations, n_starts);
  if (rc) return rc;
  if ((rc = validate_kinds(ctx, o.gate_kinds, n_gates))) return rc;
  if (!target || !init_gates || !out_gates || !out_costs)
    return fail(ctx, QF_EINVAL, "NULL pointer argument");
  if (stats && stats->cost_history && stats->cost_history_rows < 0)
    return fail(ctx, QF_EINVAL, "cost_history_rows must be >= 0");
  const int mode = resolve_mode(n, o);
  if (mode == QF_MODE_RESIDENT && n > 6) return fail(ctx, QF_EUNSUPPORTED, "resident mode needs n <= 6");
  const int rows = resident_history_rows(mode, o);
  const Layout L = make_layout(n, n_gates, n_starts, o, mode, rows);
  if (!workspace || ws_bytes < L.total)
    return fail(ctx, QF_EWORKSPACE, "workspace of %zu bytes needed, %zu given", L.total, ws_bytes);
  DeviceGuard dg(ctx->device);
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
  hipStream_t st = ctx->stream;
  const size_t gate_bytes = (size_t)n_starts * n_gates * 256;
  QF_HIP(ctx, hipMemcpyAsync(ws + L.gates, init_gates, gate_bytes, hipMemcpyDeviceToDevice, st));
  QF_HIP(ctx, hipMemcpyAsync(ws + L.locs, locations, (size_t)n_gates * 8, hipMemcpyHostToDevice, st));
  if (o.gate_kinds)
    QF_HIP(ctx, hipMemcpyAsync(ws + L.kinds, o.gate_kinds, (size_t)n_gates * 4, hipMemcpyHostToDevice, st));

  if (stats) {
    stats->pass_launches = stats->env_launches = stats->pass2_launches = 0;
    stats->pass_ms = stats->env_ms = stats->sweep_ms = stats->pass2_ms = 0.0;
  }
  RunOut out;
  if (mode == QF_MODE_RESIDENT)
    rc = run_resident(ctx, n, target, n_gates, n_starts, tol, o, ws, L, stats, rows, out);
  else
    rc = run_streaming(ctx, n, target, n_gates, locations, n_starts, tol, o, ws, L, stats, out);
  if (rc) return rc;

  int best = 0;
  bool all_numeric = true;
  for (int s = 0; s < n_starts; ++s) {
    double cs = out.final_costs[s];
    if (!std::isfinite(cs) || (s < (int)out.flags.size() && (out.flags[s] & kFlagNumeric))) cs = INFINITY;
    out.final_costs[s] = cs;
    out_costs[s] = cs;
    all_numeric = all_numeric && !std::isfinite(cs);
    if (cs < out.final_costs[best]) best = s;
  }
  QF_HIP(ctx, hipMemcpyAsync(out_gates, ws + L.gates + (size_t)best * n_gates * 256, (size_t)n_gates * 256,
                             hipMemcpyDeviceToDevice, st));
  if (out_all_gates)
    QF_HIP(ctx, hipMemcpyAsync(out_all_gates, ws + L.gates, gate_bytes, hipMemcpyDeviceToDevice, st));
  QF_HIP(ctx, hipStreamSynchronize(st));
  int status = QF_MAX_ITER;
  if (all_numeric)
    status = QF_NUMERIC;
  else if (out.final_costs[best] < tol)
    status = QF_CONVERGED;
  else if (out.decision == kStopPlateau)
    status = QF_PLATEAU;
  if (stats) {
    stats->sweeps = out.sweeps;
    stats->best_start = best;
    stats->status = status;
    stats->n_resets = out.resets;
    stats->n_rechecks = out.rechecks;
    stats->mode_used = mode;
    stats->pass_tcols = mode == QF_MODE_STREAMING ? pass_tcols(ctx, o.precision, n, n / 2 - 1, n / 2) : 0;
    stats->best_cost = out.final_costs[best];
    stats->elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (all_numeric) return fail(ctx, QF_ENUMERIC, "every start produced non-finite values");
  return QF_OK;
}

int qf_instantiate_noalloc(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations,
                           const void* init_gates, int n_starts, double tol, const qf_options* opt, void* out_gates,
                           void* out_all_gates, double* out_costs, qf_stats* stats) {
  if (!ctx) return QF_EINVAL;
  const size_t need = qf_workspace_size(n, n_gates, n_starts, opt);
  if (need == 0)  // invalid sizes or options: let qf_instantiate name the problem
    return qf_instantiate(ctx, n, target, n_gates, locations, init_gates, n_starts, tol, opt, nullptr, 0,
                          out_gates, out_all_gates, out_costs, stats);
  if (need > (size_t)QF_NOALLOC_WORKSPACE_BYTES)
    return fail(ctx, QF_EWORKSPACE,
                "qf_instantiate_noalloc: this problem needs %zu bytes of workspace, more than the fixed %zu "
                "(use qf_instantiate with a caller workspace)",
                need, (size_t)QF_NOALLOC_WORKSPACE_BYTES);
  if (stats && stats->timing)
    return fail(ctx, QF_EUNSUPPORTED, "qf_instantiate_noalloc: stats->timing creates HIP events per launch");
  if (!ctx->static_ws)
    return fail(ctx, QF_EHIP, "qf_instantiate_noalloc: the fixed workspace's device address is unavailable");
  return qf_instantiate(ctx, n, target, n_gates, locations, init_gates, n_starts, tol, opt, ctx->static_ws,
                        (size_t)QF_NOALLOC_WORKSPACE_BYTES, out_gates, out_all_gates, out_costs, stats);
}

// ------------------------------------------------------- three-qubit gates

struct Layout3 {
  size_t X = 0, R = 0, gates = 0, uold = 0, costs = 0, trace = 0, frozen = 0, ywarm = 0, total = 0;
};

Layout3 make_layout3(int n, int p, int S, int precision) {
  Layout3 L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t N = (size_t)1 << n;
  L.X = take((size_t)S * N * N * elem_bytes(precision));
  if (precision == QF_C64) L.R = take((size_t)S * N * N * 16);
  L.gates = take((size_t)S * p * 64 * 16);
  L.uold = take((size_t)S * 64 * 16);
  L.costs = take((size_t)S * 8);
  L.trace = take((size_t)S * 16);
  L.frozen = take((size_t)S * 4);
  L.ywarm = take((size_t)S * p * 2 * 64 * 16);  // warm starts of the FP64 updates, per (start, gate, half)
  L.total = off;
  return L;
}

int validate_problem3(qf_ctx* ctx, int n, int p, const int32_t* locs, int S, const qf_options& o) {
  if (n < 3 || n > 14) return fail(ctx, QF_EINVAL, "n=%d outside [3, 14] for three-qubit gates", n);
  if (p < 1) return fail(ctx, QF_EINVAL, "n_gates must be >= 1");
  if (!locs) return fail(ctx, QF_EINVAL, "locations is NULL");
  for (int g = 0; g < p; ++g) {
    const int32_t* l = locs + 3 * g;
    const bool ok = l[0] >= 0 && l[0] < n && l[1] >= 0 && l[1] < n && l[2] >= 0 && l[2] < n && l[0] != l[1] &&
                    l[0] != l[2] && l[1] != l[2];
    if (!ok) return fail(ctx, QF_EINVAL, "gate %d: location (%d, %d, %d) invalid for n=%d", g, l[0], l[1], l[2], n);
  }
  if (S < 1) return fail(ctx, QF_EINVAL, "n_starts must be >= 1");
  if (o.gate_kinds) return fail(ctx, QF_EINVAL, "gate_kinds must be NULL for three-qubit gates");
  if (o.mode == QF_MODE_RESIDENT) return fail(ctx, QF_EUNSUPPORTED, "three-qubit gates run in streaming mode only");
  return QF_OK;
}

// Alg. 1 on 8 x 8 gates, all starts on the context stream (same termination,
// multistart rule, complex64 recheck and final FP64 costs as run_streaming).
int run_streaming3(qf_ctx* ctx, int n, const void* V, int p, const int32_t* locs, int S, double tol,
                   const qf_options& o, unsigned char* ws, const Layout3& L, qf_stats* stats, RunOut& out) {
  hipStream_t st = ctx->stream;
  const int prec = o.precision;
  void* X = ws + L.X;
  void* R = prec == QF_C64 ? (void*)(ws + L.R) : nullptr;
  double* gates = reinterpret_cast<double*>(ws + L.gates);
  double* uold = reinterpret_cast<double*>(ws + L.uold);
  double* costs = reinterpret_cast<double*>(ws + L.costs);
  double* trace = reinterpret_cast<double*>(ws + L.trace);
  int32_t* frozen = reinterpret_cast<int32_t*>(ws + L.frozen);
  const int64_t gstride = (int64_t)p * 64;
  const size_t N = (size_t)1 << n;
  std::vector<Pass8Geom> geo(p);
  for (int g = 0; g < p; ++g) geo[g] = make_pass8_geom(n, locs + 3 * g);
  QF_HIP(ctx, launch_fill_i32(st, frozen, 0, (uint32_t)S));

  auto build = [&](int pr, void* dst) -> int {
    QF_HIP(ctx, launch_build_init(st, pr, V, dst, n, S));
    for (int g = 0; g < p; ++g)
      QF_HIP(ctx, launch_pass8(st, pr, dst, S, geo[g], Operand{gates + 2 * 64 * (int64_t)g, gstride, 0},
                               Operand{nullptr, 0, 0}));
    return QF_OK;
  };
  auto fp64_costs = [&](std::vector<double>& c) -> int {
    void* dst = prec == QF_C64 ? R : X;
    int rc = build(QF_C128, dst);
    if (rc) return rc;
    QF_HIP(ctx, launch_cost(st, QF_C128, dst, n, S, costs, trace));
    return read_costs(ctx, costs, S, c);
  };
  // The starts split into G groups whose sweeps run on separate streams
  // (group 0 on the caller's), staggered, so that one group's environment
  // step (the 8x8 FP64 update's latency) runs while another group's pass
  // streams.  Every start sees the same kernels in the same order, so the
  // results do not depend on G.
  int G = o.stream_groups > 0 ? o.stream_groups : kDefaultGroups3;
  G = std::min(std::min(G, kMaxGroups), S);
  if (G > 1) {
    int rc0 = ensure_aux_streams(ctx);
    if (rc0) return rc0;
  }
  struct Group3 {
    int s0 = 0, ns = 0;
    hipStream_t st = nullptr;
    void* X = nullptr;
    Env8Args ea{};
  };
  Group3 grp[kMaxGroups];
  for (int gi = 0; gi < G; ++gi) {
    Group3& q = grp[gi];
    q.s0 = gi * S / G;
    q.ns = (gi + 1) * S / G - q.s0;
    q.st = gi == 0 ? st : ctx->aux[gi - 1];
    q.X = reinterpret_cast<unsigned char*>(X) + (size_t)q.s0 * N * N * elem_bytes(prec);
    q.ea.S = q.ns;
    q.ea.do_update = 1;
    q.ea.beta = o.beta;
    q.ea.gates = gates + (size_t)q.s0 * gstride * 2;
    q.ea.gstride = gstride;
    q.ea.uold = uold + (size_t)q.s0 * 64 * 2;
    q.ea.frozen = frozen + q.s0;
    q.ea.ywstride = (int64_t)p * 128;
    q.ea.ywarm = reinterpret_cast<double*>(ws + L.ywarm) + (size_t)q.s0 * q.ea.ywstride * 2;
  }
  auto update = [&](Group3& q, int g, int half, hipEvent_t after_env) -> int {
    q.ea.half = half;
    q.ea.gidx = g;
    QF_HIP(ctx, launch_env8(q.st, prec, q.X, geo[g], q.ea));
    if (after_env) QF_HIP(ctx, hipEventRecord(after_env, q.st));
    const Operand gnew{q.ea.gates + 2 * 64 * (int64_t)g, gstride, 0};
    const Operand gold{q.ea.uold, 64, 1};
    if (half == 0)
      QF_HIP(ctx, launch_pass8(q.st, prec, q.X, q.ns, geo[g], gold, gnew));
    else
      QF_HIP(ctx, launch_pass8(q.st, prec, q.X, q.ns, geo[g], gnew, gold));
    return QF_OK;
  };
  // One TwoSidedSweep of every start (Alg. 1 order), groups interleaved,
  // forked from and joined back to the caller's stream; group k starts once
  // group k-1's first environment step is done.
  auto sweep = [&]() -> int {
    if (G > 1) {
      QF_HIP(ctx, hipEventRecord(ctx->fork, st));
      for (int gi = 1; gi < G; ++gi) QF_HIP(ctx, hipStreamWaitEvent(grp[gi].st, ctx->fork, 0));
    }
    int rc1;
    for (int g = p - 1; g >= 0; --g)
      for (int gi = 0; gi < G; ++gi) {
        const bool first = (g == p - 1);
        if (first && gi > 0) QF_HIP(ctx, hipStreamWaitEvent(grp[gi].st, ctx->stagger[gi - 1], 0));
        if ((rc1 = update(grp[gi], g, 0, (first && gi + 1 < G) ? ctx->stagger[gi] : nullptr))) return rc1;
      }
    for (int g = 0; g < p; ++g)
      for (int gi = 0; gi < G; ++gi)
        if ((rc1 = update(grp[gi], g, 1, nullptr))) return rc1;
    for (int gi = 1; gi < G; ++gi) {
      QF_HIP(ctx, hipEventRecord(ctx->join[gi], grp[gi].st));
      QF_HIP(ctx, hipStreamWaitEvent(st, ctx->join[gi], 0));
    }
    return QF_OK;
  };

  int rc = build(prec, X);
  if (rc) return rc;
  QF_HIP(ctx, launch_cost(st, prec, X, n, S, costs, trace));
  std::vector<double> c;
  if ((rc = read_costs(ctx, costs, S, c))) return rc;
  if (prec == QF_C64) {
    bool any = false;
    for (int s = 0; s < S; ++s) any = any || (c[s] < o.recheck_below);
    if (any) {
      std::vector<double> c64v = c;
      if ((rc = fp64_costs(c))) return rc;
      ++out.rechecks;
      for (int s = 0; s < S; ++s)
        if (!(c64v[s] < o.recheck_below)) c[s] = c64v[s];
    }
  }
  out.flags.assign(S, 0);
  for (int s = 0; s < S; ++s)
    if (!std::isfinite(c[s])) {
      c[s] = INFINITY;
      out.flags[s] = kFlagNumeric | kFlagPlateau;
    }
  std::vector<std::vector<double>> hist;
  hist.push_back(c);
  auto record = [&](int i, const std::vector<double>& cv) {
    if (stats && stats->cost_history && i < stats->cost_history_rows)
      for (int s = 0; s < S; ++s) stats->cost_history[(size_t)i * S + s] = cv[s];
  };
  record(0, c);
  std::vector<int32_t> frozen_host(S, 0);
  auto sync_frozen = [&]() -> int {
    bool changed = false;
    for (int s = 0; s < S; ++s) {
      const int32_t fz = (out.flags[s] & kFlagNumeric) ? 1 : 0;
      changed = changed || (fz != frozen_host[s]);
      frozen_host[s] = fz;
    }
    if (changed)
      QF_HIP(ctx, hipMemcpyAsync(frozen, frozen_host.data(), (size_t)S * 4, hipMemcpyHostToDevice, st));
    return QF_OK;
  };
  if ((rc = sync_frozen())) return rc;

  int32_t i = 0;
  int32_t decision = o.max_iter <= 0 ? kStopMaxIter : kContinue;
  while (decision == kContinue) {
    ++i;
    // warm-started FP64 updates, cold in the first sweep and every kWarmPeriod-th
    for (int gi = 0; gi < kMaxGroups; ++gi) grp[gi].ea.warm = ((i - 1) % kWarmPeriod) != 0;
    if ((rc = sweep())) return rc;
    if (o.reset_iter > 0 && i % o.reset_iter == 0) {
      if ((rc = build(prec, X))) return rc;
      ++out.resets;
    }
    QF_HIP(ctx, launch_cost(st, prec, X, n, S, costs, trace));
    if ((rc = read_costs(ctx, costs, S, c))) return rc;
    if (prec == QF_C64) {
      bool need = false;
      for (int s = 0; s < S; ++s) need = need || (!(out.flags[s] & kFlagNumeric) && c[s] < o.recheck_below);
      if (need) {
        std::vector<double> c64v = c, c64d;
        if ((rc = fp64_costs(c64d))) return rc;
        ++out.rechecks;
        for (int s = 0; s < S; ++s)
          if (c64v[s] < o.recheck_below) c[s] = c64d[s];
        if ((rc = cast_to_c64(ctx, R, X, (size_t)S * N * N))) return rc;  // refresh the builder
      }
    }
    const int32_t Lh = o.long_diff_count;
    for (int s = 0; s < S; ++s) {
      const double ci = std::isfinite(c[s]) ? c[s] : INFINITY;
      if (out.flags[s] & kFlagNumeric) {
        c[s] = INFINITY;
        continue;
      }
      const double cprev = hist[i - 1][s];
      const double cback = (Lh > 0 && i >= Lh) ? hist[i - Lh][s] : 0.0;
      out.flags[s] = start_flags_after_sweep(o, tol, i, out.flags[s], ci, cprev, cback);
      c[s] = (out.flags[s] & kFlagNumeric) ? INFINITY : ci;
    }
    hist.push_back(c);
    record(i, c);
    if ((rc = sync_frozen())) return rc;
    decision = job_decision(o, i, out.flags.data(), S);
  }
  out.sweeps = i;
  out.decision = decision;
  return fp64_costs(out.final_costs);
}

size_t qf_workspace_size3(int n, int n_gates, int n_starts, const qf_options* opt) {
  qf_options o;
  if (opt)
    o = *opt;
  else
    qf_options_default(&o);
  if (n < 3 || n > 14 || n_gates < 1 || n_starts < 1) return 0;
  if (validate_options(nullptr, o) != QF_OK) return 0;
  return make_layout3(n, n_gates, n_starts, o.precision).total;
}

int qf_instantiate3(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations,
                    const void* init_gates, int n_starts, double tol, const qf_options* opt, void* workspace,
                    size_t ws_bytes, void* out_gates, void* out_all_gates, double* out_costs, qf_stats* stats) {
  if (!ctx) return QF_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  qf_options o;
  if (opt)
    o = *opt;
  else
    qf_options_default(&o);
  if (!(tol > 0) || !std::isfinite(tol)) return fail(ctx, QF_EINVAL, "tol must be finite and > 0");
  o.dist_tol = tol;
  int rc = validate_options(ctx, o);
  if (rc) return rc;
  if ((rc = validate_problem3(ctx, n, n_gates, locations, n_starts, o))) return rc;
  if (!target || !init_gates || !out_gates || !out_costs) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  if (stats && stats->cost_history && stats->cost_history_rows < 0)
    return fail(ctx, QF_EINVAL, "cost_history_rows must be >= 0");
  const Layout3 L = make_layout3(n, n_gates, n_starts, o.precision);
  if (!workspace || ws_bytes < L.total)
    return fail(ctx, QF_EWORKSPACE, "workspace of %zu bytes needed, %zu given", L.total, ws_bytes);
  DeviceGuard dg(ctx->device);
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
  hipStream_t st = ctx->stream;
  const size_t gate_bytes = (size_t)n_starts * n_gates * 1024;
  QF_HIP(ctx, hipMemcpyAsync(ws + L.gates, init_gates, gate_bytes, hipMemcpyDeviceToDevice, st));
  if (stats) {
    stats->pass_launches = stats->env_launches = 0;
    stats->pass_ms = stats->env_ms = stats->sweep_ms = 0.0;
  }
  RunOut out;
  if ((rc = run_streaming3(ctx, n, target, n_gates, locations, n_starts, tol, o, ws, L, stats, out))) return rc;
  int best = 0;
  bool all_numeric = true;
  for (int s = 0; s < n_starts; ++s) {
    double cs = out.final_costs[s];
    if (!std::isfinite(cs) || (out.flags[s] & kFlagNumeric)) cs = INFINITY;
    out.final_costs[s] = cs;
    out_costs[s] = cs;
    all_numeric = all_numeric && !std::isfinite(cs);
    if (cs < out.final_costs[best]) best = s;
  }
  QF_HIP(ctx, hipMemcpyAsync(out_gates, ws + L.gates + (size_t)best * n_gates * 1024, (size_t)n_gates * 1024,
                             hipMemcpyDeviceToDevice, st));
  if (out_all_gates) QF_HIP(ctx, hipMemcpyAsync(out_all_gates, ws + L.gates, gate_bytes, hipMemcpyDeviceToDevice, st));
  QF_HIP(ctx, hipStreamSynchronize(st));
  int status = QF_MAX_ITER;
  if (all_numeric)
    status = QF_NUMERIC;
  else if (out.final_costs[best] < tol)
    status = QF_CONVERGED;
  else if (out.decision == kStopPlateau)
    status = QF_PLATEAU;
  if (stats) {
    stats->sweeps = out.sweeps;
    stats->best_start = best;
    stats->status = status;
    stats->n_resets = out.resets;
    stats->n_rechecks = out.rechecks;
    stats->mode_used = QF_MODE_STREAMING;
    stats->pass_tcols = 0;
    stats->best_cost = out.final_costs[best];
    stats->elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (all_numeric) return fail(ctx, QF_ENUMERIC, "every start produced non-finite values");
  return QF_OK;
}

int qf_optimize_gate3(qf_ctx* ctx, int count, const void* env, const void* u_old, double beta, void* u_new) {
  if (!ctx) return QF_EINVAL;
  if (count < 1) return fail(ctx, QF_EINVAL, "count must be >= 1");
  if (!env || !u_old || !u_new) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  if (!(beta >= 0.0 && beta <= 1.0)) return fail(ctx, QF_EINVAL, "beta must be in [0, 1]");
  DeviceGuard dg(ctx->device);
  QF_HIP(ctx, launch_optimize8(ctx->stream, count, reinterpret_cast<const double*>(env),
                               reinterpret_cast<const double*>(u_old), beta, reinterpret_cast<double*>(u_new)));
  return QF_OK;
}

size_t qf_batch_workspace_size(int n_blocks, const int32_t* block_n, const int32_t* gate_offsets, int n_starts,
                               const qf_options* opt) {
  qf_options o;
  if (opt)
    o = *opt;
  else
    qf_options_default(&o);
  if (validate_options(nullptr, o) != QF_OK) return 0;
  if (n_blocks < 1 || !block_n || !gate_offsets || n_starts < 1 || n_starts > 16) return 0;
  for (int b = 0; b < n_blocks; ++b)
    if (block_n[b] < 2 || block_n[b] > 4 || gate_offsets[b + 1] <= gate_offsets[b]) return 0;
  return make_batch_layout(n_blocks, gate_offsets[n_blocks], n_starts, o).total;
}

namespace {

// Tuner of the batched launch.  Candidates: 8 or 16 hexes per workgroup (at
// least n_starts) and 1 .. the kernel's occupancy limit (at most 4)
// workgroups per CU.  Each runs the first blocks of the processing order (up
// to 2048) for min(max_iter, 3) sweeps on the caller's own data, timed with
// events; the fastest wins.  The trials write the caller's output gates,
// which are then restored from the initial gates; with out_gates ==
// init_gates nothing can be restored, so the default (16 hexes, the
// occupancy limit) is taken untimed.  Every candidate gives bitwise the same
// results.
int tune_batch(qf_ctx* ctx, const BatchArgs& a, int n_blocks, int S, void* out_gates, const void* init_gates,
               size_t gate_bytes) {
  hipStream_t st = ctx->stream;
  int best_slots = 16, best_per = std::min(4, batch_wg_per_cu_max(16));
  if (S > 8 || out_gates == init_gates) {
    ctx->batch_cfg[S][0] = best_slots;
    ctx->batch_cfg[S][1] = best_per;
    return QF_OK;
  }
  BatchArgs t = a;
  t.n_blocks = std::min(n_blocks, 2048);
  t.opt.max_iter = std::max(1, std::min(a.opt.max_iter, 3));
  float best_ms = 0.f;
  bool have = false;
  for (int slots : {16, 8}) {
    const int per_max = std::min(4, batch_wg_per_cu_max(slots));
    for (int per = 1; per <= per_max; ++per) {
      const int grid = batch_grid(slots, per, batch_groups(t.n_blocks, S, slots));
      QF_HIP(ctx, launch_fill_i32(st, t.queue, 0, 1));
      QF_HIP(ctx, hipEventRecord(ctx->tune[0], st));
      QF_HIP(ctx, launch_batch(st, slots, grid, t));
      QF_HIP(ctx, hipEventRecord(ctx->tune[1], st));
      QF_HIP(ctx, hipEventSynchronize(ctx->tune[1]));
      float ms = 0.f;
      QF_HIP(ctx, hipEventElapsedTime(&ms, ctx->tune[0], ctx->tune[1]));
      if (!have || ms < best_ms) {
        have = true;
        best_ms = ms;
        best_slots = slots;
        best_per = per;
      }
    }
  }
  QF_HIP(ctx, hipMemcpyAsync(out_gates, init_gates, gate_bytes, hipMemcpyDeviceToDevice, st));
  ctx->batch_cfg[S][0] = best_slots;
  ctx->batch_cfg[S][1] = best_per;
  return QF_OK;
}

}  // namespace

int qf_set_batch_config(qf_ctx* ctx, int n_starts, int slots, int wg_per_cu) {
  if (!ctx) return QF_EINVAL;
  if (n_starts < 1 || n_starts > 16) return fail(ctx, QF_EINVAL, "n_starts must be in 1..16");
  if (slots == 0) {
    ctx->batch_cfg[n_starts][0] = ctx->batch_cfg[n_starts][1] = 0;
    return QF_OK;
  }
  if ((slots != 8 && slots != 16) || slots < n_starts)
    return fail(ctx, QF_EINVAL, "slots must be 8 or 16 and at least n_starts");
  DeviceGuard dg(ctx->device);
  if (wg_per_cu < 1 || wg_per_cu > batch_wg_per_cu_max(slots))
    return fail(ctx, QF_EINVAL, "wg_per_cu must be in 1..%d for %d slots", batch_wg_per_cu_max(slots), slots);
  ctx->batch_cfg[n_starts][0] = slots;
  ctx->batch_cfg[n_starts][1] = wg_per_cu;
  return QF_OK;
}

int qf_instantiate_batch(qf_ctx* ctx, int n_blocks, const int32_t* block_n, const int32_t* gate_offsets,
                         const int32_t* locations, const void* targets, const void* init_gates, int n_starts,
                         double tol, const qf_options* opt, void* workspace, size_t ws_bytes, void* out_gates,
                         double* out_costs, int32_t* out_best, int32_t* out_status, int32_t* out_sweeps,
                         qf_stats* stats) {
  if (!ctx) return QF_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  qf_options o;
  if (opt)
    o = *opt;
  else
    qf_options_default(&o);
  if (!(tol > 0) || !std::isfinite(tol)) return fail(ctx, QF_EINVAL, "tol must be finite and > 0");
  o.dist_tol = tol;
  int rc = validate_options(ctx, o);
  if (rc) return rc;
  rc = validate_batch(ctx, n_blocks, block_n, gate_offsets, locations, n_starts);
  if (rc) return rc;
  if ((rc = validate_kinds(ctx, o.gate_kinds, gate_offsets[n_blocks]))) return rc;
  if (!targets || !init_gates || !out_gates || !out_costs) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  const int total_gates = gate_offsets[n_blocks];
  const BatchLayout L = make_batch_layout(n_blocks, total_gates, n_starts, o);
  if (!workspace || ws_bytes < L.total)
    return fail(ctx, QF_EWORKSPACE, "workspace of %zu bytes needed, %zu given", L.total, ws_bytes);
  DeviceGuard dg(ctx->device);
  hipStream_t st = ctx->stream;
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);

  // Block descriptors.  Blocks run largest-first (work N^2 * p) so that the
  // queue ends on short problems, and neighbours in a workgroup are alike.
  std::vector<int32_t> order(n_blocks);
  std::vector<int64_t> tgt_off(n_blocks);
  int64_t acc = 0;
  for (int b = 0; b < n_blocks; ++b) {
    order[b] = b;
    tgt_off[b] = acc;
    acc += (int64_t)1 << (2 * block_n[b]);
  }
  auto work = [&](int b) { return ((int64_t)1 << (2 * block_n[b])) * (gate_offsets[b + 1] - gate_offsets[b]); };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  QF_HIP(ctx, hipMemcpyAsync(ws + L.order, order.data(), (size_t)n_blocks * 4, hipMemcpyHostToDevice, st));
  QF_HIP(ctx, hipMemcpyAsync(ws + L.blk_n, block_n, (size_t)n_blocks * 4, hipMemcpyHostToDevice, st));
  QF_HIP(ctx, hipMemcpyAsync(ws + L.gate_off, gate_offsets, (size_t)(n_blocks + 1) * 4, hipMemcpyHostToDevice, st));
  QF_HIP(ctx, hipMemcpyAsync(ws + L.tgt_off, tgt_off.data(), (size_t)n_blocks * 8, hipMemcpyHostToDevice, st));
  QF_HIP(ctx, hipMemcpyAsync(ws + L.locs, locations, (size_t)total_gates * 8, hipMemcpyHostToDevice, st));
  if (o.gate_kinds)
    QF_HIP(ctx, hipMemcpyAsync(ws + L.kinds, o.gate_kinds, (size_t)total_gates * 4, hipMemcpyHostToDevice, st));
  const size_t gate_bytes = (size_t)total_gates * n_starts * 256;
  if (out_gates != init_gates)
    QF_HIP(ctx, hipMemcpyAsync(out_gates, init_gates, gate_bytes, hipMemcpyDeviceToDevice, st));
  int32_t* queue = reinterpret_cast<int32_t*>(ws + L.queue);

  BatchArgs a{};
  a.n_blocks = n_blocks;
  a.S = n_starts;
  a.order = reinterpret_cast<const int32_t*>(ws + L.order);
  a.blk_n = reinterpret_cast<const int32_t*>(ws + L.blk_n);
  a.gate_off = reinterpret_cast<const int32_t*>(ws + L.gate_off);
  a.tgt_off = reinterpret_cast<const int64_t*>(ws + L.tgt_off);
  a.locs = reinterpret_cast<const int32_t*>(ws + L.locs);
  a.V = reinterpret_cast<const double*>(targets);
  a.gates = reinterpret_cast<double*>(out_gates);
  a.tol = tol;
  a.opt = o;
  a.hist = reinterpret_cast<double*>(ws + L.hist);
  a.ring = L.ring;
  a.scratch = reinterpret_cast<double*>(ws + L.scratch);
  a.ywarm = reinterpret_cast<double*>(ws + L.ywarm);
  a.out_cost = reinterpret_cast<double*>(ws + L.cost);
  a.out_best = reinterpret_cast<int32_t*>(ws + L.best);
  a.out_status = reinterpret_cast<int32_t*>(ws + L.status);
  a.out_sweeps = reinterpret_cast<int32_t*>(ws + L.sweeps);
  a.queue = queue;
  a.kinds = o.gate_kinds ? reinterpret_cast<const int32_t*>(ws + L.kinds) : nullptr;
  // Hexes per workgroup and workgroups per CU: tuned once per number of
  // starts on the caller's own first blocks, unless set (qf_set_batch_config).
  if (!ctx->batch_cfg[n_starts][0]) {
    if ((rc = tune_batch(ctx, a, n_blocks, n_starts, out_gates, init_gates, gate_bytes))) return rc;
  }
  const int slots = ctx->batch_cfg[n_starts][0];
  const int grid = batch_grid(slots, ctx->batch_cfg[n_starts][1], batch_groups(n_blocks, n_starts, slots));
  QF_HIP(ctx, launch_fill_i32(st, queue, 0, 1));
  const bool timed = stats && stats->timing;
  hipEvent_t ev[2] = {nullptr, nullptr};
  struct EvFree {
    hipEvent_t* e;
    ~EvFree() {
      for (int k = 0; k < 2; ++k)
        if (e[k]) (void)hipEventDestroy(e[k]);
    }
  } ev_free{ev};
  if (timed) {
    QF_HIP(ctx, hipEventCreate(&ev[0]));
    QF_HIP(ctx, hipEventCreate(&ev[1]));
    QF_HIP(ctx, hipEventRecord(ev[0], st));
  }
  QF_HIP(ctx, launch_batch(st, slots, grid, a));
  if (timed) QF_HIP(ctx, hipEventRecord(ev[1], st));

  std::vector<int32_t> best(n_blocks), status(n_blocks), sweeps(n_blocks);
  QF_HIP(ctx, hipMemcpyAsync(out_costs, ws + L.cost, (size_t)n_blocks * n_starts * 8, hipMemcpyDeviceToHost, st));
  QF_HIP(ctx, hipMemcpyAsync(best.data(), ws + L.best, (size_t)n_blocks * 4, hipMemcpyDeviceToHost, st));
  QF_HIP(ctx, hipMemcpyAsync(status.data(), ws + L.status, (size_t)n_blocks * 4, hipMemcpyDeviceToHost, st));
  QF_HIP(ctx, hipMemcpyAsync(sweeps.data(), ws + L.sweeps, (size_t)n_blocks * 4, hipMemcpyDeviceToHost, st));
  QF_HIP(ctx, hipStreamSynchronize(st));
  if (out_best) std::memcpy(out_best, best.data(), (size_t)n_blocks * 4);
  if (out_status) std::memcpy(out_status, status.data(), (size_t)n_blocks * 4);
  if (out_sweeps) std::memcpy(out_sweeps, sweeps.data(), (size_t)n_blocks * 4);
  if (stats) {
    int max_sweeps = 0, worst = QF_CONVERGED;
    double worst_cost = 0.0;
    for (int b = 0; b < n_blocks; ++b) {
      max_sweeps = std::max(max_sweeps, sweeps[b]);
      worst = std::max(worst, status[b]);
      worst_cost = std::max(worst_cost, out_costs[(size_t)b * n_starts + best[b]]);
    }
    stats->sweeps = max_sweeps;
    stats->best_start = 0;
    stats->status = worst;
    stats->n_resets = o.reset_iter > 0 ? max_sweeps / o.reset_iter : 0;
    stats->n_rechecks = 0;
    stats->mode_used = QF_MODE_RESIDENT;
    stats->best_cost = worst_cost;
    stats->pass_launches = stats->env_launches = 0;
    stats->pass_ms = stats->env_ms = 0.0;
    float kms = 0.0f;
    if (timed) QF_HIP(ctx, hipEventElapsedTime(&kms, ev[0], ev[1]));
    stats->sweep_ms = kms;
    stats->pass_tcols = 0;
    stats->batch_slots = slots;
    stats->batch_wg_per_cu = ctx->batch_cfg[n_starts][1];
    stats->elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return QF_OK;
}

size_t qf_gradient_workspace_size(int n, int n_gates, int n_starts, int precision) {
  if (n < 2 || n > 16 || n_gates < 1 || n_starts < 1) return 0;
  if (precision != QF_C128 && precision != QF_C64) return 0;
  return make_grad_layout(n, n_gates, n_starts, precision).total;
}

int qf_gradient(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations, const void* gates,
                int n_starts, int precision, void* workspace, size_t ws_bytes, double* cost_out, void* grad_out) {
  if (!ctx) return QF_EINVAL;
  int rc = validate_problem(ctx, n, n_gates, locations, n_starts);
  if (rc) return rc;
  if (precision != QF_C128 && precision != QF_C64) return fail(ctx, QF_EINVAL, "unknown precision");
  if (!target || !gates || !cost_out || !grad_out) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  const GradLayout L = make_grad_layout(n, n_gates, n_starts, precision);
  if (!workspace || ws_bytes < L.total)
    return fail(ctx, QF_EWORKSPACE, "workspace of %zu bytes needed, %zu given", L.total, ws_bytes);
  DeviceGuard dg(ctx->device);
  return run_gradient(ctx, n, target, n_gates, locations, reinterpret_cast<const double*>(gates), n_starts,
                      precision, reinterpret_cast<unsigned char*>(workspace), L, cost_out,
                      reinterpret_cast<double*>(grad_out));
}

int qf_su4_gates(qf_ctx* ctx, int count, const double* theta, void* gates) {
  if (!ctx) return QF_EINVAL;
  if (count < 1) return fail(ctx, QF_EINVAL, "count must be >= 1");
  if (!theta || !gates) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  DeviceGuard dg(ctx->device);
  QF_HIP(ctx, launch_su4_expm(ctx->stream, theta, count, reinterpret_cast<double*>(gates)));
  return QF_OK;
}

int qf_su4_vjp(qf_ctx* ctx, int count, const double* theta, const void* grad_gates, double* dtheta) {
  if (!ctx) return QF_EINVAL;
  if (count < 1) return fail(ctx, QF_EINVAL, "count must be >= 1");
  if (!theta || !grad_gates || !dtheta) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  DeviceGuard dg(ctx->device);
  QF_HIP(ctx, launch_su4_vjp(ctx->stream, theta, reinterpret_cast<const double*>(grad_gates), count, dtheta));
  return QF_OK;
}

void qf_lbfgs_options_default(qf_lbfgs_options* o) {
  if (!o) return;
  o->history = 10;
  o->max_iter = 1000;
  o->max_ls = 30;
  o->c1 = 1e-4;
  o->grad_tol = 1e-12;
  o->ftol_r = 1e-12;
  o->precision = QF_C128;
}

size_t qf_lbfgs_workspace_size(int n, int n_gates, int n_starts, const qf_lbfgs_options* opt) {
  qf_lbfgs_options o;
  if (opt)
    o = *opt;
  else
    qf_lbfgs_options_default(&o);
  if (n < 2 || n > 16 || n_gates < 1 || n_starts < 1) return 0;
  if (o.precision != QF_C128 && o.precision != QF_C64) return 0;
  return make_lbfgs_layout(n, n_gates, n_starts, o.precision).total;
}

int qf_lbfgs(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations, const double* theta0,
             int n_starts, double tol, const qf_lbfgs_options* opt, void* workspace, size_t ws_bytes,
             double* theta_out, double* out_costs, qf_lbfgs_result* stats) {
  if (!ctx) return QF_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  qf_lbfgs_options o;
  if (opt)
    o = *opt;
  else
    qf_lbfgs_options_default(&o);
  const int p = n_gates, S = n_starts;
  int rc = validate_problem(ctx, n, p, locations, S);
  if (rc) return rc;
  if (!(tol > 0) || !std::isfinite(tol)) return fail(ctx, QF_EINVAL, "tol must be finite and > 0");
  if (o.history < 1 || o.history > 1000) return fail(ctx, QF_EINVAL, "history must be in [1, 1000]");
  if (o.max_iter < 0 || o.max_ls < 1) return fail(ctx, QF_EINVAL, "max_iter must be >= 0 and max_ls >= 1");
  if (!(o.c1 > 0 && o.c1 < 1)) return fail(ctx, QF_EINVAL, "c1 must be in (0, 1)");
  if (!(o.grad_tol >= 0) || !(o.ftol_r >= 0)) return fail(ctx, QF_EINVAL, "grad_tol and ftol_r must be >= 0");
  if (o.precision != QF_C128 && o.precision != QF_C64) return fail(ctx, QF_EINVAL, "unknown precision");
  if (!target || !theta0 || !theta_out || !out_costs) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  if (stats && stats->cost_history && stats->cost_history_rows < 0)
    return fail(ctx, QF_EINVAL, "cost_history_rows must be >= 0");
  const LbfgsLayout L = make_lbfgs_layout(n, p, S, o.precision);
  if (!workspace || ws_bytes < L.total)
    return fail(ctx, QF_EWORKSPACE, "workspace of %zu bytes needed, %zu given", L.total, ws_bytes);
  DeviceGuard dg(ctx->device);
  hipStream_t st = ctx->stream;
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
  double* d_gates = reinterpret_cast<double*>(ws + L.gates);
  double* d_ggrad = reinterpret_cast<double*>(ws + L.ggrad);
  double* d_theta = reinterpret_cast<double*>(ws + L.theta);
  double* d_dtheta = reinterpret_cast<double*>(ws + L.dtheta);
  double* d_costs = reinterpret_cast<double*>(ws + L.costs);
  const size_t D = (size_t)p * 15;  // parameters per start
  const size_t nd = D * S;
  int evals = 0;

  // f and grad of every start at the parameters in d_theta (host copies out)
  std::vector<double> hf(S), hg(nd);
  auto evaluate = [&](const std::vector<double>& x) -> int {
    QF_HIP(ctx, hipMemcpyAsync(d_theta, x.data(), nd * 8, hipMemcpyHostToDevice, st));
    QF_HIP(ctx, launch_su4_expm(st, d_theta, S * p, d_gates));
    int r2 = run_gradient(ctx, n, target, p, locations, d_gates, S, o.precision, ws, L.G, d_costs, d_ggrad);
    if (r2) return r2;
    QF_HIP(ctx, launch_su4_vjp(st, d_theta, d_ggrad, S * p, d_dtheta));
    QF_HIP(ctx, hipMemcpyAsync(hf.data(), d_costs, (size_t)S * 8, hipMemcpyDeviceToHost, st));
    QF_HIP(ctx, hipMemcpyAsync(hg.data(), d_dtheta, nd * 8, hipMemcpyDeviceToHost, st));
    QF_HIP(ctx, hipStreamSynchronize(st));
    ++evals;
    return QF_OK;
  };
  auto dot = [&](const double* a, const double* b) {
    double acc = 0.0;
    for (size_t k = 0; k < D; ++k) acc += a[k] * b[k];
    return acc;
  };

  std::vector<double> x(nd), g(nd), xt(nd), d(nd);
  QF_HIP(ctx, hipMemcpyAsync(x.data(), theta0, nd * 8, hipMemcpyDeviceToHost, st));
  QF_HIP(ctx, hipStreamSynchronize(st));
  if ((rc = evaluate(x))) return rc;
  std::vector<double> f = hf;
  g = hg;
  for (int s = 0; s < S; ++s)
    if (!std::isfinite(f[s])) f[s] = INFINITY;
  // Per-start history (ring of s = x_{k+1} - x_k, y = g_{k+1} - g_k, rho).
  const int m = o.history;
  std::vector<std::vector<double>> sh(S, std::vector<double>((size_t)m * D)), yh(S, std::vector<double>((size_t)m * D));
  std::vector<std::vector<double>> rho(S, std::vector<double>(m, 0.0));
  std::vector<int> cnt(S, 0), head(S, 0);
  std::vector<char> active(S, 1);
  auto record = [&](int row) {
    if (stats && stats->cost_history && row < stats->cost_history_rows)
      for (int s = 0; s < S; ++s) stats->cost_history[(size_t)row * S + s] = f[s];
  };
  record(0);
  for (int s = 0; s < S; ++s) active[s] = std::isfinite(f[s]) ? 1 : 0;
  int it = 0, status = QF_MAX_ITER;
  std::vector<double> alpha(S), gd(S), fnew(S);
  std::vector<char> done_ls(S);
  auto any_converged = [&]() {
    for (int s = 0; s < S; ++s)
      if (f[s] < tol) return true;
    return false;
  };
  if (any_converged()) status = QF_CONVERGED;
  while (status == QF_MAX_ITER && it < o.max_iter) {
    bool any_active = false;
    for (int s = 0; s < S; ++s) any_active = any_active || active[s];
    if (!any_active) {
      status = QF_PLATEAU;
      break;
    }
    ++it;
    // two-loop recursion: d = -H g
    for (int s = 0; s < S; ++s) {
      double* ds = d.data() + s * D;
      const double* gs = g.data() + s * D;
      if (!active[s]) {
        std::fill(ds, ds + D, 0.0);
        continue;
      }
      for (size_t k = 0; k < D; ++k) ds[k] = -gs[k];
      std::vector<double> a(cnt[s]);
      for (int j = 0; j < cnt[s]; ++j) {
        const int slot = (head[s] - 1 - j + m) % m;
        a[j] = rho[s][slot] * dot(&sh[s][(size_t)slot * D], ds);
        const double* yv = &yh[s][(size_t)slot * D];
        for (size_t k = 0; k < D; ++k) ds[k] -= a[j] * yv[k];
      }
      if (cnt[s] > 0) {
        const int last = (head[s] - 1 + m) % m;
        const double* yv = &yh[s][(size_t)last * D];
        const double gamma = 1.0 / (rho[s][last] * dot(yv, yv));
        for (size_t k = 0; k < D; ++k) ds[k] *= gamma;
      }
      for (int j = cnt[s] - 1; j >= 0; --j) {
        const int slot = (head[s] - 1 - j + m) % m;
        const double b = rho[s][slot] * dot(&yh[s][(size_t)slot * D], ds);
        const double* sv = &sh[s][(size_t)slot * D];
        for (size_t k = 0; k < D; ++k) ds[k] += (a[j] - b) * sv[k];
      }
      gd[s] = dot(gs, ds);
      if (!(gd[s] < 0.0)) {  // not a descent direction: restart from steepest descent
        cnt[s] = head[s] = 0;
        for (size_t k = 0; k < D; ++k) ds[k] = -gs[k];
        gd[s] = dot(gs, ds);
      }
      double gn = 0.0;
      for (size_t k = 0; k < D; ++k) gn = std::max(gn, std::fabs(gs[k]));
      alpha[s] = (cnt[s] == 0) ? std::min(1.0, 1.0 / std::max(gn, 1e-300)) : 1.0;
      done_ls[s] = 0;
    }
    // backtracking line search, all starts in lockstep
    std::vector<double> gnew(nd);
    std::vector<double> xnew = x;
    for (int s = 0; s < S; ++s) done_ls[s] = active[s] ? 0 : 1;
    for (int ls = 0; ls < o.max_ls; ++ls) {
      bool pending = false;
      for (int s = 0; s < S; ++s) {
        if (done_ls[s]) continue;
        pending = true;
        for (size_t k = 0; k < D; ++k) xt[s * D + k] = x[s * D + k] + alpha[s] * d[s * D + k];
      }
      if (!pending) break;
      for (int s = 0; s < S; ++s)
        if (done_ls[s])
          for (size_t k = 0; k < D; ++k) xt[s * D + k] = xnew[s * D + k];
      if ((rc = evaluate(xt))) return rc;
      for (int s = 0; s < S; ++s) {
        if (done_ls[s]) continue;
        const double ft = std::isfinite(hf[s]) ? hf[s] : INFINITY;
        if (ft <= f[s] + o.c1 * alpha[s] * gd[s]) {
          done_ls[s] = 2;  // accepted
          fnew[s] = ft;
          std::copy(xt.begin() + s * D, xt.begin() + (s + 1) * D, xnew.begin() + s * D);
          std::copy(hg.begin() + s * D, hg.begin() + (s + 1) * D, gnew.begin() + s * D);
        } else {
          alpha[s] *= 0.5;
        }
      }
    }
    for (int s = 0; s < S; ++s) {
      if (!active[s]) continue;
      if (done_ls[s] != 2) {  // no sufficient decrease: this start stops
        active[s] = 0;
        continue;
      }
      double sy = 0.0, yy = 0.0, gmax = 0.0;
      const int slot = head[s];
      double* sv = &sh[s][(size_t)slot * D];
      double* yv = &yh[s][(size_t)slot * D];
      for (size_t k = 0; k < D; ++k) {
        sv[k] = xnew[s * D + k] - x[s * D + k];
        yv[k] = gnew[s * D + k] - g[s * D + k];
        sy += sv[k] * yv[k];
        yy += yv[k] * yv[k];
        gmax = std::max(gmax, std::fabs(gnew[s * D + k]));
      }
      if (sy > 1e-300 && yy > 0.0) {  // keep the pair only with positive curvature
        rho[s][slot] = 1.0 / sy;
        head[s] = (head[s] + 1) % m;
        cnt[s] = std::min(cnt[s] + 1, m);
      }
      const double fprev = f[s];
      f[s] = fnew[s];
      std::copy(xnew.begin() + s * D, xnew.begin() + (s + 1) * D, x.begin() + s * D);
      std::copy(gnew.begin() + s * D, gnew.begin() + (s + 1) * D, g.begin() + s * D);
      if (gmax < o.grad_tol || fprev - f[s] <= o.ftol_r * f[s]) active[s] = 0;
    }
    record(it);
    if (any_converged()) status = QF_CONVERGED;
  }
  int best = 0;
  for (int s = 0; s < S; ++s) {
    out_costs[s] = f[s];
    if (f[s] < f[best]) best = s;
  }
  QF_HIP(ctx, hipMemcpyAsync(theta_out, x.data(), nd * 8, hipMemcpyHostToDevice, st));
  QF_HIP(ctx, hipStreamSynchronize(st));
  if (status != QF_CONVERGED && f[best] < tol) status = QF_CONVERGED;
  if (stats) {
    stats->iterations = it;
    stats->evaluations = evals;
    stats->best_start = best;
    stats->status = status;
    stats->best_cost = f[best];
    stats->elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return QF_OK;
}

size_t qf_delete_gates_workspace_size(int n, int n_gates, int n_starts, const qf_options* opt) {
  const size_t inner = qf_workspace_size(n, n_gates, n_starts, opt);
  if (!inner) return 0;
  const size_t g = align_up((size_t)n_gates * 256);
  return align_up(inner) + 2 * g + 2 * align_up((size_t)n_starts * n_gates * 256) + align_up((size_t)n_gates * 4);
}

int qf_delete_gates(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations,
                    const void* gates, const void* pool, int n_starts, double tol, const qf_options* opt,
                    void* workspace, size_t ws_bytes, int32_t* keep, void* out_gates, double* out_cost,
                    qf_delete_result* result) {
  if (!ctx) return QF_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  const int p = n_gates, S = n_starts;
  int rc = validate_problem(ctx, n, p, locations, S);
  if (rc) return rc;
  if (!(tol > 0) || !std::isfinite(tol)) return fail(ctx, QF_EINVAL, "tol must be finite and > 0");
  if (!target || !gates || !pool || !keep || !out_gates || !out_cost) return fail(ctx, QF_EINVAL, "NULL pointer argument");
  qf_options o;
  if (opt)
    o = *opt;
  else
    qf_options_default(&o);
  if ((rc = validate_options(ctx, o))) return rc;
  if ((rc = validate_kinds(ctx, o.gate_kinds, p))) return rc;
  const size_t need = qf_delete_gates_workspace_size(n, p, S, &o);
  if (!workspace || ws_bytes < need)
    return fail(ctx, QF_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  DeviceGuard dg(ctx->device);
  hipStream_t st = ctx->stream;
  unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
  const size_t inner = align_up(qf_workspace_size(n, p, S, &o));
  const size_t gsz = align_up((size_t)p * 256), psz = align_up((size_t)S * p * 256);
  double2* cur = reinterpret_cast<double2*>(ws + inner);            // current circuit (compacted)
  double2* best = reinterpret_cast<double2*>(ws + inner + gsz);     // attempt result
  double2* init = reinterpret_cast<double2*>(ws + inner + 2 * gsz);  // attempt initial gates
  double2* all = reinterpret_cast<double2*>(ws + inner + 2 * gsz + psz);
  int32_t* d_idx = reinterpret_cast<int32_t*>(ws + inner + 2 * gsz + 2 * psz);

  // the given circuit must realise the target
  std::vector<double> c0(1);
  {
    qf_options o1 = o;
    o1.max_iter = 0;
    QF_HIP(ctx, hipMemcpyAsync(cur, gates, (size_t)p * 256, hipMemcpyDeviceToDevice, st));
    rc = qf_instantiate(ctx, n, target, p, locations, cur, 1, tol, &o1, ws, inner, best, nullptr, c0.data(), nullptr);
    if (rc) return rc;
    if (!(c0[0] < tol)) return fail(ctx, QF_EINVAL, "the given gates do not realise the target (cost %.3g)", c0[0]);
  }
  std::vector<int> kept;  // original indices of the gates of the current circuit
  for (int g = 0; g < p; ++g) kept.push_back(g);
  double cost_now = c0[0];
  int attempts = 0, deleted = 0, sweeps = 0;
  std::vector<int32_t> idx, sub_locs;
  for (int g = 0; g < p; ++g) {
    if (kept.size() <= 1) break;  // an empty circuit is not instantiated
    const int pos = (int)(std::find(kept.begin(), kept.end(), g) - kept.begin());
    const int q = (int)kept.size() - 1;
    idx.clear();
    sub_locs.clear();
    std::vector<int32_t> idx_cur;  // positions in the current (compacted) circuit
    for (int k = 0; k < (int)kept.size(); ++k) {
      if (k == pos) continue;
      idx.push_back(kept[k]);
      idx_cur.push_back(k);
      sub_locs.push_back(locations[2 * kept[k]]);
      sub_locs.push_back(locations[2 * kept[k] + 1]);
    }
    // start 0: the current circuit without gate g; starts 1..: the pool at the gates still present
    QF_HIP(ctx, hipMemcpyAsync(d_idx, idx.data(), (size_t)q * 4, hipMemcpyHostToDevice, st));
    {
      const int64_t tot = (int64_t)S * q * 16;
      hipLaunchKernelGGL(k_gather_gates, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                         reinterpret_cast<const double2*>(pool), (const double2*)nullptr, S, p, d_idx, q, all);
      QF_HIP(ctx, hipGetLastError());
      QF_HIP(ctx, hipMemcpyAsync(d_idx, idx_cur.data(), (size_t)q * 4, hipMemcpyHostToDevice, st));
      const int64_t tot0 = (int64_t)q * 16;
      hipLaunchKernelGGL(k_gather_gates, dim3((unsigned)((tot0 + 255) / 256)), dim3(256), 0, st,
                         reinterpret_cast<const double2*>(cur), (const double2*)nullptr, 1, (int)kept.size(), d_idx, q,
                         init);
      QF_HIP(ctx, hipGetLastError());
      QF_HIP(ctx, hipMemcpyAsync(all, init, (size_t)q * 256, hipMemcpyDeviceToDevice, st));
    }
    std::vector<double> costs(S);
    qf_stats ist{};
    qf_options oa = o;
    std::vector<int32_t> sub_kinds;
    if (o.gate_kinds) {
      for (int k : idx) sub_kinds.push_back(o.gate_kinds[k]);
      oa.gate_kinds = sub_kinds.data();
    }
    rc = qf_instantiate(ctx, n, target, q, sub_locs.data(), all, S, tol, &oa, ws, inner, best, nullptr, costs.data(),
                        &ist);
    if (rc && rc != QF_ENUMERIC) return rc;
    ++attempts;
    sweeps += ist.sweeps;
    if (rc == QF_OK && ist.best_cost < tol) {
      QF_HIP(ctx, hipMemcpyAsync(cur, best, (size_t)q * 256, hipMemcpyDeviceToDevice, st));
      kept.erase(kept.begin() + pos);
      cost_now = ist.best_cost;
      ++deleted;
    }
  }
  for (int g = 0; g < p; ++g) keep[g] = 0;
  for (int k : kept) keep[k] = 1;
  QF_HIP(ctx, hipMemcpyAsync(out_gates, cur, kept.size() * 256, hipMemcpyDeviceToDevice, st));
  QF_HIP(ctx, hipStreamSynchronize(st));
  *out_cost = cost_now;
  if (result) {
    result->attempts = attempts;
    result->deleted = deleted;
    result->sweeps = sweeps;
    result->elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return QF_OK;
}

}  // extern "C"
