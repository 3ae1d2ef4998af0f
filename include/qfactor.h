/*
 * qfactor.h -- C ABI of the MI355X (gfx950) QFactor instantiation library.
 *
 * QFactor (arXiv 2306.08152) instantiates a circuit of p general two-qubit
 * gates u_1..u_p to an n-qubit target unitary V (N = 2^n) by maximising
 * |Tr(V^dagger C)|, C = G_p ... G_1 (Sec. II, problem statement).  It keeps
 * the "circuit tensor" (here: the builder) X with Tr(X) = Tr(V^dagger C),
 * peels one gate off X, partial-traces the rest into a 4x4 environment E,
 * replaces the gate by the unitary that maximises Re Tr(E u) (SVD
 * E = X D Y^dagger -> u = Y X^dagger, Sec. III-A-1) and re-applies it on the
 * other side, sweeping p..1 and then 1..p (TwoSidedSweep of Alg. 1) until the
 * cost Delta = 1 - |Tr(V^dagger C)|/N meets a termination test (Sec. III-A-2).
 *
 * Conventions (every entry point):
 *   - complex data is interleaved (re, im); "c128" = two doubles, "c64" = two
 *     floats; matrices are row-major.
 *   - qubit 0 is the most significant bit of a row/column index; a gate on
 *     loc = (a, b) has local index 2*bit(a) + bit(b).
 *   - gates are listed in time order; C = G_p ... G_1.
 *   - the builder of one problem is an N x N matrix; a batch of S builders is
 *     S contiguous N x N matrices (start-major).  Its element type is c128
 *     (QF_C128) or c64 (QF_C64).
 *   - pointers documented as "device" must be device memory of the context's
 *     device; "host" pointers are ordinary host memory.  The caller owns
 *     every buffer; the library keeps no pointer after a call returns.
 *   - all device work is enqueued on the context's stream.  qf_instantiate
 *     returns when its outputs are final; the other calls are
 *     stream-ordered and asynchronous (synchronise the stream before reading
 *     their outputs on the host).
 *   - every call returns a qf_status; invalid arguments are rejected with
 *     QF_EINVAL before any device work is enqueued; no call throws across
 *     the ABI.  qf_last_error() gives a message for the last failure on a
 *     context.
 */
#ifndef QFACTOR_MI355X_H
#define QFACTOR_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qf_ctx qf_ctx;

typedef enum {
  QF_OK = 0,
  QF_EINVAL = -1,        /* invalid argument (checked on the host) */
  QF_EUNSUPPORTED = -2,  /* valid request that this library does not implement */
  QF_EHIP = -3,          /* HIP runtime error */
  QF_EWORKSPACE = -4,    /* workspace missing or smaller than qf_workspace_size */
  QF_ENUMERIC = -5,      /* every start produced non-finite values */
  QF_ETIMEOUT = -6       /* a bounded device-side wait gave up */
} qf_status;

typedef enum {
  QF_C128 = 0,  /* builder in complex128; everything in FP64 */
  QF_C64 = 1    /* builder in complex64; environment sums, SVD/polar step,
                   termination tests and the final cost in FP64 */
} qf_precision;

typedef enum {
  QF_MODE_AUTO = 0,       /* resident for n <= 6, streaming otherwise */
  QF_MODE_RESIDENT = 1,   /* one workgroup per start, builder in LDS (n <= 6) */
  QF_MODE_STREAMING = 2   /* builders in HBM, one fused pass per gate update */
} qf_mode;

typedef enum { QF_LEFT = 0, QF_RIGHT = 1 } qf_side;

/* Gate kinds (Sec. III-A-3, Specializing Gate Sets; the evaluation's U3 +
 * CNOT gate set).  Every gate is passed as a 4 x 4 matrix on its two
 * locations.  Single-qubit kinds act on location 0 and must be given as
 * g (x) I_2 (location 1 is only a partner qubit for the embedding); their
 * update maximises Re Tr(E2 g) over the kind's set, E2 being the partial
 * trace of the environment over the partner:
 *   QF_KIND_U4    general U(4) (SVD update, Sec. III-A-1)
 *   QF_KIND_FIXED applied, never optimised (e.g. CNOT)
 *   QF_KIND_U2    general U(2) (unitary polar factor, closed form for 2 x 2)
 *   QF_KIND_RZ    diag(1, e^{it}), t = -arg M2[1][1]
 *   QF_KIND_GPI   [[0, e^{-if}], [e^{if}, 0]], f = -arg(M2[0][1] + conj M2[1][0])
 *   QF_KIND_MS    two-qubit Molmer-Sorensen MS(f1, f2) = exp(-i pi/4
 *                 sigma_f1 (x) sigma_f2) on both locations: e^{i(f1+f2)} =
 *                 conj(w_s)/|w_s|, e^{i(f1-f2)} = conj(w_d)/|w_d| with
 *                 w_s = -i M[0][3] + i conj M[3][0], w_d = -i M[1][2] +
 *                 i conj M[2][1], M = (1-beta) E + beta u_old^dagger
 * (M2 = (1-beta) E2 + beta g_old^dagger; a zero argument keeps the gate.) */
typedef enum {
  QF_KIND_U4 = 0, QF_KIND_FIXED = 1, QF_KIND_U2 = 2, QF_KIND_RZ = 3, QF_KIND_GPI = 4, QF_KIND_MS = 5
} qf_gate_kind;

typedef enum {
  QF_CONVERGED = 0,  /* best start's final cost < tol */
  QF_PLATEAU = 1,    /* every start met a plateau test */
  QF_MAX_ITER = 2,   /* max_iter sweeps done */
  QF_NUMERIC = 3     /* every start produced non-finite values */
} qf_result_status;

/* Hyperparameters of Sec. III-A-2.  qf_options_default() sets the values the
 * paper recommends: dist_tol 1e-10, diff_tol_a 0, diff_tol_r 1e-5,
 * long_diff_count 100, long_diff_r 0.1, min_iter 0, max_iter 1e5,
 * reset_iter 40, beta 0; plus precision QF_C128, mode QF_MODE_AUTO,
 * recheck_below 1e-3, stream_groups 0 (automatic), gate_kinds NULL and
 * gate_pairs 1.
 * Readings of the garbled tests (c_i = cost after sweep i, c_0 = initial):
 *   short plateau: c_{i-1} - c_i <= diff_tol_a + diff_tol_r * c_i
 *                  (off when both are 0);
 *   long plateau:  c_{i-L} - c_i < long_diff_r * c_{i-L}, L = long_diff_count
 *                  (off when L <= 0);
 *   stop when any start has cost < tol, or every start has met a plateau
 *   test at some sweep, or after max_iter sweeps; no test before min_iter.
 * reset_iter: rebuild the builder from the gates after every reset_iter-th
 * sweep (0 = never).  beta: the SVD acts on (1-beta) E + beta u_old^dagger.
 * recheck_below (QF_C64 only): once a start's complex64 cost estimate drops
 * below this value, its cost is re-evaluated in FP64 from a freshly built
 * complex128 builder (which also refreshes the complex64 one), and the FP64
 * value is the one the tests see.  The complex64 estimate drifts by up to
 * ~1e-6 between rebuilds, so below ~1e-3 the per-sweep progress of a slowly
 * converging start is no longer resolved and the plateau test would fire on
 * rounding noise; the default keeps the tests on FP64 values from there. */
typedef struct {
  double dist_tol;
  double diff_tol_a;
  double diff_tol_r;
  int32_t long_diff_count;
  double long_diff_r;
  int32_t min_iter;
  int32_t max_iter;
  int32_t reset_iter;
  double beta;
  int32_t precision;  /* qf_precision */
  int32_t mode;       /* qf_mode */
  double recheck_below;
  int32_t stream_groups; /* streaming mode: how the environment + SVD step
                            of some starts runs under the pass of others.
                            0 = automatic: with two-gate updates (see
                            gate_pairs) three groups on separate streams
                            (the caller's and two of the library's),
                            staggered; with one pass per update four groups
                            in two pairs, each pair on one stream, every
                            launch carrying one group's environment step
                            beside the other group's pass (two groups on
                            the caller's stream for 2-3 starts; one group
                            for one start or n >= 15).  1..4 = that many
                            groups on separate streams (group 0 on the
                            caller's), staggered; at most n_starts groups.
                            Every choice gives bitwise the same results */
  const int32_t* gate_kinds; /* host, one qf_gate_kind per gate (for
                                qf_instantiate_batch: per gate of the whole
                                batch); NULL = every gate QF_KIND_U4 */
  int32_t gate_pairs;        /* streaming mode: 1 (default) runs two
                                consecutive gate updates of a sweep with one
                                partial trace and one builder pass when the
                                builder is QF_C64, the two gates span 3 or 4
                                qubits and neither is QF_KIND_FIXED (each
                                update still sees its own environment;
                                results agree with one pass per update up to
                                rounding); 2 = the same for QF_C128 builders
                                too; 0 = one pass per update */
} qf_options;

/* Outcome of qf_instantiate (host memory). */
typedef struct {
  int32_t sweeps;        /* sweeps run (lockstep over starts) */
  int32_t best_start;    /* start with the smallest final cost, lowest index on ties */
  int32_t status;        /* qf_result_status */
  int32_t n_resets;      /* builder rebuilds triggered by reset_iter */
  int32_t n_rechecks;    /* FP64 re-evaluations (QF_C64) */
  int32_t mode_used;     /* qf_mode actually run */
  double best_cost;      /* FP64 cost of the best start's returned gates */
  double elapsed_ms;     /* wall time from first launch to final outputs */
  double* cost_history;  /* in, optional (host): rows x n_starts doubles;
                            row i receives the costs after sweep i (row 0 =
                            initial gates) for i < cost_history_rows */
  int32_t cost_history_rows;
  int32_t timing;        /* in: nonzero times every pass and environment
                            kernel of the streaming sweep loop with a HIP
                            start / stop event pair that its dispatch
                            stamps (the kernel's execution); the starts
                            then run as one group (no overlap of two
                            groups' kernels), so each duration is the
                            kernel's own */
  int32_t pass_launches; /* out (timing): fused builder passes in the sweeps */
  int32_t env_launches;  /* out (timing): environment + SVD-step launches */
  double pass_ms;        /* out (timing): summed durations of those passes */
  double env_ms;         /* out (timing): summed durations of those launches */
  double sweep_ms;       /* out (timing): device time of the sweep loop */
  int32_t pass_tcols;    /* out: form of the fused pass at a mid-circuit gate:
                            tile width (columns) of the LDS-staged pass, or -1
                            for the register-direct pass; chosen on first use
                            per (precision, gate class, n) by timing the
                            candidates on the caller's builder */
  int32_t pass2_launches; /* out (timing): the two-gate passes among
                             pass_launches */
  double pass2_ms;        /* out (timing): their summed durations */
  int32_t batch_slots;    /* out (qf_instantiate_batch): instantiations per
                             workgroup of the batched launch (8 or 16) */
  int32_t batch_wg_per_cu; /* out (qf_instantiate_batch): its workgroups per
                              compute unit */
} qf_stats;

/* Create a context on `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL = the device's null stream).  This is the only call that allocates:
 * 32 KiB of pinned host memory for per-sweep cost read-back, a device
 * scratch of about 2.3 MiB for the stand-alone step calls (qf_environment,
 * qf_update_gate: environment partial sums, arrival counters and u_old; they
 * process their builders in chunks so the scratch never grows), a 4 x 4
 * identity operand, and the library's three auxiliary streams (default
 * priority) and events.  qf_instantiate and the other drivers work in the
 * caller's workspace.  qf_destroy frees everything.  A context may be used
 * by one host thread at a time. */
int qf_create(qf_ctx** ctx, int device, void* hip_stream);
int qf_destroy(qf_ctx* ctx);
int qf_set_stream(qf_ctx* ctx, void* hip_stream);
const char* qf_strerror(int status);
const char* qf_last_error(const qf_ctx* ctx);
void qf_options_default(qf_options* opt);

/* Bytes of device workspace qf_instantiate needs for this problem size
 * (0 on invalid sizes).  opt may be NULL (defaults). */
size_t qf_workspace_size(int n, int n_gates, int n_starts, const qf_options* opt);

/* InitCircuitTensor (Alg. 1): builder[s] = G_p ... G_1 V^dagger for every
 * start s, i.e. the target's conjugate transpose followed by every gate
 * applied on the output legs.  target: device N x N c128.  gates: device
 * n_starts x n_gates x 4 x 4 c128.  locations: host n_gates x 2 int32, two
 * distinct qubits in [0, n).  builder: device n_starts x N x N in
 * `precision`.  2 <= n <= 16. */
int qf_build(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations,
             const void* gates, int n_starts, int precision, void* builder);

/* ApplyRight / ApplyLeft of Alg. 1 on a batch of builders: with G = g on loc
 * (identity elsewhere), side QF_LEFT does X <- G X (output legs, "ApplyRight")
 * and QF_RIGHT does X <- X G (input legs, "ApplyLeft"); dagger != 0 applies
 * G^dagger (the inverse, which removes the gate).  gates: device
 * n_builders x 4 x 4 c128, one gate per builder (rounded to the builder's
 * precision).  loc: host int32[2]. */
int qf_apply_gate(qf_ctx* ctx, int n, int n_builders, void* builder, int precision,
                  const int32_t* loc, const void* gates, int side, int dagger);

/* CalcEnvMat of Alg. 1 (Sec. III, Fig. tensors): env[s][i][j] =
 * sum over the other qubits of X_s[(i, rest), (j, rest)], so that
 * Tr((u (x) I) X_s) = Tr(env_s u) for every 4x4 u.  Summed in FP64.
 * env_out: device n_builders x 4 x 4 c128. */
int qf_environment(qf_ctx* ctx, int n, int n_builders, const void* builder, int precision,
                   const int32_t* loc, void* env_out);

/* OptimizeGate for general unitaries (Sec. III-A-1, Eq. opt_u, with beta of
 * Sec. III-A-2): for each of `count` environments E, M = (1-beta) E +
 * beta u_old^dagger, SVD M = X D Y^dagger, u_new = Y X^dagger (FP64).  A zero
 * M keeps u_old; a non-finite M gives NaN.  env, u_old, u_new: device
 * count x 4 x 4 c128 (u_new may alias u_old). */
int qf_optimize_gate(qf_ctx* ctx, int count, const void* env, const void* u_old, double beta,
                     void* u_new);

/* One gate update of TwoSidedSweep (Alg. 1), in place, for every builder:
 * half 0 (first half-sweep): remove G^dagger on the output legs, E = Tr_rest,
 * optimise, apply the new gate on the input legs; half 1: remove on the input
 * legs, optimise, apply on the output legs.  The remove and re-apply are one
 * fused pass over the builder.  gates: device n_builders x 4 x 4 c128, in =
 * current gate, out = updated gate.  env_out: optional device
 * n_builders x 4 x 4 c128 receiving E. */
int qf_update_gate(qf_ctx* ctx, int n, int n_builders, void* builder, int precision,
                   const int32_t* loc, int half, double beta, void* gates, void* env_out);

/* Cost of each builder from its trace, FP64: trace_out[s] = Tr(X_s) (device
 * c128, optional), cost_out[s] = 1 - |Tr X_s| / N (device double). */
int qf_cost(qf_ctx* ctx, int n, int n_builders, const void* builder, int precision,
            double* cost_out, void* trace_out);

/* QFactor (Alg. 1 with the multistart rule of Sec. IV-A): instantiate
 * n_gates two-qubit gates on `locations` to `target`, from n_starts initial
 * gate sets run in lockstep; stop when any start's cost < tol, when every
 * start has plateaued, or after max_iter sweeps.
 *   target:       device N x N c128 (the unitary V)
 *   locations:    host n_gates x 2 int32
 *   init_gates:   device n_starts x n_gates x 4 x 4 c128
 *   tol:          > 0; replaces opt->dist_tol
 *   opt:          host, NULL = qf_options_default
 *   workspace:    device, >= qf_workspace_size(n, n_gates, n_starts, opt) bytes
 *   out_gates:    device n_gates x 4 x 4 c128: the best start's gates
 *   out_all_gates:optional device n_starts x n_gates x 4 x 4 c128
 *   out_costs:    host n_starts doubles: FP64 cost of each start's returned
 *                 gates, from a fresh complex128 builder
 *   stats:        optional host qf_stats
 * Non-convergence is not an error: the call returns QF_OK with status
 * QF_PLATEAU / QF_MAX_ITER.  A start whose values become non-finite is
 * frozen; QF_ENUMERIC is returned only when every start is frozen. */
int qf_instantiate(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations,
                   const void* init_gates, int n_starts, double tol, const qf_options* opt,
                   void* workspace, size_t ws_bytes, void* out_gates, void* out_all_gates,
                   double* out_costs, qf_stats* stats);

/* qf_instantiate without a caller workspace, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, behaviour and results
 * as qf_instantiate, minus workspace/ws_bytes: the workspace is a fixed
 * device array of QF_NOALLOC_WORKSPACE_BYTES (64 MiB) that the library holds
 * on every device it runs on until the process ends; the call itself
 * allocates nothing.  Problems whose qf_workspace_size exceeds it return
 * QF_EWORKSPACE before any device work.  For circuits of about 5n gates
 * it holds, in complex64 / complex128 builders: n = 10 with up to 2 / 3
 * starts, n = 9 with 10 / 15,
 * n = 8 with 40 / 62, and every resident problem (n <= 6); no n >= 11
 * problem fits.  qf_workspace_size gives the exact need.  All calls on
 * one device share the array, so calls that overlap on a device (several
 * host threads, or contexts on different streams) race and must be
 * serialised by the caller; a call leaves the array's contents behind and
 * clears what it needs at its start.  stats->timing (which creates HIP
 * events) is refused with QF_EUNSUPPORTED. */
#define QF_NOALLOC_WORKSPACE_BYTES (64u << 20)
int qf_instantiate_noalloc(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations,
                           const void* init_gates, int n_starts, double tol, const qf_options* opt, void* out_gates,
                           void* out_all_gates, double* out_costs, qf_stats* stats);

/* Form of the fused remove/re-apply pass (the hot loop of every gate update,
 * Alg. 1) used for builders of n qubits in `precision`, for one class of
 * gates: gate_class 0 = the higher of the gate's two column bits (bit
 * n-1-q of a qubit q) is >= 3, gate_class 1 = both bits are among the three
 * lowest.  tile: -1 = register-direct pass, one 4x4 block per thread (needs
 * n >= 6, else the 512-column tile is used), -2 = micro-tile register pass,
 * the two blocks of 8 adjacent columns per quad of lanes with 16-byte loads
 * (QF_C64 only; for gate_class 1 at n >= 9, else the 512-column tile is
 * used), 256 / 512 / 1024 (1024: QF_C64 only) = columns of the LDS-staged
 * tile, 0 = forget the choice (the next qf_instantiate times the candidates
 * again).  Every form gives bitwise the same builder.
 * Returns QF_EINVAL for other values. */
int qf_set_pass_tile(qf_ctx* ctx, int precision, int n, int gate_class, int tile);

/* Tiles each workgroup of the two-gate pass walks (two consecutive gate
 * updates of Alg. 1 in one builder pass) for builders of n qubits in
 * `precision`: 1, 2, 4 or 8 (the next tile's loads in flight under the
 * current tile's products), or 0 = forget the choice (the next
 * qf_instantiate times the candidates again).  Every value gives bitwise the
 * same builder.  Returns QF_EINVAL for other values or n outside [4, 16]. */
int qf_set_pass2_tiles(qf_ctx* ctx, int precision, int n, int tiles);

/* Three-qubit gates (Sec. III: the environment and the update of Eq. opt_u
 * hold for gates of any size; the k = 3 gate-set variant of Sec. III-A-3).
 * qf_instantiate for a circuit whose every gate is an 8 x 8 unitary on three
 * qubits:
 *   locations:  host, n_gates x 3 int32, three distinct qubits in [0, n)
 *               (loc[0] the gate's most significant local bit, Q1)
 *   init_gates: device, n_starts x n_gates x 8 x 8 c128 (row-major)
 *   out_gates:  device, n_gates x 8 x 8 c128, the best start's gates
 *   out_all_gates: optional device, n_starts x n_gates x 8 x 8 c128
 *   target, out_costs, tol, stats: as for qf_instantiate.
 * The same sweep order, termination tests, multistart rule, complex64
 * recheck and final FP64 costs as qf_instantiate; the starts run in
 * stream_groups staggered groups on separate streams (0 = one; results do
 * not depend on the grouping; stats->timing is ignored).  Needs
 * 3 <= n <= 14, opt->gate_kinds == NULL and mode AUTO or STREAMING (RESIDENT
 * gives QF_EUNSUPPORTED).  The caller owns the workspace
 * (qf_workspace_size3 bytes, 0 for invalid sizes).  Errors as
 * qf_instantiate. */
size_t qf_workspace_size3(int n, int n_gates, int n_starts, const qf_options* opt);
int qf_instantiate3(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations,
                    const void* init_gates, int n_starts, double tol, const qf_options* opt, void* workspace,
                    size_t ws_bytes, void* out_gates, void* out_all_gates, double* out_costs, qf_stats* stats);

/* The 8 x 8 gate update of Eq. opt_u (beta of Sec. III-A-2) for `count`
 * environments: u_new[k] = argmax over unitary u of Re Tr(M u),
 * M = (1 - beta) env[k] + beta u_old[k]^dagger.  env, u_old, u_new: device,
 * count x 8 x 8 c128 (u_new must not alias env or u_old).  A zero M (largest
 * entry below 1e-300) keeps u_old; a non-finite M gives NaN.  QF_EINVAL for
 * count < 1, NULL pointers or beta outside [0, 1]. */
int qf_optimize_gate3(qf_ctx* ctx, int count, const void* env, const void* u_old, double beta, void* u_new);

/* Batched instantiation of many small independent problems (the partitions
 * of hierarchical synthesis, Sec. II "Partitioning and Resynthesis"), each
 * run as QFactor with its own multistarts in lockstep (Sec. IV-A), all in
 * one persistent launch.  Block b has block_n[b] qubits (2 <= n <= 4) and
 * the gates gate_offsets[b] .. gate_offsets[b+1]-1 of `locations` (host,
 * total_gates x 2 int32, qubits local to the block; at least one gate).
 *   targets:    device, the blocks' N_b x N_b c128 unitaries concatenated in
 *               block order (block b starts at sum_{b'<b} N_b'^2 entries)
 *   init_gates: device, for each block in order its n_starts x p_b x 4 x 4
 *               c128 initial gates (block b starts at n_starts *
 *               gate_offsets[b] * 16 entries)
 *   n_starts:   1..16 starts per block
 *   opt:        as for qf_instantiate (mode is ignored; both precisions run
 *               complex128 builders: blocks are at most 16 x 16, held in
 *               LDS, and their sweeps are chains of FP64 gate updates, so a
 *               complex64 builder would save nothing and need FP64 cost
 *               re-evaluations);
 *               tol replaces dist_tol
 *   workspace:  device, >= qf_batch_workspace_size(...)
 *   out_gates:  device, same layout as init_gates: every start's final gates
 *   out_costs:  host, n_blocks x n_starts FP64 costs of the returned gates
 *   out_best, out_status, out_sweeps: host, n_blocks each, optional
 *   stats:      optional; sweeps = largest sweep count, status = QF_CONVERGED
 *               only if every block converged
 * Returns when all outputs are final. */
size_t qf_batch_workspace_size(int n_blocks, const int32_t* block_n, const int32_t* gate_offsets, int n_starts,
                               const qf_options* opt);

/* Shape of the batched launch for `n_starts` starts per block: `slots`
 * instantiations (8 or 16, at least n_starts) per workgroup, one per 16
 * lanes, and `wg_per_cu` workgroups per compute unit (1 .. the kernel's
 * occupancy limit).  slots = 0 forgets the choice: the next
 * qf_instantiate_batch with these starts times every candidate (8 and 16
 * slots, 1 .. min(4, occupancy limit) workgroups per CU) for up to three
 * sweeps on its own first 2048 blocks (largest first) and keeps the
 * fastest; it restores out_gates from init_gates afterwards, and takes 16
 * slots at the occupancy limit untimed when they are the same buffer or
 * n_starts > 8.  The shape changes no result: every choice gives bitwise the
 * same outputs.  Returns QF_EINVAL for other values. */
int qf_set_batch_config(qf_ctx* ctx, int n_starts, int slots, int wg_per_cu);
int qf_instantiate_batch(qf_ctx* ctx, int n_blocks, const int32_t* block_n, const int32_t* gate_offsets,
                         const int32_t* locations, const void* targets, const void* init_gates, int n_starts,
                         double tol, const qf_options* opt, void* workspace, size_t ws_bytes, void* out_gates,
                         double* out_costs, int32_t* out_best, int32_t* out_status, int32_t* out_sweeps,
                         qf_stats* stats);

/* Cost and gradient of the cost with respect to every gate matrix (the
 * derivative the gradient-based instantiation optimisers of Sec. II,
 * "Numerical Optimization in Instantiation", need; cost as in Sec. II).
 * With T = Tr(V^dagger C) = Tr(E_g u_g) (Sec. III), the real gradient packed
 * as a complex matrix is
 *     grad_g = dDelta/dRe u_g + i dDelta/dIm u_g = -(T/|T|) E_g^dagger / N
 * (zero where T = 0).  All p environments come from one half-sweep of the
 * builder with the gates held fixed, so memory is one builder per start.
 *   target:   device, N x N c128;  locations: host, n_gates x 2
 *   gates:    device, n_starts x n_gates x 4 x 4 c128 (not modified)
 *   precision QF_C128 or QF_C64 (builder precision; sums and outputs FP64)
 *   workspace: device, >= qf_gradient_workspace_size(...)
 *   cost_out: device, n_starts doubles;  grad_out: device, same layout as gates
 * Work is enqueued on the context's stream; the call does not synchronise. */
size_t qf_gradient_workspace_size(int n, int n_gates, int n_starts, int precision);
int qf_gradient(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations, const void* gates,
                int n_starts, int precision, void* workspace, size_t ws_bytes, double* cost_out, void* grad_out);

/* Parameterised two-qubit gates of the gradient-based baseline: a gate is
 * exp(i H(theta)), H = sum_k theta_k P_k over the 15 non-identity Pauli
 * products P_k = sigma_a (x) sigma_b, k = 4a + b - 1 (sigma_0..3 = I, X, Y,
 * Z); H is traceless Hermitian so the gate is in SU(4), and a gate's global
 * phase does not change the cost.  (Sec. VI discusses the parameter counts of
 * such encodings.)
 *   qf_su4_gates: theta (device, count x 15 FP64) -> gates (device, count x
 *                 4 x 4 c128)
 *   qf_su4_vjp:   grad_gates (device, count x 4 x 4 c128, packed as in
 *                 qf_gradient) -> dtheta (device, count x 15):
 *                 dtheta_k = Re Tr(grad^dagger dU/dtheta_k)
 * Asynchronous on the context's stream. */
int qf_su4_gates(qf_ctx* ctx, int count, const double* theta, void* gates);
int qf_su4_vjp(qf_ctx* ctx, int count, const double* theta, const void* grad_gates, double* dtheta);

/* L-BFGS baseline (the gradient-descent comparison optimiser of Sec. II and
 * Sec. V) over parameterised SU(4) gates, driven by qf_gradient: every
 * evaluation maps theta to gates, builds the builders, and takes the cost and
 * the gradient; the two-loop recursion and the backtracking (Armijo) line
 * search run on the host, all starts in lockstep. */
typedef struct {
  int32_t history;   /* correction pairs kept (default 10) */
  int32_t max_iter;  /* iterations (default 1000) */
  int32_t max_ls;    /* trial steps per line search (default 30) */
  double c1;         /* sufficient-decrease constant (default 1e-4) */
  double grad_tol;   /* a start stops when max |dDelta/dtheta| < grad_tol (default 1e-12) */
  double ftol_r;     /* ... or when f_{k-1} - f_k <= ftol_r * f_k (default 1e-12) */
  int32_t precision; /* builder precision, QF_C128 (default) or QF_C64 */
} qf_lbfgs_options;
void qf_lbfgs_options_default(qf_lbfgs_options* o);
size_t qf_lbfgs_workspace_size(int n, int n_gates, int n_starts, const qf_lbfgs_options* opt);
/* Outcome of qf_lbfgs (host memory). */
typedef struct {
  int32_t iterations;    /* L-BFGS iterations run (lockstep over starts) */
  int32_t evaluations;   /* cost + gradient evaluations, line-search trials included */
  int32_t best_start;    /* start with the smallest final cost, lowest index on ties */
  int32_t status;        /* QF_CONVERGED, QF_PLATEAU (every start stopped) or QF_MAX_ITER */
  double best_cost;      /* final cost of the best start */
  double elapsed_ms;     /* wall time of the call */
  double* cost_history;  /* in, optional (host): rows x n_starts doubles; row i
                            receives the costs after iteration i (row 0 = theta0) */
  int32_t cost_history_rows;
} qf_lbfgs_result;
/* theta0, theta_out: device, n_starts x n_gates x 15 FP64;  out_costs: host,
 * n_starts final costs.  The job stops when a start's cost falls below tol,
 * when every start has stopped, or after max_iter iterations.  result:
 * optional host qf_lbfgs_result. */
int qf_lbfgs(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations, const double* theta0,
             int n_starts, double tol, const qf_lbfgs_options* opt, void* workspace, size_t ws_bytes,
             double* theta_out, double* out_costs, qf_lbfgs_result* result);

/* Outcome of qf_delete_gates (host memory). */
typedef struct {
  int32_t attempts;    /* deletions tried (one re-instantiation each) */
  int32_t deleted;     /* deletions kept */
  int32_t sweeps;      /* sweeps of all the attempts' instantiations together */
  double elapsed_ms;   /* wall time of the call */
} qf_delete_result;

/* Gate deletion (the re-synthesis workflow QFactor drives in Sec. V,
 * "Circuit Optimization Scaling"): one uni-directional sweep over the gates
 * of a partition, g = 0..p-1; each step deletes gate g from the current
 * circuit and re-instantiates the reduced structure (qf_instantiate with
 * `opt`) to the partition's own unitary; the deletion is kept when the best
 * start's cost is below tol, and the re-instantiated gates become the
 * current circuit.  Start 0 of every attempt is the current circuit without
 * gate g (a warm start); starts 1..n_starts-1 take their gates from the
 * caller's pool at the positions still present.
 *   target:     device, N x N c128, the partition's unitary
 *   locations:  host, n_gates x 2
 *   gates:      device, n_gates x 4 x 4 c128: a circuit of this structure
 *               that realises target (cost below tol); not modified
 *   pool:       device, n_starts x n_gates x 4 x 4 c128 (start 0 unused)
 *   workspace:  device, >= qf_delete_gates_workspace_size(...)
 *   keep:       host, n_gates int32 out: 1 kept, 0 deleted
 *   out_gates:  device, n_gates x 4 x 4 c128 out: the kept gates in order,
 *               compacted to the front (the rest left unspecified)
 *   out_cost:   host, FP64 cost of the final circuit
 *   result:     optional host qf_delete_result
 * Returns QF_EINVAL if `gates` does not realise target within tol. */
size_t qf_delete_gates_workspace_size(int n, int n_gates, int n_starts, const qf_options* opt);
int qf_delete_gates(qf_ctx* ctx, int n, const void* target, int n_gates, const int32_t* locations,
                    const void* gates, const void* pool, int n_starts, double tol, const qf_options* opt,
                    void* workspace, size_t ws_bytes, int32_t* keep, void* out_gates, double* out_cost,
                    qf_delete_result* result);

#ifdef __cplusplus
}
#endif

#endif /* QFACTOR_MI355X_H */
