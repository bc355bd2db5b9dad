/*
 * lre.h -- C ABI of the gfx950 (MI355X) library for linear regression estimation
 * (LRE) of an n-qubit state from local Pauli measurement counts.
 *
 * Method: Hou et al., "Full reconstruction of a 14-qubit state within four hours"
 * (arXiv:1602.08604).  The library implements the paper's steps (i) and (ii):
 *   step (i)  Sec. II eq. (3) with the Pauli structure of Sec. III: the least-squares
 *             coefficients Theta = (X^T X)^{-1} sum_j p_j Gamma^(j), where every
 *             Gamma^(j) has 2^n nonzero entries and X^T X = (x)_k diag{3,1,1,1};
 *   step (ii) Sec. II eq. (4): mu = sum_i theta_i Omega_i with Omega_i of eq. (5).
 * Step (iii) (projection onto physical states) is not part of this library.
 *
 * Data layout (all device memory, row-major, caller-owned):
 *   counts : uint16 [3^n][2^n].  Row b is one measurement setting,
 *            b = sum_k b_k 3^{n-k} with b_k in {0:X, 1:Y, 2:Z} (qubit 1 most
 *            significant); column s = sum_k s_k 2^{n-k}, s_k = 0 for the +1
 *            eigenvector of the measured Pauli operator.  16-byte aligned.
 *   coef   : double [4^n].  coef[i] = e_i = 2^{n/2} theta_i, the Pauli expectation
 *            of the string with letters a_k (i = sum_k a_k 4^{n-k}, eq. 5;
 *            a_k in {0:I, 1:X, 2:Y, 3:Z}).  coef[0] = 1 for every valid input.
 *   rho    : [2^n][2^n] complex, interleaved (re, im), row r = sum_k r_k 2^{n-k}.
 *            complex128 by default, complex64 with LRE_RHO_FP32.  16-byte aligned.
 *            This is mu of eq. (4): Hermitian, unit trace, not necessarily positive.
 * Frequencies p_j are taken within each basis, p = c[b][s] / N_b, N_b the basis total.
 *
 * Conventions common to every entry point:
 *   - Calls enqueue work on `stream` (a hipStream_t; NULL = default stream) and return
 *     without synchronising.  No entry point allocates device memory except
 *     lre_create (a 64-byte flag word) and lre_batch_plan (the work list);
 *     lre_project's solver libraries allocate their own scratch.
 *   - Host-checkable problems (bad n, NULL or misaligned pointers, workspace too
 *     small) return an error before anything is launched.
 *   - Data-dependent problems are recorded in the context's device flag word and
 *     reported by lre_check: a basis whose counts do not sum to the declared total
 *     (LRE_E_SHOTS) or a basis with no counts in per-basis mode (LRE_E_EMPTY_BASIS).
 *     Outputs are unspecified when a flag is raised.
 *   - One lre_ctx per host thread, or external locking.  Calls that share a
 *     workspace must be ordered on one stream.
 *   - No C++ exception crosses this interface.
 */
#ifndef LRE_H
#define LRE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LRE_OK = 0,
  LRE_E_ARG = 1,          /* invalid argument (n out of range, NULL/misaligned pointer) */
  LRE_E_WORKSPACE = 2,    /* workspace smaller than lre_workspace_bytes() */
  LRE_E_HIP = 3,          /* a HIP runtime call failed */
  LRE_E_SHOTS = 4,        /* a basis row does not sum to its declared total */
  LRE_E_EMPTY_BASIS = 5,  /* per-basis mode: a basis with zero counts */
  LRE_E_UNSUPPORTED = 6,  /* valid request that the library does not serve */
  LRE_E_TIMEOUT = 7,      /* a batched run's bounded wait for a dependency expired */
  LRE_E_EIG = 8           /* lre_project: the eigendecomposition did not converge */
} lre_status;

#define LRE_MAX_QUBITS 14

/* Flags (bitwise or). */
#define LRE_NO_RHO 0x1u    /* skip step (ii); rho may be NULL */
#define LRE_RHO_FP32 0x2u  /* write rho as complex64 instead of complex128 */
#define LRE_WHT_MFMA 0x4u  /* signed outcome sums on int8 MFMA: the same integer sums
                              (bit-identical with uniform shots; per-basis binary64 sums
                              added in another order, equal to rounding) */

typedef struct lre_ctx lre_ctx;

/* Create a context on HIP device `hip_device`: allocates the 64-byte device flag
 * word.  *out receives the context.  Errors: LRE_E_ARG (out == NULL), LRE_E_HIP. */
lre_status lre_create(lre_ctx** out, int hip_device);

/* Destroy a context created by lre_create (NULL is ignored). */
void lre_destroy(lre_ctx* ctx);

/* Static, human-readable name of a status code ("unknown status" for a value outside
 * the enumeration). */
const char* lre_status_str(lre_status status);

/* Bytes of device workspace lre_estimate needs for this (n, shots, flags); 0 when n
 * is out of range.  shots follows lre_estimate (0 = per-basis totals). */
size_t lre_workspace_bytes(int n, uint64_t shots, uint32_t flags);

/* Steps (i) and (ii) on one instance (Sec. II eqs. 3 and 4, Sec. III).
 *   n           : 1 <= n <= LRE_MAX_QUBITS.
 *   counts      : device uint16 [3^n][2^n], 16-byte aligned.
 *   shots       : > 0  every basis totals exactly `shots` (checked); e_i is then the
 *                      correctly rounded quotient of the exact integer sum
 *                      T_i = sum_{b,s} c[b][s] 2^{n/2} gamma_i^(b,s) by 3^{n-w(i)} shots.
 *                 == 0 per-basis totals N_b: taken from n_per_basis when non-NULL
 *                      (checked against the row sums) or computed from the rows
 *                      (one extra pass over counts); e_i = 3^{-(n-w)} sum_b S_b / N_b
 *                      in binary64.
 *   n_per_basis : device uint32 [3^n] or NULL; read only when shots == 0.
 *   coef        : device double [4^n], written.
 *   rho         : device complex [2^n][2^n] (see header), written unless LRE_NO_RHO.
 *   workspace   : device memory of at least lre_workspace_bytes(n, shots, flags) bytes,
 *                 256-byte aligned, caller-owned, contents need not be initialised.
 *   flags       : LRE_NO_RHO | LRE_RHO_FP32 | LRE_WHT_MFMA.
 *   stream      : hipStream_t to enqueue on.
 * Returns LRE_OK once every kernel is enqueued. */
lre_status lre_estimate(lre_ctx* ctx, int n, const uint16_t* counts, uint64_t shots,
                        const uint32_t* n_per_basis, double* coef, void* rho, void* workspace,
                        size_t workspace_bytes, uint32_t flags, void* stream);

/* lre_estimate without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Arguments, results and errors are those of lre_estimate; the workspace
 * is a static device array of LRE_NOALLOC_SCRATCH_BYTES bytes that the library holds
 * on every device it runs on until the process ends (its per-device address is
 * resolved by lre_create).  The call allocates nothing and frees nothing.
 *   - Requests whose lre_workspace_bytes(n, shots, flags) exceed
 *     LRE_NOALLOC_SCRATCH_BYTES return LRE_E_WORKSPACE before any launch (with
 *     64 MiB: every n <= 10, any shots and flags).
 *   - Within a process, every call on one device shares that device's array, whatever
 *     the context: calls that overlap in time on one device (different streams,
 *     threads or contexts of that device) race and their results are unspecified.
 *     Order them on one stream.  The array needs no clearing between calls (no
 *     kernel of the path reads workspace it has not written in the same call).
 *   - LRE_E_HIP if lre_create could not resolve the array's address. */
#define LRE_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
lre_status lre_estimate_noalloc(lre_ctx* ctx, int n, const uint16_t* counts, uint64_t shots,
                                const uint32_t* n_per_basis, double* coef, void* rho, uint32_t flags,
                                void* stream);

/* Synchronise `stream`, read and clear the context's device flag word.  Returns
 * LRE_E_SHOTS, LRE_E_EMPTY_BASIS, LRE_E_TIMEOUT, LRE_E_HIP or LRE_OK. */
lre_status lre_check(lre_ctx* ctx, void* stream);

/* Profiling hook.  events: `count` (<= 4) caller-created hipEvent_t handles, or NULL to
 * disable.  While set, lre_estimate records them on its stream at stage boundaries:
 *   events[0] before its first kernel,        events[1] after the counts pass,
 *   events[2] after the rest of step (i),     events[3] after step (ii).
 * The caller owns the events and must keep them alive while they are set. */
lre_status lre_set_stage_events(lre_ctx* ctx, void* const* events, int count);

/* Exact integer numerators of eq. (3) with uniform shots (verification entry):
 * T[i] = sum_{b,s} c[b][s] * prod_k g(a_k, b_k, s_k), g = 2^{1/2} gamma of the one-qubit
 * projector (Sec. III), for every i < 4^n, as int64.  Same kernels as lre_estimate.
 *   shots     : the declared per-basis total (checked; bounds the partial sums).
 *   T         : device int64 [4^n].
 *   workspace : at least lre_workspace_bytes(n, shots, flags | LRE_NO_RHO) bytes. */
lre_status lre_pauli_sums(lre_ctx* ctx, int n, const uint16_t* counts, uint64_t shots,
                          int64_t* T, void* workspace, size_t workspace_bytes, uint32_t flags,
                          void* stream);

/* Signed outcome sums of selected bases (verification entry):
 * out[j][m] = sum_s c[b_j][s] (-1)^{popcount(s & m)} for m < 2^n, i.e. the per-basis
 * part sum_s c gamma^(b,s)_i of eq. (3) at the coefficient i whose support is m.
 * flags: 0 (the register / lane butterflies of the plain counts pass) or LRE_WHT_MFMA
 * (the int8-MFMA 64-outcome transform of the MFMA counts pass, n >= 6; smaller n
 * returns LRE_E_UNSUPPORTED).
 *   bases : device int64 [num_bases], each in [0, 3^n) (an out-of-range entry yields
 *           an all-zero row and raises LRE_E_ARG through lre_check).
 *   out   : device int32 [num_bases][2^n]. */
lre_status lre_signed_sums(lre_ctx* ctx, int n, const uint16_t* counts, const int64_t* bases,
                           int64_t num_bases, int32_t* out, uint32_t flags, void* stream);

/* ---------------------------------------------------------------------------------
 * Batched estimation: many independent instances (each its own n, counts and shots)
 * in one launch of a persistent kernel.  Every instance gets exactly what
 * lre_estimate returns for it (steps (i) and (ii), Sec. II eqs. 3-4): the same
 * kernels' arithmetic, bit-identical coefficients and rho.
 *
 * lre_batch_plan builds a work list (an instance of n <= 7 qubits is one item; a larger
 * one is split into its counts-pass row groups, later pass and step-(ii) blocks, in
 * dependency order) and uploads it.  lre_batch_run enqueues a fill kernel that clears the
 * item and dependency counters in the workspace, then one persistent kernel whose
 * workgroups take items from the list in order; an item that needs the results of
 * earlier items waits for their counters (a bounded wait: on expiry the item is
 * skipped and LRE_E_TIMEOUT is raised through lre_check).  For a plan with instances
 * of 7 or more qubits it then enqueues the staged form's fold and step-(ii) kernels,
 * which return at once unless the plan's shape is staged (lre_batch_tiles.staged), so
 * that a captured run replays correctly after lre_batch_set_tiles or lre_batch_tune.
 * lre_batch_run makes no allocation, copy or memset and may be captured into a HIP
 * graph.
 */
#define LRE_BATCH_MAX_QUBITS 9

typedef struct {
  int n;                   /* 1 <= n <= LRE_BATCH_MAX_QUBITS */
  const uint16_t* counts;  /* device uint16 [3^n][2^n], 16-byte aligned */
  uint64_t shots;          /* > 0: every basis totals exactly `shots`, with
                              3^n * shots < 2^31 (integer branch, checked per basis);
                              == 0: per-basis totals N_b (binary64 branch), as in
                              lre_estimate */
  const uint32_t* n_per_basis; /* shots == 0 only: device uint32 [3^n], 4-byte aligned,
                              checked against the row sums, or NULL to take the row
                              sums (one extra pass over the instance's counts) */
  double* coef;            /* device double [4^n], 8-byte aligned */
  void* rho;               /* device complex [2^n][2^n], 16-byte aligned; unused with
                              LRE_NO_RHO */
} lre_instance;

/* Work-item shape of a plan (what lre_batch_tune chooses between). */
typedef struct {
  int workers_per_cu;   /* persistent workgroups per compute unit: 1 or 2 */
  int counts_tiles;     /* counts-pass row groups (3^7 rows, all their outcomes) per item at
                           most, >= 1; an instance's groups are split into that many items
                           of equal size (to one group) */
  int fold_cols;        /* later-pass columns per item at most, multiple of 432 (split as
                           evenly as counts_tiles) */
  int rho_blocks;       /* step-(ii) work per item, >= 1: high-qubit row patterns x_hi
                           (2^(n-6) per instance of n > 7 qubits) */
  int interleave;       /* 0: stage by stage, largest instances first;
                           1: instance by instance (all stages of an instance together) */
  int staged;           /* 0: every stage in the persistent kernel's work list;
                           1: the list holds the per-basis totals, the counts pass and the
                           instances of at most 7 qubits (step (ii) of those of exactly 7
                           excepted), and the later fold and step (ii) follow as two
                           kernels of their own (one thread per column; one block per
                           step-(ii) unit), in stream order; fold_cols, rho_blocks and
                           interleave then do not matter */
} lre_batch_tiles;

typedef struct lre_batch lre_batch;

/* Plan a batch of `count` instances (count >= 1).  flags: LRE_NO_RHO | LRE_RHO_FP32
 * (applied to every instance).  The instance array is copied; the buffers it points
 * to must stay valid while the plan is used.  Allocates the device work list (once:
 * lre_batch_set_tiles and lre_batch_tune reuse it).
 * A plan with a per-basis instance (shots == 0) runs one workgroup per compute unit
 * (its binary64 accumulators fill the LDS), whatever workers_per_cu says.
 * Errors: LRE_E_ARG (bad instance: n < 1, pointer, alignment, shots too large),
 * LRE_E_UNSUPPORTED (n > LRE_BATCH_MAX_QUBITS), LRE_E_HIP. */
lre_status lre_batch_plan(lre_ctx* ctx, const lre_instance* inst, int count, uint32_t flags,
                          lre_batch** plan_out);

/* Device workspace bytes lre_batch_run needs (counters and every instance's
 * intermediate buffers); 0 for a NULL plan. */
size_t lre_batch_workspace_bytes(const lre_batch* plan);

/* Replace the plan's work-item shape and rebuild its work list (synchronous: waits
 * for the device to be idle, then uploads).  The list keeps its device address for
 * the plan's lifetime (it is allocated once by lre_batch_plan, at the length of the
 * longest shape) and the persistent kernel reads the item count from device memory,
 * so an lre_batch_run captured into a HIP graph before a retune stays valid: its
 * replays run the current list (with the grid and per-CU worker count of the
 * captured launch).  Errors: LRE_E_ARG for out-of-range fields, LRE_E_HIP. */
lre_status lre_batch_set_tiles(lre_batch* plan, const lre_batch_tiles* tiles);

/* The plan's current work-item shape and work-item count. */
lre_status lre_batch_get_tiles(const lre_batch* plan, lre_batch_tiles* tiles, int* num_items);

/* Autotuner: runs the batch (lre_batch_run) for each of 82 candidate work-item shapes
 * (72 unstaged and 10 staged; 41 for a plan with per-basis instances, which run one
 * workgroup per CU),
 * `reps` timed runs each after one warm-up, keeps the fastest shape and returns its
 * mean time in *best_ms (may be NULL).  Synchronous on `stream`; overwrites the
 * instances' outputs.  workspace as for lre_batch_run. */
lre_status lre_batch_tune(lre_batch* plan, void* workspace, size_t workspace_bytes, int reps,
                          double* best_ms, void* stream);

/* Enqueue the whole batch on `stream` (see above).  workspace: device memory of at
 * least lre_batch_workspace_bytes(plan) bytes, 256-byte aligned; calls that share a
 * workspace must be ordered on one stream.  Data errors go to the context's flag
 * word (lre_check). */
lre_status lre_batch_run(lre_batch* plan, void* workspace, size_t workspace_bytes, void* stream);

/* Free the plan and its work list (NULL is ignored). */
void lre_batch_destroy(lre_batch* plan);

/* ---------------------------------------------------------------------------------
 * Streamed estimation: counts delivered slab by slab, for instances whose counts do not
 * fit device memory (n = 15 holds 940 GB of counts), the way the paper fed its GPU one
 * group of measurement data at a time (Sec. III storage, Sec. IV GPU scheme).  Results
 * are those of lre_estimate: bit-identical coefficients with uniform shots, binary64
 * sums (order-dependent rounding) with per-basis totals.
 *
 * Slab k (0 <= k < 3^h) holds the 3^(n-h) consecutive bases k*3^(n-h) .. (k+1)*3^(n-h)-1,
 * i.e. the bases whose top h qubits carry the letters of k's base-3 digits: device (or,
 * for lre_stream_push_host, host) uint16 [3^(n-h)][2^n], rows as in `counts` above.
 * Each slab is cut into its 2^h outcome segments (fixed outcome bits of the top h
 * qubits); a segment goes through the passes of an (n-h)-qubit instance, whose rows are
 * read with the stride of the full rows, and the top h qubits are folded into `coef`,
 * which accumulates over the slabs; lre_stream_finish divides by (X^T X)_ii and runs
 * step (ii).  Slabs may come in any order, each exactly once.  Every call of one
 * stream object must be ordered on one HIP stream and use the same workspace.
 */
#define LRE_STREAM_MAX_QUBITS 15
#define LRE_STREAM_HOST 0x8u  /* lre_stream_create: reserve a staging slab for push_host */

typedef struct lre_stream lre_stream;

/* Plan a streamed estimate of n qubits with slabs fixed by the top h qubits:
 * 1 <= h <= 6, 8 <= n - h <= LRE_MAX_QUBITS, n <= LRE_STREAM_MAX_QUBITS.  shots: as in
 * lre_estimate (0 = per-basis totals).  flags: LRE_NO_RHO | LRE_RHO_FP32 | LRE_WHT_MFMA
 * | LRE_STREAM_HOST.  Host memory only (one event is created).  Errors: LRE_E_ARG,
 * LRE_E_HIP. */
lre_status lre_stream_create(lre_ctx* ctx, int n, int h, uint64_t shots, uint32_t flags, lre_stream** out);

/* Device workspace bytes every call of the stream object needs (256-byte aligned,
 * caller-owned, one buffer for all calls): one segment's pass buffers, the 2^h segment
 * sums, their row-sum parts, the staging slab with LRE_STREAM_HOST, and step (ii)'s
 * intermediate (16 * 4^n bytes, aliased onto the rest).  0 for NULL. */
size_t lre_stream_workspace_bytes(const lre_stream* s);

/* Start an estimate: coef (device double [4^n], 8-byte aligned) becomes the accumulator
 * and is cleared (a fill kernel on `stream`); forgets earlier slabs.  Errors: LRE_E_ARG,
 * LRE_E_WORKSPACE, LRE_E_HIP. */
lre_status lre_stream_begin(lre_stream* s, double* coef, void* workspace, size_t workspace_bytes, void* stream);

/* Add slab `slab` from device memory (16-byte aligned; n_per_basis: device uint32
 * [3^(n-h)] of the slab's totals or NULL for the row sums, read only with shots == 0).
 * Enqueued on `stream`; the slab's buffers must stay unchanged until the stream has
 * passed its kernels.  Data errors (totals, empty bases) go to the context's flag word.
 * Errors: LRE_E_ARG (no lre_stream_begin, slab out of range or already pushed, pointer),
 * LRE_E_WORKSPACE, LRE_E_HIP. */
lre_status lre_stream_push(lre_stream* s, int64_t slab, const uint16_t* counts, const uint32_t* n_per_basis,
                           void* workspace, size_t workspace_bytes, void* stream);

/* As lre_stream_push, for a slab in host memory (pinned memory copies at the link's
 * full rate): copied on `stream` into the workspace's staging slab (the stream object
 * must have been created with LRE_STREAM_HOST), then processed there.  Returns once the
 * copies have completed, so the host buffers may be refilled at once while the slab's
 * kernels run.  Errors as lre_stream_push. */
lre_status lre_stream_push_host(lre_stream* s, int64_t slab, const uint16_t* counts, const uint32_t* n_per_basis,
                                void* workspace, size_t workspace_bytes, void* stream);

/* After all 3^h slabs: coef[i] /= 3^{n-w(i)} (times shots in uniform mode), then step
 * (ii) into rho (device complex [2^n][2^n], 16-byte aligned) unless LRE_NO_RHO.
 * Enqueued on `stream`.  Errors: LRE_E_ARG (a slab missing, no begin, rho), LRE_E_WORKSPACE,
 * LRE_E_HIP. */
lre_status lre_stream_finish(lre_stream* s, void* rho, void* workspace, size_t workspace_bytes, void* stream);

/* Destroy a stream object (NULL is ignored). */
void lre_stream_destroy(lre_stream* s);

/* ---------------------------------------------------------------------------------
 * Reduced measurement set (Sec. VI): instead of the 3^n Pauli bases, one
 * informationally complete set of four operators E_0..E_3 per qubit (the same set on
 * every qubit, e.g. a four-outcome POVM), i.e. 4^n product operators.  The paper names
 * no set; the caller gives it by its Pauli components.  Eq. (3) is then
 *   e = 2^{n/2} theta = ((x)_k M) p,  M = 2 (G^T G)^{-1} G^T,  p_j = c_j / N,
 * since Gamma^(j) is the tensor product of the rows G[j_k][.] / sqrt 2 and
 * X^T X = 2^-n (x)_k G^T G; step (ii) is eq. (4) on e as for the Pauli bases.
 *   counts : device uint16 [4^n], outcome j = sum_k j_k 4^{n-k} (qubit 1 most
 *            significant), 16-byte aligned; N = sum of all counts.
 *   G      : device double [4][4] row-major, G[j][a] = Tr(E_j sigma_a) (sigma_0 = I,
 *            then X, Y, Z); G^T G must be invertible (else LRE_E_ARG through lre_check
 *            and coef = 0).  N = 0 raises LRE_E_EMPTY_BASIS through lre_check.
 *   coef   : device double [4^n], e_i in the layout of lre_estimate (binary64; M and
 *            the mode products in binary64, one division by N at the end).
 *   rho    : as lre_estimate; flags LRE_NO_RHO | LRE_RHO_FP32.
 *   workspace : at least lre_povm_workspace_bytes(n, flags) bytes, 256-byte aligned.
 * 1 <= n <= LRE_MAX_QUBITS.  Enqueued on `stream`. */
size_t lre_povm_workspace_bytes(int n, uint32_t flags);
lre_status lre_povm_estimate(lre_ctx* ctx, int n, const uint16_t* counts, const double* G, double* coef, void* rho,
                             void* workspace, size_t workspace_bytes, uint32_t flags, void* stream);

/* ---------------------------------------------------------------------------------
 * Step (iii) (Sec. II): the physical state closest to mu, with the fast algorithm the
 * paper cites -- eigendecompose mu, move the spectrum onto the probability simplex
 * (negative eigenvalues removed, the removed mass shared equally over the eigenvalues
 * kept), reassemble rho = V diag(lambda) V^H.
 *   mu        : device complex128 [2^n][2^n] row-major, Hermitian with trace 1 (the
 *               output of lre_estimate); only read.
 *   rho       : device complex128 [2^n][2^n] row-major, out (positive semidefinite,
 *               trace 1); must not overlap mu.
 *   eigvals   : device double [2^n] out, the eigenvalues of mu in ascending order, or
 *               NULL.
 *   workspace : at least lre_project_workspace_bytes(n) bytes, 256-byte aligned.
 * Enqueued on `stream` (eigensolver and product from rocSOLVER / rocBLAS, which may
 * allocate their own scratch).  A solver failure raises LRE_E_EIG through lre_check
 * (rho is then 0). */
size_t lre_project_workspace_bytes(int n);
lre_status lre_project(lre_ctx* ctx, int n, const void* mu, void* rho, double* eigvals, void* workspace,
                       size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Device streaming rates (diagnostics, not part of the method): plain kernels with
 * 16-byte vector accesses (each block a contiguous range), used to state the practical
 * HBM ceiling next to the datasheet peak.  Enqueued on `stream`; time them with events around the call.
 *   lre_stream_read : reads `bytes` at `buf`; `sink` is a device uint32 that may be
 *                     written (it keeps the loads from being optimised away).
 *   lre_stream_copy : copies `bytes` from `src` to `dst` (non-overlapping).
 * Pointers are device pointers, 16-byte aligned; `bytes` is a multiple of 16, else
 * LRE_E_ARG.  The caller owns every buffer. */
lre_status lre_stream_read(const void* buf, size_t bytes, uint32_t* sink, void* stream);
lre_status lre_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Compute issue rates (diagnostics, not part of the method), next to the datasheet
 * peaks the counts pass is compared with.  Each launches one kernel of `iters`
 * iterations on `stream` (time it with events around the call) and stores in *ops
 * (host pointer, may be NULL) the number of operations the launch performs:
 *   lre_peak_valu_i32 : 32-bit integer adds, 8 independent chains per lane;
 *   lre_peak_mfma_i8  : dense int8 MFMA (v_mfma_i32_16x16x64_i8, 32768 operations each),
 *                       4 independent accumulator chains per wave.
 * `sink` is a device uint32 that may be written.  iters < 1 or sink NULL: LRE_E_ARG. */
lre_status lre_peak_valu_i32(int iters, uint32_t* sink, double* ops, void* stream);
lre_status lre_peak_mfma_i8(int iters, uint32_t* sink, double* ops, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LRE_H */
