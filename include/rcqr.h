/*
 * rcqr -- randomized Householder-Cholesky QR with multisketching on one AMD Instinct MI355X.
 *
 * Method: Higgins, Szyld, Boman, Yamazaki, "Analysis of Randomized Householder-Cholesky QR
 * Factorization with Multisketching" (arXiv 2309.05868), Algorithm 3 (rand_cholQR) built on
 * Algorithm 1 (randQR) and Algorithm 2 (cholQR).  Notation: V has m rows and n columns (the
 * paper writes n rows and m columns); the CountSketch S1 has s1 rows, the Gaussian sketch S2
 * has s2 rows.
 *
 * Data layout (all FP64, all row-major, all in device memory owned by the caller):
 *   V  m x n, leading dimension ldv >= n      input, read three times, never written
 *                                             (unless Q aliases it)
 *   Q  m x n, leading dimension ldq >= n      output, orthonormal columns; may alias V
 *                                             (d_Q == d_V with ldq == ldv)
 *   R  n x n, leading dimension ldr >= n      output, upper triangular with positive
 *                                             diagonal; the strict lower triangle is
 *                                             written as zeros
 *   workspace  rcqr_workspace_bytes() bytes   caller-allocated device memory, 256-byte
 *                                             aligned; holds W1, W, R0, G, R1, partial sums,
 *                                             the CountSketch bucket index and the status
 *                                             word.  One plan uses it at a time.
 *
 * Sketch contract (the paper fixes no generator; Section 6.1 only says the sketches were
 * built explicitly).  Philox4x64-10 (Salmon et al., SC'11), key (seed, 0):
 *   row i:  y = Philox((floor(i/4), 0, 0, 1)), w = y[i mod 4],
 *           bucket h(i) = floor(w s1 / 2^64), sign = -1 if (w & 1) else +1    (S1, Section 3)
 *   S2[4b+t, k], t = 0..3:  y = Philox((k, b, 0, 2)); Box-Muller on (y0, y1) -> t = 0, 1 and
 *           (y2, y3) -> t = 2, 3 with u1 = ((ya >> 11) + 1) 2^-53, u2 = (yb >> 11) 2^-53,
 *           z = sqrt(-2 ln u1) {cos, sin}(2 pi u2);  S2[j, k] = z / sqrt(s2)        (Section 3)
 *
 * Errors: argument errors are returned synchronously.  Numerical failures are found on the
 * device and reported through rcqr_info(): RCQR_E_RANK when the Householder R0 of the sketch
 * has a zero or non-finite diagonal entry, RCQR_E_CHOL when the Cholesky factorization of
 * the Gram matrix of V R0^{-1} meets a pivot that is not positive (NaN included).  After a
 * numerical failure the contents of Q and R are unspecified.
 *
 * Streams and threads: every entry point that launches work enqueues it on the plan's HIP
 * stream and returns without waiting, except rcqr_info() and rcqr_phase_times(), which wait
 * for the stream.  A plan (and its workspace) must not be used by two host threads at once.
 */
#ifndef RCQR_H
#define RCQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rcqr_plan_s* rcqr_plan_t;

typedef enum {
  RCQR_OK = 0,
  RCQR_E_INVALID = 1,     /* bad argument (sizes, leading dimensions, null pointers, workspace) */
  RCQR_E_UNSUPPORTED = 2, /* n > 128 */
  RCQR_E_NOMEM = 3,       /* host allocation of the plan failed */
  RCQR_E_HIP = 4,         /* a HIP runtime call failed (launch, event, copy) */
  RCQR_E_RANK = 5,        /* Householder R0 of the sketch has a zero / non-finite diagonal */
  RCQR_E_CHOL = 6,        /* Cholesky of the Gram matrix met a non-positive pivot */
  RCQR_E_SCRATCH = 7      /* rcqr_factor_static: the shape's workspace exceeds the static scratch */
} rcqr_status_t;

/* Largest number of columns the kernels support. */
#define RCQR_MAX_N 128

/*
 * Plan flags (bitwise OR; 0 = the method as written, everything in FP64).
 *
 * RCQR_FLAG_SKETCH_FP32: the preconditioner is computed in single precision: W1 = S1 V accumulates
 *   V's entries rounded to FP32, W = S2 W1 runs on the FP32 matrix cores (S2 entries are the FP64
 *   contract values rounded to FP32) with FP32 accumulation, and the Householder R0 is computed
 *   in FP32 and promoted to FP64.  Everything after R0 (Q0 = V R0^{-1}, the Gram matrix, the
 *   Cholesky, the final pass) stays FP64.  Only R0's quality as a preconditioner changes
 *   (Section 5 needs S2 S1 to be an embedding and R0 backward stable): the rounding error of the
 *   sketch is about u32 kappa(V) relative to its smallest singular value, so kappa(Q0) grows like
 *   u32 kappa(V) once kappa(V) exceeds about 1/u32 = 1.7e7; combine with RCQR_FLAG_REORTH there.
 * RCQR_FLAG_GEMM_BF16 (requires RCQR_FLAG_SKETCH_FP32): the Gaussian product's operands are
 *   rounded to BF16 (FP32 accumulation), a relative perturbation of about 2^-9 of W1 and S2.
 * RCQR_FLAG_REORTH: one more Cholesky QR after the first: Rc = R1 R0, Q1 = V Rc^{-1} by row-wise
 *   substitution, R2 = chol(Q1^T Q1), Q = Q1 R2^{-1}, R = R2 Rc (one more read of V).  Needed when
 *   kappa(Q0) is far from 1, that is with the single-precision sketch at large kappa(V).
 * RCQR_FLAG_SKETCH_AT_PLAN: the CountSketch S1 is generated once, by rcqr_plan (enqueued on the
 *   plan's stream), instead of in every factorization: its bucket index (each row's bucket and
 *   sign, the rows of every bucket in ascending order) depends only on m, s1 and the seed, and
 *   stays in the workspace.  The experiments of Section 6.1 build S1 explicitly and leave its
 *   generation out of their timings; with this flag a plan's factorizations are timed the same
 *   way.  Results are bitwise those of a plan without the flag.  (No effect when s1 n is small
 *   enough for the LDS CountSketch, which hashes rows as it reads them.)  Not for batches.
 */
#define RCQR_FLAG_SKETCH_FP32 1u
#define RCQR_FLAG_GEMM_BF16 2u
#define RCQR_FLAG_REORTH 4u
#define RCQR_FLAG_SKETCH_AT_PLAN 8u

/* Bytes of device workspace a plan of this shape needs (0 if the shape or the flags are
 * invalid; the flags do not change the size).  It holds the small intermediates of Algorithm 1
 * (W1 = S1 V of s1 x n, W = S2 W1 of s2 x n, R0) and Algorithm 2 (G, R1), the partial sums of
 * the multi-workgroup passes, the CountSketch bucket index (about 8 bytes per row of V when
 * s1 n exceeds the LDS copies) and the status word; never a copy of V or Q0. */
size_t rcqr_workspace_bytes(int64_t m, int64_t n, int64_t s1, int64_t s2, uint32_t flags);

/*
 * Create a plan for V of m x n with CountSketch size s1 and Gaussian sketch size s2
 * (Algorithm 1's S1 of s1 x m and S2 of s2 x s1).  Requires 1 <= n <= 128, n <= m,
 * n <= s2 <= s1, s1 < 2^31, m < 2^31; s1 > m is accepted (the sketch is then not
 * compressive but still a CountSketch).  `stream` is a hipStream_t (NULL = default stream).
 * The workspace must stay valid until rcqr_destroy().  flags: RCQR_FLAG_* above (unknown bits,
 * or RCQR_FLAG_GEMM_BF16 without RCQR_FLAG_SKETCH_FP32, give RCQR_E_INVALID); they apply to
 * rcqr_factor only.
 */
rcqr_status_t rcqr_plan(rcqr_plan_t* plan, int64_t m, int64_t n, int64_t s1, int64_t s2, uint64_t seed,
                        uint32_t flags, void* d_workspace, size_t workspace_bytes, void* stream);

/*
 * Algorithm 3 (rand_cholQR): W = S2 (S1 V); R0 = Householder R of W (Algorithm 1); Q0 = V R0^{-1}
 * by row-wise substitution; G = Q0^T Q0; R1 = chol(G) (Algorithm 2); Q = Q0 R1^{-1};
 * R = R1 R0.  Asynchronous on the plan's stream.  In place (d_Q == d_V) is supported except
 * for a plan with RCQR_FLAG_REORTH and more than 64 columns, which returns RCQR_E_INVALID
 * (that path stores Q0 in Q and then reads V a second time).
 */
rcqr_status_t rcqr_factor(rcqr_plan_t plan, const double* d_V, int64_t ldv, double* d_Q, int64_t ldq,
                          double* d_R, int64_t ldr);

/*
 * Algorithm 4 (cholQR2) on the same plan and workspace, the comparator of Section 6: two
 * passes of Cholesky QR, R = R1 R0.  Fails with RCQR_E_CHOL once kappa(V) is beyond about
 * u^{-1/2} (Section 6.3).  Asynchronous on the plan's stream.
 */
rcqr_status_t rcqr_cholqr2(rcqr_plan_t plan, const double* d_V, int64_t ldv, double* d_Q, int64_t ldq,
                           double* d_R, int64_t ldr);

/*
 * Shifted CholeskyQR3, the other comparator of Section 6 (cited in Section 1 as stable up to
 * kappa(V) of about u^{-1}): Ra = chol(V^T V + s I) with s = 11 (m n + n (n + 1)) u ||V||_F^2,
 * u = 2^-52; Qa = V Ra^{-1}; then cholQR2 of Qa (Algorithm 4); R = Rc Rb Ra.  Qa is stored in
 * d_Q (so V is read twice and Q written twice); d_Q may alias d_V with ldq == ldv.
 * Same arguments, errors and stream semantics as rcqr_factor; a failing Cholesky reports
 * RCQR_E_CHOL through rcqr_info.
 */
rcqr_status_t rcqr_scholqr3(rcqr_plan_t plan, const double* d_V, int64_t ldv, double* d_Q, int64_t ldq,
                            double* d_R, int64_t ldr);

/* Wait for the plan's stream and report the last factorization: *status is an rcqr_status_t
 * (RCQR_OK, RCQR_E_RANK or RCQR_E_CHOL), *column the 1-based failing column or 0.  Algorithm 1
 * needs W = S2 S1 V of full column rank (the remark after Algorithm 1 in Section 4) and
 * Algorithm 2 a positive definite Gram matrix: RANK names the first column whose R0 diagonal
 * entry is zero or not finite, CHOL the first non-positive pivot of chol(G). */
rcqr_status_t rcqr_info(rcqr_plan_t plan, int32_t* status, int32_t* column);

/* Free the host-side plan (the handle rcqr_plan returned for Algorithm 3's shape and sketch
 * sizes); does not touch the caller's memory, which the caller frees after the plan's stream
 * has passed the last call that uses it. */
rcqr_status_t rcqr_destroy(rcqr_plan_t plan);

/* Static description of a status code. */
const char* rcqr_status_string(int32_t status);

/*
 * Per-phase timing.  rcqr_set_timing(plan, steps) with steps > 0 makes every rcqr_factor call
 * record HIP events on the plan's stream between its phases, into a ring of `steps` calls
 * (steps = 0 turns timing off; at most 4096).  rcqr_phase_times() waits for the stream, writes
 * the mean duration in milliseconds of up to `max` phases over the calls recorded since the
 * previous rcqr_phase_times (the last `steps` of them), resets the count and returns the phase
 * count through *count; rcqr_phase_name(i) names phase i.
 * Phases: 0 countsketch (sketch generation and W1 = S1 V), 1 gaussian (W = S2 W1),
 * 2 householder (R0), 3 trsm_gram (Q0 = V R0^{-1}, partial G), 4 cholesky (G, R1, R = R1 R0),
 * 5 reorth (the second Gram pass and Cholesky of RCQR_FLAG_REORTH; empty otherwise),
 * 6 final (Q = Q0 R1^{-1}, recomputing Q0).
 */
rcqr_status_t rcqr_set_timing(rcqr_plan_t plan, int32_t steps);
rcqr_status_t rcqr_phase_times(rcqr_plan_t plan, float* ms, int32_t max, int32_t* count);
const char* rcqr_phase_name(int32_t phase);

/*
 * Launch tuning.  Two choices change how a factorization is launched but never its result
 * (Q and R are bitwise the same for every setting):
 *   final_mode  RCQR_FINAL_RECOMPUTE (default): the final pass recomputes Q0 = V R0^{-1} from V
 *               (32 m n bytes in all); RCQR_FINAL_MATERIALIZE: the Gram pass stores Q0 in Q and
 *               the final pass applies R1^{-1} to it in place (40 m n bytes, no second
 *               substitution).  Only up to 64 columns and without RCQR_FLAG_REORTH; otherwise
 *               ignored.
 *   grid_mult   cap of the multi-row passes' grids, in workgroups per compute unit (1 .. 8,
 *               default 2).
 * rcqr_tune() times every combination (final_mode x grid_mult in {1, 2, 4}) on the caller's V
 * with `reps` factorizations each (after one warm-up) on the plan's stream, keeps the fastest in
 * the plan and returns its mean milliseconds through *best_ms (may be NULL).  It synchronises the
 * stream; Q must not alias V.  rcqr_set_tuning / rcqr_get_tuning store and read the choice
 * (for callers that cache it per shape).
 */
#define RCQR_FINAL_RECOMPUTE 0
#define RCQR_FINAL_MATERIALIZE 1
rcqr_status_t rcqr_tune(rcqr_plan_t plan, const double* d_V, int64_t ldv, double* d_Q, int64_t ldq, double* d_R,
                        int64_t ldr, int32_t reps, float* best_ms);
rcqr_status_t rcqr_set_tuning(rcqr_plan_t plan, int32_t final_mode, int32_t grid_mult);
rcqr_status_t rcqr_get_tuning(rcqr_plan_t plan, int32_t* final_mode, int32_t* grid_mult);

/*
 * HIP graphs.  rcqr_graph_create() records one factorization of the given V into Q and R
 * (method RCQR_METHOD_RAND_CHOLQR = rcqr_factor, RCQR_METHOD_CHOLQR2, RCQR_METHOD_SCHOLQR3) by
 * stream capture on the plan's stream and instantiates it; nothing runs during the capture.
 * rcqr_graph_launch() replays it on the plan's stream: one launch instead of about fifteen, for
 * callers that factor same-shaped inputs from fixed buffers (small m, where launches dominate).
 * The plan must have been created with a stream other than the legacy default stream
 * (RCQR_E_INVALID otherwise) and with timing off or on (events are not recorded in the graph).
 * The plan, its workspace, V, Q and R must stay valid while the graph is used; destroy the graph
 * before the plan.  Replays and eager calls on the same plan share its workspace: issue them on
 * the plan's stream only (they are then ordered).  A failure is reported by rcqr_info() as for
 * an eager call.
 */
typedef struct rcqr_graph_s* rcqr_graph_t;
#define RCQR_METHOD_RAND_CHOLQR 0
#define RCQR_METHOD_CHOLQR2 1
#define RCQR_METHOD_SCHOLQR3 2
rcqr_status_t rcqr_graph_create(rcqr_plan_t plan, int32_t method, const double* d_V, int64_t ldv, double* d_Q,
                                int64_t ldq, double* d_R, int64_t ldr, rcqr_graph_t* graph);
rcqr_status_t rcqr_graph_launch(rcqr_graph_t graph);
rcqr_status_t rcqr_graph_destroy(rcqr_graph_t graph);

/*
 * Batches of factorizations.  rcqr_batch_create() records `count` factorizations, each on its own
 * plan (any m, n, s1, s2, seed and flags) with its own V, Q and R (arrays of `count` entries):
 * each is captured as a HIP graph on its plan's stream.  rcqr_batch_launch() launches every
 * member's graph on its own stream, forked from the first plan's stream and joined back to it
 * with events, so the members run concurrently: one factorization's single-workgroup steps (the
 * Householder QR of the sketch, the Cholesky) overlap with the others' work, and the host issues
 * one graph launch per member instead of about fifteen kernel launches.  The batch is complete
 * when the first plan's stream reaches the launch.  (One graph holding every member as a
 * parallel branch was measured to run its branches one after another on this ROCm, hence one
 * graph per member.)  Requirements as for rcqr_graph_create on every plan (a non-default stream
 * each; distinct streams run concurrently, plans sharing a stream run one after the other).  A
 * plan may appear only once.  Each member gives bitwise the Q and R of an eager call on its plan;
 * its status is read with rcqr_info() on its plan.  Plans, workspaces and matrices must stay
 * valid while the batch exists; destroy the batch before the plans.
 * Errors: RCQR_E_INVALID (count < 1, a null pointer or array, a plan on the default stream, a
 * repeated plan, an invalid V/Q/R), RCQR_E_HIP (capture, instantiation or launch failed),
 * RCQR_E_NOMEM.
 */
typedef struct rcqr_batch_s* rcqr_batch_t;
rcqr_status_t rcqr_batch_create(int32_t count, const rcqr_plan_t* plans, int32_t method, const double* const* d_V,
                                const int64_t* ldv, double* const* d_Q, const int64_t* ldq, double* const* d_R,
                                const int64_t* ldr, rcqr_batch_t* batch);
rcqr_status_t rcqr_batch_launch(rcqr_batch_t batch);
rcqr_status_t rcqr_batch_destroy(rcqr_batch_t batch);

/*
 * Same-shaped batches in one set of launches.  rcqr_factor_batch() runs rcqr_factor (Algorithm 3)
 * on `count` matrices of the plan's shape at once: member b reads V + b * stride_v (leading
 * dimension ldv), writes Q + b * stride_q and R + b * stride_r, uses the sketch seed d_seeds[b]
 * (a device array of `count` seeds, read by the kernels; or, when d_seeds is null, the plan's
 * seed + b) and the b-th slice of the workspace, which must then hold
 * count * rcqr_workspace_bytes(m, n, s1, s2, 0) bytes (the size given to rcqr_plan).  Each
 * kernel of the factorization is launched once for the whole batch, the member being a grid
 * index, so a batch of small factorizations costs the launches of one and fills the GPU with
 * all of them.  Member b gives bitwise the Q and R of rcqr_factor on a plan with its seed.
 * Supported for plans with flags 0 and count <= 4096; otherwise RCQR_E_UNSUPPORTED.
 * Strides must keep members apart (stride_v >= m * ldv, stride_q >= m * ldq, stride_r >= n * ldr;
 * Q may be V with the same leading dimension and stride); RCQR_E_INVALID otherwise, or when the
 * workspace is too small for `count`.  Statuses: rcqr_info_member(plan, b, ...) reads member b's
 * (synchronises the plan's stream).  Timing (rcqr_set_timing) does not record batches.
 */
rcqr_status_t rcqr_factor_batch(rcqr_plan_t plan, int32_t count, const double* d_V, int64_t ldv, int64_t stride_v,
                                double* d_Q, int64_t ldq, int64_t stride_q, double* d_R, int64_t ldr, int64_t stride_r,
                                const uint64_t* d_seeds);

/*
 * Ragged batches: matrices with the plan's n, s1 and s2 but each with its own number of rows,
 * in one set of launches (Algorithm 3 on every member).  A member names its own device buffers
 * (V of m x n with leading dimension ldv, Q of m x n with ldq -- Q may be V with ldq == ldv --,
 * R of n x n with ldr), its row count n <= m <= the plan's m, and its sketch seed.
 */
typedef struct {
  const double* V;
  double* Q;
  double* R;
  int64_t m, ldv, ldq, ldr;
  uint64_t seed;
} rcqr_member_t;
/*
 * rcqr_factor_ragged() factors members[0 .. count-1] (a host array, read during the call) on the
 * plan's stream with every kernel launched once for the batch: the grids are sized for the
 * plan's m and each workgroup takes its member's rows, buffers and row-count-dependent
 * partitions (bucket-index chunks, CountSketch copies, Gram pass workgroups) from a member
 * description the call copies into the member's workspace slice (hipMemcpy2DAsync from host
 * memory; one copy of about 88 bytes per member).  Member b gives bitwise the Q and R of
 * rcqr_factor on a plan of its own shape (m_b, n, s1, s2) and seed: the partitions, and so every
 * summation order, are those of its own shape.  The workspace must hold
 * count * rcqr_workspace_bytes(plan m, n, s1, s2, 0) bytes (slice b serves member b); statuses are
 * read with rcqr_info_batch / rcqr_info_member as for rcqr_factor_batch.  Flags 0 and
 * count <= 4096 (else RCQR_E_UNSUPPORTED); RCQR_E_INVALID for a null plan or array, count < 1,
 * a workspace too small for count, or a member outside the rules above (nothing is launched then).
 */
rcqr_status_t rcqr_factor_ragged(rcqr_plan_t plan, int32_t count, const rcqr_member_t* members);
rcqr_status_t rcqr_info_member(rcqr_plan_t plan, int32_t member, int32_t* status, int32_t* column);
/* Statuses of members 0 .. count-1 into host arrays status[count], column[count] with one copy
 * (synchronises the plan's stream).  RCQR_E_INVALID for count < 1 or beyond the workspace. */
rcqr_status_t rcqr_info_batch(rcqr_plan_t plan, int32_t count, int32_t* status, int32_t* column);

/*
 * Allocation-free factorization, for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops that must not call hipMalloc, harnesses that forbid it.  Runs
 * exactly the kernels of rcqr_factor (same results, bit for bit) with the workspace taken from a
 * library-owned static device array of RCQR_STATIC_WORKSPACE_BYTES (64 MiB) instead of a plan's:
 * no plan, no hipMalloc / hipFree, no host allocation.  Each GPU the library runs on holds its own
 * copy of the array until the process ends; its device address is looked up once per device, on
 * the first call on that device (hipGetSymbolAddress, with the stream's device current).
 *   m, n, s1, s2, seed, flags: as for rcqr_plan (RCQR_FLAG_SKETCH_AT_PLAN is ignored: with no
 *   plan, the sketch is made in the call); V, Q, R: as for rcqr_factor (caller-owned device
 *   memory; Q may alias V under rcqr_factor's rule);
 *   d_info: NULL, or caller-owned device memory for two int32 that receive, in stream order, the
 *   status (RCQR_OK, RCQR_E_RANK, RCQR_E_CHOL) and the 1-based failing column, as rcqr_info reports
 *   them for a plan;
 *   stream: a hipStream_t (NULL = the default stream); the work is enqueued there, asynchronously.
 * Errors, returned synchronously before anything is launched: RCQR_E_INVALID / RCQR_E_UNSUPPORTED
 * for the arguments rcqr_plan and rcqr_factor reject; RCQR_E_SCRATCH when
 * rcqr_workspace_bytes(m, n, s1, s2, flags) exceeds RCQR_STATIC_WORKSPACE_BYTES (2,000,000 x 64 with
 * s1 = 8192, s2 = 256 needs 48.8 MiB and fits; 128 columns with s1 = 32768 need more than 72 MiB
 * and do not); RCQR_E_HIP.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (two host threads,
 * or two streams whose work is not ordered) race and give wrong results; calls ordered on one
 * stream, or on streams ordered by events, are safe.  The array keeps the last call's contents;
 * everything a call reads from it is written earlier in the same call.
 */
#define RCQR_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
rcqr_status_t rcqr_factor_static(int64_t m, int64_t n, int64_t s1, int64_t s2, uint64_t seed, uint32_t flags,
                                 const double* d_V, int64_t ldv, double* d_Q, int64_t ldq, double* d_R, int64_t ldr,
                                 int32_t* d_info, void* stream);

/* ------------------------------------------------------------------------------------------
 * Inspection entry points (same library; used by tests, never on a timed path).
 * ------------------------------------------------------------------------------------------ */

/* CountSketch bucket h(i) and sign (+1/-1) of rows row0 .. row0+count-1 under the plan's seed
 * and s1 (Section 3's S1).  d_bucket: count int32, d_sign: count int8, device memory. */
rcqr_status_t rcqr_sketch_hash(rcqr_plan_t plan, int64_t row0, int64_t count, int32_t* d_bucket, int8_t* d_sign);

/* Entries S2[j0 .. j0+nj-1, k0 .. k0+nk-1] of the Gaussian sketch (Section 3), row-major with
 * leading dimension nk, into device memory d_out (nj * nk doubles). */
rcqr_status_t rcqr_gaussian_block(rcqr_plan_t plan, int64_t j0, int64_t nj, int64_t k0, int64_t nk, double* d_out);

/* Copy the intermediates of the last rcqr_factor call from the workspace (device to device),
 * in the notation of Algorithms 1 and 2: W1 = S1 V (s1 x n), W = S2 W1 (s2 x n), R0 = the
 * Householder R of W (n x n), G = Q0^T Q0 (n x n, upper triangle; lower set to zero),
 * R1 = chol(G) (n x n).  Any pointer may be NULL; the caller owns the destinations (row-major,
 * leading dimension = number of columns).  With RCQR_FLAG_SKETCH_FP32, W1 and W are the FP32
 * values widened to FP64; with RCQR_FLAG_REORTH, G and R1 are those of the second pass.
 * Asynchronous on the plan's stream; RCQR_E_INVALID for a null plan. */
rcqr_status_t rcqr_intermediates(rcqr_plan_t plan, double* d_W1, double* d_W, double* d_R0, double* d_G,
                                 double* d_R1);

/* Q0 = V R0^{-1} (Algorithm 1, step 3, by the row-wise substitution Section 5.2 analyses) as
 * computed inside the Gram pass (d_Q0_gram) and as recomputed inside the final pass
 * (d_Q0_final), using R0 of the last rcqr_factor call on the same V.  Up to 64 columns these are
 * the kernels rcqr_factor launches: the Gram pass in the variant that stores Q0 (the
 * materialising launch choice) and the final pass given R1 = I, whose product by the identity
 * returns its recomputed Q0 unchanged.  The recompute scheme relies on the two being bitwise
 * identical: the Gram matrix that gave R1 must be the Gram matrix of the Q0 that R1 is applied
 * to.  65..128 columns store Q0 and do not recompute it (both outputs come from the same solve).
 * Both outputs m x n with leading dimension ldq, caller-owned device memory.  Overwrites the
 * plan's Gram partials; asynchronous on the plan's stream. */
rcqr_status_t rcqr_q0_twice(rcqr_plan_t plan, const double* d_V, int64_t ldv, double* d_Q0_gram,
                            double* d_Q0_final, int64_t ldq);

#ifdef __cplusplus
}
#endif

#endif /* RCQR_H */
