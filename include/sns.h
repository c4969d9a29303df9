/*
 * sns.h - C ABI of libsns: sketch-and-solve least squares on MI355X (gfx950).
 *
 * The library solves the overdetermined least-squares problem
 *     min_x || A x - b ||_2,   A in R^{m x n}, b in R^m            (Sec. 1.3, eq. 1)
 * by the sketch-and-solve paradigm of Sec. 1.2: draw a sketch S in R^{d x m}
 * (m >> n, n <= d), form SA and Sb, and solve the reduced problem
 * min || SA x - Sb || (Sec. 1.3) by Householder QR of [SA | Sb] and a
 * triangular solve.  Optionally the answer is refined with LSQR on the
 * right-preconditioned operator A R^{-1} (the sketch-and-precondition solver
 * SAP-SAS of Sec. 2.1).
 *
 * Conventions for every entry point:
 *   - All matrix/vector pointers are DEVICE pointers (memory of the current
 *     HIP device) unless stated otherwise.  The caller owns every buffer,
 *     including the workspace; the library never allocates or frees device
 *     memory on these paths and keeps no pointer after the call returns
 *     (serving requests excepted, see sns_serve_submit).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it in order; calls return without waiting
 *     unless documented.  Results are valid after the stream is synchronised.
 *   - Dense matrices are row-major with leading dimension ld >= n (elements).
 *   - Argument errors are detected on the host before anything is enqueued and
 *     returned immediately; nothing is written in that case.
 *   - Numerical outcomes (rank deficiency, non-finite values, non-convergence)
 *     are reported through sns_info, written on the stream.
 *   - Results are deterministic: the same inputs, seed and sizes give the same
 *     bits, whatever else runs on the device.  No floating-point atomics are
 *     used anywhere.
 *   - Size limits: m < 2^31; CountSketch d <= 16384; QR d <= 8192 and
 *     n <= 4096; LSQR refinement n <= 2048 with 16-byte aligned rows
 *     (values pointer and ld * element size multiples of 16).
 */
#ifndef SNS_H
#define SNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SNS_OK = 0,
  SNS_ERR_INVALID_ARG = 1,   /* null pointer, bad enum, bad option value */
  SNS_ERR_SHAPE = 2,         /* violates n >= 1, n <= d <= m, ld >= n, or a size limit */
  SNS_ERR_DTYPE = 3,         /* dtype / layout / sketch combination not supported */
  SNS_ERR_RANK_DEFICIENT = 4,/* |R_jj| <= 10 n u64 max_i |R_ii| for some j */
  SNS_ERR_NOT_CONVERGED = 5, /* LSQR reached max_iters before the stop rule held */
  SNS_ERR_NUMERICAL = 6,     /* non-finite value met in a norm or the factorisation */
  SNS_ERR_OUT_OF_MEMORY = 7, /* workspace / serving pool too small */
  SNS_ERR_QUEUE_FULL = 8,    /* serving queue full */
  SNS_ERR_NOT_READY = 9,     /* serving request still in flight */
  SNS_ERR_HIP = 10           /* a HIP runtime call failed */
} sns_status;

typedef enum { SNS_F32 = 0, SNS_F64 = 1 } sns_dtype;
typedef enum { SNS_DENSE_ROWMAJOR = 0, SNS_CSR = 1 } sns_layout;

/* Sketch operators (Sec. 1.2.1 and 1.2.2). */
typedef enum {
  SNS_SKETCH_COUNT = 0,       /* Clarkson-Woodruff CountSketch: one +-1 per column of S */
  SNS_SKETCH_GAUSSIAN = 1,    /* dense Gaussian sketch, bf16 inputs, fp32 accumulation */
  SNS_SKETCH_SPARSE_SIGN = 2, /* sparse sign embedding: zeta +-1 entries per column of S */
  SNS_SKETCH_HADAMARD = 3     /* subsampled randomized Hadamard transform */
} sns_sketch_kind;

/* A tall matrix.  Dense: values (m x n row-major, leading dimension ld).
 * CSR: row_ptr[m+1] (int32, nondecreasing, row_ptr[0] = 0, row_ptr[m] = nnz),
 * col_idx[nnz] (int32, each in [0, n), no repeated column within a row) and
 * values[nnz], all in device memory (col_idx and values may be NULL when
 * nnz = 0); ld is ignored.  The library does not
 * read these arrays on the host: entries with a column outside [0, n) are
 * ignored, and row_ptr values outside [0, nnz] are undefined behaviour.
 * `values` has the element type `dtype`. */
typedef struct {
  int64_t m, n;
  sns_dtype dtype;
  sns_layout layout;
  const void* values;
  int64_t ld;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  int64_t nnz;
} sns_matrix;

/* The sketch S in R^{d x m}, drawn from `seed`.
 * CountSketch (Sec. 1.2.2): S[h(i), i] = s(i), every other entry 0, where
 *   (w0,w1,w2,w3) = Philox4x32-10(counter (j mod 2^32, j >> 32, 0, 0),
 *                                 key (seed mod 2^32, seed >> 32)), j = i >> 1,
 *   lane = i & 1, h(i) = (w_{2 lane} * d) >> 32, s(i) = +1 if the top bit of
 *   w_{2 lane + 1} is clear, else -1.
 * Gaussian (Sec. 1.2.1): S = d^{-1/2} G with G[k, i] = T[q], q the byte
 *   (i & 15) of Philox4x32-10(counter (j mod 2^32, j >> 32, k, 1), key as
 *   above), j = i >> 4, T[q] = bf16(Phi^{-1}((q + 1/2) / 256)).  The product
 *   uses bf16(A) and bf16(b) (round to nearest even).
 * Sparse sign embedding (the sparse family of Sec. 1.2.2 with `zeta` nonzeros
 *   per column): S = sum over k = 0 .. zeta-1 of CountSketch matrices S_k,
 *   where S_k uses the CountSketch rule above with counter word 2 set to k
 *   (so zeta = 1 is the CountSketch); entries +-1 without scale, and two
 *   entries of a column that land in one row add.  Dense A only; zeta in
 *   1..64 with zeta * m < 2^31.  `zeta` is ignored by the other kinds.
 * Hadamard (Sec. 1.2.1, SRHT): A is padded with zero rows to m' = 2^L >= m;
 *   S = d^{-1/2} P H D with D = diag(s(i)), H[r, i] = (-1)^popcount(r & i),
 *   and P selecting rows r_0 .. r_{d-1} of H D A uniformly with replacement:
 *   s(i) = -1 iff the top bit of word (i & 3) of Philox4x32-10(counter
 *   (i >> 2 mod 2^32, i >> 34, 0, 2)) is set; r_k = (w * m') >> 32 with w word
 *   (k & 3) of Philox4x32-10(counter (k >> 2 mod 2^32, k >> 34, 0, 3)).  Dense
 *   fp32/fp64 A with m <= 2^26; the workspace holds m' x (n + 1) values. */
typedef struct {
  sns_sketch_kind kind;
  int64_t d;
  uint64_t seed;
  int32_t zeta;
} sns_sketch;

typedef struct {
  int refine;      /* 0: plain sketch-and-solve; 1: SAP-SAS (LSQR on A R^{-1} applied
                      implicitly); 2: SAA-SAS (Y = A R^{-1} formed, LSQR on Y; sns_lstsq only) */
  int max_iters;   /* LSQR iteration cap (refine = 1 or 2) */
  double rtol;     /* stop when ||Abar^T r|| / ||r|| <= rtol (1 - sqrt(n/d));
                      rtol = 0 runs exactly max_iters iterations */
  int accum_fp64;  /* 1: accumulate the dense CountSketch in fp64 (fp32 inputs);
                      the CSR sketch always accumulates in fp64 */
} sns_solve_opts;

typedef struct {
  int32_t status;          /* an sns_status */
  int32_t iters;           /* LSQR iterations run */
  double rel_resid_est;    /* ||Abar^T r|| / (||r|| (1 - sqrt(n/d))) at exit; 0 if refine = 0 */
  double sketch_resid;     /* ||(Q^T Sb)[n:]||, the sketched residual norm */
} sns_info;

/* Human-readable name of a status code (static string). */
const char* sns_status_string(int status);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int sns_version(void);

/* CountSketch hash of rows i0 .. i0+count-1 (definition at sns_sketch).
 * h: device uint32[count], s: device int8[count] (either may be NULL).
 * Errors: SNS_ERR_SHAPE if d < 1 or d >= 2^32, count < 0. */
sns_status sns_hash(uint64_t seed, int64_t d, int64_t i0, int64_t count,
                    uint32_t* h, int8_t* s, void* stream);

/* The 256-entry Gaussian table T used on the device, as bf16 bit patterns,
 * copied to the HOST array out[256].  Synchronous. */
sns_status sns_gaussian_table(uint16_t* out);

/* Workspace bytes sns_sketch_apply needs for this sketch and matrix. */
sns_status sns_sketch_workspace_size(const sns_sketch* sk, const sns_matrix* A, size_t* bytes);

/* SA = S A and Sb = S b (step 2 of Sec. 1.2).
 * SA: device d x n row-major (leading dimension n) of A's dtype, fully
 * overwritten (empty buckets give zero rows).  b and Sb may both be NULL;
 * otherwise b has m entries and Sb d entries of A's dtype.
 * CountSketch: one deterministic pass over [A | b]; rows are grouped by bucket
 * with a stable counting sort and each bucket is reduced in a fixed order.
 * accum_fp64 (from opts, may be NULL) selects fp64 accumulation for fp32 A.
 * CSR A (CountSketch only): the rows that hold nonzeros are compacted and
 * sorted by bucket the same way, each bucket adds its rows' nonzeros in
 * ascending row order; Sb is formed over all m rows.  Requires n <= 4096.
 * Gaussian: fp32 dense A only (SNS_ERR_DTYPE otherwise); computed on the
 * matrix cores as bf16 x bf16 products with fp32 accumulation.
 * Errors: SNS_ERR_INVALID_ARG (NULL sk/A/SA/workspace, b and Sb not both set
 * or both NULL), SNS_ERR_SHAPE (n < 1, d < 1, m < 1, ld < n, m >= 2^31,
 * d > 16384, d < n, d > m, CSR with n > 4096), SNS_ERR_OUT_OF_MEMORY
 * (ws_bytes too small). */
sns_status sns_sketch_apply(const sns_sketch* sk, const sns_matrix* A, const void* b,
                            void* SA, void* Sb, const sns_solve_opts* opts,
                            void* workspace, size_t ws_bytes, void* stream);

/* Householder QR of the augmented d x (n+1) matrix [SA | Sb] (fp64) and the
 * triangular solve R x0 = c with c = (Q^T Sb)[:n] (step 3 of Sec. 1.2).
 * SA: device d x n row-major (ld_sa >= n) and Sb: device d, both of `dtype`.
 * Outputs: x0 device fp64[n]; R (may be NULL) device fp64 n x n row-major,
 * upper triangle with the LAPACK sign convention (beta = -sign(alpha)||x||),
 * strictly lower part zero; info (host pointer, may be NULL) receives status
 * (SNS_ERR_RANK_DEFICIENT if |R_jj| <= 10 n u64 max|R_ii|) and sketch_resid.
 * Requires n <= d.  `info` is written by the stream: synchronise before
 * reading it. */
sns_status sns_qr_solve_workspace_size(int64_t d, int64_t n, size_t* bytes);
sns_status sns_qr_solve(int64_t d, int64_t n, sns_dtype dtype, const void* SA, int64_t ld_sa,
                        const void* Sb, double* x0, double* R, sns_info* info,
                        void* workspace, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * QR solve as sns_qr_solve, same arguments and outputs, with the workspace in
 * a static 64 MiB device array inside the library instead of caller memory.
 * Each device the library runs on holds its own array until the process
 * ends; its address is looked up on the first call on a device (with that
 * device current).  No device or host memory is allocated by the call.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (two streams, or two host threads) race and give undefined
 * results; serialise them.  Errors: as sns_qr_solve (argument checks first),
 * and SNS_ERR_OUT_OF_MEMORY when the workspace sns_qr_solve_workspace_size
 * reports for (d, n) exceeds 64 MiB (for example d = 4096 with n = 1000 fits,
 * d = 8192 with n = 1000 does not); nothing is enqueued then. */
sns_status sns_qr_solve_noalloc(int64_t d, int64_t n, sns_dtype dtype, const void* SA,
                                int64_t ld_sa, const void* Sb, double* x0, double* R,
                                sns_info* info, void* stream);

/* Workspace bytes sns_lstsq needs. */
sns_status sns_lstsq_workspace_size(const sns_sketch* sk, const sns_matrix* A,
                                    const sns_solve_opts* opts, size_t* bytes);

/* Solve min ||A x - b|| (Sec. 1.3): sketch (Sec. 1.2), QR + triangular solve,
 * and with opts->refine = 1 the SAP-SAS refinement (Sec. 2.1): LSQR on
 * A R^{-1} from r0 = b - A x0, x = x0 + R^{-1} dy.  Every product with A
 * accumulates in fp64; n-vectors are fp64; m-vectors are stored in A's dtype.
 * b: device, m entries of A's dtype.  x: device fp64[n].
 * info: HOST pointer (pinned memory recommended) or NULL; written on the
 * stream, valid after synchronising it.
 * With opts->refine = 2, the SAA-SAS variant named beside it in Sec. 2.1:
 * Y = A R^{-1} is formed once (fp64 products, stored in A's dtype inside the
 * workspace, m x n) and LSQR runs on Y from the same r0; x = x0 + R^{-1} dy.
 * In exact arithmetic both variants give the same iterates; SAA costs one
 * extra pass that reads A and writes Y plus about m n^2 multiply-adds, and
 * its workspace holds Y.
 * A may be CSR with refine = 0 (plain sketch-and-solve); refinement streams
 * dense rows and returns SNS_ERR_DTYPE for CSR.
 * With refinement and rtol > 0 the call holds the host thread while the
 * iterations run: the device posts its stop flag to pinned host memory after
 * each iteration, the host keeps at most two iterations enqueued ahead of the
 * last flag it has read, and returns once it has enqueued the final update
 * (the stream then completes the solve).  With rtol = 0, or while the stream
 * is being captured, all max_iters + 1 iterations are enqueued at once and the
 * call returns without waiting.
 * Errors: as sns_sketch_apply, plus SNS_ERR_INVALID_ARG for refine outside
 * 0..2, max_iters < 0 or rtol < 0. */
sns_status sns_lstsq(const sns_sketch* sk, const sns_matrix* A, const void* b, double* x,
                     const sns_solve_opts* opts, void* workspace, size_t ws_bytes,
                     sns_info* info, void* stream);

/* One problem of a batch (sns_lstsq_batched). */
typedef struct {
  sns_sketch sketch;    /* CountSketch or sparse sign embedding (other kinds: SNS_ERR_DTYPE) */
  sns_matrix A;         /* dense row-major */
  const void* b;        /* device, m entries of A's dtype */
  double* x;            /* device fp64[n], the answer */
  sns_solve_opts opts;  /* as for sns_lstsq, refine 0 or 1 (2: SNS_ERR_INVALID_ARG) */
} sns_problem;

/* Workspace bytes sns_lstsq_batched needs for these problems. */
sns_status sns_lstsq_batched_workspace_size(const sns_problem* probs, int count, size_t* bytes);

/* Solve `count` independent least-squares problems of uneven shapes together
 * (Secs. 1.2, 1.3, 2.1 per problem): every kernel of the sketch, the QR and
 * the refinement runs once for the whole batch, each work-group taking a
 * piece of one problem.  Each problem's arithmetic is the one sns_lstsq does
 * for it alone, so x and info are bit-identical to a solo sns_lstsq call.
 * The refinement iterations of all problems advance together; a problem that
 * met its stop rule skips the remaining iterations.  With use_graph != 0 a
 * chunk of refinement iterations is captured once into a HIP graph and
 * replayed until every problem has stopped.
 * probs: HOST array of count problems, all of the same dtype, CountSketch,
 * dense A (same limits as sns_lstsq).  infos: HOST array of count sns_info
 * (pinned memory recommended) or NULL, written on the stream.  The call
 * returns after the last refinement chunk has been enqueued (it waits on the
 * stream between chunks to read the number of problems still running).
 * Errors: as sns_lstsq for any problem; SNS_ERR_DTYPE if dtypes differ or a
 * problem is not a dense CountSketch problem; SNS_ERR_INVALID_ARG if count <
 * 1 or probs is NULL. */
sns_status sns_lstsq_batched(const sns_problem* probs, int count, void* workspace,
                             size_t ws_bytes, sns_info* infos, int use_graph, void* stream);

/* The set-up of a small problem (CountSketch, dense A, d <= 256, n <= 64,
 * m (n + 1) <= 2^21):
 * sketch of [A | b] (Sec. 1.2 steps 1-2), Householder QR of [SA | Sb] and
 * x0 = R^{-1} c (step 3), runs in one persistent launch shared by every such
 * problem of a sns_lstsq call, a batch or a server round: a fixed grid claims
 * row chunks of all of them from a device queue, and the work-group that
 * completes a problem's sketch factors it in registers.  Larger problems take
 * the blocked path (bucket sort, gather, panel QR).  The fused form is off by
 * default (on one MI355X the blocked path sets these problems up faster);
 * sns_fused_enable(1) turns it on for every later call and server set-up,
 * sns_fused_enable(0) back off.  Results of the two forms differ in rounding,
 * and so do workspace sizes: query them after switching.  The switch is
 * process-wide and must not change while calls or servers are in flight. */
void sns_fused_enable(int on);
int sns_fused_enabled(void);

/* ------------------------------------------------------------- serving --
 * A server solves submitted problems with continuous batching.  A scheduler
 * thread owns two HIP streams and works in rounds: it admits waiting requests
 * in arrival order while a slot is free and the request's workspace fits in
 * the pool (admission by device-memory footprint), sets the admitted ones up
 * together on the second stream (sketch, QR, X = R^{-1}; one batched launch
 * per kernel) while the first advances every request set up in an earlier
 * round by a chunk of refinement iterations (one batched launch per kernel),
 * and retires the requests whose stop rule has fired.  A request joins the
 * iterating batch in the round after its set-up, behind an event, so its
 * work shares launches with the running ones.  Each request's arithmetic is
 * the one sns_lstsq does for it alone: x and info are bit-identical to a
 * solo call whatever else is in flight. */
typedef struct sns_server sns_server;

typedef struct {
  void* pool;          /* device memory for request workspaces (caller-owned) */
  size_t pool_bytes;
  sns_dtype dtype;     /* element type of every request's A and b */
  int max_slots;       /* requests admitted at once, 1..4096 */
  int queue_capacity;  /* requests waiting for admission, >= 1 */
  int chunk_iters;     /* refinement iterations per round, >= 1 */
} sns_serve_config;

typedef struct {
  uint64_t submitted, completed;
  double p50_ms, p99_ms, mean_ms;  /* latency from submit to result, completed requests */
  double span_s;                   /* first submit to last completion */
  size_t peak_pool_bytes;          /* most pool bytes in use at once */
  int peak_slots;                  /* most requests admitted at once */
  uint64_t rounds;                 /* scheduling rounds run */
} sns_serve_stats;

/* Create a server on the current device.  Errors: SNS_ERR_INVALID_ARG (NULL
 * arguments or a field out of range), SNS_ERR_OUT_OF_MEMORY (pool too small
 * for the server's own tables), SNS_ERR_HIP. */
sns_status sns_serve_create(const sns_serve_config* cfg, sns_server** out);

/* Queue one problem (same rules as sns_lstsq: dense CountSketch, A, b and x in
 * device memory; they must stay valid until the request completes).  The
 * server's streams wait on no caller stream: every write to A, b or x that
 * the caller enqueued must be complete when this call is made (synchronise
 * the stream it went to first), and x must not be read before sns_serve_poll
 * or sns_serve_wait reports the request done.  *ticket identifies the request.  Errors: as sns_lstsq
 * (checked now), SNS_ERR_DTYPE (dtype differs from the server's),
 * SNS_ERR_OUT_OF_MEMORY (workspace larger than the pool), SNS_ERR_QUEUE_FULL. */
sns_status sns_serve_submit(sns_server* srv, const sns_problem* req, uint64_t* ticket);

/* SNS_OK and *out filled (host pointer, may be NULL) once the request has
 * completed (x written); the ticket is then released.  SNS_ERR_NOT_READY while
 * it runs; SNS_ERR_INVALID_ARG for an unknown ticket. */
sns_status sns_serve_poll(sns_server* srv, uint64_t ticket, sns_info* out);

/* As sns_serve_poll, but blocks until the request has completed. */
sns_status sns_serve_wait(sns_server* srv, uint64_t ticket, sns_info* out);

/* Counters and latency percentiles so far (host pointer). */
sns_status sns_serve_stats_get(sns_server* srv, sns_serve_stats* out);

/* Completes every submitted request, stops the scheduler and frees the
 * server (not the pool). */
sns_status sns_serve_destroy(sns_server* srv);

/* ------------------------------------------------------------ autotuner --
 * The fused refinement pass has launch-shape parameters (lanes per row,
 * 16-byte chunks per lane, work-groups, rows per step, waves per
 * work-group).  The plan for a
 * problem is taken from a tuning table entry matching its dtype, n and m
 * range; without one, a built-in rule is used.  The tuner times every valid
 * candidate on the caller's matrix with HIP events and reports the fastest;
 * a driver (paper_2409_14309_amd/autotune.py) sweeps shapes and saves the
 * table.  A plan fixes the order of the per-group partial sums, so results
 * are reproducible for a given table. */
typedef struct {
  int dtype;             /* sns_dtype */
  int n;
  int64_t m_lo, m_hi;    /* rows covered, inclusive */
  int lpr, nch, grid, unroll;
  double us;             /* measured time of one pass (informational) */
  int waves;             /* waves per work-group: 4 or 8 (0 in sns_tune_set: 4) */
} sns_tune_entry;

/* Workspace for sns_tune_pass on A. */
sns_status sns_tune_workspace_size(const sns_matrix* A, size_t* bytes);
/* Time every candidate plan of the pass on A (dense, device data; `reps`
 * timed launches each after one warm-up) and write the fastest to *best
 * (m_lo = m_hi = A->m).  Synchronous. */
sns_status sns_tune_pass(const sns_matrix* A, int reps, void* workspace, size_t ws_bytes,
                         sns_tune_entry* best, void* stream);
/* The CountSketch gather (dense A, Sec. 1.2 step 1) has two launch-shape
 * parameters: lanes per row (4..64, a power of two; one row-slot of that many
 * lanes streams a tile of lpr x 16 bytes of each row) and segments per bucket
 * (1..64, a power of two; each segment keeps at least 256 rows, and more than
 * one segment adds a fixed-order reduction of the partial sketches).  An
 * entry matches a problem by dtype, n, d and an m range.  The blocked QR
 * (Sec. 1.2 step 3) has a panel configuration (0..4: rows per thread, panel
 * width and threads of the panel work-group, holding d <= 512, 1024, 2048,
 * 4096 and 8192 rows) and the width of the trailing update's column groups
 * (1 or 2 columns reduced together; a work-group takes several groups in
 * turn); an entry matches by d range and n range.  Both change the order of the sums, so a
 * result is reproducible for a given table. */
typedef struct {
  int dtype;             /* sns_dtype */
  int n, d;
  int64_t m_lo, m_hi;    /* rows covered, inclusive */
  int lpr, nseg;
  double us;             /* measured time of one gather (informational) */
} sns_tune_gather_entry;

typedef struct {
  int d_lo, d_hi;        /* sketch rows covered, inclusive */
  int n_lo, n_hi;        /* columns covered, inclusive */
  int cfg, cb;
  double us;             /* measured time of one factorisation (informational) */
} sns_tune_qr_entry;

/* Workspace for sns_tune_gather on A with d buckets (dense A, n <= d <= m,
 * d <= 16384, n <= 4096). */
sns_status sns_tune_gather_workspace_size(const sns_matrix* A, int64_t d, size_t* bytes);
/* Bucket-sort A's rows once (seed as in sns_sketch; b: m device values of
 * A's dtype), then time every candidate gather shape (`reps` timed launches
 * each after one warm-up; candidates whose column tile is more than twice n
 * are skipped) and write the fastest to *best (m_lo = m_hi = A->m).
 * Synchronous. */
sns_status sns_tune_gather(const sns_matrix* A, const void* b, int64_t d, uint64_t seed, int reps,
                           void* workspace, size_t ws_bytes, sns_tune_gather_entry* best,
                           void* stream);
/* Workspace for sns_tune_qr of a d x n sketch (1 <= n <= d <= 8192, n <= 4096). */
sns_status sns_tune_qr_workspace_size(int64_t d, int64_t n, size_t* bytes);
/* Time the blocked QR and solve of [SA | Sb] (device, row-major SA d x n with
 * leading dimension n, Sb d; dtype SNS_F32 or SNS_F64) under every panel
 * configuration that holds d and both trailing widths, and write the fastest
 * to *best (d_lo = d_hi = d, n_lo = n_hi = n).  Synchronous. */
sns_status sns_tune_qr(int dtype, int64_t d, int64_t n, const void* SA, const void* Sb, int reps,
                       void* workspace, size_t ws_bytes, sns_tune_qr_entry* best, void* stream);

/* The table: add or replace the entry with the same key (pass: dtype, n,
 * m_lo, m_hi; gather: dtype, n, d, m_lo, m_hi; QR: d and n ranges; lookups
 * take the first entry that covers a problem); clear (all three kinds);
 * load (appends; text lines "dtype n m_lo m_hi lpr nch grid unroll us
 * [waves]" for the pass, waves 4 when absent; "G dtype n d m_lo m_hi lpr
 * nseg us" for the gather; "Q d_lo d_hi n_lo n_hi cfg cb us" for the QR;
 * '#' comments; a malformed line loads nothing from the file) and save.
 * Thread-safe. */
sns_status sns_tune_set(const sns_tune_entry* e);
sns_status sns_tune_gather_set(const sns_tune_gather_entry* e);
sns_status sns_tune_qr_set(const sns_tune_qr_entry* e);
sns_status sns_tune_clear(void);
sns_status sns_tune_load(const char* path);
sns_status sns_tune_save(const char* path);

/* Kernel timing (tracing support).  While enabled, every kernel the library
 * launches is bracketed by two HIP events on its stream; sns_timing_summary
 * waits for the recorded launches and writes one line per kernel name,
 * "name launches total_ms avg_us", after a header line, into buf (host, len
 * bytes, truncated and NUL-terminated), returning the untruncated length.
 * SNS_TRACE=1 in the environment enables timing at the first call and prints
 * the summary to stderr at exit.  Not for use while another thread launches
 * library work.  sns_timing_select restricts timing to the kernels named in
 * `names` (host string, comma-separated, copied; NULL or "" selects every
 * kernel): each timed launch adds two event records to its stream. */
void sns_timing_enable(int on);
void sns_timing_select(const char* names);
void sns_timing_reset(void);
int sns_timing_summary(char* buf, size_t len);


#ifdef __cplusplus
}
#endif

#endif /* SNS_H */
