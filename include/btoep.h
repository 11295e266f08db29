/*
 * btoep -- FFT-based matvecs with block lower-triangular Toeplitz operators on AMD MI355X.
 *
 * The operator is the discrete parameter-to-observable map F of a linear time-invariant
 * system (Venkat, Fernando, Henneking, Ghattas, arXiv 2407.13066, section 2.1,
 * eq. ShiftInvariance): Nt x Nt blocks of size Nd x Nm, block (i, j) = F_{i-j} for i >= j
 * and zero above the diagonal, given by its first block column F_0 .. F_{Nt-1}.
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - Indices are 0-based; output block i is the paper's d_{i+1} (section 2.1).
 *  - Vectors are time-outer-space-inner (the paper's TOSI ordering, section 3.1):
 *      m[r][j][p]  (r < k right-hand sides, j < Nt, p < Nm),   d[r][i][s]  (s < Nd),
 *    dense, row-major, k right-hand sides stacked outermost.
 *  - Vector element type: double for an operator stored as BTOEP_F64, float otherwise.
 *  - All vector, workspace and operator pointers given to apply/cg calls are DEVICE
 *    pointers on the operator's device.  Host pointers are accepted only where stated.
 *  - Streams are hipStream_t values passed as `void*` (NULL = the default stream).  Apply
 *    calls are asynchronous and stream-ordered; cg_solve returns when the solve is done.
 *  - Workspace: pass `ws`/`ws_bytes` of at least btoep_workspace_size(); with ws == NULL
 *    the operator's own workspace is used (grown on demand with hipMalloc, which
 *    synchronises the device), and calls on the same operator must then not overlap.
 *    Calls that pass their own workspaces may run concurrently on one operator: the
 *    stored operator is read-only after btoep_create.
 *  - Errors: arguments are validated before any kernel is launched; nothing is written on
 *    error.  A HIP failure returns BTOEP_ERR_HIP and its text is kept for
 *    btoep_last_error().  No exception crosses this interface.
 */
#ifndef BTOEP_H
#define BTOEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct btoep_op_s* btoep_op;

/* The enumerations are int-sized.  C++ translation units (the library itself) see them with
 * the fixed underlying type int, so that any int a C caller passes -- valid or not -- is a
 * value of the type and is rejected by the argument checks instead of being undefined. */
#ifdef __cplusplus
#define BTOEP_ENUM enum : int
#else
#define BTOEP_ENUM enum
#endif

typedef BTOEP_ENUM {
    BTOEP_OK = 0,
    BTOEP_ERR_INVALID_ARG = 1,
    BTOEP_ERR_OUT_OF_MEMORY = 2,
    BTOEP_ERR_HIP = 3,
    BTOEP_ERR_UNSUPPORTED = 4,
    BTOEP_ERR_NOT_CONVERGED = 5,
    BTOEP_ERR_WORKSPACE_TOO_SMALL = 6,
    BTOEP_ERR_IO = 7
} btoep_status;

/* Storage precision of the Fourier-space operator (complex FP64, FP32 or BF16 parts). */
typedef BTOEP_ENUM { BTOEP_F64 = 0, BTOEP_F32 = 1, BTOEP_BF16 = 2 } btoep_dtype;

/* Where an input given to btoep_create lives. */
typedef BTOEP_ENUM { BTOEP_HOST = 0, BTOEP_DEVICE = 1 } btoep_memory;

/* Operation selector for btoep_workspace_size and btoep_apply_batched. */
typedef BTOEP_ENUM { BTOEP_APPLY_F = 0, BTOEP_APPLY_FT = 1, BTOEP_APPLY_H = 2, BTOEP_CG = 3 } btoep_which;

/* Largest number of right-hand sides one btoep_apply_batched call accepts. */
#define BTOEP_MAX_BATCH 64

typedef struct {
    int64_t Nt, Nd, Nm;
    int64_t L;          /* padded transform length 2N, N >= Nt the smallest 7-smooth integer */
    int64_t nfreq;      /* L/2 + 1 stored frequencies                                        */
    int64_t ldF;        /* row stride (complex elements) of the stored operator               */
    btoep_dtype storage;
    btoep_dtype vector; /* BTOEP_F64 (double vectors) or BTOEP_F32 (float vectors)            */
    size_t fhat_bytes;  /* device bytes of the stored operator                                */
    int device;
} btoep_info;

/*
 * Setup (paper section 3.2, Algorithm 1): zero-pad every time series F_k[s][p], k < Nt, to
 * length L, transform it along time (computed in FP64) and store its L/2+1 non-redundant
 * frequencies, rounded to nearest (ties to even) into `storage`:
 *     Fhat_f[s][p] = sum_{k<Nt} F_k[s][p] exp(-2 pi i f k / L),  f = 0 .. L/2.
 * The frequency-outer layout Fhat[f][s][p] is the paper's TOSI form of the transformed
 * operator.
 *   blocks : FP64 first block column, [Nt][Nd][Nm] row-major, blocks[k] = F_k; in host or
 *            device memory per `where`.  Not retained; may be freed once the call returns.
 *   stream : stream for the setup work; the call returns after it has completed.
 *   out    : receives the new operator (owned by the caller; free with btoep_destroy).
 * Uses the current HIP device.  Series too long for one workgroup's local memory use the
 * four-step transforms (see btoep_set_fft).  Errors: INVALID_ARG (sizes < 1, null pointers),
 * UNSUPPORTED (Nt > 64827, i.e. more than 65535 stored frequencies; Nd > 65535; Nm > 2^30),
 * OUT_OF_MEMORY, HIP.
 */
btoep_status btoep_create(int64_t Nt, int64_t Nd, int64_t Nm, const double* blocks, btoep_memory where,
                          btoep_dtype storage, void* stream, btoep_op* out);

/*
 * Setup in pieces (paper section 3.2, Algorithm 1: each processor reads and transforms its
 * own rectangle of sensor rows x parameter columns of the block matrix).
 *
 * btoep_create_empty makes an operator of the given shape whose stored Fhat is zero (F = 0);
 * btoep_set_blocks then transforms and stores any rectangle of it, replacing what was there.
 * Every (sensor, parameter) series is transformed on its own, so setting all rectangles of a
 * partition, in any order, stores exactly (bit for bit) what btoep_create stores.  Applies
 * may run between calls; they see zero blocks where nothing was set.
 *
 * The block sequence may be given as the first block column (order BTOEP_BLOCK_COLUMN:
 * input time t holds F_t, what Nm forward solves produce) or as the last block row
 * (BTOEP_LAST_BLOCK_ROW: input time t holds F_{Nt-1-t}, what Nd adjoint solves produce;
 * section 2.3 notes that either determines F).
 *   s0, ns : sensor rows s0 .. s0+ns-1;  p0, np : parameter columns p0 .. p0+np-1
 *   src    : FP64, element (t, s, p) at src[t*ld_time + (s-s0)*ld_sensor + (p-p0)], t < Nt,
 *            host or device memory per `where`; not retained.  ld_sensor >= np and
 *            ld_time >= (ns-1)*ld_sensor + np (rows do not overlap).
 *   stream : stream for the work; the call returns after it has completed.
 * Errors: INVALID_ARG (rectangle outside the operator, bad strides or enums, null
 * pointers), OUT_OF_MEMORY, HIP.
 */
typedef BTOEP_ENUM { BTOEP_BLOCK_COLUMN = 0, BTOEP_LAST_BLOCK_ROW = 1 } btoep_block_order;

btoep_status btoep_create_empty(int64_t Nt, int64_t Nd, int64_t Nm, btoep_dtype storage, void* stream,
                                btoep_op* out);
btoep_status btoep_set_blocks(btoep_op op, int64_t s0, int64_t ns, int64_t p0, int64_t np, const double* src,
                              int64_t ld_time, int64_t ld_sensor, btoep_block_order order, btoep_memory where,
                              void* stream);

/*
 * Keeping the transformed operator for reuse (section 3.2: the setup output is stored for
 * later matvecs).  btoep_save writes Fhat as stored -- a 64-byte little-endian header (magic
 * "BTOEPFH\n", version 1, storage code, Nt, Nd, Nm, L, payload bytes) followed by
 * Fhat[f][s][p], f <= L/2, s < Nd, p < Nm, in the storage format -- and btoep_load makes a new
 * operator on the current device holding exactly those values (applies then return the same
 * bits as on the saved operator, for the same transform mode and tuning).  Both copy
 * through a 64 MiB pinned host buffer and return when done.
 * Errors: INVALID_ARG (null pointers), IO (the file cannot be opened, read or written; a
 * header that is not this format, names sizes outside the library's limits or a transform
 * length the library would not choose for Nt, or a file size that does not match it --
 * all checked before any device work), OUT_OF_MEMORY, HIP.
 */
btoep_status btoep_save(btoep_op op, const char* path, void* stream);
btoep_status btoep_load(const char* path, void* stream, btoep_op* out);

/*
 * For comparison only: the paper's alternate local matvec (appendix).  The transformed
 * blocks are kept a second time in SOTI order, Fs[s][p][f] (every sensor-parameter series
 * contiguous over frequency), and the frequency-domain step becomes elementwise products with
 * the vector spectrum in SOTI order followed by sums over block rows (F) or block columns (F^T):
 *     dhat[s][f] = sum_p Fs[s][p][f] mhat[p][f],   mhat'[p][f] = sum_s conj(Fs[s][p][f]) dhat[s][f].
 * mode 0 follows the appendix (products written to a matrix-sized buffer, then a separate
 * reduction); mode 1 forms the products inside the reduction.  Transforms and time-domain
 * steps are those of btoep_apply_F / btoep_apply_FT, with transposes between the orderings.
 * btoep_alt_prepare allocates the SOTI copy (the stored operator's size again) and, for mode 0,
 * the product buffer (the same size in the vector precision), fills the copy from the stored
 * operator and returns when done.  btoep_alt_apply applies F (which = BTOEP_APPLY_F: m [Nt][Nm]
 * -> d [Nt][Nd]) or F^T (BTOEP_APPLY_FT: d -> m) to one right-hand side, using the operator's
 * own workspace; call btoep_alt_prepare with the same mode first.
 * Errors: INVALID_ARG (bad enums, null pointers, not prepared), UNSUPPORTED (more than about
 * 2^21 frequencies or parameters, or Nd Nm >= 2^31), OUT_OF_MEMORY, HIP.
 */
btoep_status btoep_alt_prepare(btoep_op op, int mode, void* stream);
btoep_status btoep_alt_apply(btoep_op op, btoep_which which, int mode, const void* in, void* out, void* stream);

/* Releases the operator and everything it owns (synchronises its device). */
btoep_status btoep_destroy(btoep_op op);

/* Shapes, layout and sizes of an operator. */
btoep_status btoep_query(btoep_op op, btoep_info* info);

/* Device bytes of workspace one call of `which` with k right-hand sides needs. */
btoep_status btoep_workspace_size(btoep_op op, btoep_which which, int64_t k, size_t* bytes);

/*
 * d = F m (paper section 3.3, Algorithm 2 on one device): transform m along time (zero
 * padded), multiply every frequency by Fhat_f, transform back and keep the first Nt
 * samples, i.e. (F m)_i = sum_{j<=i} F_{i-j} m_j.
 *   k : right-hand sides (k >= 0; k == 0 does nothing);  m : [k][Nt][Nm];  d : [k][Nt][Nd].
 */
btoep_status btoep_apply_F(btoep_op op, int64_t k, const void* m, void* d, void* ws, size_t ws_bytes,
                           void* stream);

/*
 * m = F^T d (paper section 3.4, Algorithm 3): the same steps with the conjugate transpose
 * of every Fhat_f (eq. AdjointFFTMatvec), i.e. (F^T d)_j = sum_{i>=j} F_{i-j}^T d_i.
 *   d : [k][Nt][Nd];  m : [k][Nt][Nm].
 */
btoep_status btoep_apply_FT(btoep_op op, int64_t k, const void* d, void* m, void* ws, size_t ws_bytes,
                            void* stream);

/*
 * Hessian action (paper section 2.2, eq. LinearInverseProblem, with scalar weights):
 *     Hm = F^T (noise_prec * F m) + prior_prec * m.
 * Two passes over the stored operator; the time-domain truncation between them is applied
 * on the device.  m and Hm : [k][Nt][Nm]; they must not overlap.
 */
btoep_status btoep_apply_H(btoep_op op, int64_t k, double noise_prec, double prior_prec, const void* m, void* Hm,
                           void* ws, size_t ws_bytes, void* stream);

/*
 * The three applies without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * same launches and chunking as btoep_apply_F / _FT / _H (which = BTOEP_APPLY_F, _FT or _H;
 * noise_prec / prior_prec used by _H only; in / out laid out as for those calls), so the
 * results are bitwise the same, but the workspace is a static device array of
 * BTOEP_STATIC_SCRATCH_BYTES that the library holds on each device it runs on until the
 * process ends.  Calls on one device share that array: calls that overlap on one device
 * (other streams, other threads) race and must not be issued.  Nothing in it needs to start
 * at zero.  Errors: INVALID_ARG (as btoep_apply_*), WORKSPACE_TOO_SMALL when
 * btoep_workspace_size(op, which, min(k, BTOEP_MAX_BATCH)) exceeds BTOEP_STATIC_SCRATCH_BYTES
 * (nothing launched; btoep_last_error names both sizes), HIP.
 */
#define BTOEP_STATIC_SCRATCH_BYTES (128u << 20)
btoep_status btoep_apply_static(btoep_op op, btoep_which which, int64_t k, double noise_prec, double prior_prec,
                                const void* in, void* out, void* stream);

/*
 * Pointer-array form of the three applies for right-hand sides that do not sit in one
 * array (e.g. requests batched by a server): in[r] / out[r] (HOST arrays of k <=
 * BTOEP_MAX_BATCH device pointers) each point at one [Nt][Nm] or [Nt][Nd] vector.
 * `which` is BTOEP_APPLY_F, _FT or _H (noise_prec / prior_prec used by _H only).
 * Results equal k separate calls (each right-hand side is computed independently).
 */
btoep_status btoep_apply_batched(btoep_op op, btoep_which which, int64_t k, const void* const* in,
                                 void* const* out, double noise_prec, double prior_prec, void* ws, size_t ws_bytes,
                                 void* stream);

/*
 * Graph form of one apply, for callers that repeat the same step on new vectors (a server's
 * batches, a solver's iterations): the launches of btoep_apply_batched for k <=
 * BTOEP_MAX_BATCH right-hand sides are recorded once into a HIP graph and replayed by
 * btoep_graph_launch.  The vector addresses are not frozen into the graph: the kernels read
 * them from a device table the graph owns, which btoep_graph_launch rewrites (with a small
 * kernel on `stream`, right before the replay) from
 *   in[r], out[r]  (HOST arrays of k device pointers, as for btoep_apply_batched; both NULL
 *                   to replay on the previous launch's vectors -- INVALID_ARG, with nothing
 *                   launched, before any launch has given vectors).
 * For _H no output may overlap an input.  `ws` (caller owned, at least
 * btoep_workspace_size(op, which, k) bytes, required) and the operator are used by every
 * replay and must outlive the graph.  Launches of one graph must be ordered on one stream
 * (they share the table and the workspace).  Creation allocates the table and launches
 * nothing; destruction synchronises the device.  The results equal btoep_apply_batched's.
 */
typedef struct btoep_graph_s* btoep_graph;

btoep_status btoep_graph_create(btoep_op op, btoep_which which, int64_t k, double noise_prec, double prior_prec,
                                void* ws, size_t ws_bytes, btoep_graph* out);
btoep_status btoep_graph_launch(btoep_graph g, const void* const* in, void* const* out, void* stream);
btoep_status btoep_graph_destroy(btoep_graph g);

typedef struct {
    double rtol;        /* stop when ||b - H x||_2 <= rtol ||b||_2 (true residual, FP64)       */
    int max_outer;      /* refinement steps (outer loop)                                        */
    int max_inner;      /* CG iterations per refinement step                                    */
    double inner_rtol;  /* inner CG stops when its recurrence residual drops by this factor     */
    int check_every;    /* inner iterations between host convergence checks (>= 1)             */
    int use_graph;      /* != 0: each inner iteration (H apply, inner products, vector
                           updates) is captured once per call into a HIP graph and replayed;
                           same kernels and results as launching them one by one            */
} btoep_cg_opts;

typedef struct {
    int inner_iters;     /* CG iterations, all refinement steps                              */
    int outer_iters;     /* refinement steps taken                                           */
    int matvecs;         /* H applications (inner + residual)                                */
    int converged;       /* 1 when the true residual met rtol                                */
    double rel_residual; /* final ||b - H x|| / ||b|| computed with the refinement operator  */
} btoep_cg_result;

/*
 * Solves H x = b for k right-hand sides by conjugate gradients (paper section 2.2) with
 * iterative refinement: each outer step forms the true residual r = b - H_hi x in FP64
 * with `op_hi`, runs CG on H_lo e = r with `op_lo` (vectors in op_lo's vector type, inner
 * products and CG scalars in FP64), and updates x += e in FP64.  With op_hi == NULL, op_lo
 * must be BTOEP_F64 and serves both roles (plain FP64 CG with a true-residual check).
 *   b, x : FP64 device arrays [k][Nt][Nm]; x holds the initial guess and receives x.
 *   results : HOST array of k entries (may be NULL).
 * Returns BTOEP_ERR_NOT_CONVERGED (x still written) when some right-hand side missed rtol.
 * op_lo and op_hi must have the same Nt, Nd, Nm and device.  The workspace needs at least
 * btoep_cg_workspace_size(op_lo, op_hi, k) bytes.
 */
btoep_status btoep_cg_workspace_size(btoep_op op_lo, btoep_op op_hi, int64_t k, size_t* bytes);
btoep_status btoep_cg_solve(btoep_op op_lo, btoep_op op_hi, int64_t k, double noise_prec, double prior_prec,
                            const double* b, double* x, const btoep_cg_opts* opts, btoep_cg_result* results,
                            void* ws, size_t ws_bytes, void* stream);

/*
 * Autotuning: times every variant of the single-right-hand-side product kernels (row block
 * size, non-temporal or cached operator loads) on this operator, `reps` launches each on
 * `stream`, and keeps the fastest for later applies; when both transform modes apply (see
 * btoep_set_fft), times the vector-side transform pair in each and keeps the faster.  Uses
 * the operator's own workspace and scratch it allocates (synchronises the device) and writes
 * nothing the caller owns.  Times are milliseconds per launch; entries past `nvar` are unused.
 */
typedef struct {
    int nvar;
    int var_n, var_c;    /* chosen variants */
    double ms_n[8];      /* product for F   */
    double ms_c[8];      /* product for F^T */
    int fft_four_step;   /* transform mode kept: 1 four-step, 0 single-pass               */
    double ms_fft[2];    /* forward + inverse vector-side transforms of one right-hand
                            side, single-pass and four-step (0 when a mode does not apply) */
} btoep_tune_result;

btoep_status btoep_autotune(btoep_op op, int reps, void* stream, btoep_tune_result* out);

/*
 * Transform mode (paper section 2.4: one length-2N DFT per time series; only the order of the
 * arithmetic changes).  n1 = 0: automatic (single-pass transforms in one workgroup's LDS when
 * a length-N series fits, else four-step transforms N = N1 N2 with N1 near sqrt(N)); n1 > 1:
 * four-step transforms with first factor n1 (must divide N); n1 < 0: single-pass (when it
 * fits).  Synchronises the device; workspace sizes change with the mode (query them again).
 * BTOEP_ERR_INVALID_ARG for an n1 that does not divide N or gives factors without a column
 * tile, BTOEP_ERR_UNSUPPORTED for single-pass on a series that does not fit; the operator then
 * keeps the automatic mode.
 */
btoep_status btoep_set_fft(btoep_op op, int64_t n1);

/* Pins the variants (0 .. nvar-1) and whether k >= 2 right-hand sides use the matrix-core
 * kernels (use_mfma != 0, the default) or one single-vector product per right-hand side. */
btoep_status btoep_set_tuning(btoep_op op, int var_n, int var_c, int use_mfma);

/*
 * Matrix-core mode of the several-right-hand-side products of an FP32-stored operator:
 * mode 0 runs them on the FP32 matrix cores (FP32 operands); mode 1 on the BF16 matrix cores
 * with operator and vectors each split into a BF16 high part and a BF16 remainder, keeping
 * the three terms hi*hi + hi*lo + lo*hi (relative error of a few 1e-6 against the FP64
 * definition, within the FP32 storage's 1e-5; the FP32 matrix cores give ~1e-6).  Single
 * right-hand sides are unaffected.  INVALID_ARG for another mode or another storage.
 */
btoep_status btoep_set_gemm(btoep_op op, int mode);

/*
 * Matrix-core autotuning (several right-hand sides, FP32 or BF16 storage): the tile shapes
 * and launch shapes of the two product kernels are chosen per right-hand-side bucket
 * (2..8, 9..16, 17..32, 33..64) by timing every variant on this operator's own stored data
 * for k right-hand sides, `reps` times each, on `stream`:
 *   forward product (F): 0 right-hand sides in groups of at most 32 (four 16-column result
 *     tiles per launch), vector chunks sized by the launch width; 1 groups of up to 64 (one
 *     pass over the operator, eight tiles); 2 / 3 narrow (64-column) / wide chunks always;
 *   adjoint product (F^T): 0 the default rule (4 waves below four tiles, 8 from four on);
 *     1..4 (waves, operator K steps in flight) = (4, 0), (8, 0), (4, 1), (8, 1).
 * With allow_split != 0 an FP32-stored operator times both modes of btoep_set_gemm and keeps
 * the faster one for that bucket; otherwise the bucket's current mode is kept and timed.  The fastest choice is kept for
 * later applies in that bucket; btoep_set_gemm_variants pins one.  Every variant computes the
 * same products (same per-right-hand-side arithmetic order within a mode).  Uses the
 * operator's own workspace (grown with hipMalloc when needed; synchronises the device).
 * Errors: INVALID_ARG (k outside 2..BTOEP_MAX_BATCH, reps < 1, variants out of range),
 * UNSUPPORTED (FP64 storage, or matrix cores disabled by btoep_set_tuning), HIP.
 */
typedef struct {
    int k;
    int nvar_n, nvar_c;   /* variants timed */
    int var_n, var_c;     /* chosen */
    int split;            /* chosen mode (1: BF16 matrix cores, three-term split)   */
    double ms_n[2][8];    /* [mode][variant] ms per forward product of k vectors    */
    double ms_c[2][8];    /* [mode][variant] ms per adjoint product of k vectors    */
} btoep_gemm_tune_result;

btoep_status btoep_autotune_gemm(btoep_op op, int64_t k, int allow_split, int reps, void* stream,
                                 btoep_gemm_tune_result* out);
btoep_status btoep_set_gemm_variants(btoep_op op, int64_t k, int var_n, int var_c);

/*
 * Per-kernel timing for measurement: while enabled, every kernel an apply launches on this
 * operator is bracketed by HIP events recorded on the same stream.  btoep_profile_read waits
 * for the recorded events and returns, per kernel name, the launches and the summed
 * milliseconds since profiling was (re)enabled.  Enabling resets the totals.  Not for
 * concurrent use on one operator.
 */
typedef struct {
    char name[24];
    int64_t launches;
    double total_ms;
} btoep_kernel_time;

btoep_status btoep_profile_enable(btoep_op op, int enable);
btoep_status btoep_profile_read(btoep_op op, btoep_kernel_time* out, int max, int* count);

/*
 * Stepwise CG, for servers that batch the H applications of many solves with other work
 * (paper section 2.2).  The caller applies H itself (btoep_apply_H / btoep_apply_batched on
 * the vectors returned by btoep_cg_vectors) and then calls btoep_cg_update; everything else
 * (inner products in FP64, scalar recurrences, vector updates) runs on the device.  Because
 * the caller forms Ap, a general SPD prior R (section 2.2's prior precision operator) can be
 * used: apply H with prior_prec = 0 and add R p before the update.
 *   btoep_cg_start : state for k right-hand sides; x (op vector type, [k][Nt][Nm], caller
 *                    owned) is set to 0, r = p = b; stops a right-hand side once
 *                    ||r|| <= rtol ||b|| (recurrence residual).  Allocates its vectors.
 *   btoep_cg_vectors : device pointers of the stacked p and Ap arrays ([k][Nt][Nm] each).
 *   btoep_cg_update  : after Ap = H p: x += alpha p, r -= alpha Ap, p = r + beta p.
 *   btoep_cg_poll    : enqueue a copy of the scalars to pinned host memory on `stream`.
 *   btoep_cg_status  : non-blocking; ready = 1 once the last poll landed, then active =
 *                      right-hand sides still iterating, iters = largest iteration count,
 *                      rel_res (host [k], may be NULL) = ||r|| / ||b|| per right-hand side.
 *   btoep_cg_end     : releases the state; a state from btoep_cg_start frees its memory
 *                      (synchronises the device), one from btoep_cg_begin only its host
 *                      object (no device call that waits).
 * All calls on one state must be ordered on one stream.
 *
 * Refined stepwise CG on caller memory, for servers that must neither allocate nor wait
 * (section 2.2 with the FP64 refinement of btoep_cg_solve):
 *   btoep_cg_state_size : device and pinned-host bytes of a state for k right-hand sides.
 *   btoep_cg_begin : like btoep_cg_start, but the state lives in `dev_mem` (device, 256-byte
 *                    aligned) and `host_mem` (pinned host memory), both caller owned and at
 *                    least btoep_cg_state_size bytes; it allocates no device memory and
 *                    launches only kernels on `stream`.  With op_hi (an FP64 operator of the
 *                    same shape; op_hi may be op_lo itself when that is FP64), b and x are
 *                    FP64 and the solve is refined: the inner iteration on op_lo's vectors
 *                    stops once its recurrence residual has dropped by inner_rtol (0 < inner_rtol
 *                    < 1), or below rtol/2 relative to b, and the caller then applies H_hi to x
 *                    (btoep_cg_residual_vectors: x, and the FP64 array Hx that receives H_hi x)
 *                    and calls btoep_cg_refine.  Without op_hi, b and x have op_lo's vector type
 *                    and the state behaves as one from btoep_cg_start (inner_rtol unused).
 *                    x is set to 0.  The memory may be reused once all work enqueued on the
 *                    state has completed.
 *   btoep_cg_update  : also accumulates x (FP64 when refined) += alpha p.
 *   btoep_cg_refine  : after Hx = H_hi x: the true residual b - H_hi x in FP64, the outer test
 *                      ||b - H_hi x|| <= rtol ||b||, and a restart of the inner iteration on that
 *                      residual for the right-hand sides that missed it (INVALID_ARG unrefined).
 *   btoep_cg_report  : non-blocking; ready = 1 once the last poll landed, then per right-hand
 *                      side (HOST array of k): inner iterations, refinement steps, H
 *                      applications (updates + refinements), converged and rel_residual -- the
 *                      true FP64 residual of the last refinement when refined (the x = 0 one
 *                      before the first), else the recurrence residual.
 * Errors: INVALID_ARG (null pointers, k outside 1..BTOEP_MAX_BATCH, rtol <= 0, operators that
 * differ in shape or device, a non-FP64 op_hi, misaligned memory), WORKSPACE_TOO_SMALL (memory
 * smaller than btoep_cg_state_size), HIP.
 */
typedef struct btoep_cg_s* btoep_cg;

btoep_status btoep_cg_start(btoep_op op, int64_t k, double noise_prec, double prior_prec, const void* b, void* x,
                            double rtol, void* stream, btoep_cg* out);
btoep_status btoep_cg_state_size(btoep_op op_lo, btoep_op op_hi, int64_t k, size_t* dev_bytes,
                                 size_t* host_bytes);
btoep_status btoep_cg_begin(btoep_op op_lo, btoep_op op_hi, int64_t k, const void* b, void* x, double rtol,
                            double inner_rtol, void* dev_mem, size_t dev_bytes, void* host_mem, size_t host_bytes,
                            void* stream, btoep_cg* out);
btoep_status btoep_cg_vectors(btoep_cg cg, void** p, void** Ap);
btoep_status btoep_cg_residual_vectors(btoep_cg cg, void** x, void** Hx);
btoep_status btoep_cg_update(btoep_cg cg, void* stream);
btoep_status btoep_cg_refine(btoep_cg cg, void* stream);
btoep_status btoep_cg_poll(btoep_cg cg, void* stream);
btoep_status btoep_cg_status(btoep_cg cg, int* ready, int* active, int* iters, double* rel_res);
btoep_status btoep_cg_report(btoep_cg cg, int* ready, btoep_cg_result* results);
btoep_status btoep_cg_end(btoep_cg cg);

/*
 * Measurement support: streams one device array of `bytes` (>= 1 MiB) through a kernel of
 * non-temporal 16-byte loads, `reps` times for each of six launch shapes (4 or 8 loads in
 * flight per lane, 4, 8 or 16 workgroups per CU) on `stream` (the current device), and returns,
 * for the shape with the lowest mean, the best time and the best and mean read rates
 * (GB/s = 1e9 bytes/s).  This is the rate the
 * memory system gives one streaming read, against which the operator-streaming product
 * kernels (section 4.1 reads its kernels against peak bandwidth) are compared.  Allocates
 * and frees the array (synchronises the device).  Errors: INVALID_ARG, OUT_OF_MEMORY, HIP.
 */
btoep_status btoep_read_bandwidth(size_t bytes, int reps, void* stream, double* best_ms, double* best_gbs,
                                  double* mean_gbs);

/*
 * Measurement support: writes one device array of `bytes` (>= 1 MiB) with non-temporal 8- or
 * 16-byte stores, `reps` times for each of six launch shapes (store width 8 or 16 bytes, 4, 8
 * or 16 workgroups per CU) on `stream` (the current device), and returns, for the shape with
 * the lowest mean, the best time and the best and mean write rates (GB/s = 1e9 bytes/s): the
 * ceiling of the kernels whose traffic is mostly result writes (the adjoint products of
 * several right-hand sides, the forward transform).  Allocates and frees the array
 * (synchronises the device).  Errors: INVALID_ARG, OUT_OF_MEMORY, HIP.
 */
btoep_status btoep_write_bandwidth(size_t bytes, int reps, void* stream, double* best_ms, double* best_gbs,
                                   double* mean_gbs);

/* Static text for a status code. */
const char* btoep_status_string(btoep_status s);

/* Text of the last HIP error seen on this operator (or by the calling thread when op is NULL). */
const char* btoep_last_error(btoep_op op);

#ifdef __cplusplus
}
#endif

#endif /* BTOEP_H */
