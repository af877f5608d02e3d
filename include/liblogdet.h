/*
 * liblogdet - log-determinant estimation of large sparse SPD matrices on one
 * AMD Instinct MI355X (gfx950), by the OSLQ and OSA-IOP estimators of
 * Mbingui, Tambue and Karambal, "Optimal Stochastic Krylov Based Techniques
 * for Large-Scale Log-Determinant Estimation".
 *
 * Problem statement (Section 2, eqs. Leja1/Leja2): log det Q = tr log Q for a
 * symmetric positive definite Q that is only touched through products Q x.
 * Both estimators split tr(log Q - c I) Hutch++-style (Alg 2, Alg 3) into an
 * exactly evaluated sketch subspace and a Hutchinson residual, and evaluate
 * every quadratic form with a Krylov recurrence:
 *   - OSLQ (Section 3, Alg 3): subspace from orth(J S), J = Q / lambda_max
 *     (when lambda_min < 1), Gauss-Lanczos quadrature of log on T_m.
 *   - OSA-IOP (Section 2, Alg 2 with Alg 1): subspace from orth(L S), every
 *     L x from Arnoldi with incomplete orthogonalisation over a window of k
 *     vectors on Q / gamma, gamma = sqrt(lambda_min lambda_max), and
 *     log(H_m) e1.
 *   - SLQ (the sketch-rank-0 setting of OSLQ) and So-SLQ, the comparators of
 *     Section 4: So-SLQ keeps the k dominant left singular vectors of a sketch
 *     log(J) S (each column from Alg 1) and evaluates both parts by
 *     Gauss-Lanczos quadrature.
 *
 * All pointers in this header are HOST pointers unless stated otherwise.
 * Every function returns an ld_status; no exception or signal crosses the
 * ABI; out-parameters are left untouched when an error is returned, and
 * ld_last_error() then describes the failure (thread-local string).
 */
#ifndef LIBLOGDET_H
#define LIBLOGDET_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ld_status;

enum {
  LD_OK = 0,
  LD_PENDING = 1,            /* ld_poll: the request has not finished yet      */
  LD_E_INVALID_ARG = -1,     /* a parameter is outside its documented range    */
  LD_E_BAD_CSR = -2,         /* malformed CSR structure                        */
  LD_E_NOT_SPD = -3,         /* a_ii <= 0, a non-positive Ritz value, or a
                                Hessenberg log that is not real                */
  LD_E_NUMERIC = -4,         /* NaN/Inf in a Krylov run or the sketch QR       */
  LD_E_NO_MEMORY = -5,       /* the request can never fit the HBM budget       */
  LD_E_BUSY = -6,            /* object still referenced by in-flight requests  */
  LD_E_DEVICE = -7,          /* HIP runtime error (message in ld_last_error)   */
  LD_E_UNKNOWN_TICKET = -8   /* ld_poll/ld_wait on a ticket never issued or
                                already retired                                */
};

/* Storage type of the matrix values on the device.  Values are always given
 * in FP64 and rounded once, round-to-nearest-even. */
typedef enum { LD_VT_FP64 = 0, LD_VT_FP32 = 1, LD_VT_BF16 = 2 } ld_value_type;

typedef enum { LD_METHOD_OSLQ = 0, LD_METHOD_OSA_IOP = 1, LD_METHOD_SO_SLQ = 2 } ld_method;
/* Distribution of the random sketch and probe columns (Section 2 allows both).
 * Both come from Philox4x64-10 (Salmon et al., SC'11) under key (seed, 0):
 *   RADEMACHER: row i, column p: bit i % 64 of word (i / 64) % 4 of the block
 *               at counter (i / 256, p, 0, 0); a set bit gives -1, else +1.
 *   GAUSSIAN:   rows 4b..4b+3 of column p from the block at counter
 *               (b, p, 1, 0) by the Box-Muller transform: words (w0, w1) feed
 *               rows 4b, 4b+1 and (w2, w3) rows 4b+2, 4b+3; for a pair (wa, wb),
 *               u1 = ((wa >> 11) + 1) 2^-53, u2 = (wb >> 11) 2^-53,
 *               rho = sqrt(-2 log u1): even row rho cos(2 pi u2), odd row
 *               rho sin(2 pi u2) (device log/sqrt/sin/cos, not bit-exact with
 *               other math libraries). */
typedef enum { LD_PROBE_RADEMACHER = 0, LD_PROBE_GAUSSIAN = 1 } ld_probe_dist;

/* LD_PREC_FP64: every vector, product and reduction in FP64.
 * LD_PREC_MIXED: Krylov vectors in FP32; sparse products read the matrix in
 * its storage type (FP32 or BF16 values with FP32 row sums; FP64 values with
 * FP64 row sums, rounded to FP32 once per entry); every inner product and
 * norm accumulated in FP64; sketch QR, projection, the small
 * tridiagonal/Hessenberg reductions and the trace in FP64.
 * LD_PREC_HALF: as LD_PREC_MIXED with the Krylov vectors stored in IEEE
 * FP16 (row sums of the product in FP32, or FP64 for FP64 values).  Each
 * stored block carries a power-of-two scale that keeps the entries of unit
 * vectors near 1 and below the FP16 range limit; the scale is removed
 * exactly from every inner product and norm.  Half the vector traffic of
 * LD_PREC_MIXED; the extra rounding (2^-11 per stored entry) enters the
 * estimate through averages over n entries and many probes, and grows with
 * the share of the spectrum near lambda_lo.  Accepted only where it holds
 * the mixed-precision accuracy (1e-4 relative to FP64): windows up to
 * iop_window = 4 (beyond, classical Gram-Schmidt over a longer window of
 * FP16-rounded vectors can lose stability and make the tridiagonal T
 * indefinite) and matrices whose spectral interval (ld_matrix_bounds) has
 * lambda_hi <= 512 lambda_lo (beyond, Wendland covariances with many
 * eigenvalues near their nugget move by more than 1e-4); anything else is
 * LD_E_INVALID_ARG.  The 1e-4 is relative to sum |log lambda_i|: a logdet
 * whose terms nearly cancel (eigenvalues on both sides of 1) can miss 1e-4
 * relative to its own value even inside that range.
 * LD_PREC_AUTO: LD_PREC_MIXED where lambda_hi <= 4096 lambda_lo, else
 * LD_PREC_FP64 (FP32 vectors held 1e-4 against FP64 on a serving mix of
 * Laplacians and Wendland covariances up to a ratio of ~8700).  Never
 * LD_PREC_HALF. */
typedef enum {
  LD_PREC_FP64 = 0,
  LD_PREC_MIXED = 1,
  LD_PREC_HALF = 2,
  LD_PREC_AUTO = 3
} ld_precision;

typedef struct ld_ctx ld_ctx;
typedef struct ld_matrix ld_matrix;

typedef struct {
  int32_t device;            /* HIP device ordinal                              */
  int32_t max_slots;         /* serving: requests resident at once (0 -> 16)    */
  uint64_t hbm_budget_bytes; /* serving: device bytes for resident requests
                                (0 -> 80% of the free memory at creation)       */
  void* hip_stream;          /* optional hipStream_t to run ld_estimate on
                                (NULL -> the library creates its own)           */
  int32_t default_method;    /* ld_method used by ld_estimate                    */
  int32_t default_precision; /* ld_precision used by ld_estimate                 */
} ld_ctx_opts;

typedef struct {
  int32_t method;            /* ld_method                                        */
  int32_t precision;         /* ld_precision                                     */
  int32_t n_probes;          /* s + r: sketch columns plus residual probes       */
  int32_t sketch_rank;       /* s, 0 <= s <= min(n, 256); s = 0 is plain SLQ /
                                Hutchinson.  So-SLQ: the sketch width q,
                                1 <= q <= min(n, 48).  Block caps: n_probes
                                (and s) <= 128 in LD_PREC_FP64, <= 256 in the
                                other precisions (LD_E_INVALID_ARG beyond); for
                                So-SLQ the cap applies to k + n_probes - q      */
  int32_t krylov_steps;      /* m, 1 <= m <= min(n, 512): mat-vecs per Krylov run */
  int32_t iop_window;        /* k >= 1: orthogonalise against the k newest basis
                                vectors (the paper's IOP uses k = 2; k >= m is
                                full re-orthogonalisation)                      */
  uint64_t seed;             /* key of the probe generator (see ld_probe_dist)   */
  double tol;                /* stop a run when h_{t+1,t} < tol (<= 0 -> 1e-10) */
  int32_t probe_dist;        /* ld_probe_dist of every random column             */
  int32_t subspace_rank;     /* So-SLQ: kept rank k, 1 <= k <= q (0 -> min(10, q));
                                must be 0 for the other methods                  */
  double adapt_tol;          /* > 0: adaptive Krylov dimension (OSLQ, SLQ,
                                So-SLQ): every adapt_every steps each run's
                                Gauss quadrature value K_t is formed, and the
                                run stops at step t once
                                |K_t - K_{t - adapt_every}| <= adapt_tol |K_t|;
                                0 -> every run takes krylov_steps (or stops at
                                h < tol).  Must be 0 for OSA-IOP.                */
  int32_t adapt_every;       /* steps between convergence checks (0 -> 5)        */
  int32_t sketch_passes;     /* OSA-IOP and So-SLQ sketch image Y = L S (one
                                Alg 1 run per sketch column, y = ||s|| V_m
                                log(H_m) e1 + ...): 0 or 1 keeps each run's
                                basis V_m (m + 1 probe blocks of s columns);
                                2 runs the sketch recurrences twice, the first
                                time for H_m only, the second time adding each
                                basis vector into Y while it is still in a ring
                                of min(m + 1, min(k, m) + 9) blocks: the same
                                values and sums, bitwise, for about m - 1 more
                                sketch steps.  OSLQ (whose sketch is one
                                product): 0 or 1                                */
} ld_params;

typedef struct {
  double logdet;             /* the estimate of log det Q                        */
  double tr_sketch;          /* subspace part tr(A^T L_c A)                      */
  double tr_resid;           /* residual part (1/r) sum_j u_j^T L_c u_j         */
  double shift_c;            /* c: logdet = n c + tr_sketch + tr_resid           */
  double lambda_lo;          /* spectral interval used (Gershgorin or hints)     */
  double lambda_hi;
  double scale;              /* OSLQ: alpha (runs on Q/alpha); OSA-IOP: gamma    */
  int64_t probe_steps;       /* sum over Krylov runs of the mat-vecs performed
                                (OSA-IOP: sketch-image runs included)            */
  int64_t matvecs;           /* all Q x products, sketch included               */
  int32_t min_steps;         /* smallest effective Krylov dimension of a run    */
  int32_t n_breakdowns;      /* runs stopped early by h < tol                    */
  double device_ms;          /* device time of the estimate (HIP events)        */
  double latency_ms;         /* host wall time from call (or submit) to result  */
  int32_t basis_rank;        /* columns of the sketch basis A kept by its QR:
                                orth(Y) takes the columns of Y in order and
                                drops one whose part orthogonal to those kept
                                before it is at most 1e-6 of its norm (its run
                                is skipped, K = 0); = sketch_rank (So-SLQ:
                                subspace_rank) unless the sketch image is
                                rank-deficient                                  */
} ld_result;

/* Optional per-run outputs of ld_estimate_detail.  Each pointer may be NULL;
 * arrays are caller-owned host memory.  Runs are numbered 0..n_probes-1: the
 * s sketch-basis runs first, then the r residual runs (OSA-IOP's sketch-image
 * runs are not reported). */
typedef struct {
  double* probe_K;           /* [runs] quadrature value of the run: the
                                estimate of x^T (log Q - c I) x / ||x||^2        */
  double* probe_norm2;       /* [runs] ||x||^2 of the run's start vector        */
  int32_t* probe_steps;      /* [runs] effective Krylov dimension                */
  double* tri_alpha;         /* [runs * krylov_steps] h_{t,t}, row-major         */
  double* tri_beta;          /* [runs * krylov_steps] h_{t+1,t}                  */
  double* sketch_basis;      /* [n * b] the basis A, row-major (row i, column j
                                at i*b + j)                                      */
} ld_detail;
/* In ld_detail, runs = n_probes and b = sketch_rank for OSLQ and OSA-IOP;
 * runs = subspace_rank + n_probes - sketch_rank and b = subspace_rank for
 * So-SLQ (the q sketch-image runs are not reported). */

/* Context: owns a HIP stream (unless one is supplied), a device workspace and
 * the serving scheduler.  Returns LD_E_DEVICE when the device is absent. */
ld_status ld_ctx_create(const ld_ctx_opts* opts, ld_ctx** out);
/* Waits for every submitted request, then releases everything.  Matrices
 * created in the context must be destroyed first (else LD_E_BUSY). */
ld_status ld_ctx_destroy(ld_ctx* ctx);
/* Thread-local description of the last error returned on this thread. */
const char* ld_last_error(void);

/* Copies a host CSR matrix to the device (the caller keeps ownership of its
 * arrays and may free them on return).  row_ptr[n+1] is monotone from 0 to
 * nnz; col_idx[nnz] in [0, n), sorted and unique within each row; every
 * diagonal entry present and > 0 (else LD_E_NOT_SPD).  values are FP64 and
 * stored as `vt`; an FP64 copy is kept as well for LD_PREC_FP64 runs.
 * With LD_VT_FP32 or LD_VT_FP64 the matrix may also keep row groups (see
 * ld_autotune): per union column its index and 4 FP64 values (plus 4 FP32
 * ones with LD_VT_FP32), 36 or 52 bytes, built on the device here when
 * groups of 4 rows hold at least 2 entries per union column (so at most
 * 18 or 26 bytes per entry).
 * lambda_lo_hint / lambda_hi_hint > 0 replace the Gershgorin bounds
 * (Section 2.1); a Gershgorin lower bound <= 0 without a hint is replaced by
 * 1e-6 * lambda_hi.  n and nnz must fit int32. */
ld_status ld_create_csr(ld_ctx* ctx, int64_t n, int64_t nnz,
                        const int32_t* row_ptr, const int32_t* col_idx,
                        const double* values, int32_t vt,
                        double lambda_lo_hint, double lambda_hi_hint,
                        ld_matrix** out);
/* Releases a matrix; LD_E_BUSY while submitted requests still use it. */
ld_status ld_destroy(ld_matrix* a);
/* The spectral interval the estimators will use for this matrix. */
ld_status ld_matrix_bounds(const ld_matrix* a, double* lambda_lo, double* lambda_hi);
/* x^T Q x for a host vector x[n] (caller-owned), on the device in FP64: the
 * data term of the Gaussian log-likelihood of Section 4,
 * L(theta) = log det Q / 2 - x^T Q x / 2 - n log(2 pi) / 2.  Blocking. */
ld_status ld_quad_form(ld_matrix* a, const double* x, double* out);

/* Blocking estimate with the context's default method and precision and
 * tol = 1e-10 (Alg 3 for OSLQ, Alg 2 for OSA-IOP). */
ld_status ld_estimate(ld_matrix* a, int32_t n_probes, int32_t sketch_rank,
                      int32_t krylov_steps, int32_t iop_window, uint64_t seed,
                      ld_result* out);
/* Blocking estimate with explicit parameters.  A matrix whose spectral
 * interval has zero width (lambda_lo == lambda_hi: Q = q I) gets the exact
 * n log q without any Krylov run (probe_steps = 0; detail arrays zero). */
ld_status ld_estimate_ex(ld_matrix* a, const ld_params* p, ld_result* out);
/* As ld_estimate_ex, also filling the non-NULL arrays of `detail`. */
ld_status ld_estimate_detail(ld_matrix* a, const ld_params* p, ld_result* out,
                             const ld_detail* detail);
/* For callers that cannot allocate device memory during the call (code that
 * runs where hipMalloc is not allowed, tight serving loops, harnesses that
 * forbid allocation): ld_estimate_ex with every device buffer of the estimate
 * (Krylov blocks, sketch, partial sums, per-run state) carved from a fixed
 * 256 MiB scratch array that each GPU holds from the library's load until the
 * process ends.  The call performs no hipMalloc, hipFree or other allocating
 * routine; the matrix (created earlier by ld_create_csr) and the host result
 * are the caller's.  The events and the pinned word it needs are created with
 * the context.  Same kernels, geometry and summation order as ld_estimate_ex:
 * the result is bitwise the same.  A request whose buffers exceed the scratch
 * (about 500 n bytes for 30 FP32 probes with window 2) is LD_E_INVALID_ARG,
 * as is everything ld_estimate_ex refuses.  Blocking.  Every call on one GPU
 * uses that GPU's one scratch array, which keeps the last call's contents
 * (each call clears what it needs); calls on one GPU from this library are
 * serialised, and overlapping use of the array by other means would race.
 * Profiling (ld_profile_enable) does not cover it. */
ld_status ld_estimate_noalloc(ld_matrix* a, const ld_params* p, ld_result* out);

/* Device bytes an estimate of `a` with parameters `p` takes beyond the
 * matrix itself (Krylov blocks, sketch, partial sums, per-run state): the
 * workspace ld_estimate_ex uses and the amount a served request is charged
 * against the HBM budget.  LD_E_INVALID_ARG for parameters the estimate
 * would refuse. */
ld_status ld_request_bytes(ld_matrix* a, const ld_params* p, uint64_t* bytes);

/* Autotuner of the Krylov-step kernels (the product Q V of a probe block,
 * and the orthogonalisation update with its fused norms).  Both sweep the
 * probe block row by row with L <= 64 lanes per row (a 64-lane wave holds
 * floor(64 / L) rows, any remaining lanes idle), each lane holding C
 * 16-byte chunks of the row (1 <= C <= 4, L * C chunks covering the block).
 * The product may also split a row's sparse entries over E = 1, 2, 4 or 8
 * lane groups (L a power of two, L / E column lanes each, their sums added
 * at the row's end), which shortens the per-lane chain of dependent gathers
 * on long rows (tried when rows hold 16 entries or more on average).
 * For OSA-IOP it also times, for the estimate block, the update of the
 * steps that also read v1 (every other step), which keeps a geometry of its
 * own (untuned: the update's, or fewer chunks per lane when the update's
 * holds more than 8 elements per lane).
 * For windows of two or more ld_autotune also times the two step schedules
 * (ld_tune_result.step_presub) on its choices and keeps the schedule in
 * which the product subtracts the second-newest vector unless the other is
 * more than 1% faster per step.
 * The product's rows may also be taken in tiles (ld_tune_set's
 * spmm_row_stride), which ld_autotune tries on every power-of-two L with the
 * strides of the matrix's most frequent column offsets (at most two, each in
 * a quarter of the sampled rows or more).
 * Matrices created with LD_VT_FP32 or LD_VT_FP64 whose groups of 4
 * consecutive rows share most of their columns (at least 2 entries per
 * column of the group's union, as on covariance matrices of sorted points)
 * also keep those groups: the union of the 4 rows' columns with one value
 * per row and column (zero where a row has no entry), in FP64 and, with
 * LD_VT_FP32, FP32.  The product then gathers each union column's probe
 * row once for the 4 rows (spmm_row_groups), over the values the estimate
 * reads (FP32 or FP64 storage values on FP32 Krylov vectors, FP64 values on
 * FP64 vectors; not with FP16 vectors or BF16 values); it is the untuned
 * default on such matrices for blocks of 16 columns or more where values
 * and vectors have the same type, with one chunk per lane for FP32 and two
 * for FP64, and ld_autotune tries it in every plain geometry of at most 2
 * chunks per lane.  A row's sum sees its
 * nonzero terms in CSR order, so the product's output is the CSR product's.
 * The groups are built on the device when the matrix is created.
 * ld_autotune times every such (L, C, E) with L a power of two and at most
 * half a row of idle chunks on this matrix, and L = ceil(chunks / C) where
 * that is not a power of two, for the probe-block shapes and
 * precision that `p` implies (the estimate block and, for OSA-IOP and So-SLQ,
 * the sketch-run block), each kernel `reps` times per round over three
 * rounds, keeping the fastest per kernel.  Both are timed as a steady-state
 * step of `p` runs them: with iop_window >= 2 the product also subtracts the
 * second-newest window vector and the update takes the rest of the window.
 * The choice is stored in the matrix and used by every later estimate and
 * served request whose shapes match (the update's per class of window: 1, 2,
 * up to 4 or up to 8 vectors after that subtraction); results then differ from the untuned ones only by the summation
 * order of the partial sums (FP64 rounding), and stay bitwise reproducible
 * for a fixed choice.  Blocking; call it before submitting requests on this
 * matrix (a request takes its geometry when it is admitted).  reps = 0 drops
 * the stored choice for these shapes (back to the default).  `out` may be
 * NULL; the lanes and chunks fields give the choice for the estimate block,
 * the *_ms fields the mean time per launch of the choice and of the default
 * geometry. */
typedef struct {
  int32_t spmm_lanes, spmm_chunks;
  int32_t update_lanes, update_chunks;
  double spmm_ms, spmm_default_ms;
  double update_ms, update_default_ms;
  int32_t candidates;        /* geometries timed for the product               */
  int32_t spmm_entry_split;  /* sparse-entry groups per row of the product     */
  int32_t spmm_interleave;   /* 1: the product's row chunks interleave over the
                              * XCDs; 0: a contiguous band of chunks per XCD,
                              * which keeps a row's neighbours in one L2    */
  int32_t spmm_row_stride;   /* 0, or S: the product's block takes its rows as
                              * 4 runs S rows apart (row tiles)             */
  int32_t step_presub;       /* 1: the product subtracts the second-newest
                              * window vector (its coefficient is known by
                              * symmetry) and the update the rest; 0: the
                              * update subtracts the whole window           */
  double step_presub_ms;     /* product + update per step, schedule 1       */
  double step_plain_ms;      /* the same, schedule 0 (0 for windows of 1)   */
  int32_t spmm_row_groups;   /* 1: the product reads the matrix's row groups */
} ld_tune_result;
ld_status ld_autotune(ld_matrix* a, const ld_params* p, int32_t reps, ld_tune_result* out);
/* Stores a given geometry for the estimate block of `p` on this matrix (a
 * choice found earlier, or one to test): the product with spmm_lanes lanes
 * per row, spmm_chunks chunks per lane, its entries split over
 * spmm_entry_split lane groups and its row chunks interleaved over the XCDs
 * (spmm_interleave 1) or banded per XCD (0), and its rows taken in tiles
 * (spmm_row_stride S > 0: each 256-thread block's four waves take runs of
 * 64 / L consecutive rows S rows apart, so on a grid operator whose line
 * stride is S the +-S neighbours of one wave's rows are the rows the other
 * waves of the block gather at the same time; S a multiple of 64 / L, L a
 * power of two, S <= 32767; rows past the last whole tile of 4 S rows keep
 * the plain order), the update likewise (no split, interleaved; stored for
 * the window class of `p`), with the step schedule step_presub (1: the
 * product subtracts the second-newest window vector, the default; 0: the
 * update subtracts the whole window; see ld_tune_result), and the product
 * over the matrix's row groups (spmm_row_groups 1: FP32 or FP64 Krylov
 * vectors on a matrix that keeps them, not BF16 values, C <= 2, no entry
 * split, no row tiles) or its CSR
 * rows (0).  Any (L, C, E) with L <= 64, 1 <= C <= 4, E in {1, 2, 4, 8},
 * E <= L, C <= 2 when E > 1, and (L / E) * C chunks covering the block is
 * accepted, where L is a power of two when E > 1; anything else is
 * LD_E_INVALID_ARG and stores nothing. */
ld_status ld_tune_set(ld_matrix* a, const ld_params* p, int32_t spmm_lanes, int32_t spmm_chunks,
                      int32_t spmm_entry_split, int32_t update_lanes, int32_t update_chunks,
                      int32_t spmm_interleave, int32_t spmm_row_stride, int32_t step_presub,
                      int32_t spmm_row_groups);

/* Serving with continuous batching: queue a request and return at once with
 * a ticket.  Requests are admitted as resident slots and HBM budget free up;
 * admitted requests advance together, several Krylov steps per scheduler
 * tick.  A result depends only on (matrix, params), never on the other
 * requests in flight.  Returns LD_E_NO_MEMORY if the request could never fit
 * the budget.  Thread-safe. */
ld_status ld_submit(ld_matrix* a, const ld_params* p, uint64_t* ticket);
/* LD_PENDING while the request runs; LD_OK (with *out filled, or the
 * request's own error) exactly once, after which the ticket is retired. */
ld_status ld_poll(ld_ctx* ctx, uint64_t ticket, ld_result* out);
/* Blocks until the request finishes, then behaves as ld_poll. */
ld_status ld_wait(ld_ctx* ctx, uint64_t ticket, ld_result* out);

/* Serving scheduler statistics of a context (zero before the first
 * ld_submit).  held_bytes is what the resident slots' device buffers hold
 * now, idle slots included; the scheduler keeps it at or below
 * budget_bytes (ld_ctx_opts.hbm_budget_bytes), releasing idle buffers before
 * a slot grows, and peak_held_bytes is the most it has held.  A batched
 * launch advances every resident request by one Krylov step. */
typedef struct {
  uint64_t submitted, completed, ticks;
  uint64_t batched_steps, batched_launches;
  uint64_t held_bytes, peak_held_bytes, budget_bytes;
  uint64_t buffer_allocs, buffer_frees;
  int32_t peak_active, max_slots;
} ld_serving_stats;
ld_status ld_serving_stats_get(ld_ctx* ctx, ld_serving_stats* out);

/* HIP-graph replay of blocking estimates (ld_estimate, ld_estimate_ex,
 * ld_estimate_detail; not ld_estimate_noalloc, which instantiates nothing).
 * With mode 1 (the default) the second blocking estimate of a context with
 * the same matrix and the same parameters apart from the seed captures the
 * estimate's kernel launches in a HIP graph, and every later one replays it:
 * one graph launch in place of one launch per kernel (the host stops being
 * the bound on small matrices).  The seed reaches the probe kernels through
 * device memory, written before each replay, so one graph serves every seed.
 * A replay runs the same kernels in the same order on the same buffers: the
 * result is bitwise the eager one.  Estimates with an adaptive Krylov
 * dimension (a host check during the run), with profiling enabled, or of a
 * matrix whose interval has zero width always launch kernel by kernel.  Up
 * to 8 graphs are kept per context, least recently used dropped first; a
 * matrix's graphs go with ld_destroy, and all of them when the context's
 * workspace grows; a new autotune result makes a new graph.  Should the
 * runtime refuse a capture, the context switches itself to mode 0 and the
 * estimate runs kernel by kernel (capture_failed below).  Mode 0
 * launches every estimate kernel by kernel and drops the kept graphs.
 * Thread-safe (estimates of a context run one at a time). */
ld_status ld_graph_mode(ld_ctx* ctx, int32_t mode);
typedef struct {
  uint64_t captures;  /* graphs captured                                      */
  uint64_t replays;   /* estimates run as a graph replay                      */
  uint64_t eager;     /* blocking estimates launched kernel by kernel         */
  uint64_t cached;    /* graphs kept now                                      */
  int32_t mode;       /* the ld_graph_mode setting                            */
  int32_t capture_failed; /* 1: a capture or instantiation failed; the context
                           * then switched to mode 0 and ran that estimate
                           * kernel by kernel                                 */
} ld_graph_stats;
ld_status ld_graph_stats_get(ld_ctx* ctx, ld_graph_stats* out);

/* Instrumentation (off by default).  While enabled, every launch of a kernel
 * family in `family_mask` is bracketed by two HIP events recorded on the
 * stream the kernel runs on.  ld_profile_query returns, for the families in
 * `family` (summed), the number of launches, the summed device time (ms) and
 * the summed algorithmic bytes: the minimum HBM traffic each launch implies
 * (matrix, vectors read, vectors written; partial sums excluded).  Enabling
 * (or disabling) resets the counters.  Times are harvested when a blocking
 * estimate returns. */
enum {
  LD_PROF_SPMM = 1,     /* CSR x probe block                                 */
  LD_PROF_DOTS = 2,     /* window inner products                             */
  LD_PROF_UPDATE = 4,   /* orthogonalisation update + norms                  */
  LD_PROF_REDUCE = 8,   /* fixed-order reductions of partial sums            */
  LD_PROF_SMALL = 16,   /* per-probe bookkeeping, quadrature, Hessenberg log */
  LD_PROF_SKETCH = 32,  /* Gram, Cholesky, triangular solve, projection      */
  LD_PROF_PROBES = 64,  /* Rademacher generation                             */
  LD_PROF_ALL = 127
};
ld_status ld_profile_enable(ld_ctx* ctx, uint32_t family_mask);
ld_status ld_profile_query(ld_ctx* ctx, uint32_t family, int64_t* launches, double* total_ms,
                           double* total_bytes);

/* Test hook: the Rademacher probe columns col_begin..col_end-1 (n rows) as
 * generated on the device, copied to host memory out[n * (col_end -
 * col_begin)], row-major. */
ld_status ld_debug_rademacher(ld_ctx* ctx, uint64_t seed, int64_t n,
                              int32_t col_begin, int32_t col_end, double* out);
/* Test hook: the quadrature value K_p = e1^T log(T_p) e1 of `runs`
 * symmetric tridiagonal matrices, computed as the estimates compute it (the
 * trapezoidal rule on the Stieltjes integral of log for [a, b], the
 * Golub-Welsch rule for a T_p with an eigenvalue outside [a/1000, 1000 b]).
 * T_p has dimension dims[p] <= m, diagonal alpha[p*m + t] and off-diagonal
 * beta[p*m + t] (t < dims[p] - 1), host arrays.  need[p] = 1 where the
 * Golub-Welsch rule gave K_p.  LD_E_NUMERIC on a non-positive Ritz value or
 * a non-finite K. */
ld_status ld_debug_quad_log(ld_ctx* ctx, int32_t runs, int32_t m, const double* alpha,
                           const double* beta, const int32_t* dims, double a, double b,
                           double* K, int32_t* need);
/* Test hook: as ld_debug_rademacher for either distribution (ld_probe_dist). */
ld_status ld_debug_probes(ld_ctx* ctx, uint64_t seed, int64_t n, int32_t col_begin,
                          int32_t col_end, int32_t dist, double* out);

/* Calibration hook: copies `bytes` (rounded down to 16) between two device
 * buffers with a plain 16-byte-per-lane copy kernel, `reps` times, and
 * returns the mean device time per copy in *ms.  Used to scale hardware
 * byte counters (FETCH_SIZE / WRITE_SIZE) against a transfer of known size
 * and to measure attainable HBM bandwidth. */
ld_status ld_debug_copy(ld_ctx* ctx, uint64_t bytes, int32_t reps, double* ms);
/* Calibration hook: attainable streaming bandwidth at a read:write mix.  A
 * plain stream kernel (four 16-byte items per lane in flight, streaming
 * loads and stores, up to 32768 short blocks: the fastest shape measured)
 * reads `reads` (1..3) device buffers of `bytes` each and, with writes = 1,
 * writes their elementwise sum to a fourth (writes = 0: reads only).  Runs `reps` times after a warm-up and
 * returns the mean device time per run in *ms; the bytes moved are
 * (reads + writes) * bytes. */
ld_status ld_debug_stream(ld_ctx* ctx, uint64_t bytes, int32_t reads, int32_t writes,
                          int32_t reps, double* ms);
/* Debug: the matrix's row groups (the product's alternative storage, see
 * ld_autotune).  *n_union = the number of union columns (0: the matrix
 * keeps none).  When gp, col and val are all non-NULL, also copies into
 * them (caller-owned host memory, sized from a first call with NULL
 * arrays) the group pointers gp[ceil(n / 4) + 1], the union columns
 * col[n_union] and their FP64 values val[4 n_union] (val[4 u + r]: row r
 * of the group, zero where that row has no entry).  Blocking. */
ld_status ld_debug_row_groups(ld_matrix* a, int64_t* n_union, int32_t* gp, int32_t* col,
                              double* val);

#ifdef __cplusplus
}
#endif
#endif /* LIBLOGDET_H */
