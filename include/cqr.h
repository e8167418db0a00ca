/*
 * libcqr: CholeskyQR2 with block Gram-Schmidt on AMD Instinct MI355X (gfx950).
 *
 * Thin QR factorisation A = Q R of a tall-and-skinny FP64 matrix (m >= n)
 * by the two schedules of Mijic, Kaushik and Davidovic, "QR factorization of
 * ill-conditioned tall-and-skinny matrices on distributed-memory systems"
 * (arXiv 2405.04237):
 *
 *   CQR_SCHED_ORIG  CholeskyQR2 with Gram-Schmidt (CQR2GS): block
 *                   Gram-Schmidt CholeskyQR (Algorithm 6, distributed form
 *                   Algorithm 8) applied twice, R = R2 R1 (Algorithm 7).
 *   CQR_SCHED_MOD   modified CQR2GS (mCQR2GS, Algorithm 9): CholeskyQR2 of the
 *                   first panel, then per panel one projection/update against
 *                   the previous (fully orthogonal) panel, CholeskyQR,
 *                   re-orthogonalisation against all previous panels, and
 *                   CholeskyQR again.
 *   CQR_SCHED_SCQR3 shifted CholeskyQR3 (sCQR3, Algorithm 5): shifted
 *                   CholeskyQR (Algorithm 4: W = A^T A + s I with
 *                   s = sqrt(m) u ||A||_F^2, u = 2^-53, W = R1^T R1,
 *                   Q1 = A R1^{-1}), then CholeskyQR2 of Q1 (Algorithm 3),
 *                   R = (R3 R2) R1. A whole-matrix algorithm: b is ignored
 *                   and n must not exceed CQR_MAX_PANEL. ||A||_F^2 is the
 *                   trace of the computed Gram matrix (the same sum of
 *                   squares, no extra pass over A).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrices are FP64 and column-major (LAPACK layout). A and Q are m x n
 *   with leading dimension lda >= max(1, m); R is n x n with leading
 *   dimension n. All pointers are device pointers unless marked "host".
 * - Panel j covers columns [j b, min((j+1) b, n)); the last panel may be
 *   narrower. b = 0 selects a default width; b > n is clamped to n. After
 *   clamping 1 <= b <= CQR_MAX_PANEL (a wider b returns
 *   CQR_ERR_UNSUPPORTED). The Cholesky factor and inverse of a panel's b x b
 *   Gram matrix are formed by one workgroup: for b <= 128 entirely in its
 *   local data share (128 x 128 FP64 = 128 KiB of the 160 KiB a gfx950
 *   workgroup may hold), for 128 < b <= 256 with the matrix in device
 *   workspace and 16-row blocks and the last 128 x 128 block in LDS (the
 *   same right-looking steps and block back substitution).
 * - A is only read. Q may equal A (in-place factorisation); any other
 *   overlap of A, Q, R, the workspace or the info word is an error the
 *   library does not detect.
 * - On success R is upper triangular with a positive diagonal and an exactly
 *   zero strict lower triangle.
 * - Calls are asynchronous and ordered on `stream` (a hipStream_t; NULL is
 *   the default stream). No entry point synchronises except cqr_get_info and
 *   cqr_profile_query. Results are bitwise reproducible for fixed arguments.
 * - Numerical breakdown is reported asynchronously through an info word in
 *   device memory: 0 = success; j > 0 = the Gram matrix of a panel was not
 *   numerically positive definite at global column j (1-based), i.e. a
 *   Cholesky pivot was not > 0 or was NaN (the failure mode the paper names
 *   in sections "CholeskyQR" and "CholeskyQR2"). Once set, the remaining
 *   kernels of that factorisation do nothing and Q, R are undefined.
 *   Nothing is retried or silently repaired, and only CQR_SCHED_SCQR3,
 *   whose shift is part of the algorithm, shifts a Gram matrix. (A NaN or
 *   infinite entry reaches every diagonal entry through that shift, so
 *   CQR_SCHED_SCQR3 reports such input at column 1.)
 * - Return values: CQR_OK, or a negative status (argument errors are
 *   detected before any device work is queued).
 */
#ifndef LIBCQR_CQR_H
#define LIBCQR_CQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum cqr_status {
  CQR_OK = 0,
  CQR_ERR_ARG = -1,         /* invalid argument; nothing was launched */
  CQR_ERR_HIP = -2,         /* a HIP runtime call or kernel launch failed */
  CQR_ERR_NOMEM = -3,       /* the library could not allocate its workspace */
  CQR_ERR_WORKSPACE = -4,   /* caller workspace smaller than required */
  CQR_ERR_UNSUPPORTED = -5  /* a size this build does not handle */
};

#define CQR_MAX_PANEL 256

enum cqr_schedule {
  CQR_SCHED_MOD = 0,   /* mCQR2GS, Algorithm 9 (default) */
  CQR_SCHED_ORIG = 1,  /* CQR2GS, Algorithm 7 */
  CQR_SCHED_SCQR3 = 2  /* shifted CholeskyQR3, Algorithms 4-5; n <= CQR_MAX_PANEL */
};

typedef struct cqr_options {
  int schedule;            /* enum cqr_schedule */
  int *d_info;             /* device int for the breakdown column; NULL = the
                              library's internal word (read by cqr_get_info) */
  void *workspace;         /* device scratch of >= cqr_workspace_bytes(...)
                              bytes, 256-byte aligned; NULL = a workspace the
                              library allocates once per device and keeps */
  size_t workspace_bytes;  /* size of `workspace` */
  int lookahead;           /* CQR_SCHED_MOD only. 1: overlap each panel's
                              CholeskyQR / re-orthogonalisation chain with the
                              trailing update of the panels after it (the
                              look-ahead the paper proposes as future work,
                              section "Conclusion"): the update is split into
                              the next panel's columns and the rest, and the
                              panel's chain runs on a library-owned side
                              stream (default priority) forked from and joined
                              back into `stream` with events. Same kernels on
                              the same operands: results are bitwise those of
                              lookahead = 0. 0: everything on `stream`. Zero-
                              initialise the struct; other schedules ignore
                              it. */
  int adaptive;            /* CQR_SCHED_MOD only. 1: the run-time choice of
                              CholeskyQR repetitions the paper proposes as
                              future work (section "Conclusion"): a repeated
                              CholeskyQR of a panel is left out (U = I) when
                              its input's Gram matrix W has ||W - I||_F <=
                              CQR_ADAPTIVE_TOL, and the re-orthogonalisation
                              update when its coefficients have ||Z||_F <=
                              CQR_ADAPTIVE_TOL (Z := 0). Decided on the device
                              (no synchronisation); the accuracy bounds are
                              kept, and well-conditioned panels cost fewer
                              passes. 0: every repetition runs. */
  int update_tile;         /* kernel variant of the trailing updates
                              A_rest -= Q_j Y and Qt -= Q_{1:j-1} Z (enum
                              cqr_tile; the panel width b is the paper's
                              tuning knob, section "CholeskyQR2 with
                              Gram-Schmidt", and these are the GPU's): every
                              variant computes each entry with the same
                              operations in the same order, so the choice
                              changes speed only, never the bits. A variant
                              that does not apply to a shape or alignment
                              falls back to CQR_TILE_AUTO. */
  int proj_tile;           /* kernel variant of the projections
                              Y = Q_j^T A_rest and Z = Q_{1:j-1}^T Qt (enum
                              cqr_tile: CQR_TILE_WIDE or CQR_TILE_NARROW;
                              same bits either way). */
} cqr_options;

/* Kernel variants of the streaming products (cqr_options.update_tile and
 * proj_tile); values outside the enum return CQR_ERR_ARG. */
enum cqr_tile {
  CQR_TILE_AUTO = 0,   /* the library's default for the shape */
  CQR_TILE_SLAB = 1,   /* update: 64-column slab of Y in LDS, rows streamed
                          (inner dimension <= 128) */
  CQR_TILE_WIDE = 2,   /* 64 x 128 output tile per wave, accumulators held
                          over the whole inner dimension (update and
                          projection) */
  CQR_TILE_NARROW = 3, /* update: 32 x 64 tiles, four waves per workgroup;
                          projection: 64 x 64 tiles */
  CQR_TILE_RESIDENT = 4 /* update: each wave's rows of Q_j held in registers
                           while it sweeps every 64-column slab of the
                           update (Q_j read once), inner dimension <= 128
                           and a multiple of 16 */
};

/* Tolerance of cqr_options.adaptive (a Frobenius norm). */
#define CQR_ADAPTIVE_TOL 1e-14

/* Factor A = Q R with the default schedule (mCQR2GS). Q has leading
 * dimension lda, R leading dimension n. Uses the library's internal
 * workspace and info word (read the info word with cqr_get_info), so
 * concurrent calls on different streams of one device must use
 * cqr_factor_ex with their own workspace instead.
 *
 * The internal workspace is allocated by the first call on a device and
 * grown, when a later call needs more, in stream order on `stream`: that
 * stream waits (an event, not the host) for the last call that used the old
 * buffer, which is then released with hipFreeAsync, and the new buffer comes
 * from hipMallocAsync. The host never waits for the device. A call made
 * while `stream` is being captured into a graph must not use the internal
 * workspace (it returns CQR_ERR_ARG: pass a workspace to cqr_factor_ex), and
 * the first call on a device, which allocates the info word, must not be
 * captured. */
int cqr_factor(int64_t m, int64_t n, int64_t b, const double *A, int64_t lda,
               double *Q, double *R, void *stream);

/* As cqr_factor, with the schedule, info word and workspace chosen by the
 * caller (opt may be NULL for the defaults). */
int cqr_factor_ex(int64_t m, int64_t n, int64_t b, const double *A, int64_t lda,
                  double *Q, double *R, void *stream, const cqr_options *opt);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * cqr_factor_ex with a caller workspace, but the workspace is a fixed
 * CQR_NOALLOC_SCRATCH_BYTES array in the library's device code, one per
 * device, created when the library's device code is loaded on that device
 * and held until the process ends. The call allocates nothing (no hipMalloc
 * or hipFree, no events; per-kernel profiling does not bracket it), and the
 * caller still owns A, Q, R and the info word.
 *   schedule  enum cqr_schedule; the look-ahead and adaptive options are off.
 *   d_info    device int, required (NULL is CQR_ERR_ARG); 0 or the 1-based
 *             breakdown column, as for cqr_factor_ex.
 * Sizes whose in-place workspace (cqr_workspace_bytes(m, n, b, schedule))
 * exceeds CQR_NOALLOC_SCRATCH_BYTES return CQR_ERR_WORKSPACE before any
 * device work. An aliasing lda (a multiple of 1024 doubles) is factored in
 * place, never through a staging copy. Results are bitwise those of
 * cqr_factor_ex with the same arguments and a caller workspace of that size.
 * Every call on a device shares that device's array, and nothing in it needs
 * to start at zero (each call writes every region before reading it): calls
 * that overlap in time on one device, on any streams, race and give
 * undefined results. The first call on a device looks up the array's device
 * address (hipGetSymbolAddress) and must not be made during stream capture;
 * later calls may be captured. */
#define CQR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int cqr_factor_noalloc(int64_t m, int64_t n, int64_t b, const double *A, int64_t lda,
                       double *Q, double *R, int schedule, int *d_info, void *stream);

/* Bytes of device workspace cqr_factor_ex needs for these sizes and leading
 * dimension (host arithmetic only; 0 for invalid sizes, lda < m included).
 * The info word is not included. When lda is a multiple of 1024 doubles the
 * column lines the split-m products read at one row share a few cache sets;
 * such a call factors a copy with a shifted stride, and the workspace
 * includes room for it (lda * n doubles). A caller workspace without that
 * room (at least the size for a non-aliasing lda) is accepted, and the call
 * then factors in place at the aliasing stride (same results, slower). */
size_t cqr_workspace_bytes_ld(int64_t m, int64_t n, int64_t b, int64_t lda, int schedule);

/* cqr_workspace_bytes_ld with lda = m (a tightly packed matrix). */
size_t cqr_workspace_bytes(int64_t m, int64_t n, int64_t b, int schedule);

/* Panel width used when b = 0 is passed (n for CQR_SCHED_SCQR3, which has
 * no panels). */
int64_t cqr_default_panel(int64_t m, int64_t n, int schedule);

/* Batched factorisation: many independent matrices of uneven shape in one
 * persistent launch. Each workgroup takes the next work item from a queue
 * ordered longest-first (work ~ the bytes a matrix moves, m n (1 + n / b))
 * and runs mCQR2GS (Algorithm 9) on it, with its panel reductions over rows
 * finished in the workgroup's local memory. A matrix whose work exceeds one
 * workgroup's fair share is split by rows over a team of up to four
 * workgroups (at least 2048 rows each); in a batch of at most one matrix
 * per eight resident workgroups every matrix is split over up to sixteen
 * (at least 128 rows each), so that a few matrices still fill the device.
 * Team members add their row-reduced products in a fixed member order
 * through device memory (the paper's distributed form, Algorithm 8, with
 * workgroups for ranks); every member repeats the small Cholesky steps.
 * All workgroups of the launch are
 * resident at once, so team members always find their partners; a wait
 * that still exceeds a spin limit of a few seconds ends with info = -1.
 *
 * cqr_plan_batched (host shapes; allocates and synchronises, so call it
 * outside graph capture): h_m[i], h_n[i] the shape of matrix i, h_b[i] its
 * panel width (h_b == NULL or 0 = min(ceil(n / 2), 32); clamped to n). Limits of this
 * form: n <= 128, panel width <= 32, m <= 2^33; schedule must be CQR_SCHED_MOD
 * (CQR_ERR_UNSUPPORTED otherwise).
 *
 * cqr_factor_batched enqueues a reset kernel (queue word, team counters) and
 * one persistent kernel on `stream` and nothing else: no allocation, no
 * memset, no synchronisation,
 * so the call can be captured into a HIP graph and replayed. d_A, d_lda,
 * d_Q, d_R are device arrays (indexed by matrix id) of device pointers and
 * leading dimensions: A_i and Q_i are m_i x n_i column-major with leading
 * dimension d_lda[i] >= m_i (Q_i may equal A_i), R_i is n_i x n_i
 * column-major with leading dimension n_i. d_info[i] receives 0, the
 * 1-based breakdown column of matrix i, or -1 (a team wait timed out); in
 * both error cases Q_i and R_i are undefined. Calls that use the same plan
 * must not overlap in time (they share its queue and team buffers). */
typedef struct cqr_batch_plan cqr_batch_plan;
int cqr_plan_batched(int64_t batch, const int64_t *h_m, const int64_t *h_n, const int64_t *h_b,
                     int schedule, cqr_batch_plan **plan);
int cqr_factor_batched(const cqr_batch_plan *plan, const double *const *d_A,
                       const int64_t *d_lda, double *const *d_Q, double *const *d_R,
                       int *d_info, void *stream);
void cqr_plan_destroy(cqr_batch_plan *plan);

/* Reverse-mode derivative (adjoint) of the thin QR map A -> (Q, R), m >= n,
 * for full-column-rank A with R's diagonal positive:
 *     dA = (dQ + Q copyltu(M)) R^{-T},   M = R dR^T - dQ^T Q,
 * copyltu(M) = tril(M) + tril(M, -1)^T. The paper does not differentiate the
 * factorisation; this is the published QR adjoint, computed with the same
 * kernel shapes as the forward factorisation: one split-m pass for the lower
 * triangle of dQ^T Q (a fixed-order reduction), n x n work for R^{-1} and
 * copyltu(M) R^{-T}, and one streaming pass dA = [dQ | Q] [R^{-T}; C R^{-T}].
 *
 * Q, A, dQ and dA are m x n column-major with leading dimension lda; R and dR
 * are n x n column-major with leading dimension n. Q == NULL selects the
 * recompute mode: Q = A R^{-1} is never formed, products with Q are applied
 * as products with A followed by R^{-1} on the n x n side (A must then be
 * non-NULL; otherwise A is ignored). dQ and dR may be NULL (zero cotangent);
 * the strict lower triangle of dR is ignored. dA must not overlap any input.
 * 1 <= n <= CQR_MAX_PANEL (R^{-1} is formed by one workgroup, as the
 * factorisation's U^{-1}).
 * workspace: >= cqr_backward_workspace_bytes(m, n, batch) bytes of device
 * memory, 256-byte aligned, or NULL for a buffer the library keeps per device
 * (grown in stream order as cqr_factor's workspace; a call during stream
 * capture must pass its own and otherwise returns CQR_ERR_ARG).
 * Asynchronous on `stream`; bitwise reproducible. R^{-1} is computed on a
 * library-owned side stream of default priority, forked from and joined back
 * into `stream` with events, so it overlaps the first pass (a graph capture
 * of `stream` records the fork and join; the first call on a device, which
 * creates that stream, must not be made during a capture). Returns CQR_OK
 * or a negative status (argument errors before any device work). */
size_t cqr_backward_workspace_bytes(int64_t m, int64_t n, int64_t batch);
int cqr_backward(int64_t m, int64_t n, const double *Q, const double *A, int64_t lda,
                 const double *R, const double *dQ, const double *dR, double *dA, void *stream,
                 void *workspace, size_t workspace_bytes);

/* The adjoint of `batch` equally shaped factorisations in one set of launches
 * (batch index on the grid). Matrix i of Q, A, dQ and dA starts at base +
 * i * stride (stride >= lda * n doubles); R and dR at base + i * n * n.
 * batch <= 65535. */
int cqr_backward_batched(int64_t batch, int64_t m, int64_t n, const double *Q, const double *A,
                         int64_t lda, int64_t stride, const double *R, const double *dQ,
                         const double *dR, double *dA, void *stream, void *workspace,
                         size_t workspace_bytes);

/* Wait for `stream` and copy the library's internal info word of the current
 * device into *info (host). */
int cqr_get_info(void *stream, int *info);

/* Human-readable text of a status code (static storage). */
const char *cqr_status_string(int status);

/* Per-kernel timing. While enabled, every kernel launch of the library is
 * bracketed by HIP events on its stream and credited with its algorithmic
 * flops and bytes (the paper's Table 1/2 counts: Gram m w^2, forming Q
 * m w^2, projection and update 2 m p q each). cqr_profile_query waits for
 * the recorded events and returns, for kernel class `kind` (enum
 * cqr_kernel_kind), the number of launches, their summed duration in
 * milliseconds and their summed algorithmic flops and bytes. */
enum cqr_kernel_kind {
  CQR_K_GRAM = 0,     /* split-m Gram partials of a panel (SYRK) */
  CQR_K_PROJ = 1,     /* split-m projection partials Y = Q_j^T Z */
  CQR_K_UPDATE = 2,   /* trailing update Z -= Q_j Y, inner dimension <= 128 */
  CQR_K_TRSM = 3,     /* Q_j = X U^{-1} (explicit inverse, streaming GEMM) */
  CQR_K_REDUCE = 4,   /* fixed-order sum of split-m partials */
  CQR_K_CHOL = 5,     /* b x b Cholesky + triangular inverse, one workgroup */
  CQR_K_SMALL = 6,    /* small R-block products, fills and the sCQR shift */
  CQR_K_BATCHED = 7,  /* the persistent batched factorisation (whole launch) */
  CQR_K_COPY = 8,     /* copy into the staging buffer */
  CQR_K_UPDATE_LONG = 9, /* update Qt -= Q_{1:j-1} Z, inner dimension > 128 */
  CQR_K_COUNT = 10
};
int cqr_profile_enable(int on);
/* Restrict the bracketing to the kernel classes whose bit (1u << kind) is
 * set in kind_mask (default: all), so that a timed run can carry events
 * around one class only. */
int cqr_profile_select(unsigned kind_mask);
int cqr_profile_reset(void);
int cqr_profile_query(int kind, int64_t *launches, double *ms, double *flops,
                      double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* LIBCQR_CQR_H */
