/*
 * bks.h -- C ABI of libbks: block Krylov-Schur (BKS) and HOOI for the best
 * rank-(r, r, r3) approximation of large sparse (1,2)-symmetric tensors on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: L. Elden and M. Dehghan, "A Krylov-Schur like method for computing
 * the best rank-(r1,r2,r3) approximation of large and sparse tensors".
 *
 * Problem (eq. main min, eq. max): given A in R^{m x m x n} with
 * A(i,j,k) = A(j,i,k) (Definition of a (1,2)-symmetric tensor, section "Notation"),
 * find U (m x r) and W (n x r3) with orthonormal columns maximising
 * ||A.(U, U, W)||; the optimal core is F = A.(U, U, W) (eq. Rayleigh).  The
 * large tensor is touched only through the tensor-times-block products
 * exported here as bks_ttmc (section "Block-Krylov methods", Algorithm 3).
 *
 * Conventions
 *   - Indices are 0-based.  Dense matrices passed to bks_ttmc are row-major
 *     with a leading dimension in elements (row i at ptr + i*ld).  Solver
 *     inputs and outputs (U, W, F) are host FP64 arrays in column-major
 *     (Fortran) order.
 *   - Return value 0 is success, negative values are errors, BKS_ENOTCONV
 *     (positive) means the iteration cap was reached; results are written.
 *     bks_last_error(ctx) gives a message for the last failure on that ctx.
 *   - Ownership: the caller owns every buffer it passes.  Handles (ctx,
 *     tensor, server) are owned by the library until destroyed/freed.  A ctx
 *     is used by one host thread at a time.
 *   - Streams: `stream` arguments are hipStream_t values passed as void*;
 *     NULL means the null stream.
 *   - Devices: a call on a ctx (or on a tensor of one) makes the ctx's
 *     device current on the calling thread and leaves it so;
 *     bks_server_create restores the caller's.
 *
 * Environment (the first six are read once per process; results do not
 * depend on them unless stated)
 *   BKS_HOST_THREADS      host threads of the inner solve (default: hardware
 *                         concurrency, at most 8)
 *   BKS_DEVICE_CORE_MIN   cores with at least this many entries (k1^2 k3) form
 *                         their dense products on the device (default 1e5;
 *                         results change only by rounding order)
 *   BKS_DEVICE_HOOI_MIN   of those, cores with at least this many entries also
 *                         run the HOOI steps' and the objective's products on
 *                         the device (default 1e5; rounding order only)
 *   BKS_DEVICE_SOLVE_MIN  Newton systems of at least this order are factorised
 *                         on the device (default 256; rounding order only)
 *   BKS_NARROW_REG        bit mask of the narrow products that take the
 *                         register-direct kernel instead of the LDS-staged
 *                         one: 1 FREE3 symmetric half, 2 FREE3 with X != Y,
 *                         4 MODE3 (and FREE1's first step), 8 FREE1's second
 *                         step (default 8; rounding order only)
 *   BKS_DEBUG_INNER=1     one line per inner solve on stderr
 *   BKS_FAIL_NEXT_ALLOC=1 checked at every device allocation: the next one
 *                         fails with BKS_ENOMEM and the variable is cleared
 *                         (tests of the error paths)
 */
#ifndef BKS_H
#define BKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bks_ctx_s *bks_ctx;
typedef struct bks_tensor_s *bks_tensor;
typedef struct bks_server_s *bks_server;

/* status codes */
#define BKS_OK 0
#define BKS_EINVAL (-1)   /* bad argument (sizes, ranks, leading dimensions) */
#define BKS_EINDEX (-2)   /* index out of range in uploaded coordinates */
#define BKS_EVALUE (-3)   /* NaN or Inf value */
#define BKS_EASYM (-4)    /* (i,j,k) and (j,i,k) given with different values */
#define BKS_ENOMEM (-5)   /* device allocation failed or over the ctx budget */
#define BKS_EDEVICE (-6)  /* HIP runtime error */
#define BKS_ENOTFOUND (-7)/* unknown request id */
#define BKS_EDUP (-8)     /* repeated position without BKS_SUM_DUPLICATES */
#define BKS_ECANCELED (-9)/* request cancelled (bks_server_cancel) */
#define BKS_ENOTCONV 1    /* iteration cap reached; results still written */

/* value / compute precisions */
#define BKS_F32 0           /* FP32 values, factors, accumulation, output */
#define BKS_F64 1           /* FP64 factors, accumulation and output */
#define BKS_F32IN_F64ACC 2  /* FP32 tensor values, FP64 factors/accum/output */

/* tensor-times-block operations (section "Multilinear tensor-matrix multiplication"; section "Block-Krylov methods for (1,2)-symmetric tensors") */
#define BKS_FREE3 0  /* T3 = A.(X, Y)_{1,2}: n x q */
#define BKS_FREE1 1  /* T1 = A.(Y, Z)_{2,3}: m x (py*pz) */
#define BKS_MODE3 2  /* t = A.(Z)_3 on the stored pair pattern: P x pz */

/* upload flags */
#define BKS_DEVICE_PTRS 1     /* i, j, k, val are device pointers */
#define BKS_SUM_DUPLICATES 2  /* repeated canonical positions are summed */
#define BKS_FULL_SYMMETRIC 4  /* input lists both (i,j,k) and (j,i,k) */
#define BKS_SCALE_FROBENIUS 8   /* scale every slice A(:,:,k) to Frobenius norm 1 */
#define BKS_SCALE_LAMBDA_MAX 16 /* scale every slice so its largest eigenvalue is 1 */

/* solver variants (Tables 1-3) and precision modes */
#define BKS_VARIANT_BK 0
#define BKS_VARIANT_MIN 1
#define BKS_VARIANT_MAX 2
#define BKS_PREC_FP64 0   /* every product in FP64 */
#define BKS_PREC_MIXED 1  /* FP32 expansion/core products, FP64 elsewhere */

/* Create a context on HIP device `device`.  `mem_budget_bytes` caps the
 * device memory the ctx may hold (0 = no cap).  Errors: BKS_EDEVICE. */
int bks_ctx_create(int device, size_t mem_budget_bytes, bks_ctx *out);
void bks_ctx_destroy(bks_ctx ctx);
/* Message for the last nonzero status returned on ctx (never NULL). */
const char *bks_last_error(bks_ctx ctx);
/* Library version string. */
const char *bks_version(void);

/* Kernel timing on ctx: with enable = 1 every tensor-times-block launch made
 * through ctx (bks_ttmc and the solvers) is bracketed by HIP events on the
 * stream it runs on; statistics are reset.  enable = 0 stops recording. */
int bks_ctx_profile(bks_ctx ctx, int enable);
/* Read profile entry `idx` (0-based; BKS_ENOTFOUND past the end): kernel
 * class name, launches, total milliseconds (from the events), and the
 * algorithmic bytes and flops summed over those launches (the stored tensor
 * read once, factors read once, output written once; 2 flops per FMA).
 * Synchronises the recorded streams. */
int bks_ctx_profile_read(bks_ctx ctx, int idx, char *name, int name_len, int64_t *calls,
                         double *ms, double *bytes, double *flops);

/* Upload a (1,2)-symmetric tensor given as coordinates (Definition of a
 * (1,2)-symmetric tensor, section "Notation").  Each entry (i, j, k, val) names the
 * positions (i,j,k) and (j,i,k) of A; (i,j) is canonicalised to
 * (min, max).  With BKS_FULL_SYMMETRIC the input is expected to hold both
 * orientations of off-diagonal entries and one copy is kept (values must
 * agree, else BKS_EASYM).  Repeated canonical positions are summed with
 * BKS_SUM_DUPLICATES, else BKS_EDUP.  `val_dtype` is BKS_F32 or BKS_F64;
 * FP64 values are kept in FP64 as well as rounded to FP32.  The library
 * builds its device formats (slice-major and row-major sorted segments, the
 * stored-pair pattern) once here and owns them until bks_tensor_free.
 * Slice scaling (section "Experiments": Example 3 normalises every slice of
 * a graph tensor so that its largest eigenvalue is 1, Example 4 scales every
 * slice to Frobenius norm 1): with BKS_SCALE_FROBENIUS each slice, as the
 * full symmetric matrix, is divided by its Frobenius norm; with
 * BKS_SCALE_LAMBDA_MAX by its spectral radius, the largest eigenvalue of a
 * nonnegative (adjacency) slice and its largest eigenvalue magnitude in
 * general (dense eigensolver on the slice's touched rows up to 400 of them,
 * else Lanczos with full reorthogonalisation to a 1e-14 relative residual).
 * Zero slices stay zero; the scaled values are what the tensor holds
 * (frob_norm of bks_tensor_info included).  Both flags at once: BKS_EINVAL.
 * With BKS_DEVICE_PTRS the four arrays are device memory that the caller
 * has finished writing (its stream synchronised); they are copied to the
 * host and not kept.  The call returns once the device formats are
 * resident.
 * Errors: BKS_EINVAL (m, n < 1, nnz < 0, or 2 n m^2 >= 2^64: the
 * upload sorts by 64-bit keys over (k, i, j)), BKS_EINDEX, BKS_EVALUE,
 * BKS_EASYM, BKS_EDUP, BKS_ENOMEM, BKS_EDEVICE. */
int bks_tensor_upload(bks_ctx ctx, int64_t m, int64_t n, int64_t nnz, const int32_t *i,
                      const int32_t *j, const int32_t *k, const void *val, int val_dtype,
                      unsigned flags, bks_tensor *out);
/* Sizes of an uploaded tensor: m, n, stored entries (i <= j), distinct
 * stored (i <= j) pairs, ||A||_F (full tensor, FP64) and device bytes held.
 * Any output pointer may be NULL. */
int bks_tensor_info(bks_tensor t, int64_t *m, int64_t *n, int64_t *nnz_stored,
                    int64_t *npairs, double *frob_norm, size_t *dev_bytes);
/* Copy the stored pair pattern (i <= j, sorted by (i, j)) that orders the
 * rows of a BKS_MODE3 result into host arrays of length npairs. */
int bks_tensor_pairs(bks_tensor t, int32_t *pi, int32_t *pj);
void bks_tensor_free(bks_tensor t);

/* Tensor-times-block product on device memory, asynchronous on `stream`
 * (section "Multilinear tensor-matrix multiplication" mode products; Algorithm 3 step (i); section "Block-Krylov methods for (1,2)-symmetric tensors").
 *
 *   BKS_FREE3: B1 = X (m x p1), B2 = Y (m x p2) or NULL for Y = X.
 *     out(k, a + p1*b) = sum_{i,j} A(i,j,k) X(i,a) Y(j,b)     (n x p1*p2)
 *     With sym_half (Y = X): the upper triangle a <= b only, column
 *     b*(b+1)/2 + a (triunfold_3, section "Block-Krylov methods for (1,2)-symmetric tensors")              (n x p1(p1+1)/2)
 *   BKS_FREE1: B1 = Y (m x p1), B2 = Z (n x p2).
 *     out(i, b + p1*c) = sum_{j,k} A(i,j,k) Y(j,b) Z(k,c)     (m x p1*p2)
 *   BKS_MODE3: B2 = Z (n x p2); B1 unused.
 *     out(q, c) = sum_k A(i_q, j_q, k) Z(k, c) for the q-th stored pair
 *     (i_q <= j_q) of bks_tensor_pairs                        (P x p2)
 *
 * prec: BKS_F32 (B1, B2, out are float), BKS_F64 or BKS_F32IN_F64ACC
 * (double).  ld1/ld2/ldo are row strides in elements.  Widths p1, p2 must be
 * >= 1; FREE1 and X != Y products need p1*p2 <= 1600.  The result overwrites
 * out; every output row is written.  Device workspace (block-packed factor
 * copies, split-segment partial rows) is owned by ctx and grows on demand:
 * calls on one ctx whose execution overlaps on different streams race on
 * it, so use one stream per ctx (or one ctx per stream).
 * Errors: BKS_EINVAL, BKS_ENOMEM, BKS_EDEVICE. */
int bks_ttmc(bks_ctx ctx, bks_tensor t, int op, const void *B1, int64_t ld1, int p1,
             const void *B2, int64_t ld2, int p2, int sym_half, int prec, void *out,
             int64_t ldo, void *stream);

/* bks_ttmc for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * products, the same kernels and bit-identical results, but every device
 * workspace of the call -- block-packed factor copies, the partial rows of
 * split segments and the work schedule -- is carved out of a fixed scratch
 * array that the library holds on each device it runs on, so no device
 * memory is allocated or freed.  The scratch is 256 MiB per device, held
 * until the process ends; a product that needs
 * more returns BKS_EINVAL with a message, as do symmetric halves wider than
 * 24 columns (the core product; use bks_ttmc).  The tensor's formats are
 * those of bks_tensor_upload; B1, B2, out are as for bks_ttmc.  The schedule
 * is copied from host memory kept by the tensor with hipMemcpyAsync on
 * `stream`.  All calls on one device share its scratch: calls whose
 * execution overlaps (other streams, other contexts, other threads) race
 * and must be serialised by the caller; the scratch keeps the last call's
 * contents and nothing in it needs clearing.
 * Errors: BKS_EINVAL, BKS_EDEVICE. */
int bks_ttmc_noalloc(bks_ctx ctx, bks_tensor t, int op, const void *B1, int64_t ld1, int p1,
                     const void *B2, int64_t ld2, int p2, int sym_half, int prec, void *out,
                     int64_t ldo, void *stream);

typedef struct {
    int r, r3;          /* target multilinear rank (r, r, r3) */
    int s, p;           /* stages and block width: BKS(s, p; k1, k3); 0 = defaults 2, 4 */
    int variant;        /* BKS_VARIANT_* */
    int precision;      /* BKS_PREC_* */
    double tol;         /* ||grad|| / ||F|| stop; <= 0: 1e-13 (FP64), 1e-11 (mixed) */
    double inner_tol;   /* inner Newton-Grassmann tolerance; <= 0: 1e-13 */
    int max_outer;      /* <= 0: 200 */
    int hooi_warm;      /* HOOI steps on the core before Newton; < 0: 5 */
    int ng_max;         /* <= 0: 50 */
    const double *U0;   /* optional host start, m x r column-major (orthonormalised here) */
    const double *W0;   /* optional host start, n x r3 column-major */
    uint64_t seed;      /* start drawn from this seed when U0/W0 are NULL */
    int inner_start;    /* 0: HOSVD + HOOI warm-up (section "Experiments"); 1: the current
                           point (the restart point is the projected problem's
                           leading coordinates) */
} bks_params;

typedef struct {
    int outer_iters;    /* outer iterations (restarts) done */
    int converged;      /* 1 if rel_grad <= tol */
    int k1, k3;         /* basis dimensions of the last expansion */
    double rel_grad;    /* ||grad|| / ||F|| at the returned point */
    double normF, normA;
    double svals1[65];  /* s_1..s_r, s_{r+1} of mode 1 (section "Conditioning of the best approximation problem") */
    double svals3[65];  /* s_1..s_r3, s_{r3+1} of mode 3 */
    double t_expand, t_core, t_inner, t_step, t_total;  /* seconds per phase */
    int n_hist;
    double rel_hist[512];  /* per outer iteration */
    double normF_hist[512];
    double svals2[65];  /* s_1..s_r2, s_{r2+1} of mode 2 (general tensors; = svals1 when U = V) */
    int fp64_from;      /* mixed precision: the first outer iteration (HOOI: iteration) whose
                           products ran in FP64 because the FP32 ones had reached their
                           rounding floor; -1: none */
} bks_info;

/* Block Krylov-Schur solve (Algorithm 5 with U = V, section "A Tensor Krylov-Schur like method"): outputs U
 * (m x r), W (n x r3) and F (r x r x r3, column-major) to host memory.
 * Requires 1 <= r <= m, 1 <= r3 <= n, r3 <= r(r+1)/2 (else W0 cannot be
 * spanned by the first products).  k1 > m or k3 > n is capped
 * (section "BK method").  Returns BKS_ENOTCONV if max_outer is reached.  `info` may be NULL.
 * Runs on the ctx's stream with the ctx's workspaces (device buffers,
 * coherent pinned host staging buffers, 1 MiB plus the size of the inner
 * solve's transfers, the rocBLAS handle): solves on one ctx
 * must not overlap; concurrent solves use one ctx each (or a server).
 * Errors: BKS_EINVAL, BKS_ENOMEM, BKS_EDEVICE. */
int bks_solve(bks_ctx ctx, bks_tensor t, const bks_params *prm, double *U, double *W,
              double *F, bks_info *info);

typedef struct {
    int r, r3;
    int precision;      /* BKS_PREC_FP64 or BKS_PREC_MIXED */
    double tol;         /* <= 0: 1e-13 */
    int max_iter;       /* <= 0: 2000 */
    int grad_every;     /* <= 0: 10 (section "Higher Order Orthogonal Iteration") */
    const double *U0, *W0;
    uint64_t seed;
} hooi_params;

/* Symmetric HOOI (section "Higher Order Orthogonal Iteration").  Same outputs and errors as bks_solve;
 * info->outer_iters counts HOOI iterations. */
int hooi_solve(bks_ctx ctx, bks_tensor t, const hooi_params *prm, double *U, double *W,
               double *F, bks_info *info);

/* ---- general (non-symmetric) tensors --------------------------------- */

/* Upload a general tensor A in R^{l x m x n} from coordinates (i < l, j < m,
 * k < n; 0-based).  Repeated positions are summed with BKS_SUM_DUPLICATES,
 * else BKS_EDUP.  The library keeps three segmented streams (entries grouped
 * by their mode-1, mode-2 and mode-3 index), each holding every entry once.
 * The handle works with bks_gttmc, bks_gsolve, bks_tensor_info (which
 * reports m = l, npairs = the mode-2 size m, and n) and bks_tensor_free.
 * Errors: BKS_EINVAL (sizes, or l m n >= 2^64), BKS_EINDEX, BKS_EVALUE,
 * BKS_EDUP, BKS_ENOMEM, BKS_EDEVICE. */
int bks_gtensor_upload(bks_ctx ctx, int64_t l, int64_t m, int64_t n, int64_t nnz,
                       const int32_t *i, const int32_t *j, const int32_t *k, const void *val,
                       int val_dtype, unsigned flags, bks_tensor *out);

/* Product of a general tensor with one free mode (section "Multilinear
 * tensor-matrix multiplication"; Algorithm 3 step (i) in each mode), device
 * memory, asynchronous on `stream`:
 *   mode 0: out(i, a + p1 b) = sum_{j,k} A(i,j,k) B1(j,a) B2(k,b)  (l x p1 p2)
 *   mode 1: out(j, a + p1 b) = sum_{i,k} A(i,j,k) B1(i,a) B2(k,b)  (m x p1 p2)
 *   mode 2: out(k, a + p1 b) = sum_{i,j} A(i,j,k) B1(i,a) B2(j,b)  (n x p1 p2)
 * Layouts, precisions, workspace and errors as for bks_ttmc; p1 p2 <= 1600. */
int bks_gttmc(bks_ctx ctx, bks_tensor t, int mode, const void *B1, int64_t ld1, int p1,
              const void *B2, int64_t ld2, int p2, int prec, void *out, int64_t ldo,
              void *stream);

typedef struct {
    int r1, r2, r3;     /* target multilinear rank */
    int s, p;           /* stages and block width (0: 2, 4) */
    int precision;      /* BKS_PREC_* */
    double tol;         /* ||grad|| / ||F|| stop; <= 0: 1e-13 (FP64), 1e-11 (mixed) */
    double inner_tol;   /* inner tolerance; <= 0: 1e-13 */
    int max_outer;      /* <= 0: 200 */
    const double *U0, *V0, *W0;  /* optional host starts (l x r1, m x r2, n x r3, column-major) */
    uint64_t seed;      /* start drawn from this seed when a start is NULL */
} bks_gparams;

/* Block Krylov-Schur for a general tensor (Algorithm 5, section "A Tensor
 * Krylov-Schur like method"): three bases grown by the block-Krylov step of
 * Algorithm 3 in every mode -- the min-BK rule per mode: stage t makes
 * U_t from (Vbar_{t-1}, Wbar_{t-1}), V_t from (Ubar_{t-1}, Wbar_{t-1}), W_t
 * from (Ubar_{t-1}, Vbar_{t-1}), bars the first p columns (U0, V0, W0
 * whole) -- the core A.(X, Y, Z), its best rank-(r1, r2, r3) approximation
 * by truncated HOSVD and HOOI on the host, the restart, and the three-term
 * gradient of Proposition 3.2.  Outputs U (l x r1), V (m x r2), W (n x r3)
 * and F (r1 x r2 x r3), column-major host FP64; info->svals1/2/3 hold the
 * S-values of the three modes, info->k1 and k3 the mode-1 and mode-3 basis
 * sizes.  Requires 1 <= r_k <= min(dim_k, 64) and each r_k at most the
 * product of the other two.  Returns BKS_ENOTCONV at max_outer.
 * Errors: BKS_EINVAL, BKS_ENOMEM, BKS_EDEVICE. */
int bks_gsolve(bks_ctx ctx, bks_tensor t, const bks_gparams *prm, double *U, double *V,
               double *W, double *F, bks_info *info);

/* ---- serving: continuous batching of BKS solves ---------------------- */
typedef struct {
    int max_active;          /* sessions on the device at once (<= 0: 8) */
    int host_workers;        /* host threads for the small dense solves (<= 0: 4) */
    size_t mem_budget_bytes; /* device bytes the admitted sessions may hold (0: 75% free) */
} bks_server_params;

typedef struct {
    int status;              /* solve status (0, BKS_ENOTCONV, BKS_ECANCELED or an error) */
    int done;                /* 1 when finished */
    double t_submit, t_start, t_end;  /* seconds on the server clock */
    bks_info info;
    size_t footprint;        /* device bytes the request was admitted with */
    size_t dev_peak;         /* most device bytes its session held while it ran
                                (library buffers; the BLAS library's own
                                workspace is not counted) */
    char error[160];         /* message of a failed request, else empty */
} bks_result;

/* Create a server on ctx's device.  Requests are admitted while their
 * memory footprint fits the budget and a slot is free: a free slot takes the
 * oldest waiting request that fits, passing over one that does not fit at
 * most 16 times before it waits for that one.  The device work of admitted
 * sessions runs on per-session streams and overlaps.  Every slot's stream is
 * made here: BKS_EDEVICE (and no server) if one cannot be, or if the free
 * memory query fails when no budget is given.  The calling thread's current
 * device is left as it was. */
int bks_server_create(bks_ctx ctx, const bks_server_params *prm, bks_server *out);
/* Submit a solve of an uploaded tensor (the tensor must outlive the
 * request).  U, W, F are host buffers written when the request completes. */
int bks_server_submit(bks_server s, bks_tensor t, const bks_params *prm, double *U,
                      double *W, double *F, uint64_t *id);
/* Submit with upload: coordinates on the host are copied and uploaded by
 * the server when the request is admitted; the tensor is freed after. */
int bks_server_submit_coo(bks_server s, int64_t m, int64_t n, int64_t nnz, const int32_t *i,
                          const int32_t *j, const int32_t *k, const float *val,
                          const bks_params *prm, double *U, double *W, double *F,
                          uint64_t *id);
/* Non-blocking status of request id; res->done tells whether it finished. */
int bks_server_poll(bks_server s, uint64_t id, bks_result *res);
/* Block until request id finishes. */
int bks_server_wait(bks_server s, uint64_t id, bks_result *res);
/* Cancel request id.  A waiting request is removed from the queue and
 * finishes at once with status BKS_ECANCELED (its U, W, F untouched); a
 * running one stops at the start of its next outer iteration and finishes
 * with status BKS_ECANCELED, its U, W, F and info holding the point of its
 * last restart (or its start).  Returns 0 when the cancellation took effect
 * or is pending, BKS_ENOTFOUND for an unknown id, BKS_EINVAL when the
 * request had already finished. */
int bks_server_cancel(bks_server s, uint64_t id);
/* Seconds on the server clock (the clock of t_submit/t_start/t_end). */
double bks_server_now(bks_server s);
void bks_server_destroy(bks_server s);

#ifdef __cplusplus
}
#endif

#endif /* BKS_H */
