/*
 * lspca.h -- C ABI of the MI355X (gfx950) Lazy SPCA library, liblspca.so.
 *
 * Method: M. Wojnowicz, D. Nguyen, L. Li, X. Zhao, "Lazy stochastic principal
 * component analysis", arXiv 1709.07175. Lazy SPCA (Algorithm 2; streaming
 * form Algorithm 4) sketches the data X (m samples x n features) as
 * U = X Omega (eq. (rp), c = 1), forms the k x n factor F = U^T X
 * (eq. (simplified_approx_svd)) and returns the right singular vectors V of F:
 * the dimensionality-reduction map pi(x) = V^T x (eq. (dim_reduction_maps)).
 * SPCA (Algorithm 1) orthonormalises U by a QR first; both span the same
 * subspace (Proposition 2) and give identical pairwise distances
 * (Proposition 3). The library uses l = k (the paper's experiments do).
 *
 * Conventions shared by every entry point
 *  - Pointers named X, Omega, F, G, V, sigma, sigma_x and Z are DEVICE
 *    pointers (HIP global memory) owned by the caller; the library never
 *    frees caller memory. Host buffers are not accepted.
 *  - Matrices are row-major. X has leading dimension ldx >= n (elements):
 *    row i (one sample) starts at X + i*ldx. V is n x k, F is k x n, G is
 *    k x k, Z is r x k, all dense (leading dimension = number of columns).
 *  - Status: every call returns LSPCA_OK (0) or a negative lspca_status.
 *    No C++ exception crosses the ABI. On an error no output is written
 *    except where stated; lspca_last_error() gives a thread-local message.
 *  - Work is queued on opts->stream (a hipStream_t; NULL = the null stream).
 *    lspca_fit, spca_fit and lspca_factor return after the device work is
 *    complete (their status depends on it). lspca_accumulate, lspca_omega
 *    and lspca_transform only enqueue: outputs are ready when the stream is.
 *  - The library keeps a per-device workspace (grown on demand, freed at
 *    process exit). Calls that overlap on one device from several host
 *    threads are serialised by a lock, and on the device each call's work
 *    waits for the previous call's last use of the workspace (an event the
 *    library records after each call), whichever streams the two calls
 *    were queued on. Caller buffers are not ordered by the library: a
 *    caller that hands one call's output to a call on another stream orders
 *    the two streams itself.
 *  - X is never centred (Sec. I-B: the SPCA subspace does not need it).
 *  - Exceptions to "device pointers only": X of lspca_accumulate_host and
 *    lspca_fit_host lives in host memory, and the projection server's
 *    requests may.
 */
#ifndef LSPCA_H
#define LSPCA_H

#include <stddef.h>
#include <stdint.h>

#if defined(LSPCA_BUILDING)
#define LSPCA_API __attribute__((visibility("default")))
#else
#define LSPCA_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* Storage / compute type of X. F, G, V and sigma are always FP64. */
typedef enum {
  LSPCA_F64 = 0,  /* FP64 X, FP64 matrix-core products (v_mfma_f64) */
  LSPCA_F32 = 1,  /* FP32 X, FP32 matrix-core products, FP32 accumulation */
  LSPCA_BF16 = 2, /* BF16 X, BF16 products, FP32 accumulation */
  LSPCA_F16 = 3   /* FP16 X, FP16 products, FP32 accumulation */
} lspca_dtype;

/* Random test matrix Omega (n x k) of eq. (rp); Sec. I-A lists both kinds. */
typedef enum {
  LSPCA_OMEGA_GAUSSIAN = 0,    /* Omega_ij iid N(0,1) */
  LSPCA_OMEGA_VERY_SPARSE = 1  /* {-1,0,+1} w.p. {1/(2p), 1-1/p, 1/(2p)} */
} lspca_omega_kind;

typedef enum {
  LSPCA_OK = 0,
  LSPCA_EINVAL = -1,    /* bad argument (NULL pointer, size, ldx, kind, dtype) */
  LSPCA_ENOMEM = -2,    /* device workspace could not be allocated */
  LSPCA_EHIP = -3,      /* a HIP runtime call failed */
  LSPCA_ERANK = -4,     /* the sketch or F is rank deficient (see below) */
  LSPCA_E2BIG = -5,     /* request larger than a configured limit */
  LSPCA_EAGAIN = -6,    /* server: no capacity right now; retry */
  LSPCA_ENOTSUP = -7,   /* combination not supported */
  LSPCA_ETIMEDOUT = -8, /* server: wait timed out */
  LSPCA_ENOTFOUND = -9, /* server: unknown or already collected ticket */
  LSPCA_ENOCONV = -10   /* small stage: one-sided Jacobi reached its sweep
                           limit with rotations still pending */
} lspca_status;

/*
 * Omega specification (seeded, counter based; the paper names no generator).
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
 * key = (seed & 0xffffffff, seed >> 32).
 *  Gaussian: one call with counter (q, j & 0xffffffff, j >> 32, 0x47415553)
 *    gives words x0..x3; u1 = ((x1*2^32+x0) >> 11) * 2^-53 + 2^-54,
 *    u2 = ((x3*2^32+x2) >> 11) * 2^-53, r = sqrt(-2 ln u1);
 *    Omega[j][2q] = r cos(2 pi u2), Omega[j][2q+1] = r sin(2 pi u2) (FP64).
 *  Very sparse (p a power of two, 1 <= p <= 2^30): one call with counter
 *    (q, j & 0xffffffff, j >> 32, 0x53505253) gives Omega[j][4q+t] from word
 *    x_t: +1 if x_t < 2^32/(2p), -1 if x_t < 2^32/p, else 0.
 *  Type: Gaussian values are rounded FP64 -> FP32 for FP32 data, and
 *    FP64 -> FP32 -> BF16/FP16 for 16-bit data (round to nearest even).
 *  The very sparse kind is never materialised by the fit: each workgroup
 *  regenerates the nonzeros it needs from the seed.
 */

typedef struct lspca_opts {
  uint32_t struct_size; /* sizeof(lspca_opts); older/smaller structs accepted */
  uint32_t sparse_p;    /* p of the very sparse kind; 0 means 64 */
  int32_t refine;       /* 16-bit X only: -1 default (on), 0 off, 1 on. On:
                           F = Y_hi^T X + Y_lo^T X with Y = Y_hi + Y_lo split
                           into two 16-bit parts, X read once */
  int32_t timing;       /* nonzero: record per-phase device times, read back
                           with lspca_last_timings() */
  void *stream;         /* hipStream_t; NULL = null stream */
  int32_t small_route;  /* truncated SVD of F (Algorithm 2 step 3): 0 = Cholesky
                           QR of F^T (twice) and one-sided Jacobi SVD of R
                           (default; relative accuracy ~ u kappa(F)); 1 = the
                           route of the caption of the paper's algorithm table:
                           eigendecomposition F F^T = W Lambda W^T, D =
                           Lambda^(1/2), V = F^T W D^-1, then one Cholesky QR
                           pass on V (accuracy ~ u kappa(F)^2: D_k is resolved
                           only down to about sqrt(u) D_1) */
  int32_t reserved;     /* 0 */
  int64_t stripe_rows;  /* rows per stripe of the pass (Algorithm 4's slices);
                           0 = auto (a 4 GiB sketch stripe) */
} lspca_opts;

/* Per-phase device times (ms) of the last call on this thread that had
 * opts->timing set; phases not run are 0. */
typedef struct lspca_timings {
  double omega_ms;      /* Omega generation (Gaussian kind) */
  double sketch_ms;     /* Y = X Omega (Algorithm 2 step 1) */
  double factor_ms;     /* F += Y^T X, G += Y^T Y (step 2) */
  double reduce_ms;     /* FP64 reduction of partial F, G */
  double small_ms;      /* small FP64 stage (truncated SVD of F; step 3) */
  double qr_ms;         /* spca_fit: tall-skinny Householder QR of Y */
  double pass2_ms;      /* spca_fit: F = Q^T X */
  double transform_ms;  /* Z = X V */
  double total_ms;      /* whole call */
  double layout_ms;     /* sparse X: column-order (CSC) build of each stripe;
                           FP16 X: the sketch scaled and split into 16-bit parts */
} lspca_timings;

/* Version string, e.g. "lspca 0.1 gfx950". */
LSPCA_API const char *lspca_version(void);
/* Static text for a status code. */
LSPCA_API const char *lspca_strerror(int status);
/* Thread-local message describing the last failure on this thread. */
LSPCA_API const char *lspca_last_error(void);
/* Copies the timings of the last timed call on this thread. */
LSPCA_API int lspca_last_timings(lspca_timings *out);

/*
 * lspca_omega -- materialise Omega (n x k, row-major) in the type `dtype`
 * as the fit uses it (specification above; eq. (rp), Sec. I-A).
 *  Omega: device buffer of n*k elements of `dtype` (FP64, FP32, BF16, FP16).
 *  p: sparse p (power of two; 0 means 64); ignored for the Gaussian kind.
 *  Errors: EINVAL (n < 1, k < 1, bad kind/dtype/p, Omega NULL).
 */
LSPCA_API int lspca_omega(int64_t n, int32_t k, lspca_omega_kind kind, uint64_t seed,
                uint32_t p, lspca_dtype dtype, void *Omega, void *stream);

/*
 * lspca_accumulate -- one step of Algorithm 4 (Streaming Lazy SPCA) for the
 * horizontal slice X (m x n): U_s = X Omega, F += U_s^T X and G += U_s^T U_s.
 *  F: k x n FP64 (device), accumulated in place (caller zeroes it first).
 *  G: k x k FP64 (device) or NULL to skip the Gram. G feeds sigma_x.
 *  Products run in the type of X with FP32 accumulation (FP64 for F64).
 *  Each FP32 partial sum spans at most 65,536 rows of the slice; the
 *  partials are added into F and G in FP64 in a fixed order, so results
 *  are deterministic for a given input and device.
 *  Errors: EINVAL (m < 1, n < 1, k < 1, k > n, ldx < n, NULL X/F, bad kind),
 *  ENOMEM, EHIP. Asynchronous on opts->stream.
 */
LSPCA_API int lspca_accumulate(const void *X, lspca_dtype xdt, int64_t m, int64_t n,
                     int64_t ldx, int32_t k, lspca_omega_kind kind,
                     uint64_t seed, const lspca_opts *opts, double *F,
                     double *G);

/*
 * lspca_factor -- the final step of Algorithms 2 and 4: truncated SVD of the
 * k x n factor F (FP64, on the device), F = U~ D V^T.
 *  V: n x k FP64 right singular vectors, columns in decreasing order of D,
 *     each column's largest-magnitude entry positive (lowest index on ties).
 *  sigma: k FP64, D (singular values of F = U^T X).
 *  sigma_x: k FP64 or NULL. When given (and G given), the approximate
 *     singular values Sigma^s of X (eq. (approx_svd)), from the k x k route
 *     R = chol(G), Q^T X = R^-T F (no tall QR).
 *  Errors: EINVAL, ENOMEM, EHIP, ERANK if F is numerically rank deficient
 *  (D_k <= 64 * n * eps * D_1) or, when sigma_x is requested, if chol(G)
 *  fails (Lemma of the footnote to Corollary 1 assumes rank(U) = k),
 *  ENOCONV if a one-sided Jacobi run stopped at its sweep limit (60 for
 *  k < 128, else 40) while its last sweep still rotated a column pair
 *  further than 1e-8 (relative to the column norms) from orthogonal (a
 *  sweep whose rotations all stay within that ends the run: the next one
 *  would not rotate). Synchronous.
 */
LSPCA_API int lspca_factor(const double *F, const double *G, int32_t k, int64_t n,
                 const lspca_opts *opts, double *V, double *sigma,
                 double *sigma_x);

/*
 * lspca_fit -- Lazy SPCA (Algorithm 2) of X resident on the device:
 * lspca_accumulate over all of X, then lspca_factor. Each stripe of rows
 * goes through two kernels, the sketch and then F = U^T X, so X is read
 * twice from device memory for FP32/FP64 data and streamed by two kernels
 * per stripe for 16-bit data.
 * Arguments as above; 1 <= k <= min(m, n) (Corollary 1 requires
 * l <= min{m, n}). Synchronous. Errors as lspca_accumulate/lspca_factor.
 */
LSPCA_API int lspca_fit(const void *X, lspca_dtype xdt, int64_t m, int64_t n,
              int64_t ldx, int32_t k, lspca_omega_kind kind, uint64_t seed,
              const lspca_opts *opts, double *V, double *sigma,
              double *sigma_x);

/*
 * lspca_accumulate_host -- Algorithm 4 (Streaming Lazy SPCA) over X in
 * HOST memory, the regime where X exceeds device memory: the rows stream
 * through two device staging buffers of stripe_rows rows (0: about 1 GiB
 * of X each), the copy of one stripe overlapping the pass over the
 * previous one. F (k x n) and G (k x k or NULL) are FP64 device
 * accumulators as in lspca_accumulate: together they are the whole state
 * of a streaming fit, so a caller can save them after any call and resume
 * with the remaining rows later. X should be pinned (hipHostMalloc) for
 * full copy rate; pageable memory works, slower. Synchronous: X may be
 * released on return. Errors as lspca_accumulate, EINVAL for device X or
 * stripe_rows < 0.
 */
LSPCA_API int lspca_accumulate_host(const void *X, lspca_dtype xdt, int64_t m, int64_t n,
                          int64_t ldx, int32_t k, lspca_omega_kind kind, uint64_t seed,
                          const lspca_opts *opts, int64_t stripe_rows, double *F, double *G);

/*
 * lspca_fit_host -- Lazy SPCA (Algorithm 4) of X in host memory:
 * lspca_accumulate_host over all rows, then lspca_factor. Outputs as
 * lspca_fit (device pointers). Synchronous.
 */
LSPCA_API int lspca_fit_host(const void *X, lspca_dtype xdt, int64_t m, int64_t n, int64_t ldx,
                   int32_t k, lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts,
                   int64_t stripe_rows, double *V, double *sigma, double *sigma_x);

/*
 * spca_fit -- SPCA (Algorithm 1), the non-lazy baseline: Y = X Omega (pass 1,
 * stored m x k), tall-skinny Householder QR Y = Q R with explicit thin Q,
 * F = Q^T X (pass 2), truncated SVD of F.
 *  V: n x k FP64 (V^s); sigma: k FP64 (Sigma^s). Same conventions as
 *  lspca_fit. Synchronous. Errors: EINVAL, ENOMEM, EHIP, ERANK.
 */
LSPCA_API int spca_fit(const void *X, lspca_dtype xdt, int64_t m, int64_t n,
             int64_t ldx, int32_t k, lspca_omega_kind kind, uint64_t seed,
             const lspca_opts *opts, double *V, double *sigma);

/*
 * spca_fit_stream -- Streaming SPCA (Algorithm 3), the one-pass baseline:
 * per stripe U_s = X_s Omega, F += U_s^T X_s and R <- R of qr([R; U_s])
 * (a tall-skinny Householder QR of U_s without Q, merged into the running
 * R); then F = R^-T F and its truncated SVD. X is read once.
 *  V: n x k FP64 (V^s); sigma: k FP64 (Sigma^s). Same conventions and
 *  limits as spca_fit (k <= 256, FP64 data: k <= 128). Synchronous.
 *  Errors: EINVAL, ENOMEM, EHIP, ERANK, ENOTSUP.
 */
LSPCA_API int spca_fit_stream(const void *X, lspca_dtype xdt, int64_t m, int64_t n,
                    int64_t ldx, int32_t k, lspca_omega_kind kind, uint64_t seed,
                    const lspca_opts *opts, double *V, double *sigma);

/*
 * lspca_transform -- Z = X V, the map pi(x) = V^T x of eq.
 * (dim_reduction_maps) applied to each of the r rows of X.
 *  V: n x k FP64 (device). Z: r x k, FP64 for F64 data, FP32 otherwise.
 *  BF16/FP16 X use V split in two 16-bit parts (V = V_hi + V_lo, two
 *  products into one FP32 accumulator); FP32 X uses V rounded to FP32.
 *  Each output row depends only on its input row, with a fixed reduction
 *  order, so a row's result does not depend on r or on the other rows.
 *  r = 0 is allowed (no work). Errors: EINVAL, ENOMEM, EHIP. Asynchronous.
 */
LSPCA_API int lspca_transform(const void *X, lspca_dtype xdt, int64_t r, int64_t n,
                    int64_t ldx, const double *V, int32_t k, void *Z,
                    const lspca_opts *opts);

/*
 * lspca_transform_noalloc -- lspca_transform for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. Same arguments, kernels and results as
 * lspca_transform (bitwise), but the one buffer the projection needs beyond
 * X, V and Z (V^T in the type of X, two parts for BF16/FP16) lives in a
 * fixed device array of LSPCA_NOALLOC_SCRATCH_BYTES that each device holds
 * until the process ends; the call allocates nothing (no hipMalloc or
 * hipFree, no library workspace, no events).
 *  Limit: parts * size(X element) * n * k <= LSPCA_NOALLOC_SCRATCH_BYTES,
 *  parts = 2 for BF16/FP16 and 1 otherwise, each part rounded up to 256
 *  bytes: n * k <= 2^21 for FP64, 2^22 for FP32, BF16 and FP16. Larger
 *  requests return E2BIG. opts->timing is ignored.
 *  Every call on one device shares that device's array, which keeps the
 *  last call's contents: calls that overlap on one device (several host
 *  threads, or several streams whose work overlaps) race on it; the caller
 *  orders them. Calls do not wait for other entry points, whose workspace
 *  is separate.
 *  The array's device address is looked up on the first call on each device
 *  (with that device current). Errors: EINVAL, E2BIG, ENOTSUP (device
 *  ordinal >= 64), EHIP. Asynchronous on opts->stream.
 */
#define LSPCA_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
LSPCA_API int lspca_transform_noalloc(const void *X, lspca_dtype xdt, int64_t r, int64_t n,
                    int64_t ldx, const double *V, int32_t k, void *Z,
                    const lspca_opts *opts);

/*
 * Sparse X (Experiment 1, "Data and Method": the data are horizontal slices
 * of a sparse matrix with FP32 values; Proposition 4 prices both products
 * of the pass at O(nnz(X) l)). X is given in CSR form, all arrays on the
 * device and owned by the caller:
 *  rowptr: m + 1 int64; row i's entries are at positions
 *     [rowptr[i], rowptr[i + 1]) of colidx and values. rowptr[0] >= 0 (a
 *     row slice of a larger CSR matrix is rowptr + r0 with the same colidx
 *     and values), nondecreasing, rowptr[m] = nnz.
 *  colidx: int32 column indices in [0, n), at least nnz entries; order
 *     within a row is free and repeated columns add (X[i][j] is the sum of
 *     row i's values with column j).
 *  values: FP32 or FP64 (vdt), at least nnz entries.
 * The arrays are checked on the device before any other kernel reads them
 * (EINVAL names the broken array); these calls wait for that check.
 * Products run in the value type (FP32 sums for FP32 data) except F, which
 * accumulates in FP64; each row's and each column's entries are summed in
 * storage / row order, so results are deterministic. Omega is the one of
 * lspca_omega for the value type.
 */

/*
 * lspca_accumulate_csr -- Algorithm 4 step for a CSR slice: U_s = X Omega,
 * F += U_s^T X, G += U_s^T U_s (G may be NULL). F k x n and G k x k FP64
 * device accumulators as in lspca_accumulate. Rows are processed in
 * stripes; each stripe's X is also put in column order on the device (a
 * stable sort; workspace about 28 bytes per entry of the stripe).
 *  Errors: EINVAL (bad sizes, NULL pointers, bad CSR arrays, bad kind or
 *  p), ENOTSUP (values not FP32/FP64, k > 4096, 2^31 entries in one stripe
 *  of 64 rows), ENOMEM, EHIP. Returns once the work is queued after the
 *  check; outputs are ready when opts->stream is.
 */
LSPCA_API int lspca_accumulate_csr(const int64_t *rowptr, const int32_t *colidx, const void *values,
                                   lspca_dtype vdt, int64_t m, int64_t n, int64_t nnz, int32_t k,
                                   lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts,
                                   double *F, double *G);

/*
 * lspca_fit_csr -- Lazy SPCA (Algorithm 2) of a CSR X resident on the
 * device: lspca_accumulate_csr over all rows, then lspca_factor. Outputs as
 * lspca_fit; 1 <= k <= min(m, n). Synchronous. Errors as
 * lspca_accumulate_csr and lspca_factor.
 */
LSPCA_API int lspca_fit_csr(const int64_t *rowptr, const int32_t *colidx, const void *values,
                            lspca_dtype vdt, int64_t m, int64_t n, int64_t nnz, int32_t k,
                            lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts, double *V,
                            double *sigma, double *sigma_x);

/*
 * spca_fit_csr -- SPCA (Algorithm 1), the non-lazy baseline, for a CSR X:
 * U = X Omega for all rows (kept, m x k), tall-skinny Householder QR U = Q R
 * with explicit thin Q, F = Q^T X (a second pass over X), truncated SVD of
 * F. Outputs as spca_fit (V^s, Sigma^s); limits as spca_fit (k <= 256, FP64
 * values: k <= 128). Synchronous. Errors as lspca_fit_csr, ENOTSUP.
 */
LSPCA_API int spca_fit_csr(const int64_t *rowptr, const int32_t *colidx, const void *values,
                           lspca_dtype vdt, int64_t m, int64_t n, int64_t nnz, int32_t k,
                           lspca_omega_kind kind, uint64_t seed, const lspca_opts *opts, double *V,
                           double *sigma);

/*
 * lspca_transform_csr -- Z = X V (eq. (dim_reduction_maps)) for the r rows
 * of a CSR X. V: n x k FP64 (device; rounded to FP32 for FP32 values).
 * Z: r x k of the value type. Each row of Z is the sum of its row's
 * entries times rows of V, in storage order. r = 0: no work. Errors:
 * EINVAL, ENOTSUP, ENOMEM, EHIP. Asynchronous after the check.
 */
LSPCA_API int lspca_transform_csr(const int64_t *rowptr, const int32_t *colidx, const void *values,
                                  lspca_dtype vdt, int64_t r, int64_t n, int64_t nnz, const double *V,
                                  int32_t k, void *Z, const lspca_opts *opts);

/*
 * Projection server: continuous batching of requests Z = X V, the map
 * pi(x) = V^T x of eq. (dim_reduction_maps), with V resident on the device.
 *
 * A request is r rows of X (r x n, rows contiguous, in the server's dtype)
 * and its output Z (r x k, rows contiguous; FP32, FP64 for an F64 server).
 * Requests enter a FIFO queue. The server's scheduler thread admits them in
 * order while fewer than max_inflight requests are admitted and unfinished
 * and, for host requests, while the staging arena has room for X and Z.
 * Admitted requests are packed, up to 64 at a time, into one launch of
 * persistent kernels that walk the launch's row tiles across requests: for
 * BF16/FP16 data, requests of few rows (at most 8,192) take 32 x 64 tiles,
 * so many workgroups share their walk over n, and the others the standard
 * tiles. A launch passes its request table in the kernel arguments (no
 * upload step) and starts only the kernels of the tile classes it uses;
 * launches rotate over several streams, so requests that arrive while others
 * are on the device are launched at once and overlap them. A request is launched from lspca_server_submit itself
 * when a launch slot is free, else by the server's scheduler thread.
 * Every tile shape computes an output element by the same chain of
 * matrix-core steps as lspca_transform, so a result is bitwise the same
 * alone, in any mix of requests, and as lspca_transform.
 * X and Z are both device pointers, or both host pointers (hipHostMalloc
 * memory gives asynchronous copies): host requests are copied into the
 * arena, projected there and copied back before they complete.
 * Latency is measured by the server from lspca_server_submit to the moment
 * its scheduler sees the request's launch (and copies) complete.
 * All functions are thread-safe for one server.
 */
typedef struct lspca_server lspca_server;

typedef struct {
  uint32_t struct_size;             /* sizeof(lspca_server_stats) */
  uint32_t max_requests_per_launch; /* largest batch packed into one launch */
  uint32_t max_concurrent_launches; /* most launches in flight at once */
  uint32_t reserved;
  uint64_t submitted, completed, launches, rows_completed;
  uint64_t arena_peak_bytes;        /* most staging bytes held at once */
  /* Latency breakdown, summed over requests (divide by completed): */
  uint64_t queue_ns;                /* submit -> its launch enqueued */
  uint64_t enqueue_ns;              /* host time of the enqueue calls of its launch */
  uint64_t device_ns;               /* launch enqueued -> completion seen */
} lspca_server_stats;

/*
 * lspca_server_create -- V: n x k FP64 (device, caller-owned; copied and
 *  converted at creation, so it may be freed afterwards). xdt: dtype of X
 *  (BF16/FP16 use V split in two 16-bit parts, as lspca_transform).
 *  arena_bytes: device staging memory for host requests (0 = device
 *  requests only). max_inflight: admitted, unfinished requests (>= 1).
 *  *out receives the server (library-owned, freed by lspca_server_destroy).
 *  Errors: EINVAL (n < 1, k < 1, bad dtype, NULL), ENOMEM, EHIP.
 */
LSPCA_API int lspca_server_create(const double *V, int64_t n, int32_t k, lspca_dtype xdt,
                        size_t arena_bytes, int32_t max_inflight, lspca_server **out);

/*
 * lspca_server_submit -- queue Z = X V for r rows; *ticket identifies the
 *  request for lspca_server_wait. X and Z must stay valid and untouched
 *  until the request completes, and any device work producing X (or still
 *  using Z) must be complete when submitting: the server's streams do not
 *  wait on the caller's. r = 0 completes at once.
 *  Errors: EINVAL (NULL, r < 0, X and Z of different memory kinds, device X
 *  not 16-byte aligned), E2BIG (host request larger than the arena),
 *  EAGAIN (queue full: 16 * max_inflight requests waiting for admission).
 */
LSPCA_API int lspca_server_submit(lspca_server *srv, const void *X, int64_t r, void *Z,
                        uint64_t *ticket);

/*
 * lspca_server_wait -- wait up to timeout_us (< 0: no limit; 0: poll) for
 *  the request to complete. On completion returns its status, writes its
 *  latency in ms (if latency_ms is not NULL) and forgets the ticket.
 *  Errors: ENOTFOUND (unknown or already waited ticket), ETIMEDOUT (still
 *  running; the ticket stays valid), EHIP (its launch failed).
 */
LSPCA_API int lspca_server_wait(lspca_server *srv, uint64_t ticket, int64_t timeout_us,
                      double *latency_ms);

/*
 * lspca_server_pause -- paused != 0: start no new launches (launches in
 *  flight finish; submissions still queue and are admitted); 0: resume.
 */
LSPCA_API int lspca_server_pause(lspca_server *srv, int paused);

/* lspca_server_get_stats -- counters since creation (out->struct_size set by the caller). */
LSPCA_API int lspca_server_get_stats(lspca_server *srv, lspca_server_stats *out);

/*
 * lspca_server_destroy -- finish every submitted request, then free the
 *  server. Tickets not yet waited are dropped. NULL is allowed.
 */
LSPCA_API int lspca_server_destroy(lspca_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* LSPCA_H */
