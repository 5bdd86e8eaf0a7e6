/*
 * psdp.h -- warm-started approximate projection onto the PSD cone, MI355X.
 *
 * The library computes Pi(X) = argmin_{Y psd} ||X - Y||_F for a dense
 * symmetric n x n matrix X (paper §1, definition of the projection and
 * eq. `projection`) with a warm-started block eigensolver of the LOBPCG
 * family (paper §5.1, Alg. 3) applied to whichever spectral side is smaller
 * (§5.1, "When is projecting with LOBPCG most efficient"; §6 side rule), and
 * returns the gap-free a-posteriori error bound of §5.2 (Thm `bound`):
 *
 *     ||Vt Lt Vt^T - Pi(A)||_F^2 <= 2 ||R||_F^2 + ||Pi(Vt_perp^T A Vt_perp)||_F^2
 *
 * where (Vt, Lt) are the positive Ritz pairs with Lt = Vt^T A Vt and
 * R = A Vt - Vt Lt.  The last term (the tail) is certified by default: an
 * FP64 Cholesky factorization of (delta - eta) I - P A P + c Vt Vt^T,
 * P = I - Vt Vt^T, completes only if every eigenvalue of Vt_perp^T A Vt_perp
 * is below delta (eta bounds the rounding of forming and factoring the
 * matrix), and then tail <= sqrt(n - m~) delta (certified = 1).  §5.2 leaves
 * this term out of its experiments.  A certificate that fails leaves the
 * tail unbounded (tail_est = err_bound = +inf, PSDP_NOT_CONVERGED, or the
 * exact path with fallback_full).  Without the certificate (certify = 0) the
 * tail is estimated from the largest non-positive Ritz pair (theta_g, r_g)
 * as sqrt(n - m~) max(theta_g + r_g, 0) (certified = 0).
 *
 * Conventions for every entry point:
 *   - matrices are column-major (Fortran order) with a leading dimension;
 *   - pointers named X, V, lambda, Pi are DEVICE pointers (HIP, on the
 *     handle's device) unless stated otherwise; options/info are HOST;
 *   - X is read-only and only its LOWER triangle is read (LAPACK uplo='L');
 *   - work is enqueued on the handle's stream; psdp_project and
 *     psdp_full_eig_project synchronise that stream before returning because
 *     they fill the host info struct;
 *   - no entry point aborts: each returns a psdp_status; arguments are
 *     validated on the host before any launch;
 *   - the caller owns X, V, lambda and Pi; the handle owns its workspace;
 *   - a handle is not thread safe: use one handle per host thread.
 */
#ifndef PSDP_H
#define PSDP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psdp_handle_s *psdp_handle;

typedef enum {
    PSDP_OK = 0,                 /* converged to tol; Pi, V, lambda valid        */
    PSDP_NOT_CONVERGED = 1,      /* max_iter reached; Pi valid with its (larger)  */
                                 /* bound in info->err_bound                      */
    PSDP_FELL_BACK_FULL_EIG = 2, /* exact full eigendecomposition was used       */
    PSDP_PENDING = 3,            /* server request not finished yet (wait/poll)  */
    PSDP_ERR_INVALID_ARG = -1,   /* bad size, pointer, stride or option          */
    PSDP_ERR_HIP = -2,           /* a HIP/ROCm call failed (e.g. no device)      */
    PSDP_ERR_OUT_OF_MEMORY = -3, /* workspace allocation failed                  */
    PSDP_ERR_NUMERICAL = -4,     /* non-finite input or breakdown not recovered  */
    PSDP_ERR_CAPACITY = -5       /* block would exceed m_cap and no fallback     */
} psdp_status;

typedef enum {
    PSDP_SIDE_AUTO = 0, /* paper §6: positive side if the estimated count of    */
                        /* positive eigenvalues is < side_threshold*n, negative */
                        /* side if the negative count is, else full eig; with   */
                        /* no estimate (pos_hint < 0) the full eig is used      */
    PSDP_SIDE_POS = 1,  /* approximate the positive pairs of X (eq. projection, */
                        /* middle)                                              */
    PSDP_SIDE_NEG = 2,  /* approximate the positive pairs of -X and use the     */
                        /* Moreau identity Pi(X) = X + Pi(-X) (eq. projection,  */
                        /* right)                                               */
    PSDP_SIDE_FULL = 3  /* exact full eigendecomposition                        */
} psdp_side;

typedef enum {
    PSDP_PREC_FP64 = 0, /* block products in FP64 (MFMA f64)                    */
    PSDP_PREC_FP32 = 1, /* block products in FP32 (MFMA f32), FP64 elsewhere     */
    PSDP_PREC_BF16 = 2  /* block products BF16 x BF16 -> FP32 (MFMA), FP64      */
                        /* elsewhere                                            */
} psdp_prec;

typedef struct {
    int side;               /* psdp_side                                          */
    int prec;               /* psdp_prec of the block products                    */
    double tol;             /* absolute 2-norm tolerance on each positive Ritz    */
                            /* residual (paper §5.2/§6 stopping rule); <= 0 picks */
                            /* 1e-8 * ||X||_F / sqrt(2 m)                          */
    int max_iter;           /* LOBPCG iteration cap (all phases together)         */
    int refine_fp64;        /* low-precision runs: finish with the FP64 residual- */
                            /* correction sweep (default 1)                       */
    int ladder;             /* on a stalled low-precision residual move BF16 ->   */
                            /* FP32 -> FP64 products (default 1); 0 = raw path    */
    int certify;            /* 1 (default): certify the tail term (FP64 Cholesky */
                            /* of (delta - eta) I - P A P + c Vt Vt^T); a failed */
                            /* certificate makes the result PSDP_NOT_CONVERGED,  */
                            /* or the full eig when fallback_full is set; 0: the */
                            /* tail is the estimate from the guard Ritz pair     */
    unsigned long long seed;/* counter-based RNG seed (cold start, expansion);    */
                            /* the stream also takes the handle's call count, so */
                            /* repeated cold starts draw different columns       */
    double side_threshold;  /* AUTO side rule threshold, default 1/3 (paper §6)   */
    int expand_cols;        /* columns added per expansion, 0 = ceil(n/50)        */
                            /* (paper §5.1 expansion rule)                        */
    int pos_hint;           /* estimated count of positive eigenvalues for AUTO,  */
                            /* e.g. the previous call's info.n_pos; -1 = none     */
    int fallback_full;      /* 1: when LOBPCG is not converged at max_iter or the */
                            /* block outgrows m_cap, use the full eig instead     */
    int block_guard;        /* cold start block = hint + max(block_guard,         */
                            /* ceil(0.2 hint)); default 4                         */
    int batch_variant;      /* psdp_project_batched launch shape: -1 = autotuned  */
                            /* (default), 0..3 = a fixed variant                  */
    int batch_graph;        /* psdp_project_batched: 1 = replay the launch        */
                            /* sequence from a captured hipGraph (default),       */
                            /* 0 = plain launches                                 */
    double bound_rel_max;   /* > 0 with fallback_full = 1 (psdp_project): a       */
                            /* converged result whose a-posteriori bound (paper   */
                            /* §5.2, residual and tail terms) exceeds             */
                            /* bound_rel_max * ||Pi||_F is replaced by the full   */
                            /* eig (PSDP_FELL_BACK_FULL_EIG); 0 = off (default)   */
    double certify_delta;   /* certificate threshold delta (> 0); 0 (default) =   */
                            /* sqrt(2 max(m~, 1)) tol / sqrt(n), so that the      */
                            /* certified tail is at most the residual part the    */
                            /* stopping rule allows; raised to 4 eta when the     */
                            /* rounding margin eta is larger                      */
    int warm_side;          /* side the warm-start block V belongs to, PSDP_SIDE_ */
                            /* POS or _NEG (the previous call's info.block_side); */
                            /* a call that resolves to the other side starts      */
                            /* cold; PSDP_SIDE_AUTO (default): the side this call */
                            /* uses                                               */
    int method;             /* psdp_method (default PSDP_METHOD_LOBPCG)           */
    int method_param;       /* BLOCK_KRYLOV: block iterations (0 = 1);            */
                            /* TOP_R: r, the block width (>= 1);                  */
                            /* CHEBYSHEV: largest filter degree per pass (0 = 24, */
                            /* at most 64)                                        */
} psdp_options;

/* Eigensolvers behind psdp_project (paper §5, the block Krylov discussion,
 * and §1 on truncated projections). */
typedef enum {
    PSDP_METHOD_LOBPCG = 0,       /* Alg. 3 until every positive Ritz pair meets */
                                  /* tol (the paper's method)                    */
    PSDP_METHOD_BLOCK_KRYLOV = 1, /* Rayleigh-Ritz on span(X, AX) from the warm  */
                                  /* start, method_param times (one block        */
                                  /* Lanczos iteration each, restarted), no      */
                                  /* convergence loop; OK only when the stopping */
                                  /* rule then holds                             */
    PSDP_METHOD_TOP_R = 2,        /* the r = method_param largest Ritz pairs     */
                                  /* (fixed block, no guard, no expansion) and   */
                                  /* Pi~ = sum_{i<=r} max(theta_i, 0) v_i v_i^T; */
                                  /* status says whether the r pairs met tol;    */
                                  /* info.trunc_bound = sqrt(n - r) max(theta_r, */
                                  /* 0), the bound that assumes exact pairs      */
    PSDP_METHOD_CHEBYSHEV = 3     /* polynomial subspace extraction (§1): passes */
                                  /* of X <- T_d((A - c) / e) X, the Chebyshev   */
                                  /* polynomial of degree d damping [lo, theta_m]*/
                                  /* (lo from 10 Lanczos steps, theta_m the      */
                                  /* block's smallest Ritz value), each followed */
                                  /* by Rayleigh-Ritz on span(X) with an FP64    */
                                  /* product, until the same stopping rule as    */
                                  /* LOBPCG holds and the certificate succeeds   */
                                  /* (at most min(max_iter, 40) passes and three */
                                  /* failed certificates); filter products at    */
                                  /* opt.prec while the largest residual is 10x  */
                                  /* above that precision's rounding floor, else */
                                  /* FP64; the same bound; info.iters = passes.  */
                                  /* The 10 Lanczos steps run on a second stream */
                                  /* the handle creates (non-blocking, default   */
                                  /* priority) after the input is ingested; the  */
                                  /* call waits for it before any return, so the */
                                  /* stream semantics of the call are unchanged  */
} psdp_method;

typedef struct {
    double err_bound;   /* sqrt(2 ||R||_F^2 + tail_est^2), absolute Frobenius     */
    double res_fro;     /* ||R||_F of the final positive Ritz pairs (FP64)        */
    double tail_est;    /* bound on ||Pi(Vt_perp^T A Vt_perp)||_F: sqrt(n - m~)   */
                        /* cert_delta when certified, +inf when the certificate  */
                        /* failed, the guard estimate when certify = 0           */
    double pi_fro;      /* ||Pi||_F of the returned projection (host estimate     */
                        /* sqrt(sum lt^2) for the positive side)                  */
    double theta_guard; /* largest non-positive Ritz value kept in the block      */
    double tol_used;    /* tolerance actually applied                            */
    int n_pos;          /* positive Ritz pairs of the approximated side (m~)     */
    int m_out;          /* columns returned in V                                  */
    int iters;          /* LOBPCG iterations (all phases)                         */
    int side_used;      /* PSDP_SIDE_POS, _NEG or _FULL                           */
    int certified;      /* 1: the tail term is certified (the Cholesky            */
                        /* certificate succeeded, or m~ = n, or the exact path   */
                        /* was used); 0: tail_est is an estimate                 */
    int status;         /* same as the return value                               */
    int expansions;     /* block expansions performed                             */
    int prec_final;     /* product precision in the last LOBPCG phase             */
    int n_pos_full;     /* eigenvalue count of X above 0 (full eig path) or -1    */
    int pos_est;        /* estimated count of positive eigenvalues of X, the      */
                        /* pos_hint for the next call on a nearby matrix (paper   */
                        /* §6 side rule): n_pos (positive side), n - n_pos        */
                        /* (negative side) or n_pos_full (exact path)             */
    int block_side;     /* side the returned V belongs to (PSDP_SIDE_POS or _NEG; */
                        /* the exact path returns leading pairs of X: POS), the   */
                        /* warm_side of the next call                             */
    double cert_delta;  /* threshold the certificate proved (NaN when not run)    */
    double cert_eta;    /* its rounding margin eta (NaN when not run)             */
    double trunc_bound; /* PSDP_METHOD_TOP_R: sqrt(n - r) max(theta_r, 0), else  */
                        /* NaN                                                    */
    double spec_lower;  /* PSDP_METHOD_CHEBYSHEV: the lower end of the damped     */
                        /* interval (an estimate at or below the smallest         */
                        /* eigenvalue: the lowest Lanczos Ritz value less twice   */
                        /* its residual and 2 %, not a proven bound), else NaN    */
    int products;       /* PSDP_METHOD_CHEBYSHEV: products with A (filter,        */
                        /* Rayleigh-Ritz and Lanczos), else 0                     */
} psdp_info;

/* Fill *opt with the defaults documented above. */
void psdp_default_options(psdp_options *opt);

/* Create a handle on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Returns PSDP_ERR_HIP when the
 * device is absent.  Allocates nothing until the first call needs it. */
psdp_status psdp_create(psdp_handle *h, int device, void *hip_stream);

/* Release the handle and all of its device memory. */
psdp_status psdp_destroy(psdp_handle h);

/* Change the stream later calls enqueue on. */
psdp_status psdp_set_stream(psdp_handle h, void *hip_stream);

/* Device workspace bytes a psdp_project call of order n with block capacity
 * m_cap and product precision prec needs (host-only computation). */
psdp_status psdp_workspace_bytes(int n, int m_cap, int prec, size_t *bytes);

/* Project one matrix (paper §5.1 Alg. 3 + §5.2 Thm `bound`).
 *   n        order of X (n >= 1)
 *   X, ldx   symmetric input, lower triangle read, ldx >= n (device)
 *   V, ldv   n x m_cap block (device).  On entry its first *m_inout columns
 *            are the warm start (the previous call's Ritz block; 0 = cold
 *            start from seeded N(0,1) columns).  On exit it holds the m_out
 *            Ritz vectors of the approximated side (of -X on the negative
 *            side), orthonormal.
 *   m_cap    column capacity of V and lambda (>= 1)
 *   m_inout  in: warm-start columns (0..m_cap); out: m_out
 *   lambda   m_cap doubles (device): Ritz values of the approximated side's
 *            matrix (X on the positive side, -X on the negative side) for the
 *            returned columns of V, in descending order
 *   Pi, ldpi n x n output Pi(X), both triangles written (device); Pi may not
 *            alias X
 * Returns PSDP_OK, PSDP_NOT_CONVERGED (Pi still valid, bound larger),
 * PSDP_FELL_BACK_FULL_EIG, or an error.  info (host) is filled on return.
 * On the full-eig side, V/lambda return the leading eigenpairs, largest
 * first: the p positive ones and max(4, ceil(0.2 p)) more as guard columns,
 * at most m_cap; m_out is their count and info->n_pos_full = p. */
psdp_status psdp_project(psdp_handle h, int n, const double *X, int ldx,
                         double *V, int ldv, int m_cap, int *m_inout,
                         double *lambda, double *Pi, int ldpi,
                         const psdp_options *opt, psdp_info *info);

/* Project `count` independent cones of uneven size in one persistent
 * launch (paper §6.1: block-diagonal SDPs split into many smaller PSD
 * variables).  Every array argument is a HOST array of length count whose
 * elements are device pointers or sizes:
 *   n[i]        order of cone i, 1 <= n[i] <= 256
 *   X[i]        n[i] x n[i], leading dimension n[i], lower triangle read
 *   V[i]        n[i] x m_cap[i] (leading dimension n[i]): warm start on entry
 *               (first m_inout[i] columns), Ritz block on exit
 *   m_cap[i]    >= 1; the block of cone i is limited to min(m_cap[i], 32, n[i])
 *   m_inout[i]  (host) warm-start width on entry, m_out on exit; 0 = cold
 *               start from min(m_cap[i], 32, n[i]) seeded N(0,1) columns
 *   lambda[i]   m_cap[i] doubles: Ritz values, descending
 *   Pi[i]       n[i] x n[i] output, both triangles, may not alias X[i]
 * One workgroup solves one cone at a time from a queue ordered by
 * decreasing n^2 m.  opt->side POS or AUTO approximates the positive part
 * of every cone, NEG the positive part of -X (Moreau); FULL is rejected.
 * opt->prec FP64 selects FP64 products, FP32 and BF16 select FP32 products;
 * orthogonalization, Rayleigh-Ritz, the final sweeps and the bound are FP64.
 * tol <= 0 picks 1e-8 ||X_i||_F / sqrt(2 m) per cone.  With
 * opt->fallback_full, cones that do not converge are projected exactly by
 * psdp_full_eig_project_batched in the same call (status
 * PSDP_FELL_BACK_FULL_EIG).  The tail term of each cone's bound is the
 * estimate sqrt(n - m~) max(theta_g + r_g, 0) from its largest
 * non-positive Ritz pair (info.certified = 0): the batched engine does not
 * run the certificate, whatever opt->certify says.  Results do not
 * depend on the queue order or the launch shape beyond rounding of the
 * product sums.  info is a HOST array[count]; a cone that does not converge
 * reports PSDP_NOT_CONVERGED with its bound, a non-finite cone
 * PSDP_ERR_NUMERICAL (its outputs untouched).  Returns the most severe
 * status (errors first).  Synchronises the handle's stream. */
psdp_status psdp_project_batched(psdp_handle h, int count, const int *n,
                                 const double *const *X, double *const *V,
                                 const int *m_cap, int *m_inout,
                                 double *const *lambda, double *const *Pi,
                                 const psdp_options *opt, psdp_info *info);

/* Exact projection of `count` cones (n[i] <= 256) through full FP64
 * eigendecompositions (paper §1), batched: cones are zero-padded to buckets
 * of order round_up(n, 32) and each bucket is one batched rocSOLVER syevd.
 * Arrays as in psdp_project_batched; V may be NULL (then m_cap, m_inout and
 * lambda are ignored), else V[i]/lambda[i] receive the leading eigenpairs
 * (positive ones plus max(4, ceil(0.2 p)) guard columns, at most m_cap[i])
 * and m_inout[i] their count.  info[i].n_pos = n_pos_full = p. */
psdp_status psdp_full_eig_project_batched(psdp_handle h, int count, const int *n,
                                          const double *const *X, double *const *V,
                                          const int *m_cap, int *m_inout,
                                          double *const *lambda, double *const *Pi,
                                          psdp_info *info);

/* Launch shape (0..3) the last psdp_project_batched call used and the
 * device time of its launch in milliseconds (hipEvents on the handle's
 * stream); -1 and 0 before the first call. */
psdp_status psdp_batched_tuning(psdp_handle h, int *variant, double *last_ms);

/* Exact projection through a full FP64 eigendecomposition (rocSOLVER
 * syevd), clip and rebuild: the exact fallback and the baseline path
 * (paper §1: full eigendecomposition with syevr in COSMO).
 *   lambda_all  n doubles (device, may be NULL): all eigenvalues ascending
 *   Pi, ldpi    n x n output (device). */
psdp_status psdp_full_eig_project(psdp_handle h, int n, const double *X, int ldx,
                                  double *lambda_all, double *Pi, int ldpi);

/* The block product of one LOBPCG iteration on its own (paper §5.1: the
 * O(n^2 m) term): Y = sym(X) S with sym(X) the symmetric matrix whose lower
 * triangle is that of X, rounded to `prec` (psdp_prec), on the matrix cores
 * (MFMA FP64, FP32, or BF16 with FP32 accumulation).  S is n x k (lds),
 * Y is n x k (ldy), FP64 device pointers, 1 <= k <= 144.  Synchronises the
 * handle's stream. */
psdp_status psdp_block_product(psdp_handle h, int n, const double *X, int ldx,
                               const double *S, int lds, int k, int prec,
                               double *Y, int ldy);

/* psdp_block_product for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same product, same kernels and same results, with every
 * buffer beyond X, S and Y (the copies of A, the staged S, the split-K
 * partial sums) in a 64 MiB device array the library holds on each GPU it
 * runs on until the process ends.  No allocation happens in the call (the
 * handle's own lazily allocated workspace is not used either).  The array
 * fits n <= 2048 with any k <= 144 in every precision; a larger request
 * returns PSDP_ERR_CAPACITY before any launch.  All calls on one GPU share
 * that GPU's array and each call leaves its contents behind: calls that
 * overlap on one GPU (several handles, streams or threads) race.
 * Synchronises the handle's stream. */
psdp_status psdp_block_product_noalloc(psdp_handle h, int n, const double *X, int ldx,
                                       const double *S, int lds, int k, int prec, double *Y,
                                       int ldy);

/* The tail certificate on its own (paper §5.2, Thm `bound`, second term
 * ||Pi(V_perp^T A V_perp)||_F with A = sym(X)): proves that every eigenvalue
 * of V_perp^T A V_perp is below delta through an FP64 Cholesky factorization
 * of (delta - eta) I - P A P + c V V^T, P = I - V V^T, c = ||A||_F / sqrt(n).
 *   X, ldx     n x n symmetric, lower triangle read (device)
 *   V, ldv     n x m with orthonormal columns (device), 0 <= m <= 48
 *   delta      > 0
 *   certified  (host) 1: proven; 0: a pivot was not positive (some eigenvalue
 *              of V_perp^T A V_perp is at least about delta)
 *   delta_eff  (host, may be NULL) threshold proven: max(delta, 4 eta)
 *   eta        (host, may be NULL) bound on the rounding of forming and
 *              factoring the matrix
 * PSDP_ERR_NUMERICAL for non-finite X.  Synchronises the handle's stream. */
psdp_status psdp_certify_tail(psdp_handle h, int n, const double *X, int ldx, const double *V,
                              int ldv, int m, double delta, int *certified, double *delta_eff,
                              double *eta);

/* ------------------------------------------------------------------------
 * Serving: a request loop for many concurrent ADMM solves (paper §6: every
 * PSD variable is projected once per ADMM iteration, warm-started from its
 * previous Ritz block).  A session is one such variable; its warm-start
 * block stays in device memory owned by the server.  Requests are admitted
 * while device-memory estimates stay within hbm_budget, run concurrently on
 * `slots` worker streams (single-cone path) and on one batching lane that
 * gathers every waiting small request (n <= small_n, positive side, block
 * <= 32) into one persistent batched launch; a request the lane does not
 * converge is redone on a worker through the full eigendecomposition.  Requests of one session run
 * in submission order; requests of different sessions overlap on the GPU.
 * The server owns its worker threads, handles and streams; the caller owns
 * X and Pi of each request until psdp_server_wait reports it done.
 * ------------------------------------------------------------------------ */
typedef struct psdp_server_s *psdp_server;

typedef struct {
    int slots;              /* concurrent single-cone workers, default 4         */
    size_t hbm_budget;      /* device bytes for workspaces; 0 = 16 GiB           */
    int batch_lane;         /* 1 (default): small requests share batched launches */
    int small_n;            /* largest order for the batching lane (<= 256)      */
    int max_batch;          /* most requests per batched launch, default 512     */
    psdp_options opt;       /* options of every request; side AUTO resolves per  */
                            /* session from its last inertia; fallback_full is   */
                            /* forced on so that every request returns Pi         */
} psdp_server_config;

typedef struct {
    psdp_info info;         /* the projection's info                             */
    long long ticket;
    int session;
    int lane;               /* 0 = single-cone worker, 1 = batching lane         */
    int batch_size;         /* requests in its launch (1 on a worker)            */
    double queue_ms;        /* submit -> start on the device                     */
    double latency_ms;      /* submit -> result complete                         */
} psdp_result;

typedef struct {
    long long submitted, completed, rejected;
    double p50_ms, p99_ms, mean_ms, max_ms;  /* latency of completed requests     */
    double throughput;      /* completed / (last completion - first submission) */
    size_t hbm_held;        /* current workspace estimate                        */
    size_t hbm_peak;        /* its maximum                                       */
    int active, queued;     /* requests on the device / waiting now             */
    int max_active;         /* most requests on the device at once              */
    long long batched_launches, batched_requests;
    long long lane_fallbacks; /* lane results not converged, redone exactly     */
} psdp_server_stats;

/* Defaults documented above (opt from psdp_default_options). */
void psdp_server_default_config(psdp_server_config *cfg);

/* Start the worker threads on HIP device `device`. */
psdp_status psdp_server_create(psdp_server *srv, int device, const psdp_server_config *cfg);

/* Wait for every submitted request, stop the workers, free everything. */
psdp_status psdp_server_destroy(psdp_server srv);

/* Open a session of order n (1 <= n) with block capacity m_cap (<= 48) and an
 * estimate of its positive eigenvalue count (-1: unknown, first request uses
 * the full eig).  Allocates its device block (n x m_cap) now. */
psdp_status psdp_server_open_session(psdp_server srv, int n, int m_cap, int pos_hint,
                                     int *session);

/* Close a session after its requests completed (PSDP_PENDING otherwise). */
psdp_status psdp_server_close_session(psdp_server srv, int session);

/* Submit Pi(X) for a session: X and Pi are n x n device matrices with
 * leading dimension n (lower triangle of X read, both triangles of Pi
 * written).  producer_stream (hipStream_t or NULL) is the stream that wrote
 * X: the request waits for it.  Returns at once with *ticket. */
psdp_status psdp_server_submit(psdp_server srv, int session, const double *X, double *Pi,
                               void *producer_stream, long long *ticket);

/* Wait up to timeout_ms (< 0: no limit) for a request; PSDP_OK fills *out
 * (the projection's status is out->info.status), PSDP_PENDING on timeout.
 * A ticket can be waited for until the next psdp_server_wait on it returns
 * PSDP_OK; afterwards it is forgotten. */
psdp_status psdp_server_wait(psdp_server srv, long long ticket, double timeout_ms,
                             psdp_result *out);

/* Wait until every submitted request has completed. */
psdp_status psdp_server_drain(psdp_server srv);

/* Copy a session's warm-start block (device, n x m, leading dim ldv) and
 * its Ritz values (device, m) out; *m = its width.  NULL V/lambda: width only. */
psdp_status psdp_server_session_block(psdp_server srv, int session, double *V, int ldv,
                                      double *lambda, int *m);

/* Counters and latency percentiles since creation (or the last reset). */
psdp_status psdp_server_stats_get(psdp_server srv, psdp_server_stats *st);
psdp_status psdp_server_stats_reset(psdp_server srv);

/* ------------------------------------------------------------------------
 * Approximate ADMM for semidefinite programs (paper §2, Alg. 1; §6: every
 * PSD projection by the warm-started block eigensolver on the side chosen
 * from the previous iterate's inertia, stopped at residual
 * tol_scale / k^tol_power; §6.2: infeasibility from successive differences).
 *
 * Problem, standard form:  minimize <C, Y>  s.t.  <A_i, Y> = b_i (i < p),
 * Y psd (n x n).  In the paper's form (P): x = Y, P = 0, q = C,
 * A x = (<A_i, Y>)_i stacked over Y itself, cone C = {b} x S_+.  The A_i are
 * given by their lower-triangle entries and their supports must be
 * disjoint (diagonal constraints, single off-diagonal entries, a trace, ...),
 * which makes the linear system of Alg. 1's first line exact in closed form:
 * A_eq^* A_eq acts on each A_i as ||A_i||_F^2 and as zero on their
 * orthogonal complement.
 * ------------------------------------------------------------------------ */
typedef struct {
    int n;                  /* order of Y                                         */
    int p;                  /* equality constraints                               */
    const double *C;        /* DEVICE n x n cost, lower triangle read             */
    int ldc;                /* >= n                                               */
    int nnz;                /* constraint entries (HOST arrays below, length nnz) */
    const int *con;         /* constraint of each entry, nondecreasing, 0..p-1;   */
                            /* every constraint has at least one entry            */
    const int *row;         /* row >= col, both in 0..n-1; no position twice      */
    const int *col;
    const double *val;      /* A_con holds val (finite, nonzero) at (row, col)    */
                            /* and (col, row)                                     */
    const double *b;        /* HOST p right-hand sides                            */
} psdp_sdp;

typedef struct {
    double rho, sigma, alpha; /* Alg. 1 parameters (0.1, 1e-6, 1.6)               */
    int max_iter;           /* iteration limit (2500)                             */
    int check_every;        /* iterations between termination and infeasibility   */
                            /* checks (40)                                        */
    double eps_abs, eps_rel; /* termination on the residuals of (P) (1e-5, 1e-5)  */
    double eps_inf;         /* infeasibility certificates (1e-5)                  */
    int exact;              /* 1: exact projections (full eig, the baseline);     */
                            /* 0 (default): psdp_project                          */
    double tol_scale;       /* projection residual tolerance at iteration k:      */
    double tol_power;       /* tol_scale / k^tol_power (10, 1.01: paper §6)       */
    int prec;               /* psdp_prec of the block products (FP64)             */
    int m_cap;              /* block capacity of the projections (48)             */
    int method;             /* eigensolver of the projections: PSDP_METHOD_LOBPCG */
                            /* (default) or PSDP_METHOD_CHEBYSHEV                 */
} psdp_admm_options;

enum {
    PSDP_ADMM_SOLVED = 0,
    PSDP_ADMM_MAX_ITER = 1,
    PSDP_ADMM_PRIMAL_INFEASIBLE = 2,  /* certificate: A^T dy ~ 0, b^T dy < 0, its  */
                                      /* PSD part negative semidefinite          */
    PSDP_ADMM_DUAL_INFEASIBLE = 3     /* certificate: A_eq dY ~ 0, dY psd,        */
                                      /* <C, dY> < 0 (the objective is unbounded) */
};

typedef struct {
    int status;             /* PSDP_ADMM_*                                        */
    int iters;              /* iterations run                                     */
    double obj;             /* <C, Y> at the last check                           */
    double r_prim, r_dual;  /* residuals of (P) at the last check                 */
    double proj_ms;         /* wall time of the projections (host clock)          */
    double total_ms;        /* wall time of the solve                             */
    int proj_block;         /* projections by the block eigensolver               */
    int proj_full;          /* projections by the exact path                      */
    int proj_not_certified; /* of those, block attempts that fell back            */
} psdp_admm_info;

/* Fill *opt with the defaults documented above. */
void psdp_admm_default_options(psdp_admm_options *opt);

/* Solve the SDP *prob with approximate ADMM.  Outputs (DEVICE): Y (n x n,
 * ldy) the primal matrix, y (p) the multipliers of the equality
 * constraints, W (n x n, ldw) the multiplier of the PSD block (at a solution
 * -W = C + sum_i y_i A_i is the dual slack, psd, and <W, Y> = 0).  Returns
 * PSDP_OK with info->status saying how the iteration ended, or an error
 * (PSDP_ERR_INVALID_ARG for overlapping supports or bad entries, before any
 * launch).  Allocates its buffers (about 10 n^2 doubles) for the duration of
 * the call and runs on the handle's stream, synchronising it. */
psdp_status psdp_admm_solve(psdp_handle h, const psdp_sdp *prob, const psdp_admm_options *opt,
                            double *Y, int ldy, double *y, double *W, int ldw,
                            psdp_admm_info *info);

/* Static string for a status code. */
const char *psdp_status_str(psdp_status s);

/* Per-kernel timing on the handle's stream (hipEvents around every launch of
 * the named kernel family while enabled).  Families: "product", "gram",
 * "tsmm", "small", "rebuild", "ingest", "batched".  *launches is the count,
 * *total_ms the summed event time, *bytes and *flops the algorithmic HBM
 * bytes and flops of those launches.  Reset by psdp_profile_enable. */
psdp_status psdp_profile_enable(psdp_handle h, int on);
psdp_status psdp_profile_get(psdp_handle h, const char *family, long *launches,
                             double *total_ms, double *bytes, double *flops);

/* Restricts the timing of psdp_profile_enable to the comma-separated kernel
 * families in `families` (e.g. "rr"); NULL or "" times every family.  Each
 * timed family adds two hipEvent records per launch group to the stream,
 * and every record costs the stream a few microseconds, so a throughput
 * measurement times only the family it reports.  The filter is kept by the
 * handle until changed; PSDP_ERR_INVALID_ARG for a null handle. */
psdp_status psdp_profile_filter(psdp_handle h, const char *families);

/* Device-to-host copies the library has made (in every call and thread of
 * the process, the server's workers included) since the last reset: their
 * count, total bytes and largest single copy.  They are state snapshots,
 * norms and eigenvalue counts, never a warm-start block: a session's block
 * (n x m doubles) stays on the device between requests.  reset != 0 clears
 * the counters after reading them. */
psdp_status psdp_transfer_stats(long long *copies, long long *bytes, long long *max_bytes,
                                int reset);

/* Library version string. */
const char *psdp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSDP_H */
