/*
 * cpasvt.h - C ABI of the MI355X (gfx950) library for singular value
 * shrinkage by Chebyshev polynomial approximation (CPA), after Onuki, Ono,
 * Shirai, Tanaka, "Fast Singular Value Shrinkage with Chebyshev Polynomial
 * Approximation Based on Signal Sparsity".
 *
 * What is computed.  For X (m x n) and a shrinkage response h on the
 * eigenvalues of the Gram (Sec. IV-A, eq. filter_response_ours; g(s) = s h(s^2)),
 * the library returns
 *     Y = X * hat H(X^T X)          (m >= n, Sec. III-B, eq. sing_shrink_from_eig_shrink)
 *     Y = hat H(X X^T) * X          (m <  n, the same identity on X^T)
 * where hat H is the K-term Chebyshev interpolant of h on [0, Lambda]
 * (Sec. III-A, eqs. chebychev_series_matrix, chebychev_coeff_shifted) and
 * Lambda >= lambda_max(Gram).  This is Algorithm 1 (Sec. III-B) with the
 * sparsifying transform T = Id and no truncation, evaluated with the sum
 * distributed over X: Y_0 = X, Y_1 = X hat B, Y_{k+1} = 2 Y_k hat B - Y_{k-1},
 * Y = c_0/2 Y_0 + sum_k c_k Y_k, hat B = (2/Lambda) Gram - Id.  No SVD or EVD is
 * computed.
 *
 * Conventions for every entry point.
 *   - Matrices are row-major with a leading dimension (elements between the
 *     starts of consecutive rows) >= the column count.
 *   - Pointers named *_dev are device memory owned by the caller; the library
 *     never frees them.  Pointers named *_host are host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it.  A call returns after enqueueing unless its
 *     description says it synchronises `stream`.
 *   - Argument errors are detected before anything is enqueued.  Nothing throws
 *     or aborts across this interface; every call returns a cpa_status, and
 *     cpa_last_error() gives a message for the calling thread.
 *   - The library owns its workspace (grown on demand inside the context with
 *     hipMalloc, freed by cpa_destroy).  Calls that share a context must not
 *     run concurrently on different host threads or streams.
 */
#ifndef CPASVT_H
#define CPASVT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CPA_OK = 0,
    CPA_ERR_ARG = 1,          /* invalid argument (null pointer, K < 1, aliasing, bad enum) */
    CPA_ERR_SHAPE = 2,        /* negative size, leading dimension too small, size above limits */
    CPA_ERR_ALLOC = 3,        /* device workspace allocation failed */
    CPA_ERR_HIP = 4,          /* a HIP runtime call failed */
    CPA_ERR_NONFINITE = 5,    /* a spectral bound came out NaN or infinite */
    CPA_ERR_BOUND = 6,        /* growth check failed even with the guaranteed bound */
    CPA_ERR_UNSUPPORTED = 7,  /* option combination not supported */
    CPA_ERR_IO = 8            /* a file could not be read or written, or is not a model file */
} cpa_status;

/* Members of the shrinkage family of Sec. IV-A (eq. filter_response_ours),
 * h(x; w(x)/rho, tau) = (sqrt(x) - w(x)/rho) / sqrt(x) if sqrt(x) > tau, else 0:
 *   CPA_SOFT            h(x; tau, tau)            g(s) = max(s - tau, 0)  (tau = 1/rho)
 *   CPA_HARD            h(x; 0, tau)              g(s) = s if s > tau else 0
 *   CPA_WEIGHTED_CONST  h(x; tau, tau)            a constant weight w/rho = tau
 *   CPA_WEIGHTED_FN     h(x; w(x), w(x))          w(x) = w_c / (sqrt(max(x - w_sigma, 0)) + w_eps)
 * The threshold test is strict (sqrt(x) == tau gives 0) and x <= 0 gives 0. */
typedef enum { CPA_SOFT = 0, CPA_HARD = 1, CPA_WEIGHTED_CONST = 2, CPA_WEIGHTED_FN = 3 } cpa_kind;

typedef struct {
    int32_t kind;       /* cpa_kind */
    int32_t reserved;   /* must be 0 */
    double tau;         /* threshold (SOFT, HARD, WEIGHTED_CONST) */
    double w_c;         /* WEIGHTED_FN numerator */
    double w_sigma;     /* WEIGHTED_FN offset subtracted from x = s^2 */
    double w_eps;       /* WEIGHTED_FN regulariser, > 0 */
} cpa_shrinkage;

/* How the spectral bound Lambda >= lambda_max(Gram) is obtained (Algorithm 1,
 * the maximum-eigenvalue step; the paper does not fix a method):
 *   CPA_BOUND_POWER      power iteration on the Gram: start vector entry i =
 *                        2u - 1, u = (SplitMix64(seed + (i+1)*0x9E3779B97F4A7C15) >> 11) * 2^-53;
 *                        w = Gram v, mu = v.w, stop when |mu_t - mu_{t-1}| <= power_tol * mu_t
 *                        or after power_iters products; ||r|| = sqrt(max(||w||^2 - mu^2, 0));
 *                        Lambda = min(mu + max(margin * mu, ||r||), (1 + margin) ||Gram||_F)
 *   CPA_BOUND_GIVEN      Lambda = opts.Lambda (must be >= 0 and finite)
 *   CPA_BOUND_FROBENIUS  Lambda = ||Gram||_F (always an upper bound)
 *   CPA_BOUND_LEARNED    the predictor network opts.model (see cpa_predictor_forward) on the
 *                        features (log ||X||_F, log ||Gram||_F^2, log(m n)), outputs (y0, y1):
 *                        Lambda = (1 + margin) ||Gram||_F exp(min(y0, 0)); K stays opts.K
 *                        (the per-matrix order is the batched path's,
 *                        cpa_shrink_batched_predicted).  With check = 1 a failed check
 *                        recomputes with the power-iteration bound (power_iters, power_tol).
 *                        Dense entry points only (cpa_shrink_dense, _noalloc,
 *                        cpa_spectral_bound); the others return CPA_ERR_UNSUPPORTED
 *   CPA_BOUND_LANCZOS    k-step Lanczos on the Gram from the power rule's start vector (or the
 *                        warm-start vector): q_1 = v/||v||, u = Gram q_j - beta_{j-1} q_{j-1},
 *                        alpha_j = q_j.u, u -= alpha_j q_j, beta_j = ||u||, q_{j+1} = u/beta_j
 *                        (no reorthogonalisation; k = min(lanczos_steps, d) steps, fewer if a
 *                        beta_j is exactly 0 or, with power_tol > 0, at the first step j >= 2
 *                        whose Ritz value theta_j (largest eigenvalue of T_j) satisfies
 *                        |theta_j - theta_{j-1}| <= power_tol theta_j; power_tol = 0 runs all
 *                        k steps); theta = largest eigenvalue of the tridiagonal
 *                        T_k, ||r|| = beta_k |s_k| with s its unit eigenvector;
 *                        Lambda = min(theta + max(margin * theta, ||r||), (1 + margin) ||Gram||_F).
 *                        The Ritz vector sum_j s_j q_j is the next warm start; info.mu and
 *                        info.resid report theta and ||r||, power_iters_done the steps.
 *                        Gram sides up to 4096 on the dense FP32 entry points (cpa_shrink_dense,
 *                        _noalloc, cpa_spectral_bound, cpa_shrink_dense_sparsified), the FP64
 *                        entry point, the CSR entry points (cpa_shrink_csr, cpa_svt_complete:
 *                        the operator form S^T S, n <= 4096), the RPCA and inpainting
 *                        drivers, and every matrix of the batched path (d <= 64);
 *                        CPA_ERR_UNSUPPORTED on larger sides, and where the (lanczos_steps
 *                        + 2) d doubles of Lanczos vectors do not fit an idle workspace
 *                        buffer (the FP64 path's m x n product buffer; the CSR path's
 *                        n x n or m x n recurrence buffers, rows padded to 32) */
typedef enum {
    CPA_BOUND_POWER = 0,
    CPA_BOUND_GIVEN = 1,
    CPA_BOUND_FROBENIUS = 2,
    CPA_BOUND_LEARNED = 3,
    CPA_BOUND_LANCZOS = 4
} cpa_bound_rule;

/* Arithmetic of the recurrence products (the Gram and the bound are always FP32
 * MFMA with FP64 reductions).
 *   CPA_PREC_FP32    FP32 MFMA with FP32 accumulation.
 *   CPA_PREC_BF16X3  each FP32 operand split into bf16 hi + lo (round to nearest
 *                    even); A_hi B_hi + A_hi B_lo + A_lo B_hi on the BF16 matrix
 *                    cores with FP32 accumulation.  Y_k, the accumulator and the
 *                    coefficients stay FP32 / FP64. */
typedef enum { CPA_PREC_FP32 = 0, CPA_PREC_BF16X3 = 1, CPA_PREC_FP64 = 2 } cpa_precision;
/* CPA_PREC_FP64 is accepted by cpa_shrink_dense_f64 only (FP64 inputs and
 * arithmetic); the FP32 entry points reject it. */

/* How the polynomial hat H(Gram) = c_0/2 I + sum_k c_k T_k(hat B) reaches X (dense path).
 *   CPA_EVAL_RECURRENCE  the three-term recurrence distributed over X (Algorithm 1's
 *                        loop applied to Y_k = X T_k(hat B)): K - 1 products of size
 *                        max(m,n) x d x d, d = min(m, n).
 *   CPA_EVAL_POLYNOMIAL  the matrix polynomial on the d x d side first (Algorithm 1's
 *                        H), then one product with X.  The polynomial is formed with
 *                        baby steps / giant steps in the Chebyshev basis: T_1..T_s by
 *                        the recurrence (s = ceil(sqrt K), at most 32), then
 *                        p = sum_j R_j T_j(T_s) by Clenshaw's recurrence, using
 *                        T_j(T_s(x)) = T_{js}(x): about 2 sqrt(K) products of d x d x d.
 *                        Same polynomial; rounding differs.  K <= 1024.
 *   CPA_EVAL_AUTO        POLYNOMIAL when K <= 1024 and it costs fewer flops,
 *                        otherwise RECURRENCE. */
typedef enum { CPA_EVAL_AUTO = 0, CPA_EVAL_RECURRENCE = 1, CPA_EVAL_POLYNOMIAL = 2 } cpa_eval;

/* Which Gram the bound and the polynomial use (eq. sing_shrink_from_eig_shrink:
 * X h(X^T X) = h(X X^T) X, so both give the same matrix; they differ in cost
 * and rounding).
 *   CPA_SIDE_AUTO   the smaller one: X^T X (n x n) when m >= n, else X X^T
 *   CPA_SIDE_RIGHT  X^T X, products with X on the right (Y_k Ghat)
 *   CPA_SIDE_LEFT   X X^T, products on the left (Ghat Y_k)
 * The sparse path forms S^T S (AUTO or RIGHT); the batched path takes AUTO. */
typedef enum { CPA_SIDE_AUTO = 0, CPA_SIDE_RIGHT = 1, CPA_SIDE_LEFT = 2 } cpa_side;
/* Damping of the Chebyshev coefficients, g_k for degree N = K - 1 (the kernel
 * polynomial method's factors):  Jackson ((N - k + 1) cos(pi k/(N+1)) +
 * sin(pi k/(N+1)) cot(pi/(N+1))) / (N + 1);  Lanczos sin(pi k/(N+1)) / (pi k/(N+1));
 * g_0 = 1. */
typedef enum { CPA_DAMP_NONE = 0, CPA_DAMP_JACKSON = 1, CPA_DAMP_LANCZOS = 2 } cpa_damping;

typedef struct {
    int32_t K;            /* number of Chebyshev coefficients (the paper's order alpha), >= 1 */
    int32_t bound;        /* cpa_bound_rule */
    double Lambda;        /* used with CPA_BOUND_GIVEN */
    int32_t power_iters;  /* maximum Gram-vector products, >= 1 */
    int32_t warm_start;   /* 1: start from the context's last power vector when its length matches */
    double power_tol;     /* relative tolerance on successive Rayleigh quotients */
    double margin;        /* relative margin delta added to the Rayleigh quotient */
    uint64_t seed;        /* start-vector seed */
    int32_t check;        /* 1: a-posteriori check of the bound (consequence of |T_k| <= 1 on
                             [-1, 1], Sec. II-B), with one recompute on failure at Lambda =
                             ||Gram||_F (at the power bound after CPA_BOUND_LEARNED)
                             (synchronises the stream).  Recurrence route: the growth
                             max_k ||Y_k||_F / ||X||_F <= 1 + growth_tol.  Matrix-polynomial
                             route: the Gram-weighted means of the baby steps,
                             max_{q=2..s} <Gram, T_q(Ghat)>_F / tr Gram <= 1 + growth_tol
                             (= sum_i lambda_i T_q(x_i) / sum_i lambda_i, at most 1 when every
                             eigenvalue maps into [-1, 1]) */
    int32_t precision;    /* cpa_precision */
    double growth_tol;    /* tolerance of the growth check */
    int32_t eval;         /* cpa_eval (dense and sparse paths; the batched path uses the recurrence) */
    int32_t side;         /* cpa_side */
    int32_t damping;      /* cpa_damping: coefficients times Jackson or Lanczos factors (not in the
                             paper; a ripple reducer for steep responses such as the high-order hard
                             threshold).  Dense, CSR and sparsified paths and the drivers; the
                             batched path rejects it */
    int32_t lanczos_steps; /* CPA_BOUND_LANCZOS: Lanczos steps in [1, 32]; 0 selects 12 */
    const float* model;   /* CPA_BOUND_LEARNED: the predictor model, CPA_PRED_MODEL_FLOATS floats in
                             device memory (caller-owned); ignored by the other rules */
    const double* coeffs; /* NULL: the shrinkage's Chebyshev coefficients (Sec. III-A).  Else K
                             doubles in device memory (caller-owned, read by the stream's kernels)
                             used as c_0..c_{K-1} of p(x) = c_0/2 + sum_k c_k T_k(2x/Lambda - 1),
                             e.g. another design from cpa_design_coeffs.  Needs CPA_BOUND_GIVEN
                             (the coefficients belong to that Lambda), check = 0 and no damping;
                             taken by cpa_shrink_dense, cpa_shrink_dense_noalloc and
                             cpa_shrink_csr, CPA_ERR_UNSUPPORTED elsewhere */
} cpa_opts;

/* Per-call report (host struct).  Filling it synchronises the stream. */
typedef struct {
    double Lambda;        /* bound used by the final evaluation */
    double mu;            /* last Rayleigh quotient, or the Ritz value theta with CPA_BOUND_LANCZOS
                             (0 with the other rules) */
    double resid;         /* last residual norm ||Gram v - mu v|| (the Ritz residual with Lanczos) */
    double fro_gram;      /* ||Gram||_F */
    double max_growth;    /* recurrence route: max_k ||Y_k||_F / ||X||_F over k = 1..K-1 (0 if
                             K == 1); matrix-polynomial route: the check's largest weighted
                             mean when check = 1, else 0 */
    int32_t power_iters_done; /* power products, or Lanczos steps */
    int32_t fallback;     /* 1 when the check forced Lambda = ||Gram||_F */
    int32_t side;         /* 0: Gram = X^T X (right side), 1: Gram = X X^T (left side) */
    int32_t reserved;
} cpa_info;

typedef struct cpa_ctx cpa_ctx;

/* Context bound to one HIP device.  Allocates no device memory until first use
 * (the first context on a device looks up that device's address of the static
 * scratch array of cpa_shrink_dense_noalloc, which loads the library's code on it). */
cpa_status cpa_create(cpa_ctx** ctx_out, int device);
cpa_status cpa_destroy(cpa_ctx* ctx);

/* Static text for a status code. */
const char* cpa_status_string(cpa_status s);
/* Message describing the last failure on the calling thread ("" if none). */
const char* cpa_last_error(void);

/* Fills opts with defaults: K = 16, POWER bound, power_iters = 100, power_tol = 1e-7,
 * margin = 0.01, seed = 0, warm_start = 0, check = 0, FP32, growth_tol = 1e-3,
 * eval = CPA_EVAL_AUTO. */
void cpa_default_opts(cpa_opts* opts);

/* Chebyshev coefficients on the host in FP64 (Sec. III-A, eq. chebychev_coeff_shifted;
 * Algorithm 1, coefficient step):
 *   c_k = (2/K) sum_{l=1..K} cos(k theta_l) h(Lambda/2 (cos theta_l + 1)),
 *   theta_l = pi (l - 1/2) / K,  k = 0..K-1.
 * c_host must hold K doubles.  Lambda == 0 gives all zeros.  Pure host code. */
cpa_status cpa_chebyshev_coeffs(const cpa_shrinkage* shrink, double Lambda, int K, double* c_host);

/* Other polynomial designs of degree K - 1 on [0, Lambda] for the shrinkage's response h,
 * the alternatives Sec. IV-B compares CPA with (eq. l_p_norm_for_approximation: p = 2 and
 * p = infinity), returned in the convention of opts.coeffs so the same kernels evaluate them:
 *   CPA_DESIGN_CHEBYSHEV  the CPA coefficients themselves (as cpa_chebyshev_coeffs; n unused)
 *   CPA_DESIGN_LSQ        least squares over the n uniform samples x_i = Lambda i / (n - 1),
 *                         i = 0..n-1 (n >= K, n >= 2; 2000 when n == 0), solved by Householder
 *                         QR in the Chebyshev basis (the same polynomial as the paper's
 *                         pseudo-inverse of the monomial Vandermonde matrix, without its
 *                         ill-conditioning at large K)
 *   CPA_DESIGN_MINIMAX    best uniform approximation on the n-point grid
 *                         x_i = (Lambda/2)(1 - cos(pi i / (n - 1))) (n >= 2 K + 1; 8000 when
 *                         n == 0) by the Remez exchange, started at the grid points nearest the
 *                         extrema of T_K, stopped when the largest grid error is within a
 *                         relative 1e-10 of the levelled error (at most 200 exchanges)
 * c_host receives K doubles.  err_host (may be NULL) receives the largest |h - p| over the
 * design's own points (samples, grid; the K Chebyshev nodes for CPA_DESIGN_CHEBYSHEV).
 * Lambda == 0 gives all zeros.  Pure host code; O(n K^2) time.  Errors: CPA_ERR_ARG for an
 * invalid shrinkage, Lambda, NULL c_host, unknown design or n out of range; K outside
 * [1, 1024] (CPA_ERR_ARG); CPA_ERR_NONFINITE if a reference system of the exchange is
 * singular. */
typedef enum { CPA_DESIGN_CHEBYSHEV = 0, CPA_DESIGN_LSQ = 1, CPA_DESIGN_MINIMAX = 2 } cpa_design;
cpa_status cpa_design_coeffs(const cpa_shrinkage* shrink, double Lambda, int K, int design, int n, double* c_host,
                             double* err_host);

/* The damping factors g_0..g_{K-1} of the kind (cpa_damping), host FP64; the
 * shrink uses c_k g_k.  Errors: K outside [1, 4096] or an unknown kind. */
cpa_status cpa_damping_factors(int K, int kind, double* g_host);

/* The device bound alone: forms the Gram of X (FP32 MFMA) and applies opts->bound
 * to it.  Writes Lambda to *Lambda_host and fills *info_host if non-null.
 * Synchronises the stream. */
cpa_status cpa_spectral_bound(cpa_ctx* ctx, void* stream, int m, int n,
                              const float* X_dev, int64_t ldx, const cpa_opts* opts,
                              double* Lambda_host, cpa_info* info_host);

/* Device bytes the context's workspace grows to for cpa_shrink_dense (and
 * cpa_spectral_bound) on an m x n input with these options: the Gram, two Y
 * buffers, the power vectors, the scalar block, the matrix-polynomial buffers
 * when that route runs, and the warm-start vector.  The context allocates them
 * on first use and keeps them (a larger call grows them); nothing is allocated
 * by this query.  (The RPCA driver adds one m x n buffer and its E_t partials.) */
cpa_status cpa_workspace_bytes(cpa_ctx* ctx, int m, int n, const cpa_opts* opts, size_t* bytes_host);

/* Dense shrinkage Y = hat G(X) of Algorithm 1 (T = Id), FP32 in and out.
 * X_dev (m x n, ldx) is read only; Y_dev (m x n, ldy) is written and must not
 * overlap X_dev (CPA_ERR_ARG).  m == 0 or n == 0 is a no-op.  Lambda == 0 (X == 0)
 * gives Y = 0.  Asynchronous unless info_host != NULL or opts->check == 1. */
cpa_status cpa_shrink_dense(cpa_ctx* ctx, void* stream, int m, int n,
                            const float* X_dev, int64_t ldx, float* Y_dev, int64_t ldy,
                            const cpa_shrinkage* shrink, const cpa_opts* opts,
                            cpa_info* info_host);

/* For callers that cannot allocate device memory (work recorded under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the shrinkage
 * of cpa_shrink_dense with the same kernels, arguments, options, results, errors
 * and synchronisation, but its workspace (Gram, power vectors, scalar block,
 * matrix-polynomial or Y ping-pong buffers, warm-start vector) lives in a static
 * 64 MiB device array that each GPU holds from its first cpa_create until the
 * process ends.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine; info is read through a fixed host buffer; per-launch timing is
 * skipped).  Limits: Gram side d = min(m, n) (or the side opts->side picks) at
 * most 4096, and the workspace for (m, n, K) at most 64 MiB - 32 KiB: d^2 floats
 * for the Gram plus, on the matrix-polynomial route, (s + ceil(K/s) + 3) d^2 floats
 * (s = ceil(sqrt K)), or on the recurrence route 2 m n floats; e.g. 1024 x 1024 at
 * K = 30 (61 MB) fits, at K = 64 it does not.  Larger requests return
 * CPA_ERR_SHAPE before anything is enqueued.  Every call on a GPU shares that
 * GPU's array, whose contents persist between calls (the scalar block is cleared
 * by a fill kernel at the start of each call; everything else is written before
 * it is read): calls that overlap on one GPU, from any stream, thread or context,
 * race and give wrong results.  With opts->warm_start the power iteration starts
 * from the vector the previous call on that GPU left, when its length matches. */
cpa_status cpa_shrink_dense_noalloc(cpa_ctx* ctx, void* stream, int m, int n,
                                    const float* X_dev, int64_t ldx, float* Y_dev, int64_t ldy,
                                    const cpa_shrinkage* shrink, const cpa_opts* opts,
                                    cpa_info* info_host);

/* The same shrinkage with FP64 input, output and arithmetic (Algorithm 1, with
 * the recurrence of eq. recurrence_our_method distributed over X as in the FP32
 * path): FP64 Gram (side as opts->side), the bound and the coefficients in FP64
 * (power iteration on the FP64 Gram), K - 1 FP64 products Y_k Gram (or Gram Y_k)
 * each followed by the three-term update, the sum accumulated in Y_dev.
 * opts->precision may be CPA_PREC_FP32 or CPA_PREC_FP64 (the arithmetic is FP64
 * either way); eval RECURRENCE or AUTO (the matrix polynomial is FP32-only);
 * check = 0.  Layout, aliasing, edge cases and synchronisation as
 * cpa_shrink_dense.  Workspace: a d x d and three m x n FP64 buffers. */
cpa_status cpa_shrink_dense_f64(cpa_ctx* ctx, void* stream, int m, int n,
                                const double* X_dev, int64_t ldx, double* Y_dev, int64_t ldy,
                                const cpa_shrinkage* shrink, const cpa_opts* opts,
                                cpa_info* info_host);

/* RPCA background modelling by ADMM (Appendix B, eq. admm_algorithm_mod) for
 *   min ||L||_* + eta ||S||_1  s.t.  I = L + S,   z = K [l; s], K = [[Id,0],[0,Id],[Id,Id]].
 * One iteration:
 *   a = (z1-u1) + (z3-u3), b = (z2-u2) + (z3-u3), l = (2a-b)/3, s = (2b-a)/3;
 *   z1 = CPA soft shrinkage of (l + u1) with tau = inv_rho   (the nuclear-norm prox);
 *   z2 = sgn(s+u2) max(|s+u2| - eta_over_rho, 0);  z3 = I;
 *   u1 += l - z1, u2 += s - z2, u3 += l + s - I;
 *   E_t = ||l_new - l_old||_2 / ||l_new||_2.
 * State: state_dev holds cpa_rpca_state_floats(m, n) floats laid out as seven
 * consecutive m x n row-major blocks [l, s, z1, z2, u1, u2, u3] (z3 = I is not
 * stored).  After any number of iterations L = block 0 and S = block 1.
 * cpa_rpca_init writes the start l = s = u1 = u2 = u3 = 1 and z1 = z2 = 1; the
 * third block of z is I from the start (the paper leaves z_0 unstated; z_0 =
 * [l_0; s_0; I] is the reading used, since that block is the projection onto
 * the observed data at every iteration).
 * cpa_rpca_iterate runs `iters` iterations from the given state; the spectral
 * bound of each shrink uses opts (power iteration warm-started across
 * iterations when opts->warm_start == 1).  Et_dev (device, `iters` doubles, may
 * be NULL) receives E_t.  I_dev (m x n, ld = n) is read only.  Asynchronous. */
int64_t cpa_rpca_state_floats(int m, int n);
cpa_status cpa_rpca_init(cpa_ctx* ctx, void* stream, int m, int n, float* state_dev);
cpa_status cpa_rpca_iterate(cpa_ctx* ctx, void* stream, int m, int n, const float* I_dev,
                            float* state_dev, int iters, double inv_rho, double eta_over_rho,
                            const cpa_opts* opts, double* Et_dev);

/* The same ADMM in one call: from the start state, iterations until
 * E_t <= tol (the paper's stopping rule, Sec. V-B) or max_iters, then L and S
 * (m x n, contiguous, caller-owned) receive the result.  E_t is checked after
 * every iteration, so the call synchronises the stream once per iteration and
 * stops at the first iteration with E_t <= tol; Et_host (max_iters doubles,
 * nullable) receives E_1, E_2, ... and *iters_done the number of iterations run.
 * The state lives in the context (7 m n floats).  I, L and S must not overlap. */
cpa_status cpa_rpca_admm(cpa_ctx* ctx, void* stream, int m, int n, const float* I_dev, float* L_dev,
                         float* S_dev, double inv_rho, double eta_over_rho, int max_iters, double tol,
                         const cpa_opts* opts, double* Et_host, int* iters_done);

/* Texture inpainting by ADMM (Sec. V-C, eq. texture_repaire4; Appendix A,
 * eq. admm_algorithm_inp) for
 *   min ||L||_* + eta ||Psi l||_1 + iota_I(Omega l) + iota_D(l) + iota_M(Omega_bar l),
 *   z = K l, K = [Id; Psi; Omega; Id; Omega_bar],
 * Psi the orthonormal 2-D DCT (Psi l = D_m L D_n^T, DCT-II matrices built on the
 * device), Omega the observed pixels (omega_dev != 0) and Omega_bar the region to
 * recover (omega_dev == 0).  One iteration:
 *   l = (K^T K)^{-1} K^T (z - u)   (K^T K = 4 Id; 3 Id + Omega without the mean term);
 *   z1 = CPA soft shrinkage of l + u1 with tau = inv_rho;
 *   z2 = sgn(y) max(|y| - eta_over_rho, 0), y = Psi l + u2;
 *   z3 = Omega I (the observed pixels);  z4 = clip(l + u4, 0, 1);
 *   z5 = y5 + (c - mean of y5 over the region) on the region, y5 elsewhere, with
 *        y5 = Omega_bar l + u5 and c = the mean of I over border_dev != 0 (the
 *        pixels surrounding the region; the caller chooses them);
 *   u += K l - z;  E_t = ||l_new - l_old||_2 / ||l_new||_2.
 * border_dev == NULL drops the mean term (z5, u5 untouched), as in the
 * random-corruption experiment of Sec. V-F.  An empty border or region makes
 * the shift 0.
 * State: cpa_inpaint_state_floats(m, n) floats, eleven consecutive m x n
 * row-major blocks [l, z1, z2, z3, z4, z5, u1, u2, u3, u4, u5]; L = block 0.
 * cpa_inpaint_init writes the start l = u = 1 and z = K l (the paper gives
 * l_0 = u_0 = 1; z_0 = K l_0 is the reading used).  cpa_inpaint_iterate runs
 * `iters` iterations (launched directly, no graph); Et_dev (device, `iters`
 * doubles, may be NULL) receives E_t.  I, omega and border (m x n floats, ld = n)
 * are read only and must not overlap the state.  Asynchronous. */
int64_t cpa_inpaint_state_floats(int m, int n);
cpa_status cpa_inpaint_init(cpa_ctx* ctx, void* stream, int m, int n, const float* omega_dev, float* state_dev);
cpa_status cpa_inpaint_iterate(cpa_ctx* ctx, void* stream, int m, int n, const float* I_dev, const float* omega_dev,
                               const float* border_dev, float* state_dev, int iters, double inv_rho,
                               double eta_over_rho, const cpa_opts* opts, double* Et_dev);

/* Sparse shrinkage, CSR input (row pointers int32[m+1], sorted column indices
 * int32[nnz], FP32 values), m >= n (for m < n shrink the transpose, i.e. pass the
 * CSC arrays as CSR of S^T, and transpose the result).  The result is dense:
 * Y_dev (m x n, ldy) = hat G(S), evaluated in
 * operator form (Algorithm 1 with T = Id, sum distributed over S, and
 * X p(X^T X) = p(X X^T) X from eq. sing_shrink_from_eig_shrink):
 *   W = S^T Y_k (n x n),  Y_{k+1} = 2((2/Lambda) S W - Y_k) - Y_{k-1},  Y_0 = S,
 * so S^T S is never formed.  The power bound iterates v <- S^T (S v) and caps at
 * (1 + margin) tr(S^T S) = (1 + margin) ||S||_F^2.  The transposed pattern is built
 * on the device and cached in the context until the CSR pointers or sizes change;
 * a new pattern is first validated on the device (rowptr[0] = 0, rowptr[m] = nnz,
 * nondecreasing, 0 <= colidx < n), which synchronises once, and a malformed one
 * returns CPA_ERR_ARG before any kernel indexes with it.
 * FP32 only; opts->check must be 0.  Fills *info_host (synchronising) if non-null. */
cpa_status cpa_shrink_csr(cpa_ctx* ctx, void* stream, int m, int n, int64_t nnz, const int32_t* rowptr_dev,
                          const int32_t* colidx_dev, const float* val_dev, float* Y_dev, int64_t ldy,
                          const cpa_shrinkage* shrink, const cpa_opts* opts, cpa_info* info_host);

/* Matrix completion by singular value thresholding (Cai, Candes, Shen; the paper
 * uses the nuclear-norm prox of Sec. V-B.1 inside its solvers) on the observed
 * entries P_Omega(M) given in CSR (the pattern is Omega; columns strictly
 * increasing within a row):
 *   Y^0 = k0 delta P_Omega(M), k0 = ceil(tau / (delta ||P_Omega(M)||_2)),
 *   X^t = shrink_tau(Y^{t-1})  (the CSR shrinkage, soft threshold tau),
 *   Y^t = Y^{t-1} + delta P_Omega(M - X^t).
 * The iterate Y^t lives on Omega (nnz values in CSR order).  On the
 * matrix-polynomial route with n <= 4096 the iterations before the last form only
 * the observed entries of X^t (the Gram by rows of Y, the polynomial p on the
 * n x n side, then (Y p)[r][c] for (r, c) in Omega); the last iteration forms the
 * dense X^iters.  X_dev (m x n dense, ldx >= n) receives X^iters.  resid_dev
 * (device, iters doubles, nullable) receives ||P_Omega(M - X^t)||_F / ||P_Omega M||_F.
 * Y0_vals_dev (device, nnz floats, nullable): start from this iterate instead of
 * k0 delta P_Omega(M) (k0 is then neither computed nor reported: *k0_host = 0);
 * Y_vals_dev (device, nnz floats, nullable; may equal Y0_vals_dev, must not
 * partly overlap it): receives Y^iters, so a later call can continue the run.
 * Lambda_dev (device, iters doubles, nullable): the bound of each iteration's
 * shrink.  *k0_host (nullable) receives k0.  Synchronises once (for k0 and the
 * norm of P_Omega M). */
cpa_status cpa_svt_complete(cpa_ctx* ctx, void* stream, int m, int n, int64_t nnz, const int32_t* rowptr_dev,
                            const int32_t* colidx_dev, const float* Mobs_dev, double tau, double delta, int iters,
                            float* X_dev, int64_t ldx, const cpa_opts* opts, double* resid_dev, double* k0_host,
                            const float* Y0_vals_dev, float* Y_vals_dev, double* Lambda_dev);

/* Batched shrinkage of many small matrices in one persistent launch (each
 * matrix: Algorithm 1 with T = Id, evaluated as in cpa_shrink_dense, inside one
 * workgroup; workgroups take matrices from an atomic queue).
 *   m_dev, n_dev, off_dev: device arrays of `batch` entries; matrix j is row-major
 *     m_j x n_j (leading dimension n_j) at X_dev + off_j, and its result is written
 *     at Y_dev + off_j (same shape).  X and Y must not overlap.
 *   Limits per matrix: min(m_j, n_j) <= 64, max(m_j, n_j) <= 128; other matrices
 *     are skipped with status 2.
 *   shrink_dev: device array of `batch` cpa_shrinkage records, or NULL to apply
 *     *shrink_host to every matrix.
 *   opts: K <= 64; bound CPA_BOUND_POWER (per-matrix power iteration, as in the
 *     dense path), CPA_BOUND_GIVEN (Lambda_dev[j]), CPA_BOUND_FROBENIUS; precision
 *     CPA_PREC_FP32, or CPA_PREC_BF16X3 (each recurrence product as three BF16
 *     matrix-core products of hi/lo parts with FP32 accumulation, as in
 *     cpa_shrink_dense; the Gram and the bound stay FP32); warm_start is not used.  With check = 1 every matrix is
 *     tested after its recurrence: ||Y_{K-1}||_F <= (1 + growth_tol) ||X_j||_F
 *     (inside [0, Lambda] every |T_k| <= 1; above it T_k grows with k, so the
 *     last term is the largest); a failing matrix is redone once with
 *     Lambda = (1 + margin) ||Gram||_F.  No synchronisation.
 *   Lambda_out_dev, status_dev: optional device arrays of `batch` entries
 *     (bound used; status 0 = done, 1 = redone with the fallback bound,
 *     2 = shape outside the limits, 3 = growth check failed at the last bound).
 * Asynchronous. */
cpa_status cpa_shrink_batched(cpa_ctx* ctx, void* stream, int batch, const int32_t* m_dev, const int32_t* n_dev,
                              const int64_t* off_dev, const float* X_dev, float* Y_dev,
                              const cpa_shrinkage* shrink_dev, const cpa_shrinkage* shrink_host,
                              const cpa_opts* opts, const double* Lambda_dev, double* Lambda_out_dev,
                              int32_t* status_dev);

/* ---- Sparsified shrinkage (Sec. III-B, Algorithm 1 with a transform and
 * truncation).  The Gram G (side as opts->side) is transformed,
 * Phi = T G T^T (eq. sing_shrink_exact_sparse), its entries below
 * eps = the keep-th largest |Phi_ij| are set to zero (eq. threshold_components;
 * entries equal to eps are kept, so an off-diagonal keep-th value also keeps its
 * mirror), the bound and the coefficients are taken from the truncated matrix,
 * hat H = hat h(truncated Phi) is formed, and Y = X T^T hat H T (or
 * T^T hat H T X on the left side).  Phi is formed exactly symmetric (block
 * transforms: FP64 transform of the FP32 Gram, upper tiles mirrored).
 * hat H is computed on the rows of the truncated matrix that keep an entry: an
 * empty row (and, by symmetry, column) is an eigenvector with eigenvalue 0, where
 * hat H is hat h(0).  opts->eval selects how:
 *   AUTO / POLYNOMIAL (2 <= K <= 1024): the bound and the baby-step / giant-step
 *     matrix polynomial on that block as a dense matrix (zero-padded to full
 *     64 x 64 tiles).  Its size is read back once: the call waits for the
 *     stream once, after the truncation.
 *   RECURRENCE (and K = 1 or K > 1024): Algorithm 1's recurrence with the block
 *     stored sparse (one sparse-dense product per step), the bound on the whole
 *     truncated matrix; no wait unless info/eps/nnz are requested.
 *   transform: CPA_TRANSFORM_BLOCK_DCT8 (the 8 x 8 block DCT, T = kron(I, D_8)),
 *              CPA_TRANSFORM_HAAR1 (the one-level orthonormal Haar DWT),
 *              CPA_TRANSFORM_HAAR1_LOWPASS (the same, with every entry of Phi in
 *              a high-frequency row or column set to zero before the threshold,
 *              as in the experiments of Sec. V),
 *              CPA_TRANSFORM_DCT (the orthonormal DCT-II over the whole side, dense:
 *              T G T^T and T^T hat H T by FP32 products, Phi then symmetrised), or
 *              CPA_TRANSFORM_IDENTITY (truncation of the Gram itself).
 *   threshold: CPA_THRESHOLD_KEEP: eps = the keep-th largest |Phi_ij|,
 *              1 <= keep <= d^2 (d: the Gram side, a multiple of 8) -- the
 *              K(|Phi|, k) of eq. (recommendation_epsilon);
 *              CPA_THRESHOLD_ABSOLUTE: eps given (finite, >= 0; the experiments
 *              of Table III fix eps), compared with the FP32 |Phi_ij| after rounding
 *              to FP32; keep is ignored.  An eps above every |Phi_ij| keeps nothing:
 *              the truncated matrix is zero, its bound is 0 and Y = 0 (on both
 *              routes; the kept count is read back, so the call waits for the
 *              stream once on the recurrence route too).
 * FP32, check = 0 only.  eps_host and nnz_host (nullable) receive the threshold
 * and the number of kept entries (synchronising).
 * The truncated matrix need not be positive semidefinite: its spectrum can leave
 * [0, Lambda] on the negative side, where Chebyshev series grow, so the keep
 * count must retain the transform's significant entries. */
typedef enum {
    CPA_TRANSFORM_IDENTITY = 0,
    CPA_TRANSFORM_BLOCK_DCT8 = 1,
    CPA_TRANSFORM_HAAR1 = 2,
    CPA_TRANSFORM_HAAR1_LOWPASS = 3,
    CPA_TRANSFORM_DCT = 4
} cpa_transform;

typedef enum { CPA_THRESHOLD_KEEP = 0, CPA_THRESHOLD_ABSOLUTE = 1 } cpa_threshold;

typedef struct {
    int32_t transform;  /* cpa_transform */
    int32_t threshold;  /* cpa_threshold */
    int64_t keep;       /* CPA_THRESHOLD_KEEP: eps = the keep-th largest |Phi_ij| */
    double eps;         /* CPA_THRESHOLD_ABSOLUTE: the threshold itself */
} cpa_sparsify;

cpa_status cpa_shrink_dense_sparsified(cpa_ctx* ctx, void* stream, int m, int n, const float* X_dev, int64_t ldx,
                                       float* Y_dev, int64_t ldy, const cpa_shrinkage* shrink, const cpa_opts* opts,
                                       const cpa_sparsify* sparsify, cpa_info* info_host, double* eps_host,
                                       int64_t* nnz_host);

/* Adaptive keep count of eq. (recommendation_epsilon) (Sec. V, with the counts
 * k_1, k_2, k_3 of Table IV) for a d x d transformed Gram and the ADMM change E_t:
 *   *keep = ceil(d^2 / 20000)    (0.5e-4 d^2) if E_t > E_l,
 *           ceil(3 d^2 / 20000)  (1.5e-4 d^2) if E_l >= E_t > E_m,
 *           ceil(d^2 / 2000)     (0.5e-3 d^2) otherwise,
 * in exact integer arithmetic, clamped to [1, d^2].  The paper's switch points are
 * E_l = CPA_SCHEDULE_E_L and E_m = CPA_SCHEDULE_E_M.  E_t = +inf (no previous
 * iteration) gives the first case.  Host only; CPA_ERR_ARG for a NaN E_t, a NULL
 * keep, or switch points that are not finite with 0 <= E_m <= E_l; CPA_ERR_SHAPE
 * for d <= 0. */
#define CPA_SCHEDULE_E_L 0.03
#define CPA_SCHEDULE_E_M 6e-4
cpa_status cpa_keep_schedule(double E_t, int d, double E_l, double E_m, int64_t* keep);

/* Texture inpainting (as cpa_inpaint_iterate, Appendix A) with z1 by the
 * sparsified shrink (cpa_shrink_dense_sparsified with `transform`) and its keep
 * count from eq. (recommendation_epsilon): iteration t uses
 * cpa_keep_schedule(E_{t-1}, d, E_l, E_m), d the Gram side, with E_prev before the
 * first iteration of the call (+inf on a fresh start; the last E_t of the previous
 * call to continue a run).  Et_dev (device, `iters` doubles) is required: the call
 * reads each E_t back, so it waits for the stream once per iteration (and the
 * sparsified shrink once more).  keep_host (host, `iters` int64, may be NULL)
 * receives the keep counts.  The Gram side must be a multiple of 8; FP32 only.
 * Errors as cpa_inpaint_iterate and cpa_keep_schedule, plus CPA_ERR_ARG for an
 * unknown transform or a NULL Et_dev.  The paper's experiment (Table IV) uses the
 * DCT; the truncated matrix can be indefinite for data that the transform does not
 * sparsify (cpa_shrink_dense_sparsified), and the iteration then need not converge. */
cpa_status cpa_inpaint_iterate_scheduled(cpa_ctx* ctx, void* stream, int m, int n, const float* I_dev,
                                         const float* omega_dev, const float* border_dev, float* state_dev, int iters,
                                         double inv_rho, double eta_over_rho, const cpa_opts* opts, int32_t transform,
                                         double E_prev, double E_l, double E_m, double* Et_dev, int64_t* keep_host);

/* ---- Batched plans: the batched shrink as one captured graph, tuned once.
 * Not in the paper (it shrinks one matrix at a time); the per-matrix
 * computation is exactly that of cpa_shrink_batched.
 *
 * cpa_batched_plan_create binds every argument of cpa_shrink_batched (same
 * meaning, layout and limits; the arrays must stay allocated, and m_dev, n_dev,
 * off_dev unchanged, for the plan's lifetime), picks a launch configuration and
 * captures the launch (queue reset + kernel) in a HIP graph.  With tune = 1 it
 * runs the batch under every configuration of the search space (persistent
 * workgroups per CU: 1 or the occupancy limit; recurrence output blocks per MFMA
 * group: 1 or 2; queue order: by index, or largest d^2 e first), four times
 * each, on `stream`, writing Y_dev and the optional outputs, and keeps the
 * fastest; with tune = 0 it takes the configuration cpa_shrink_batched uses.
 * Every configuration yields the same bits.  Creation synchronises `stream`
 * (the shapes are read to build the largest-first order).
 * cpa_batched_plan_execute replays the graph on `stream` (asynchronous; reads
 * the current contents of X_dev, Lambda_dev and shrink_dev).  Replays of one
 * plan must not overlap (they share its queue counter).
 * cpa_batched_plan_tuning reports the choice; cpa_batched_plan_destroy
 * synchronises the device and frees the plan (NULL is accepted). */
typedef struct cpa_batched_plan cpa_batched_plan;

typedef struct {
    int32_t grid;         /* workgroups launched */
    int32_t pair;         /* recurrence output blocks per MFMA group */
    int32_t order;        /* 0: queue by index, 1: largest first */
    int32_t candidates;   /* configurations timed (0: not tuned) */
    double best_us;       /* mean launch time of the chosen configuration (0 if not tuned) */
    double default_us;    /* mean launch time of cpa_shrink_batched's configuration (0 if not tuned) */
} cpa_batched_tuning;

cpa_status cpa_batched_plan_create(cpa_ctx* ctx, void* stream, int batch, const int32_t* m_dev, const int32_t* n_dev,
                                   const int64_t* off_dev, const float* X_dev, float* Y_dev,
                                   const cpa_shrinkage* shrink_dev, const cpa_shrinkage* shrink_host,
                                   const cpa_opts* opts, const double* Lambda_dev, double* Lambda_out_dev,
                                   int32_t* status_dev, int32_t tune, cpa_batched_plan** plan_out);
cpa_status cpa_batched_plan_execute(cpa_batched_plan* plan, void* stream);
cpa_status cpa_batched_plan_tuning(const cpa_batched_plan* plan, cpa_batched_tuning* out);
cpa_status cpa_batched_plan_destroy(cpa_batched_plan* plan);

/* ---- Learned bound and order predictor (not in the paper).  It stands in for
 * the maximum-eigenvalue step of Algorithm 1 and chooses the order alpha per
 * matrix, for the batched path.
 *
 * Model: a perceptron 3 -> 64 -> 64 -> 2 with tanh hidden units, stored as
 * CPA_PRED_MODEL_FLOATS floats (device memory, 16-byte aligned):
 *   W1[64][3] | b1[64] | W2[64][64] | b2[64] | W3[2][64] | b3[2]   (out x in, row-major;
 *   CPA_PRED_PARAMS trainable parameters) | mean[3] | inv_std[3] | 2 unused.
 * Features of a matrix X (m x n, Gram G): f = (log ||X||_F, log ||G||_F^2, log(m n));
 * the network sees x = (f - mean) * inv_std and returns y = (y0, y1), read as
 *   Lambda = (1 + margin) ||G||_F exp(min(y0, 0))      (never above the Frobenius bound)
 *   K_j    = clamp(ceil(exp(y1)), K_min, opts.K).
 * Training loss: pinball (quantile) loss, mean over samples and both outputs of
 * max(q_o r, (q_o - 1) r), r = target - y; a high q_0 makes y0 err on the side
 * of a larger Lambda.  Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrected). */
#define CPA_PRED_PARAMS 4546
#define CPA_PRED_MODEL_FLOATS 4554

/* Features of every matrix of a batch (layout as in cpa_shrink_batched):
 * feat_dev receives batch x 3 floats, computed exactly as the predicted path
 * computes them (FP32 MFMA Gram, FP64 sums).  A zero matrix gives -inf for the
 * first two.  status_dev (nullable): 0, or 2 for a shape outside the limits
 * (its features are not written).  Asynchronous. */
cpa_status cpa_batched_features(cpa_ctx* ctx, void* stream, int batch, const int32_t* m_dev, const int32_t* n_dev,
                                const int64_t* off_dev, const float* X_dev, float* feat_dev, int32_t* status_dev);

/* cpa_shrink_batched with the bound and the order taken from the predictor
 * model_dev (see above) instead of a power iteration: per matrix the Gram, its
 * features, the network, then the coefficients and the recurrence at
 * (Lambda, K_j).  opts.K is the largest order (<= 64), K_min the smallest.
 * With opts.check = 1, a matrix whose growth test fails is redone once with the
 * power-iteration bound of opts (status 1).  K_out_dev (nullable, int32 per
 * matrix) receives K_j; Lambda_out_dev and status_dev as in cpa_shrink_batched.
 * Asynchronous. */
cpa_status cpa_shrink_batched_predicted(cpa_ctx* ctx, void* stream, int batch, const int32_t* m_dev,
                                        const int32_t* n_dev, const int64_t* off_dev, const float* X_dev,
                                        float* Y_dev, const cpa_shrinkage* shrink_dev,
                                        const cpa_shrinkage* shrink_host, const cpa_opts* opts,
                                        const float* model_dev, int32_t K_min, double* Lambda_out_dev,
                                        int32_t* K_out_dev, int32_t* status_dev);

/* Model files (host file IO, synchronising): magic "CPAPRED1", int32 version 1,
 * int32 count = CPA_PRED_MODEL_FLOATS, then the floats (little-endian).  Load
 * checks the magic, the version and the count (CPA_ERR_IO otherwise) before it
 * writes model_dev. */
cpa_status cpa_predictor_save(cpa_ctx* ctx, void* stream, const float* model_dev, const char* path);
cpa_status cpa_predictor_load(cpa_ctx* ctx, void* stream, const char* path, float* model_dev);

/* Network outputs for n feature rows: y_dev (n x 2) = net(feat_dev (n x 3)).
 * Asynchronous. */
cpa_status cpa_predictor_forward(cpa_ctx* ctx, void* stream, int64_t n, const float* feat_dev,
                                 const float* model_dev, float* y_dev);

/* Gradient of the pinball loss over all n samples (targets targ_dev, n x 2;
 * quantiles_host[2] in (0, 1)) with respect to the CPA_PRED_PARAMS parameters:
 * grad_dev receives CPA_PRED_PARAMS floats; loss_dev (nullable, one double)
 * receives the loss.  Per-workgroup partials are summed in a fixed order, so
 * the result does not depend on scheduling.  Asynchronous. */
cpa_status cpa_predictor_grad(cpa_ctx* ctx, void* stream, int64_t n, const float* feat_dev, const float* targ_dev,
                              const float* quantiles_host, const float* model_dev, float* grad_dev,
                              double* loss_dev);

/* Minibatch training: `epochs` passes over the n samples in their stored order,
 * minibatches of batch_size (<= 16384; the last one of a pass may be smaller),
 * one Adam step per minibatch on the parameters of model_dev (updated in place;
 * the normalisation entries are not trained).  adam_dev holds 2 x CPA_PRED_PARAMS
 * floats (first moments, then second moments), zero before the first call;
 * *step_io_host is the Adam step count, 0 before the first call, advanced by
 * the steps taken.  epoch_loss_dev (nullable, `epochs` doubles) receives the
 * mean minibatch loss of every pass, measured before each step's update.
 * Asynchronous (the host only enqueues). */
cpa_status cpa_predictor_train(cpa_ctx* ctx, void* stream, int64_t n, const float* feat_dev, const float* targ_dev,
                               const float* quantiles_host, int32_t batch_size, int32_t epochs, float lr,
                               float* model_dev, float* adam_dev, int64_t* step_io_host, double* epoch_loss_dev);

/* Instrumentation: per-launch timing with HIP events.  While enabled, every
 * launch of the recurrence and full matrix-polynomial GEMMs (which = 0), of the
 * Gram GEMM (which = 1) and of the matrix-polynomial products computed as
 * symmetric pieces (which = 2) is bracketed by a pair of events recorded on the
 * caller's stream.
 * cpa_timing_enable resets the record; cpa_timing_read waits for the recorded
 * events and returns the summed kernel time in milliseconds and the number of
 * launches since the last reset. */
cpa_status cpa_timing_enable(cpa_ctx* ctx, int enable);
cpa_status cpa_timing_read(cpa_ctx* ctx, int which, double* total_ms_host, int64_t* launches_host);

/* Achievable matrix-core throughput (measurement support for roofline figures,
 * not part of the method): launches a kernel whose waves issue `iters` rounds
 * of eight independent MFMAs on register operands (kind 0:
 * v_mfma_f32_16x16x4f32, 1: v_mfma_f32_16x16x32_bf16; four waves per SIMD, no
 * memory traffic), twice, and returns the second launch's rate in TFLOP/s
 * (dense flops).  clock_ghz_host (nullable) receives the shader clock during the
 * second launch's MFMA loop: the first wave's shader-cycle count over its span of
 * the constant-rate wall counter (hipDeviceAttributeWallClockRate).  Synchronises
 * `stream`. */
cpa_status cpa_peak_mfma(cpa_ctx* ctx, void* stream, int kind, int iters, double* tflops_host,
                         double* clock_ghz_host);

#ifdef __cplusplus
}
#endif

#endif /* CPASVT_H */
