/*
 * fastcpd.h -- C ABI of libfastcpd.so, a gfx950 (MI355X) implementation of the
 * EM iteration of Fast Coherent Point Drift (Feng, Feng & Zhu, "Fast Coherent
 * Point Drift", arXiv 2006.06281) and of the original CPD M-step it replaces.
 *
 * Problem statement (Section I and Section II): a model set X in R^{M x D}
 * moves onto a scene set Y in R^{N x D} through f(X) = X + Phi W (eq. 9-10),
 * Phi_ij = exp(-|x_i - x_j|^2 / (2 beta^2)) (eq. 11).  One EM iteration:
 *   E-step  posterior p_mn with a uniform outlier term of weight w (eq. 4),
 *           rows renormalised to sum to 1 (the corresponding constraint, eq. 5);
 *   M-step  Fast CPD: W = U (Lam + lambda sigma^2 I)^-1 U^T (Yt - X) (eq. 17),
 *           optionally with the top-K eigenpairs only (eq. 20);
 *           original CPD: W = (Phi + lambda sigma^2 d(P1)^-1)^-1
 *                             (d(P1)^-1 P Y - X)                    (eq. 21);
 *   sigma^2 update (eq. 18).
 *
 * Conventions for every entry point:
 *   - All arrays are row-major and contiguous.  Point arrays are M x D or
 *     N x D.  "device" means a pointer into memory of the current HIP device.
 *   - Floating-point point arrays are double when precision == CPD_PREC_FP64
 *     and float otherwise.
 *   - The library never allocates device memory.  The caller allocates one
 *     workspace of cpd_workspace_size() bytes (256-byte aligned) and keeps it
 *     alive until cpd_destroy().  The handle itself is host memory, as is
 *     the small pinned buffer (two copies of the iteration scalars) that
 *     the first cpd_register on a handle allocates and cpd_destroy frees.
 *     The one exception is a fixed 64 MiB device array per device, part of
 *     the library's code object, that only cpdnet_forward_noalloc uses.
 *   - All device work is enqueued on the stream given to cpd_init.  Calls
 *     that return host scalars synchronise that stream.
 *   - Errors are reported through the return code only; arguments are
 *     validated before any device work is enqueued.  cpd_last_error() holds a
 *     message for the last failing call on a handle.  A handle is not
 *     thread-safe; distinct handles are independent.
 */
#ifndef FASTCPD_H
#define FASTCPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPD_ABI_VERSION 1

typedef enum {
  CPD_OK = 0,
  CPD_NOT_CONVERGED = 1,   /* max_iter reached before |dsigma^2| < tol       */
  CPD_E_ARG = -1,          /* invalid argument (nothing was enqueued)         */
  CPD_E_STATE = -2,        /* call out of order (e.g. step before prepare)    */
  CPD_E_WORKSPACE = -3,    /* workspace missing, misaligned or too small      */
  CPD_E_DEVICE = -4,       /* no usable gfx950 device, or a HIP runtime error */
  CPD_E_NUMERIC = -5,      /* non-finite sigma^2, failed factorisation, ...   */
  CPD_E_UNSUPPORTED = -6   /* valid but not implemented combination           */
} cpd_status;

typedef enum {
  CPD_METHOD_ORIGINAL = 0, /* eq. 21: M x M SPD solve every iteration          */
  CPD_METHOD_FAST = 1,     /* eq. 5 + eq. 17 (eq. 20 when K < M)               */
  CPD_METHOD_ORIGINAL_LOWRANK = 2 /* CPD-L (Section IV-B): eq. 21 with the
                              rank-K Gram of eq. 19, through a K x K system;
                              eigen-prep as for FAST; FP32 / FP64            */
} cpd_method;

typedef enum {
  CPD_PREC_FP64 = 0,       /* everything in double                             */
  CPD_PREC_FP32 = 1,       /* E-step and M-step in float; eig and sigma^2 FP64 */
  CPD_PREC_BF16X = 2       /* E-step squared distances from bf16 products on
                              the matrix cores, fp32 accumulate and exp; the
                              row sums (P1, P Y) are a second bf16 product
                              with each posterior value split into two bf16
                              parts (16 significant bits); its
                              exponent error grows as 1/sigma^2, so sigma^2 is
                              not lowered below 1e-7 D times the data's
                              closed-form sigma^2_0 in this mode              */
} cpd_precision;

typedef enum {
  CPD_EIG_FULL = 0,        /* all eigenpairs of Phi that are not round-off     */
  CPD_EIG_TOPK = 1,        /* the K largest eigenpairs (eq. 19), randomized    */
  CPD_EIG_IMPORT = 2       /* caller supplies U (M x K) and Lam (K)            */
} cpd_eig_mode;

/* Bits of cpd_params.flags (0 = defaults).  By default a single handle sorts
   its point sets along a Hilbert curve at init (the caller sees every
   per-point array in its own order; the permutation is internal) and the
   E-step skips tile pairs (64-point tiles in FP32 / FP64, 16-point tiles in
   BF16X) whose exponentials all underflow to +0, which leaves every result
   bit-identical to the unskipped computation on the same order.  Batch
   members do the same per instance. */
#define CPD_FLAG_NO_SORT 1       /* keep the caller's order (implies NO_CULL)   */
#define CPD_FLAG_NO_CULL 2       /* sort, but evaluate every tile               */

typedef struct {
  int32_t abi_version;     /* must be CPD_ABI_VERSION                          */
  int32_t M, N, D;         /* 1 <= M, N <= 2^26; 1 <= D <= 3                   */
  double beta;             /* kernel width, > 0 (eq. 10-11)                    */
  double lambda;           /* regularisation weight, > 0 (eq. 7, eq. 11)       */
  double w;                /* outlier weight, 0 <= w < 1 (eq. 2)               */
  double sigma2_init;      /* <= 0: sum_mn |y_n - x_m|^2 / (D M N)             */
  int32_t method;          /* cpd_method                                       */
  int32_t precision;       /* cpd_precision                                    */
  int32_t eig_mode;        /* cpd_eig_mode (Fast only)                         */
  int32_t K;               /* TOPK / IMPORT: number of eigenpairs, 1 <= K <= M */
  int32_t oversample;      /* TOPK: extra columns p (default 20 when <= 0)     */
  int32_t power_iters;     /* TOPK: subspace iterations q (default 2 when < 0) */
  uint64_t seed;           /* TOPK: seed of the Gaussian test matrix           */
  double tol;              /* stop when |sigma2_new - sigma2| < tol            */
  int32_t max_iter;        /* iteration cap of cpd_register (> 0)              */
  int32_t flags;           /* CPD_FLAG_* bits, 0 for the defaults              */
} cpd_params;

typedef struct {
  int32_t iter;            /* iterations completed on this handle              */
  int32_t converged;       /* |dsigma2| < tol after this step                  */
  double sigma2;           /* sigma^2 after the step                           */
  double dsigma2;          /* |sigma^2 after - sigma^2 before|                 */
  double loglik;           /* eq. 3 at the state the E-step saw                */
} cpd_step_info;

typedef struct {
  int32_t iters, converged;
  double sigma2;
  double t_c;              /* E-step time (s), as the paper's t_c              */
  double t_eig;            /* eigendecomposition time (s) (t_eig)              */
  double t_iter;           /* M-step time (s) (t_iter)                         */
  double t_o;              /* everything else (s) (t_o)                        */
} cpd_result;

typedef struct cpd_ctx* cpd_handle;

/* Bytes of device workspace needed for these parameters (no device call). */
cpd_status cpd_workspace_size(const cpd_params* p, size_t* bytes);

/* Create a handle.  X (M x D) and Y (N x D) are device arrays of the working
 * precision; they are copied into the workspace, so the caller may reuse them
 * after this call returns.  Sets Xt = X and sigma^2 to sigma2_init (or the
 * standard start, computed on the device).  hip_stream may be NULL (the null
 * stream).  On failure *h is set to NULL. */
cpd_status cpd_init(cpd_handle* h, const cpd_params* p, const void* X,
                    const void* Y, void* workspace, size_t workspace_bytes,
                    void* hip_stream);

/* One-time preparation before the iterations (Section III, eq. 16 and 19).
 *   FAST + FULL   all eigenpairs of Phi (Jacobi on the dense Phi up to 1024
 *                 points; above that, randomized subspace iteration whose width
 *                 grows until the trailing Ritz value is round-off of lam_1,
 *                 at most 2048 columns: when even that basis ends above
 *                 round-off (slow spectral decay: small beta, many points)
 *                 the call returns CPD_NOT_CONVERGED, keeps the top 2016
 *                 pairs (the handle is usable, eq. 19 instead of eq. 16) and
 *                 cpd_last_error names the trailing Ritz value).
 *   FAST + TOPK   the K largest eigenpairs: randomized range finder with
 *                 power_iters subspace iterations and a Rayleigh-Ritz step on
 *                 K + oversample columns.  omega (device, M x (K+oversample)
 *                 doubles) is the Gaussian test matrix; NULL draws it on the
 *                 device from `seed`.
 *   FAST + IMPORT U_import (device, M x K doubles, orthonormal columns) and
 *                 lam_import (device, K doubles), e.g. from cpd_eig_export.
 *   ORIGINAL      builds the M x M Gram matrix Phi.
 * Arguments not used by the mode must be NULL. */
cpd_status cpd_eig_prepare(cpd_handle h, const double* U_import,
                           const double* lam_import, const double* omega);

/* Number of eigenpairs held after cpd_eig_prepare (K, or the adaptive count
 * of FULL mode). */
cpd_status cpd_eig_count(cpd_handle h, int32_t* K_out);

/* Copy the eigenpairs out (device, M x K and K doubles, descending order;
 * eigenvalues are reported as computed, before clamping at 0). */
cpd_status cpd_eig_export(cpd_handle h, double* U_out, double* lam_out);

/* One EM iteration from the current state (E-step at (Xt, sigma^2), M-step
 * with lambda sigma^2, Xt <- X + Phi W, then the sigma^2 update).  With
 * info == NULL the call only enqueues work; otherwise it waits and fills
 * info.  Returns CPD_E_NUMERIC if sigma^2 became non-finite. */
cpd_status cpd_step(cpd_handle h, cpd_step_info* info);

/* Iterate from the current state until |dsigma^2| < tol or max_iter steps.
 * W0 (device, M x D, nullable) first starts a new run from Xt = X + Phi W0
 * (warm start) with sigma^2 = sigma2_init when that is > 0, else the standard
 * start sum_mn |y_n - xt_m|^2 / (D M N) at that Xt; the previous run's
 * sigma^2 is never reused.  X_out (device, M x D) receives Xt; W_out
 * (nullable) receives W.  res (host, nullable) gets counts and the timing
 * split of the paper's runtime protocol (Section IV).  Returns
 * CPD_NOT_CONVERGED when the cap was hit. */
cpd_status cpd_register(cpd_handle h, const void* W0, void* X_out,
                        void* W_out, cpd_result* res);

/* Overwrite the iterate: Xt (device, M x D) and sigma^2 (> 0). */
cpd_status cpd_set_state(cpd_handle h, const void* Xt, double sigma2);

/* Read the iterate: Xt and W (device, M x D, nullable) and sigma^2 (host,
 * nullable).  Synchronises the stream. */
cpd_status cpd_get_state(cpd_handle h, void* Xt_out, void* W_out,
                         double* sigma2_out);

/* E-step alone at the current state (eq. 4-5), results to device arrays of
 * the working precision, each nullable:
 *   logd (N)   natural log of eq. 4's denominator sum_k exp(-|y_n-xt_k|^2/2s2) + c
 *   P1 (M)     row sums of the eq. 4 posterior
 *   Yt (M x D) P'Y with P' the row-normalised posterior (eq. 5)
 *   tbar (M)   sum_n p'_mn |y_n - xt_m|^2
 * The iterate is not changed. */
cpd_status cpd_estep(cpd_handle h, void* logd, void* P1, void* Yt, void* tbar);

/* Kernel timing for benchmarks and tuning: runs `reps` full iterations from
 * the current state (the iterate advances) and reports the average device
 * time in milliseconds of each stage, measured with HIP events on the
 * handle's stream, into out_ms[8]:
 *   [0] E-step pass A, column sums        [1] pass A merge and exact fix-up
 *   [2] E-step pass B, row sums           [3] pass B merge and exact fix-up
 *   [4] M-step                            [5] sigma^2 update
 *   [6] prescale                          [7] whole iteration
 * Synchronises the stream. */
cpd_status cpd_time_kernels(cpd_handle h, int32_t reps, double* out_ms);

/* Two-way registration for a scene with missing points (Section IV-A): the
   scene is first registered onto the model, one-to-one correspondences are
   taken from that result, and the model's transformation is solved from
   them.  These two calls provide the steps on top of cpd_register.

   cpd_matches: for every scene point n of h (caller's row order) the
   caller's row of the nearest transformed model point, -1 when mutual_only
   and n is not also that point's nearest scene point (squared Euclidean
   distance in the working precision, lowest index on ties).  match_out:
   device, N int32.  Synchronises h's stream.

   cpd_solve_matches: the transformation from given one-to-one
   correspondences, eq. 21 with P1_m = 1 and PY_m = y_match[m] for matched
   model points and P1_m = 0 (an infinite penalty: w_m = 0) for the rest,
   evaluated with h's eigenpairs through the K x K system of CPD-L; every
   model point moves (Xt = X + U z).  match: device, M int32, caller's scene
   row or -1 (out-of-range entries count as unmatched).  sigma2 > 0 sets the
   handle's sigma^2 (typically the first registration's final value).
   X_out, W_out: device M x D or NULL; the handle's state becomes the result.
   h: a prepared FAST or CPD-L handle (CPD_E_STATE otherwise); a system that
   is not positive definite returns CPD_E_NUMERIC. */
cpd_status cpd_matches(cpd_handle h, int32_t mutual_only, int32_t* match_out);
cpd_status cpd_solve_matches(cpd_handle h, const int32_t* match, double sigma2, void* X_out,
                             void* W_out);

/* Release the handle (host memory only; the workspace stays the caller's). */
cpd_status cpd_destroy(cpd_handle h);

/* ------------------------------------------------------------------ batch
 * Many independent registrations of uneven sizes advanced together: every
 * stage of an EM iteration (E-step passes, Fast M-step, sigma^2) runs as one
 * launch whose workgroups walk a work list over all instances' tiles, the
 * whole iteration is captured once as a HIP graph and replayed, and an
 * instance that has converged (or hit its max_iter) drops out: its work items
 * return at once.  Per-instance parameters follow cpd_params (Fast method,
 * FP32, D = 3, FULL or TOPK eigen-prep).  Points are packed: instance i owns
 * rows x_off[i] .. x_off[i+1]-1 of X_packed (float, device, sum M_i x 3) and
 * likewise for Y with y_off (host arrays of B + 1 offsets).  One caller
 * workspace of cpd_batch_workspace_size() bytes holds everything: each
 * instance's iteration state, and the eigen-prep scratch (FP64 eigenvectors,
 * bases, Gram partials) once per preparing host thread (at most 32) rather
 * than once per instance, since an instance needs it only while it prepares.
 * Each instance keeps its points in Hilbert order with far-tile culling,
 * as a single handle does (CPD_FLAG_NO_SORT / CPD_FLAG_NO_CULL per instance). */
typedef struct cpd_batch_ctx* cpd_batch;

cpd_status cpd_batch_workspace_size(int32_t B, const cpd_params* p, size_t* bytes);

cpd_status cpd_batch_init(cpd_batch* hb, int32_t B, const cpd_params* p,
                          const float* X_packed, const float* Y_packed,
                          const int64_t* x_off, const int64_t* y_off,
                          void* workspace, size_t workspace_bytes,
                          void* hip_stream);

/* Eigen-prep of every instance (Section III, eq. 16/19; host threads drive up
 * to four streams), then the choice of the E-step plan, then the graph
 * capture.  Leaves every instance at its start state.  The plan is a split
 * length among {1024, 2048, 512, 4096} points and a tile of 1024 or 512
 * points per workgroup (the 8 candidates of cpd_batch_info):
 *   tune == 1        time two batched iterations of every candidate, keep
 *                    the fastest;
 *   tune == 0        candidate 0 (split 1024, tile 1024), untimed;
 *   2 <= tune <= 9   candidate tune - 2, untimed (tests, reproducible runs).
 * Other values: CPD_E_ARG. */
cpd_status cpd_batch_prepare(cpd_batch hb, int32_t tune);

/* Iterate all instances from their start state until each has converged or
 * reached its max_iter.  W0_packed (device, nullable, sum M_i x 3) starts
 * instance i at Xt = X + Phi W0_i with the standard sigma^2 start at that Xt
 * (warm start); NULL starts at Xt = X.  sigma2_start (host, nullable, B
 * values) overrides the start of sigma^2 for every instance whose entry is
 * > 0 (a warm start that knows its expected error); entries <= 0 keep the
 * default.  X_out_packed (device, nullable) receives every Xt;
 * res (host, nullable, B entries) gets per-instance iterations, convergence
 * and sigma^2, with t_eig per instance and t_o = the whole batched run. */
cpd_status cpd_batch_register(cpd_batch hb, const float* W0_packed, const double* sigma2_start,
                              float* X_out_packed, cpd_result* res);

/* What cpd_batch_prepare chose, every output optional (NULL skips it):
 *   chunk    the split length of the E-step partials (points per split);
 *   tile     the E-step tile (points per workgroup, 512 or 1024);
 *   tune_ms  8 doubles: one batched iteration's time (ms) per candidate,
 *            candidate c = split length {1024, 2048, 512, 4096}[c / 2] with
 *            tile {1024, 512}[c % 2]; 0 when not tuned;
 *   K        B int32: each instance's eigenpair count (the M-step's width). */
cpd_status cpd_batch_info(cpd_batch hb, int32_t* chunk, int32_t* tile, double* tune_ms,
                          int32_t* K);

cpd_status cpd_batch_destroy(cpd_batch hb);

/* --------------------------------------------------------- warm start net
 * A point-set network predicting initial GRBF coefficients W0 (M x 3) from a
 * model set X and a scene set Y, for f(X) = X + Phi W (Section III, eq. 9-11):
 * a shared per-point MLP on [p, flag] (4 -> 256 -> 256 -> 256 -> 256, ReLU),
 * max-pooled per set into g_X and g_Y, and a head per model point
 * z = relu(f(x_m) Wa + g_X Wb + g_Y Wc + bh), W0_m = z Wo + bo.  The 256 x 256
 * products run on the matrix cores with fp32 accumulation; `precision`
 * selects how activations, inter-layer gradients and the 256 x 256 weight
 * copies are stored: CPDNET_BF16 (the training and inference mode) or
 * CPDNET_FP32 (the same kernels in fp32, a reference for the bf16 mode).  The
 * parameters are one fp32 array (order W1 b1 W2 b2 W3 b3 W4 b4 Wa Wb Wc bh
 * Wo bo, every W as [fan_in][fan_out]).  Training minimises the displacement
 * error |Phi W0 - V*|^2 / M averaged over a batch (Phi formed on the fly in
 * fp32).  All arrays are device float arrays; a batch packs `batch`
 * instances of M model and N scene points each, row-major x 3.  The
 * workspace (256-byte aligned) is sized by cpdnet_workspace_size for the
 * same (batch, M, N, precision). */
#define CPDNET_BF16 0
#define CPDNET_FP32 1

cpd_status cpdnet_param_count(size_t* count);
cpd_status cpdnet_init(float* params, uint64_t seed, float out_scale, void* hip_stream);
cpd_status cpdnet_workspace_size(int32_t batch, int32_t M, int32_t N, int32_t precision,
                                 size_t* bytes);
cpd_status cpdnet_forward(const float* params, const float* X, const float* Y, int32_t batch,
                          int32_t M, int32_t N, int32_t precision, float* W0_out,
                          void* workspace, size_t workspace_bytes, void* hip_stream);
/* cpdnet_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and result, with the workspace taken from a device array
 * the library owns (64 MiB, one per device, held until the process ends)
 * instead of a caller buffer.  Nothing is allocated by this call.  Returns
 * CPD_E_WORKSPACE when cpdnet_workspace_size(batch, M, N, precision) exceeds
 * 64 MiB (e.g. bf16 with batch 4 at M = N = 2000 fits, batch 8 does not).
 * Every call on one device shares that array: calls that overlap on a device
 * (several streams or host threads) race and must be serialised by the
 * caller. */
cpd_status cpdnet_forward_noalloc(const float* params, const float* X, const float* Y,
                                  int32_t batch, int32_t M, int32_t N, int32_t precision,
                                  float* W0_out, void* hip_stream);
/* Loss (host double, nullable; non-NULL waits for the stream) and its
 * gradient (device, param_count floats). */
cpd_status cpdnet_loss_grad(const float* params, const float* X, const float* Y, const float* V,
                            int32_t batch, int32_t M, int32_t N, int32_t precision, double beta,
                            float* grad_out, double* loss_out, void* workspace,
                            size_t workspace_bytes, void* hip_stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the fp32 master; m, v
 * are param_count floats each; step counts from 1. */
cpd_status cpdnet_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                       float lr, void* hip_stream);
/* Training pairs on the device at any M: model points on the unit sphere
 * (CPDNET_SHAPE_SPHERE, the 500-point recipe) or on a surface without
 * symmetries, r(u) = 1 + six Gaussian bumps of random centre and height
 * N(0, 0.25^2) (CPDNET_SHAPE_BUMPS), plus N(0, jitter^2); W* ~ N(0, coef^2),
 * V* = Phi W* (displacement of every model point), Y = X + V* with a
 * fraction outlier_frac of rows replaced by U[-1.5, 1.5]^3 (N = M).
 * Instance b draws from counter-based stream seed0 + b.  W_scratch holds W*. */
#define CPDNET_SHAPE_SPHERE 0
#define CPDNET_SHAPE_BUMPS 1
cpd_status cpdnet_synth(float* X, float* Y, float* V, float* W_scratch, int32_t batch, int32_t M,
                        int32_t shape, double beta, double coef, double jitter,
                        double outlier_frac, uint64_t seed0, void* hip_stream);

const char* cpd_status_str(cpd_status s);
const char* cpd_last_error(cpd_handle h);   /* h may be NULL: global message */

/* Library build information: ABI version and the offload target. */
int32_t cpd_abi_version(void);
const char* cpd_build_info(void);

#ifdef __cplusplus
}
#endif
#endif /* FASTCPD_H */
