/*
 * gpr.h -- C ABI of libgpr, an MI355X (gfx950) library for exact Gaussian-
 * process regression with the squared-exponential kernel.
 *
 * What it computes (Sec. 4.1 of the paper):
 *   k(a, b) = v * exp(-sum_d (a_d - b_d)^2 / (2 l))            eq. (1)
 *   K = k(X, X) + sigma^2 I        (noise by index, training set only)
 *   mean = K_{X*,X} K^{-1} y                                   eq. (2)
 *   cov  = K_{X*,X*} - K_{X*,X} K^{-1} K_{X,X*}                 eq. (3)
 * through the Cholesky factor K = L L^T, computed with the right-looking
 * tiled algorithm of Sec. 4.2 (Fig. 1: POTRF, TRSM, SYRK and GEMM tile tasks),
 * followed by the triangular solves L beta = y, L^T alpha = beta, and
 * L V = K_{X,X*}, W = V^T V.
 *
 * Readings taken where the paper is silent or garbled:
 *   - eq. (1) divides by 2 l, as printed (l acts as a squared lengthscale);
 *   - the noise term is an index Kronecker delta on the training set only, so
 *     k(X*, X) and k(X*, X*) carry no noise and cov is the latent posterior;
 *   - the hyperparameters are (l, v, sigma^2), sigma^2 a variance;
 *   - the TRSM of Fig. 1 is L_IJ = K_IJ L_JJ^{-T}, the operation that makes
 *     K = L L^T hold for row-major lower tiles;
 *   - everything is row-major and 0-based (Sec. 4.3).
 *
 * Conventions for every call:
 *   - matrices are row-major double arrays; X is n x D, Xs is n_test x D;
 *   - pointers to data are DEVICE pointers unless stated otherwise; the
 *     caller owns them and keeps them alive until the stream reaches the call;
 *   - `stream` is a hipStream_t (NULL = the null stream); all work is
 *     stream-ordered and asynchronous to the host unless stated; calls on one
 *     context are additionally ordered among themselves, whatever stream
 *     they use;
 *   - the library owns gpr_ctx, gpr_tiled and its workspace;
 *   - return value: GPR_OK or a negative error code. Argument errors are
 *     detected on the host before any work is queued. A non-positive-definite
 *     pivot is found on the device: it is reported through `info_dev` and by
 *     gpr_sync (GPR_ENOTPD), never by the call that queued the work.
 *   - sizes: n >= 1 training points; any n is accepted. Internally the
 *     problem is padded to a whole number of tiles (K with an identity block,
 *     the cross covariance with zeros), which leaves every result unchanged.
 *     tile must be a multiple of 32 in [32, 1024].
 */
#ifndef GPR_H
#define GPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPR_ABI_VERSION 10

/* Status codes. */
enum {
    GPR_OK = 0,
    GPR_ENOTPD = 1,   /* a pivot of the Cholesky factorisation was not > 0 */
    GPR_EINVAL = -1,  /* bad argument (null pointer, size, hyperparameter)  */
    GPR_ENOMEM = -2,  /* device allocation failed or exceeded the cap      */
    GPR_EHIP = -3,    /* a HIP runtime call failed                         */
    GPR_ENODEV = -4,  /* no usable GPU                                     */
    GPR_ENOTSUP = -5  /* option not available in this library              */
};

/* Hyperparameters of eq. (1): lengthscale l, vertical variance v and noise
 * variance sigma^2 (Sec. 4.1). All must be > 0, except that sigma^2 may be
 * any finite value (a negative one makes K indefinite, which the Cholesky
 * then reports as GPR_ENOTPD). */
typedef struct {
    double lengthscale;
    double vertical_variance;
    double noise_variance;
} gpr_hyper;

/* Precision of the off-diagonal tile updates (GEMM/SYRK) of the Cholesky and
 * of the covariance solve. POTRF, TRSM, the vector solves and the residual
 * of the iterative refinement are always FP64. Mixed modes keep FP64 tile
 * storage and subtract an FP32 MFMA accumulator into it. */
typedef enum {
    GPR_FP64 = 0,
    GPR_MIXED_FP32 = 1,
    GPR_MIXED_BF16 = 2
} gpr_precision;

/* How the tile task graph is executed (the task graph of Fig. 1, Sec. 4.2,
 * with the covariance rows of Sec. 4.1 appended). GPR_EXEC_STREAMS: batched
 * tile-task launches on three HIP streams with one step of look-ahead.
 * GPR_EXEC_PERSISTENT: one launch per sweep; resident workgroups take work
 * items (POTRF row panels, TRSM strips, update blocks) from a ticket list in
 * a precomputed priority order and wait on per-tile progress counters in
 * device memory. Both give bitwise-identical results. The persistent
 * executor runs the FP64 and FP32-update sweeps; the BF16 sweeps of a context
 * created with it run on the streams. GPR_EXEC_AUTO chooses per sweep: the
 * persistent executor for tiles of at most GPR_AUTO_PERSIST_TILE rows when
 * the swept matrix (training rows, plus the test rows of a prediction sweep)
 * has at most GPR_AUTO_PERSIST_ROWS rows, where its single launch beats the
 * per-step launches of small tiles (measured on MI355X: about 2x at
 * n = n_test = 128, tile 32), and the streams otherwise. */
typedef enum {
    GPR_EXEC_STREAMS = 0,
    GPR_EXEC_PERSISTENT = 1,
    GPR_EXEC_AUTO = 2
} gpr_executor;
#define GPR_AUTO_PERSIST_TILE 64
#define GPR_AUTO_PERSIST_ROWS 4096

/* Order of the tile tasks of the factorisation (Sec. 4.2: the right-looking
 * algorithm of Fig. 1, and its left-looking variant).
 * GPR_RIGHT_LOOKING: after POTRF and the TRSMs of tile column J, every later
 * tile is updated with column J (one rank-m update per step).
 * GPR_LEFT_LOOKING: tile column K receives the products of all earlier
 * columns just before it is factored: its terms 0 .. K-2 in one update task
 * per tile, accumulated in registers and subtracted once (issued while
 * column K-1 is being factored; a long task is split over several workgroups
 * whose parts are added in a fixed order), then its last term; the test
 * block of the covariance (eq. (3)) takes all its terms in one task per tile
 * after the last column. Each tile is then read and written a few times
 * instead of once per step. The two orders give the same factor up to
 * rounding (different summation order); each is deterministic. */
typedef enum {
    GPR_RIGHT_LOOKING = 0,
    GPR_LEFT_LOOKING = 1
} gpr_variant;

typedef struct gpr_ctx gpr_ctx;      /* device, streams, events, workspace   */
typedef struct gpr_tiled gpr_tiled;  /* lower-tiled symmetric / triangular n x n matrix */

/* How alpha was refined against a mixed-precision factor L~ (the paper
 * has no mixed mode; these follow the usual FP64 refinement of a
 * low-precision Cholesky factor). GPR_REFINE_IR: plain refinement
 * r = y - K alpha, alpha += L~^{-T} L~^{-1} r, throughout.
 * GPR_REFINE_PCG: plain refinement contracted too slowly (a step gained
 * less than a factor 4 with ||r|| / ||y|| > 1e-12, as happens when
 * kappa(K) times the unit roundoff of the updates is not small), and the
 * remaining steps were conjugate gradients on K alpha = y preconditioned by
 * L~ L~^T, which converge to the same FP64 alpha. */
enum { GPR_REFINE_IR = 0, GPR_REFINE_PCG = 1 };

/* Host-side refinement statistics, filled when gpr_predict returns in a
 * mixed precision (it synchronises the stream in that case). */
typedef struct {
    int32_t iters;              /* refinement steps taken (both kinds)           */
    double rel_residual;        /* ||y - K alpha||_2 / ||y||_2 after the last one */
    int32_t fallback_precision; /* precision the factor was finally computed in  */
    int32_t method;             /* GPR_REFINE_IR or GPR_REFINE_PCG                */
} gpr_ir_stats;

/* Tiled-matrix states. */
enum { GPR_STATE_EMPTY = 0, GPR_STATE_K = 1, GPR_STATE_L = 2 };

/* ---- context ------------------------------------------------------------ */

/* Creates a context on `device` (HIP ordinal). n_streams: number of streams
 * the executor may use (>= 1; it uses at most 3 -- the caller's stream for
 * the critical path, a panel stream and a bulk-update stream; Sec. 4.3 uses
 * a user-sized pool). With 1, every launch runs on the caller's stream in
 * schedule order (no overlap; useful to time kernels in isolation); with 2
 * the panel work shares the caller's stream.
 * Returns GPR_ENODEV if the device does not exist, GPR_ENOTSUP for an
 * executor this library lacks. On success *out must later go to
 * gpr_ctx_destroy.
 * Device-memory cap: if the environment variable GPR_MAX_DEVICE_BYTES holds a
 * positive integer when the context is created, the device memory held by
 * the context's workspace and by the handles it creates may not exceed that
 * many bytes in total; a call whose allocation would exceed it returns
 * GPR_ENOMEM (as does a failed allocation). Handles keep counting against
 * the cap after the context is destroyed, until they are freed. */
int gpr_ctx_create(gpr_ctx** out, int device, int n_streams, gpr_executor ex);

/* Waits for all work of the context, frees its workspace and the context. */
int gpr_ctx_destroy(gpr_ctx* ctx);

/* Chooses the task order of every later factorisation of the context
 * (gpr_cholesky, gpr_fit_predict, gpr_fit_predict_var, the forward sweep of
 * gpr_nlml_grad and gpr_fit_hyper) and of the covariance solve of
 * gpr_predict. Default GPR_RIGHT_LOOKING. A context made for
 * GPR_EXEC_PERSISTENT runs left-looking sweeps on the streams. Host call;
 * GPR_EINVAL for an unknown variant. */
int gpr_ctx_set_variant(gpr_ctx* ctx, gpr_variant v);

/* ---- the hot path --------------------------------------------------------- */

/* Assembles K = k(X, X) + sigma^2 I (eq. (1)) into lower tiles of size
 * tile x tile (Sec. 4.2: only the lower tiles are stored and computed).
 * X: device, n x D row-major. If *K_inout is NULL a new handle is allocated
 * (library-owned device memory); otherwise the handle is reused and must have
 * been made with the same n and tile. Afterwards the handle holds K. */
int gpr_assemble(gpr_ctx* ctx, const double* X, int64_t n, int32_t D,
                 gpr_hyper h, int32_t tile, gpr_tiled** K_inout, void* stream);

/* Factorises K = L L^T in place with the tiled right-looking algorithm of
 * Sec. 4.2 (Fig. 1). The handle must hold K (GPR_EINVAL otherwise); it holds
 * L afterwards, plus the inverse of every diagonal tile of L and of the
 * blocks of G x G tiles that the solves take in one step (G = 4 for tiles up
 * to 256, and up to 512 with FP32 or BF16 updates, whose refinement runs many
 * solves; else 2; see gpr_solve_plan_describe). prec chooses the precision of
 * the GEMM/SYRK updates.
 * info_dev (optional, device int32): set to 0, or to the 1-based global
 * column of the first pivot that was not > 0 (LAPACK convention); gpr_sync
 * then returns GPR_ENOTPD. After a failed pivot the rest of the
 * factorisation is skipped and the handle's contents are meaningless. */
int gpr_cholesky(gpr_ctx* ctx, gpr_tiled* K, gpr_precision prec,
                 int32_t* info_dev, void* stream);

/* Dense variant for tests: A is n x n row-major (device), only its lower
 * triangle is read; on return its lower triangle holds L and its strict
 * upper triangle is zero. Uses the same tile kernels via a scratch handle. */
int gpr_cholesky_dense(gpr_ctx* ctx, double* A, int64_t n, int32_t tile,
                       gpr_precision prec, int32_t* info_dev, void* stream);

/* Predictive mean (eq. (2)) and, if cov != NULL, the full posterior
 * covariance (eq. (3)) at the n_test rows of Xs.
 * L: handle produced by gpr_cholesky from k(X, X) + sigma^2 I with the same
 * X, n and h (GPR_EINVAL if it does not hold a factor or n differs).
 * y: device, n. mean: device, n_test. cov: device, n_test x n_test
 * row-major, both triangles written (exactly symmetric), or NULL.
 * n_test == 0 is a no-op. In a mixed precision the mean is recovered by FP64
 * iterative refinement (stop at ||r|| / ||y|| <= 1e-14, stagnation, or 50
 * steps; preconditioned conjugate gradients take over when plain
 * refinement contracts too slowly, see GPR_REFINE_PCG), the call
 * synchronises the stream and fills *ir if non-NULL. */
int gpr_predict(gpr_ctx* ctx, gpr_tiled* L, const double* X, const double* y,
                int64_t n, const double* Xs, int64_t n_test, int32_t D,
                gpr_hyper h, double* mean, double* cov, gpr_ir_stats* ir,
                void* stream);

/* The whole path in one call: assembles K = k(X, X) + sigma^2 I into
 * *K_inout (allocated if NULL, reused otherwise, as in gpr_assemble),
 * factorises it and, in the same tile sweep, turns the appended test rows
 * into V^T = K_{X*,X} L^{-T} and the test block into
 * K_{X*,X*} - V^T V (eq. (3)); then the mean (eq. (2)). The results equal
 * those of gpr_assemble + gpr_cholesky + gpr_predict bit for bit; the single
 * sweep gives every step more independent tile updates to overlap with the
 * diagonal-tile chain. Afterwards *K_inout holds the factor L (usable by
 * gpr_predict and gpr_solve). cov may be NULL (mean only: no covariance
 * rows are swept). info_dev as in gpr_cholesky. */
int gpr_fit_predict(gpr_ctx* ctx, const double* X, const double* y, int64_t n,
                    const double* Xs, int64_t n_test, int32_t D, gpr_hyper h,
                    int32_t tile, gpr_precision prec, gpr_tiled** K_inout,
                    double* mean, double* cov, int32_t* info_dev,
                    gpr_ir_stats* ir, void* stream);

/* gpr_predict and gpr_fit_predict with the predictive variances as a third
 * output: var (device, n_test, or NULL) receives diag of the posterior
 * covariance, k(x*_i, x*_i) - ||V_{:,i}||^2 (Sec. 4.1: its diagonal holds the
 * predictive variances). With cov == NULL and var != NULL only V^T is formed:
 * the sweep skips the updates of the test block (the n_test^2 n flops of
 * eq. (3)) and the variances are row sums of squares of V^T. With both,
 * var is the diagonal of cov (bitwise). Other arguments and errors as in
 * gpr_predict / gpr_fit_predict, which are these calls with var == NULL. */
int gpr_predict_var(gpr_ctx* ctx, gpr_tiled* L, const double* X, const double* y,
                    int64_t n, const double* Xs, int64_t n_test, int32_t D,
                    gpr_hyper h, double* mean, double* cov, double* var,
                    gpr_ir_stats* ir, void* stream);
int gpr_fit_predict_var(gpr_ctx* ctx, const double* X, const double* y, int64_t n,
                        const double* Xs, int64_t n_test, int32_t D, gpr_hyper h,
                        int32_t tile, gpr_precision prec, gpr_tiled** K_inout,
                        double* mean, double* cov, double* var, int32_t* info_dev,
                        gpr_ir_stats* ir, void* stream);

/* x = K^{-1} b through the factor: forward substitution L beta = b, then
 * backward substitution L^T x = beta (the solve recipe after eq. (2)).
 * L: handle holding a factor; b, x: device vectors of length n (may alias).
 */
int gpr_solve(gpr_ctx* ctx, gpr_tiled* L, const double* b, double* x, void* stream);

/* gpr_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same launches and the same result bit for bit, with no allocation of any
 * kind in the call. Its work vectors live in a fixed device array of the
 * library (3 GPR_NOALLOC_MAX_N doubles, 3 MiB, one copy per GPU, held until
 * the process ends; its address is taken when a context is created on that
 * GPU). Every call on one GPU shares that array: calls that overlap on one
 * GPU (other streams, other contexts, other threads) race and give wrong
 * results; calls ordered on one stream or by the caller's synchronisation
 * are safe. L, b, x as in gpr_solve; n rounded up to whole tiles must not
 * exceed GPR_NOALLOC_MAX_N (GPR_EINVAL otherwise). */
#define GPR_NOALLOC_MAX_N 131072
int gpr_solve_noalloc(gpr_ctx* ctx, gpr_tiled* L, const double* b, double* x, void* stream);

/* Negative log marginal likelihood
 *   NLML = 1/2 y^T K^{-1} y + 1/2 log det K + n/2 log(2 pi)
 *        = 1/2 beta^T beta + sum_i log L_ii + n/2 log(2 pi),  beta = L^{-1} y,
 * with K = K(X, X) + sigma^2 I of eq. (1) factored by the tiled Cholesky
 * (Sec. 4.2), and its gradient with respect to (l, v, sigma^2). The gradient
 * runs reverse-mode through the computation: the solve adjoint gives the
 * adjoint of the factor, Lbar = -tril(alpha beta^T) + diag(1 / L_ii), and a
 * reverse sweep over the tile tasks of Fig. 1 (the Cholesky adjoint) turns it
 * into Kbar = 1/2 (K^{-1} - alpha alpha^T); then
 *   dNLML/dtheta = sum_ij Kbar_ij dK_ij/dtheta,
 *   dK/dl = v e s / (2 l^2), dK/dv = e, dK/dsigma^2 = I   (e = exp(-s / (2 l))).
 * X: device n x D row-major; y: device n. tile: as gpr_assemble.
 * prec: GPR_FP64 (the mixed precisions return GPR_ENOTSUP: the log
 * determinant is taken from the FP64 factor).
 * out_nlml: device, 1 double. out_grad3: device, 3 doubles in the order
 * (l, v, sigma^2), or NULL. out_Kbar: device n x n row-major, receives the
 * symmetric Kbar (gradient with respect to K for any kernel), or NULL. With
 * both NULL only the NLML is computed (no reverse sweep).
 * Asynchronous on `stream`. A failed pivot writes NaN to every output and is
 * reported by gpr_sync (GPR_ENOTPD). Workspace (two lower-tiled n x n arrays
 * plus a few tiles) is kept in the context for the next call. */
int gpr_nlml_grad(gpr_ctx* ctx, const double* X, const double* y, int64_t n,
                  int32_t D, gpr_hyper h, int32_t tile, gpr_precision prec,
                  double* out_nlml, double* out_grad3, double* out_Kbar,
                  void* stream);

/* Hyperparameter fit: Adam on z = log theta (theta = (lengthscale, vertical
 * variance, noise variance); the log keeps theta > 0) minimising the NLML of
 * gpr_nlml_grad, from theta0. Each step evaluates the NLML and its gradient
 * at theta = exp(z) on the GPU (FP64), then takes the bias-corrected Adam
 * step with (lr, beta1, beta2, eps). The paper fixes the hyperparameters
 * (Sec. 3); this is the usual maximum-likelihood fit of the same model.
 * The loop is device-resident: z, the moments and theta stay in device
 * memory, the kernels of each evaluation read theta from there, and a
 * one-thread kernel takes the Adam step, so the host does not wait between
 * steps; it reads the stop flag every 4 steps (evaluations issued after the
 * stop leave the result unchanged).
 * Stops after max_steps, or once the NLML changed by at most tol relative to
 * the previous evaluation (tol = 0: never). theta0, theta_out (3 doubles),
 * nlml_trace (max_steps doubles, the NLML before each step; may be NULL) and
 * steps_done (may be NULL) are HOST pointers; X and y are device arrays as in
 * gpr_nlml_grad. Returns after synchronising the stream. Errors as in
 * gpr_nlml_grad; GPR_ENOTPD if K(theta) stopped being positive definite
 * along the way (theta_out is then not written). */
int gpr_fit_hyper(gpr_ctx* ctx, const double* X, const double* y, int64_t n,
                  int32_t D, int32_t tile, const double* theta0, int32_t max_steps,
                  double lr, double beta1, double beta2, double eps, double tol,
                  double* theta_out, double* nlml_trace, int32_t* steps_done,
                  void* stream);

/* ---- handles and utilities ----------------------------------------------- */

/* Shape and state of a handle (host call, no device work); any out pointer
 * may be NULL. */
int gpr_tiled_info(const gpr_tiled* T, int64_t* n, int32_t* tile,
                   int32_t* state);

/* Copies the handle into a dense n x n row-major device array. For a factor
 * (state L) the strict upper triangle is written as 0; for K both triangles
 * are written (mirrored from the stored lower tiles). */
int gpr_tiled_to_dense(gpr_ctx* ctx, const gpr_tiled* T, double* out,
                       void* stream);

/* Frees a handle (waits for the device to finish with it first). */
int gpr_tiled_free(gpr_tiled* T);

/* Blocks until `stream` has finished the context's queued work, then
 * returns GPR_ENOTPD if any factorisation queued since the previous gpr_sync
 * hit a non-positive pivot (its column in *column if non-NULL, else 0),
 * GPR_OK otherwise. GPR_EHIP: a HIP call failed, or a device-side wait
 * between the workgroups of a factorisation (POTRF, persistent sweep) hit its
 * spin limit; the results of every call queued since the previous gpr_sync
 * are then invalid. The record is cleared when it is reported, so the
 * context stays usable and later calls are unaffected. */
int gpr_sync(gpr_ctx* ctx, void* stream, int64_t* column);

/* ---- instrumentation ------------------------------------------------------
 * Per-kernel timers (the role APEX plays in Sec. 3.1): while enabled, every
 * launch the context issues is bracketed by HIP timing events on the stream
 * it runs on. Kinds: 0 POTRF, 1 inverse of the diagonal tiles, 2 TRSM,
 * 3 tile update (GEMM / SYRK), 4 assembly, 5 triangular vector solve,
 * 6 kernel matvec (mean / residual), 7 export to dense, 8 adjoint tile
 * products of the reverse sweep, 9 adjoint seed and gradient reduction,
 * 10 persistent sweep (one launch per sweep; flops of all its tile tasks). */
int gpr_profile_enable(gpr_ctx* ctx, int on);

/* Totals for one kind over the launches recorded since the last reset:
 * number of launches, summed device time in ms, and summed algorithmic
 * flops (GEMM tile 2 m^3, SYRK / TRSM tile m^3, POTRF and inverse m^3 / 3 each,
 * triangular vector solve 2 m^2 per tile read, kernel matvec 2 per entry, adjoint tile product 2 m^3
 * per term) and bytes (assembly and export: bytes written; adjoint seed and
 * reduction: bytes of the lower tiles). Blocks until the recorded work is done. reset != 0 clears
 * all kinds after reading. Any out pointer may be NULL. */
int gpr_profile_read(gpr_ctx* ctx, int kind, int64_t* launches, double* total_ms,
                     double* flops, double* bytes, int reset);

/* Static description of a status code. */
const char* gpr_strerror(int status);

/* ---- schedule introspection (host only, no device needed) -----------------
 * The executor turns the tile task graph into a list of batched launches on
 * two streams. This call returns that list for M training tile rows and
 * Mhat test tile rows without running anything, so the schedule can be
 * checked on a machine without a GPU.
 * mode: 0 = Cholesky only, 1 = covariance solve with a given factor
 * (rows M..M+Mhat-1 only), 2 = both in one sweep, 3 and 4 = modes 1 and 2
 * without the updates of the test block (only V^T: predictive variances).
 * tasks: host array of 5 int32 per task: kind (0 POTRF, 1 TRSM, 2 SYRK,
 * 3 GEMM), I, K, J, launch index. Tile (I, K) is the one written; for POTRF
 * I = K = J, for TRSM K = J. Rows I >= M are test rows.
 * launches: host array of 5 int32 per launch: stream (0 critical, 1 panel,
 * 2 bulk), the indices of up to three launches on other streams that must
 * finish before it starts (-1 where unused), and the launch kind (0 POTRF,
 * 1 TRSM, 2 tile updates). Launches on one stream run in list order.
 * Capacities are in records; counts are always written. Returns
 * GPR_EINVAL if a capacity is too small (counts still written). */
int gpr_schedule_describe(int32_t M, int32_t Mhat, int32_t mode,
                          int32_t* tasks, int64_t task_cap, int64_t* n_tasks,
                          int32_t* launches, int64_t launch_cap,
                          int64_t* n_launches);

/* gpr_schedule_describe for either task order. tasks: 6 int32 per task:
 * kind, I, K, J, nk, launch index; an update task (kind 2 or 3) of tile
 * (I, K) holds the nk products of columns J .. J + nk - 1 (nk = 1 throughout
 * for GPR_RIGHT_LOOKING, whose list equals gpr_schedule_describe's). */
int gpr_schedule_describe_variant(int32_t M, int32_t Mhat, int32_t mode, int32_t variant,
                                  int32_t* tasks, int64_t task_cap, int64_t* n_tasks,
                                  int32_t* launches, int64_t launch_cap,
                                  int64_t* n_launches);

/* The reverse sweep of gpr_nlml_grad as a list of batched tile-product
 * launches, for M tile rows and a split of the long row sums into chunks of
 * G terms, without running anything (host only).
 * Operands are symbolic (matrix, I, J): matrix 0 L (factor tile (I, J)),
 * 1 Lbar, 2 Abar (tile (I, J) of the lower-tiled adjoint arrays), 3 inverse
 * of diagonal tile I, 4 partial tile I, 5 / 6 / 7 single scratch tiles Q, G, X;
 * -1 none. Each task computes
 *   out = [cin] + sum_terms alpha op(A) op(B) + sum of partial tiles
 *         part0 .. part0 + npart - 1,
 * then its epilogue (0 none, 1 lower triangle with the diagonal halved,
 * 2 mirror the lower triangle into the upper one).
 * tasks: 12 int32 per task: out (3), cin (3), part0, npart, first_term,
 * nterm, epilogue, 0. terms: 8 int32 per term: A (3), B (3), alpha (+1 or -1),
 * flags (1 A transposed, 2 B transposed, 4 A lower-triangular, 8 B
 * lower-triangular). launches: 6 int32 per launch: kind (0 TRSM adjoint,
 * 1 partial sums, 2 diagonal sum, 3 POTRF adjoint, 4 sums of the partial
 * tiles into the column's Lbar tiles), step, first task, task count, stream
 * (0 the caller's, 1 a second stream), and the index of a launch on the
 * other stream that must finish first (-1 if none). Launches on one stream
 * run in list order, tasks of one launch in parallel. The sweep is
 * left-looking: step J collects into column J everything the later steps
 * contribute to it (M - J tile products per tile), then runs its TRSM and
 * POTRF adjoints; the contributions that do not involve column J + 1 run on
 * the second stream during step J + 1. Capacities in records; counts always
 * written; GPR_EINVAL if one is too small. */
int gpr_adjoint_describe(int32_t M, int32_t G, int32_t* tasks, int64_t task_cap,
                         int64_t* n_tasks, int32_t* terms, int64_t term_cap,
                         int64_t* n_terms, int32_t* launches, int64_t launch_cap,
                         int64_t* n_launches);

/* The tile products that build the group inverses of the vector solves
 * (Sec. 4.1: beta = L^{-1} y and alpha = L^{-T} beta by block substitution,
 * G tile rows per step) for M tile rows of size `tile`, without running
 * anything (host only), as for an FP64 factor. *group receives G (4 for
 * tiles up to 256, else 2). The plan depends on M and G only: a factor with
 * FP32 or BF16 updates and a tile above 256 and up to 512 (G = 4) has the plan
 * returned for the same M and tile 256.
 * Group g holds tiles gG .. gG + G - 1; the off-diagonal tile (i, j), i > j,
 * of the inverse of its block goes to W slot g G (G - 1) / 2 + i (i - 1) / 2
 * + j. Operands are symbolic (kind, a, b): kind 0 tile (a, b) of L, 1 the
 * inverse of diagonal tile a, 2 W slot a, 3 scratch slot a. Each task
 * computes out = sum over its terms of alpha A B, the terms first_term ..
 * first_term + nterm - 1 counted from the first term of its launch; the
 * launches run in order. tasks: 6 int32 per task: launch, out (3),
 * first_term, nterm. terms: 7 int32 per term: A (3), B (3), alpha (+1 or -1).
 * Either array may be NULL; capacities in records; counts always written;
 * GPR_EINVAL if a capacity is too small or M < 1 or the tile is invalid. */
int gpr_solve_plan_describe(int32_t M, int32_t tile, int32_t* group, int32_t* tasks,
                            int64_t task_cap, int64_t* n_tasks, int32_t* terms,
                            int64_t term_cap, int64_t* n_terms);

/* The ticket order of the persistent executor for one sweep shape (host
 * only): M, Mhat, mode as for gpr_schedule_describe, tile m, update block
 * size `block` (divides m), and `workers` resident workgroups assumed by the
 * planner. items: 5 int32 per ticket (kind 0 POTRF row panel, 1 TRSM strip,
 * 2 update block; sub-index; I, K, J as in gpr_schedule_describe). waits:
 * 8 int64 per ticket: the number of waits (0..3), then (counter, value) x 3
 * -- the item starts once counter >= value (-1, 0 where unused) -- and the
 * counter the item increments when done. Counter (I, K) = I (I + 1) / 2 + K
 * over the tile rows of the extended matrix. Either array may be NULL;
 * cap in tickets; *n_items always written; GPR_EINVAL if cap is too small. */
int gpr_persist_describe(int32_t M, int32_t Mhat, int32_t mode, int32_t tile, int32_t block,
                         int32_t workers, int32_t* items, int64_t* waits, int64_t cap,
                         int64_t* n_items);

/* ABI version of the loaded library (GPR_ABI_VERSION it was built with). */
int gpr_abi_version(void);

/* First 16 hex digits of the SHA-256 of the sources the library was built
 * from (static string owned by the library), so that a loader can refuse a
 * binary that does not match its source tree. */
const char* gpr_source_hash(void);

#ifdef __cplusplus
}
#endif

#endif /* GPR_H */
