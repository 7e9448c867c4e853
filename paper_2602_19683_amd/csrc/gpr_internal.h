// gpr_internal.h -- declarations shared by the libgpr sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "gpr.h"
#include "persist.h"

namespace gpr {

// ---------------------------------------------------------------------------
// Tile addressing
// ---------------------------------------------------------------------------

// A grid of m x m row-major tiles, each contiguous (leading dimension m).
// layout 0: lower tiles of a symmetric / triangular matrix, tile (I, J) with
//           J <= I at index I (I + 1) / 2 + J  (Sec. 4.2: lower tiles only).
// layout 1: full rectangular grid with `ncolt` tiles per tile row, tile (I, J)
//           at index I * ncolt + J.
struct TileMat {
    double* base;
    int m;
    int layout;
    int ncolt;
};

__host__ __device__ inline size_t tile_index(const TileMat& T, int I, int J)
{
    return T.layout == 0 ? (size_t)I * (I + 1) / 2 + J : (size_t)I * T.ncolt + J;
}

__host__ __device__ inline double* tile_ptr(const TileMat& T, int I, int J)
{
    return T.base + tile_index(T, I, J) * (size_t)T.m * T.m;
}

// ---------------------------------------------------------------------------
// Task descriptors consumed by the batched tile kernels
// ---------------------------------------------------------------------------

enum : int { TASK_DIAG = 1 };  // symmetric update: only lower 128-blocks needed

// C -= A * B^T on m x m tiles (GEMM of Fig. 1; SYRK when A == B and
// flags & TASK_DIAG).
struct UpdateTask {
    double* C;
    const double* A;
    const double* B;
    int ldc, lda, ldb, flags;
    // nk consecutive products: C -= sum_{t < nk} A_t B_t^T with A_t = A + t kstride,
    // B_t = B + t kstride (the tiles (I, k), k = k0 .. k0 + nk - 1, of one tile
    // row are kstride = m^2 apart), summed in t order into one accumulator.
    int nk = 1;
    int pad = 0;
    long long kstride = 0;
    // part != null: store the accumulated sum there (leading dimension ldc)
    // instead of subtracting it from C (one part of a split update).
    double* part = nullptr;
};

// C -= part_0 + ... (subtracted one part after the other, in order) over the
// tile, the lower 128-row blocks only for a symmetric task (flags & TASK_DIAG);
// parts are m x m with leading dimension m, `stride` doubles apart.
struct ReduceTask {
    double* C;
    const double* part;
    long long stride;
    int ldc, nparts, flags, pad;
};

// B := B * L_JJ^{-T} in place (TRSM of Fig. 1 read as L_IJ = K_IJ L_JJ^{-T}).
// L: the factored diagonal tile; Dinv: an array whose 32 x 32 diagonal blocks
// hold the inverses of L's 32 x 32 diagonal blocks. B32 (optional): also
// write the result rounded to FP32 there (m x m, leading dimension m).
struct TrsmTask {
    double* B;
    const double* L;
    const double* Dinv;
    float* B32;
    int ldb, ldl, ldd, pad;
};

// Tile product task of the adjoint sweep (k_tgemm.hip):
//   C = beta Cin + sum_t alpha_t op(A_t) op(B_t) + sum_p part[p * part_stride],
// then the epilogue. All tiles m x m; partial tiles have leading dimension m.
enum : int { TG_TRANS_A = 1, TG_TRANS_B = 2, TG_TRI_A = 4, TG_TRI_B = 8 };
// TG_EPI_PHI: keep the lower triangle, halve the diagonal, zero the upper.
// TG_EPI_SYM: write the lower triangle and mirror it into the upper one.
enum : int { TG_EPI_NONE = 0, TG_EPI_PHI = 1, TG_EPI_SYM = 2 };

struct TGemmTerm {
    const double* A;
    const double* B;
    double alpha;
    int lda, ldb, flags, pad;
};

struct TGemmTask {
    double* C;
    const double* Cin;
    const double* part;
    long long part_stride;
    double beta;
    int ldc, ldcin, npart, first_term, nterm, epi;
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the k_*.hip files). All return hipError_t of
// the launch; grid sizes are derived from the arguments.
// ---------------------------------------------------------------------------

// Assemble `ntiles` tiles of T (lower tiles if layout 0, all if layout 1).
// Entry (i, j) of the padded matrix: for i < na and j < nb,
// v exp(-|a_i - b_j|^2 / (2 l)) plus s2 where diag_noise and i == j;
// otherwise (padding) 1 where identity_pad and i == j, else 0.
// hyp (nullable, device, 3 doubles): when given, (l, v, s2) are read from it
// by the kernel instead (hyperparameters kept on the device). copy (nullable):
// a second tile array of T's layout that receives the same values.
hipError_t launch_assemble(const TileMat& T, int tile_rows, const double* A, int64_t na,
                           const double* B, int64_t nb, int D, double l, double v,
                           double s2, bool diag_noise, bool identity_pad,
                           hipStream_t s, const double* hyp = nullptr, double* copy = nullptr);

// Dense row-major n x n (ld) -> lower tiles of T (padding: identity).
hipError_t launch_dense_to_tiled(const double* A, int64_t n, int64_t lda, const TileMat& T,
                                 int tile_rows, hipStream_t s);

// Lower tiles of T -> dense row-major n x n (ld). mirror: upper triangle
// copied from the lower one; else the strict upper triangle is zero.
hipError_t launch_tiled_to_dense(const TileMat& T, int64_t n, double* out, int64_t ldo,
                                 bool mirror, hipStream_t s);

// Tile updates and TRSM strips of a sweep. abort_info (nullable, device):
// the factorisation's failed-pivot record; when it is > 0 at a launch's start
// the launch returns at once (nothing of a failed factorisation is used).
// Pass it only for sweeps that factorise, where it was reset beforehand.
// Block edge (128, 64 or 32) of the update kernels for a launch of ntask m x m
// tasks.
int update_block_size(int ntask, int m);
hipError_t launch_update_f64(const UpdateTask* d_tasks, int ntask, int m, const int* abort_info,
                             hipStream_t s);
// The part sums of split updates (ReduceTask).
hipError_t launch_update_reduce(const ReduceTask* d_tasks, int ntask, int m, const int* abort_info,
                                hipStream_t s);
hipError_t launch_trsm_f64(const TrsmTask* d_tasks, int ntask, int m, const int* abort_info,
                           hipStream_t s);
// POTRF of one diagonal tile, m / 32 cooperating workgroups ordered by
// flags[0 .. 2 m/32) (set to `epoch` as parts of a row panel are done; epoch
// must differ from every value the flags hold). *err is set if a wait hits
// its limit. syrk (nullable): an m x m tile S (ld m); A -= S S^T is applied
// first, by the POTRF's own workgroups (the tile's last SYRK update; FP32
// operands and accumulation if syrk_f32).
hipError_t launch_potrf_f64(double* A, int lda, int m, double* Tinv, int ldt, int* info,
                            int64_t col_base, unsigned* flags, unsigned epoch, int* err,
                            hipStream_t s, const double* syrk = nullptr, bool syrk_f32 = false);
// POTRF of one diagonal tile and the TRSM task *trsm (the tile below it) in
// one launch, the TRSM strips following the POTRF row panels (2 m/32
// workgroups). ready (nullable): the strips first wait until *ready ==
// ready_val (stored by launch_signal after the tile's last update on another
// stream).
hipError_t launch_potrf_trsm_f64(double* A, int lda, int m, double* Tinv, int ldt, int* info,
                                 int64_t col_base, unsigned* flags, unsigned epoch, int* err,
                                 const TrsmTask* trsm, const unsigned* ready, unsigned ready_val,
                                 hipStream_t s, const double* syrk = nullptr, bool syrk_f32 = false);
// *flag = v (release, device scope) once the launches before it on s are done.
hipError_t launch_signal(unsigned* flag, unsigned v, hipStream_t s);
// Inverses of the M factored diagonal tiles (J, J) of the lower-tiled K;
// the inverse of tile J goes to Tinv + J m^2 (leading dimension m), whose
// 32 x 32 diagonal blocks must already hold the block inverses.
hipError_t launch_trtri_f64(const TileMat& K, int M, double* Tinv, hipStream_t s);
// Tile rows per step of the vector solves for tile size m and the precision
// of the factor's updates (4 or 2).
int trsv_group(int m, int prec);
// x = L^{-1} b (trans: L^{-T} b) over the lower tiles of L with the inverses of
// its diagonal tiles (Tinv, M tiles); r: scratch of length M m (b is copied
// there first). W (nullable): the off-diagonal tiles of the inverses of the
// G x G blocks of tiles (G = 4 with m <= 512, or 2; group g = tiles g G ..),
// Inv_ij (i > j, relative indices) at tile g G (G - 1) / 2 + i (i - 1) / 2 + j;
// with it, two launches per group of tile rows, else per tile row.
hipError_t launch_trsv(const TileMat& L, const double* Tinv, const double* W, int G, int M,
                       const double* b, double* r, double* x, bool trans, hipStream_t s);

// out_i = base_i - k(A_i, B) x  (subtract) or out_i = k(A_i, B) x  (base == nullptr),
// where k(A_i, B) x = sum_j k(a_i, b_j) x_j + (noise ? s2 x_i : 0) over j < nb.
// work: device scratch of matvec_chunks(na, nb) * na doubles.
int matvec_chunks(int64_t na, int64_t nb);
hipError_t launch_kernel_matvec(const double* A, int64_t na, const double* B, int64_t nb,
                                int D, double l, double v, double s2, bool noise,
                                const double* x, const double* base, double* out,
                                double* work, hipStream_t s);

// Mixed-precision tile updates (prec GPR_MIXED_FP32 or GPR_MIXED_BF16); m % 64 == 0.
hipError_t launch_update_mixed(const UpdateTask* d_tasks, int ntask, int m, int prec,
                               const int* abort_info, hipStream_t s);

// out[0] = sum x_i^2 (deterministic).
hipError_t launch_sumsq(const double* x, int64_t n, double* out, hipStream_t s);
// out[0] = sum x_i y_i (deterministic).
hipError_t launch_dot(const double* x, const double* y, int64_t n, double* out, hipStream_t s);
// y += x
hipError_t launch_axpy(double* y, const double* x, int64_t n, hipStream_t s);
// Conjugate-gradient updates, scalars in device memory: with w = -K p,
// a = rz / -pw, x += a p, r += a w; and p = z + (rz_new / rz_old) p.
hipError_t launch_cg_xr(double* x, double* r, const double* p, const double* w,
                        const double* rz, const double* pw, int64_t n, hipStream_t s);
hipError_t launch_cg_p(double* p, const double* z, const double* rz_new, const double* rz_old,
                       int64_t n, hipStream_t s);
// out = base - K x (base null: out = -K x) for K stored as M lower tiles
// (diagonal tiles full), rows < n; work: symv_work_doubles(M, m) doubles of
// partial products (m a multiple of 32, at most 1024).
size_t symv_work_doubles(int M, int m);
hipError_t launch_symv_tiled(const TileMat& K, int M, const double* x, const double* base,
                             double* out, int64_t n, double* work, hipStream_t s);

// Adjoint sweep tile products; bm in {32, 64, 128} divides m.
int tgemm_block(int ntask, int m);
hipError_t launch_tgemm_f64(const TGemmTask* d_tasks, int ntask, const TGemmTerm* d_terms, int m,
                            int bm, hipStream_t s);
// NLML seed of the adjoint: W (lower tiles) = -tril(alpha beta^T) + diag(1 / L_ii),
// zero above the diagonal of the diagonal tiles.
hipError_t launch_lbar_init(const TileMat& W, const TileMat& L, int M, const double* alpha,
                            const double* beta, hipStream_t s);
// Per-workgroup partial sums (3 per workgroup) of
//   sum_{i >= j, i, j < n} A_ij (e_ij s_ij, e_ij, delta_ij),  e_ij = exp(-s_ij / (2 l)),
// over the lower tiles of A; returns the number of partial triples written.
int grad_reduce_parts(int M, int m);
hipError_t launch_grad_reduce(const TileMat& A, int M, const double* X, int64_t n, int D,
                              double l, double* parts, hipStream_t s, const double* hyp = nullptr);
// Dense symmetric adjoint from the lower-convention Abar: out_ij = Abar_ii on the
// diagonal, Abar_{max(i,j), min(i,j)} / 2 elsewhere (n x n, row-major).
hipError_t launch_kbar_export(const TileMat& A, int64_t n, double* out, hipStream_t s);
// out_nlml = 1/2 beta^T beta + sum log L_ii + n/2 log(2 pi); out_grad3 (if not
// null) from the partial triples. NaN if info[0] > 0.
hipError_t launch_nlml_finish(const TileMat& L, const double* beta, int64_t n,
                              const double* parts, int nparts, double l, double v,
                              const int* info, double* out_nlml, double* out_grad3,
                              hipStream_t s, const double* hyp = nullptr);

// Adam on z = log theta kept on the device (the hyperparameter fit). theta =
// exp(z) is what the next evaluation reads (as its `hyp` array).
struct AdamState {
    double z[3], m[3], s[3], theta[3];
    double b1t, b2t, prev;
    int t;     // steps taken
    int stop;  // 0 running, 1 stopped (tolerance or step limit), 2 non-finite NLML
};
// state := start at z0 (moments zero, theta = exp(z0)).
hipError_t launch_adam_init(AdamState* st, double z0, double z1, double z2, hipStream_t s);
// One bias-corrected Adam step from fit = (nlml, d/dl, d/dv, d/dsigma^2) at
// theta, unless the state has stopped: trace[t] = nlml, the moments and z
// updated with the gradient in log theta (theta_k d/dtheta_k), theta =
// exp(z); stops once |nlml - previous| <= tol |previous| (tol > 0, from the
// second step on), at max_steps, or on a non-finite NLML (trace not written).
hipError_t launch_adam_step(AdamState* st, const double* fit, double* trace, int max_steps,
                            double lr, double beta1, double beta2, double eps, double tol,
                            hipStream_t s);

// var_i = v - sum_j V^T_ij^2 over the M tiles of test-tile row i / m of V
// (layout 1), i < n_test; and out_i = S_ii for the lower-tiled S, i < n.
hipError_t launch_rowsq_var(const TileMat& V, int M, int64_t n_test, double v, double* var,
                            hipStream_t s);
hipError_t launch_tile_diag(const TileMat& S, int64_t n, double* out, hipStream_t s);
// mean_i = sum_j V^T_ij beta_j over the M tiles of test-tile row i / m of V
// (layout 1), i < n_test; beta: M m entries.
hipError_t launch_rowdot_mean(const TileMat& V, int M, int64_t n_test, const double* beta,
                              double* mean, hipStream_t s);

hipError_t launch_set_int(int* p, int value, hipStream_t s);
hipError_t launch_copy_f64(const double* src, double* dst, int64_t n, int64_t n_pad,
                           hipStream_t s);

// ---------------------------------------------------------------------------
// Schedule of the tiled sweep (host only; schedule.cpp)
// ---------------------------------------------------------------------------

enum TaskKind : int { K_POTRF = 0, K_TRSM = 1, K_SYRK = 2, K_GEMM = 3 };
enum LaunchKind : int { LK_POTRF = 0, LK_TRSM = 1, LK_UPDATE = 2 };
// SWEEP_PREDICT_V / SWEEP_FUSED_V: as SWEEP_PREDICT / SWEEP_FUSED without the
// updates of the test block (only V^T is formed: predictive variances).
enum SweepMode : int { SWEEP_CHOLESKY = 0, SWEEP_PREDICT = 1, SWEEP_FUSED = 2,
                       SWEEP_PREDICT_V = 3, SWEEP_FUSED_V = 4 };

inline bool sweep_factors(int mode) { return mode == SWEEP_CHOLESKY || mode == SWEEP_FUSED ||
                                             mode == SWEEP_FUSED_V; }
inline bool sweep_test_rows(int mode) { return mode != SWEEP_CHOLESKY; }
inline bool sweep_test_block(int mode) { return mode == SWEEP_PREDICT || mode == SWEEP_FUSED; }

struct SchedTask {
    int kind, I, K, J;
    int nk = 1;  // update tasks: products of columns J .. J + nk - 1 (left-looking)
};

struct SchedLaunch {
    int stream;        // 0 critical, 1 panel, 2 bulk
    int wait[3];       // launches on other streams to wait for (-1: none)
    int nwait;
    int kind;          // LaunchKind
    int first, count;  // task range
    int step;          // J
};

struct Schedule {
    std::vector<SchedTask> tasks;
    std::vector<SchedLaunch> launches;
};

// Reverse sweep of the tiled Cholesky (adjoint.cpp). Operands are symbolic:
// matrix id and tile coordinates, resolved to pointers by the executor.
enum AdjMat : int { AM_NONE = -1, AM_L = 0, AM_LBAR = 1, AM_ABAR = 2, AM_TINV = 3, AM_PART = 4,
                    AM_Q = 5, AM_G = 6, AM_X = 7 };
enum AdjLaunchKind : int { AK_TRSM = 0, AK_PART = 1, AK_DIAG_SUM = 2, AK_POTRF = 3, AK_PUSH = 4 };

struct AdjRef {
    int mat, I, J;  // AM_TINV: tile I; AM_PART: partial tile I; AM_Q/G/X: single tiles
};
struct AdjTerm {
    AdjRef A, B;
    int alpha;  // +1 or -1
    int flags;  // TG_*
};
struct AdjTask {
    AdjRef out, cin;  // cin.mat == AM_NONE: beta = 0
    int part0, npart;
    int first_term, nterm;
    int epi;
};
struct AdjLaunch {
    int kind, step, first, count;
    int stream;  // 0: the caller's stream (the chain of each step), 1: a second stream
    int wait;    // launch on the other stream to wait for, or -1
};
struct AdjPlan {
    std::vector<AdjTask> tasks;
    std::vector<AdjTerm> terms;
    std::vector<AdjLaunch> launches;
    int max_part = 0;  // partial tiles needed
};
AdjPlan build_adjoint(int M, int G);

// Tile sweep over M training tile rows and Mhat test tile rows (see gpr.h,
// gpr_schedule_describe).
Schedule build_schedule(int M, int Mhat, int mode);
// The left-looking task order (multi-term update tasks), and the schedule of
// a variant (GPR_RIGHT_LOOKING: build_schedule).
Schedule build_schedule_left(int M, int Mhat, int mode);
Schedule build_schedule_variant(int M, int Mhat, int mode, int variant);

// The tile products that build the off-diagonal tiles of the group inverses
// of the vector solves (solve_plan.cpp), with symbolic operands: TR_L tile
// (a, b) of L, TR_TINV the inverse of diagonal tile a, TR_W / TR_Y slot a of
// the result / scratch tiles. A task computes out = sum over its terms of
// alpha A B; first_term counts from its launch's first term.
enum : int { TR_L = 0, TR_TINV = 1, TR_W = 2, TR_Y = 3 };
struct TinvRef {
    int kind, a, b;
};
struct TinvTaskPlan {
    TinvRef out;
    int first_term, nterm;
};
struct TinvTermPlan {
    TinvRef A, B;
    double alpha;
};
struct TinvLaunchPlan {
    int first_task = 0, ntask = 0, first_term = 0, nterm = 0;
};
struct TinvPlan {
    int G = 1;
    long long nslot = 0;   // W slots (and as many Y slots)
    std::vector<TinvTaskPlan> tasks;
    std::vector<TinvTermPlan> terms;
    std::vector<TinvLaunchPlan> launches;
};
TinvPlan plan_tinv_groups(int M, int G);
// every task's terms lie inside its launch's terms
bool tinv_plan_valid(const TinvPlan& P);

// Persistent executor (persist.cpp, k_persist.hip): geometry, ticket order for
// `workers` resident workgroups, update block size for a tile size, the
// number of workgroups that fit at once, and the launch (which first clears
// the ncnt progress counters and the ticket at d_cnt[ncnt]). prec: GPR_FP64
// or GPR_MIXED_FP32 (precision of the update items).
PGeom persist_geom(int M, int Mhat, int mode, int m, int bm);
std::vector<PItem> build_persist_order(int M, int Mhat, int mode, int m, int bm, int workers);
int persist_block(int m);
int persist_workers(int bm, int prec);
hipError_t launch_persist(const PItem* d_items, int64_t nitems, const PGeom& g, int m, int bm,
                          int prec, int workers, const TileMat& K, double* tinv, const TileMat& V,
                          const TileMat& S, unsigned* d_cnt, int64_t ncnt, unsigned* flags,
                          unsigned epoch0, int* info, int* err, hipStream_t s);

}  // namespace gpr
