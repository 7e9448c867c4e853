// k_potrf.hip -- POTRF of a diagonal tile (Fig. 1, task 1) and the inverse
// of the resulting triangular factor, which turns every TRSM and triangular
// vector solve into a product.
//
// POTRF, left-looking over 32-row panels, one workgroup per row panel w of
// the m x m tile (m / 32 workgroups). Workgroup w computes its blocks in
// column order q = 0 .. w:
//     acc = K[w, q] - L[w, 0:32q] L[q, 0:32q]^T      (FP64 MFMA, LDS-staged)
//     L[w, q] = acc Dinv_q^T                          (q < w)
//     L[w, w] = chol(K[w, w] - sum_q L[w, q] L[w, q]^T), Dinv_w = L[w, w]^{-1}
// The diagonal block's sum is accumulated as each L[w, q] is formed, so no
// long product sits between the last handoff and the 32 x 32 factorisation.
// Workgroup q publishes two flags (release / acquire at device scope, so they
// hold across XCDs): its off-diagonal blocks L[q, 0:q] are stored (before its
// diagonal factorisation), and its diagonal block and Dinv_q are stored.
// The long product for block (w, q) needs only the first, so it overlaps the
// factorisation of panel q; only the 32 x 32 product with Dinv_q waits for
// the second. A workgroup only ever waits for lower-numbered workgroups,
// which the hardware dispatches first, so every wait ends; a spin limit
// turns a broken invariant into an error report instead of a hang.
//
// TRTRI: block column c of Tinv = L^{-1} is X_c = Dinv_c and
//     X_r = -Dinv_r sum_{s=c}^{r-1} L[r, s] X_s,   r > c,
// one workgroup per block column, sequential in r; one launch inverts many
// diagonal tiles at once (it is off the critical path: TRSM uses only the
// 32 x 32 block inverses).
#include "gpr_internal.h"
#include "k_accum.h"
#include "k_common.h"
#include "k_potrf_dev.h"
#include "k_trsm_dev.h"

namespace gpr {

__global__ __launch_bounds__(256) void k_potrf_f64(double* __restrict__ A, int lda, int m,
                                                   double* __restrict__ Tinv, int ldt,
                                                   int* __restrict__ info, int64_t col_base,
                                                   unsigned* __restrict__ flags, unsigned epoch,
                                                   int* __restrict__ err,
                                                   const double* __restrict__ syrk, int syrk_f32)
{
    // a pivot already failed in an earlier tile: nothing of this factorisation
    // is used any more. Failures of this launch are recorded as columns
    // > col_base, so every workgroup of the launch takes the same branch.
    if (info != nullptr) {
        const int f = *info;
        if (f > 0 && f <= col_base) return;
    }
    __shared__ PotrfLds sh;
    potrf_panel(A, lda, m, Tinv, ldt, info, col_base, flags, epoch, err, blockIdx.x, sh,
                threadIdx.x, syrk, syrk_f32 != 0);
}

// POTRF of the diagonal tile (J, J) and the TRSM of the tile below it,
// (J + 1, J), in one launch: workgroups 0 .. P-1 are the POTRF row panels
// as above, workgroups P .. 2P-1 the TRSM's 32-row strips. A strip takes
// column block p as soon as row panel p of the factor is final (the panel's
// second flag), so the TRSM runs beside the factorisation instead of after
// it; the strips only wait for lower-numbered workgroups. The TRSM also needs
// the last update of its own tile, done by a launch on another stream: that
// launch is followed by a one-thread kernel that stores `ready_val` to
// *ready (release), and the strips acquire it before they start (ready may be
// null when the update is ordered by the stream itself). With syrk given, the
// POTRF panels first apply the tile's last SYRK update themselves (with FP32
// operands and accumulation if syrk_f32, the form of a mixed FP32 sweep).
__global__ __launch_bounds__(256) void k_potrf_trsm_f64(
    double* __restrict__ A, int lda, int m, double* __restrict__ Tinv, int ldt,
    int* __restrict__ info, int64_t col_base, unsigned* __restrict__ flags, unsigned epoch,
    int* __restrict__ err, const TrsmTask* __restrict__ trsm, const unsigned* __restrict__ ready,
    unsigned ready_val, const double* __restrict__ syrk, int syrk_f32)
{
    if (info != nullptr) {
        const int f = *info;
        if (f > 0 && f <= col_base) return;
    }
    __shared__ union {
        PotrfLds potrf;
        TrsmLds trsm;
    } sh;
    const int P = m / NB;
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < P) {
        potrf_panel(A, lda, m, Tinv, ldt, info, col_base, flags, epoch, err, blockIdx.x, sh.potrf,
                    tid, syrk, syrk_f32 != 0);
        return;
    }
    if (ready != nullptr) {
        if (tid == 0 && !wait_flag(ready, ready_val, err)) flag_error(err);
        __syncthreads();
    }
    const unsigned* diag_done = flags + P;
    trsm_strip(*trsm, (int)blockIdx.x - P, m, sh.trsm, tid, [&](int p) {
        if (tid == 0 && !wait_flag(diag_done + p, epoch, err)) flag_error(err);
        __syncthreads();
    });
}

// Marks the end of the launches before it on its stream (see above).
__global__ void k_signal(unsigned* __restrict__ flag, unsigned v)
{
    __hip_atomic_store(flag, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void k_trtri_f64(TileMat K, double* __restrict__ Tall)
{
    __shared__ double As[2][KC][SP];
    __shared__ double Bs[2][KC][SP];
    __shared__ double Sacc[NB][NB + 1];
    const int m = K.m;
    const int P = m / NB;
    const int J = blockIdx.x / P, c = blockIdx.x % P;
    const double* __restrict__ L = tile_ptr(K, J, J);
    double* __restrict__ Tinv = Tall + (size_t)J * m * m;
    const int lda = m, ldt = m;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int qi = wave >> 1, qj = wave & 1;

    // blocks above the diagonal in this block column are zero
    for (int e = tid; e < c * NB * NB; e += 256) {
        const int r = e / NB, cc = e % NB;
        Tinv[(size_t)r * ldt + c * NB + cc] = 0.0;
    }
    for (int r = c + 1; r < P; ++r) {
        // acc = sum_{s=c}^{r-1} L[r, s] X_s  (X_s = Tinv block (s, c))
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        acc = accum32<false, KC>(L + (size_t)r * NB * lda + c * NB, lda,
                             Tinv + (size_t)c * NB * ldt + c * NB, ldt, NB * (r - c), acc, 1.0,
                             As, Bs, tid);
#pragma unroll
        for (int v = 0; v < 4; ++v) Sacc[16 * qi + drow(lk, v)][16 * qj + lr] = acc[v];
        __syncthreads();
        // X_r = -Dinv_r acc
        const double* dr = Tinv + (size_t)(r * NB + 16 * qi + lr) * ldt + r * NB + lk;
        dbl4 o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < NB; k += 4) o = mfma16(-dr[k], Sacc[k + lk][16 * qj + lr], o);
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Tinv[(size_t)(r * NB + 16 * qi + drow(lk, v)) * ldt + c * NB + 16 * qj + lr] = o[v];
        __syncthreads();
    }
}

hipError_t launch_potrf_f64(double* A, int lda, int m, double* Tinv, int ldt, int* info,
                            int64_t col_base, unsigned* flags, unsigned epoch, int* err,
                            hipStream_t s, const double* syrk, bool syrk_f32)
{
    hipLaunchKernelGGL(k_potrf_f64, dim3(m / NB), dim3(256), 0, s, A, lda, m, Tinv, ldt, info,
                       col_base, flags, epoch, err, syrk, syrk_f32 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_potrf_trsm_f64(double* A, int lda, int m, double* Tinv, int ldt, int* info,
                                 int64_t col_base, unsigned* flags, unsigned epoch, int* err,
                                 const TrsmTask* trsm, const unsigned* ready, unsigned ready_val,
                                 hipStream_t s, const double* syrk, bool syrk_f32)
{
    hipLaunchKernelGGL(k_potrf_trsm_f64, dim3(2 * (m / NB)), dim3(256), 0, s, A, lda, m, Tinv, ldt,
                       info, col_base, flags, epoch, err, trsm, ready, ready_val, syrk,
                       syrk_f32 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_signal(unsigned* flag, unsigned v, hipStream_t s)
{
    hipLaunchKernelGGL(k_signal, dim3(1), dim3(1), 0, s, flag, v);
    return hipGetLastError();
}

hipError_t launch_trtri_f64(const TileMat& K, int M, double* Tinv, hipStream_t s)
{
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_trtri_f64, dim3(M * (K.m / NB)), dim3(256), 0, s, K, Tinv);
    return hipGetLastError();
}

}  // namespace gpr
