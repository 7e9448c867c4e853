// k_trsm.hip -- batched TRSM tasks of Fig. 1, B := B L_JJ^{-T} (the reading
// L_IJ = K_IJ L_JJ^{-T}), by left-looking blocked substitution.
//
// One workgroup owns a strip of 32 rows of one tile, in place. For each
// 32-column block p, left to right:
//     acc = B_p - X[:, 0:32p] L_JJ[32p:32p+32, 0:32p]^T    (FP64 MFMA)
//     X_p = acc Dinv_p^T                                    (Dinv_p = inverse of the
//                                                            32 x 32 diagonal block p
//                                                            of L_JJ, made by POTRF)
// X_p is final when computed and is written over B_p (and, if asked, also as
// an FP32 copy). Only the 32 x 32 diagonal-block inverses are needed, so no
// full inverse of L_JJ sits on the critical path. The strip stays in global
// memory (the workgroup's own rows, cached): the workgroup needs only the
// small LDS staging of the block product, so it can share a compute unit
// with the tile-update workgroups that run beside it on other streams.
#include "gpr_internal.h"
#include "k_accum.h"
#include "k_common.h"

namespace gpr {

namespace {
constexpr int TK = 16;  // k-chunk of the block product
}

__global__ __launch_bounds__(256) void k_trsm_f64(const TrsmTask* __restrict__ tasks, int m)
{
    __shared__ double As[2][TK][36];
    __shared__ double Bs[2][TK][36];
    __shared__ double Sacc[32][33];
    const int strips = m / 32;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lid / strips, s = lid - t * strips;
    const TrsmTask tk = tasks[t];
    double* __restrict__ B = tk.B + (size_t)s * 32 * tk.ldb;
    const int ldb = tk.ldb, ldl = tk.ldl, ldd = tk.ldd;
    float* __restrict__ B32 = tk.B32 ? tk.B32 + (size_t)s * 32 * m : nullptr;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int qi = wave >> 1, qj = wave & 1;
    const int P = m / 32;
    for (int p = 0; p < P; ++p) {
        const int c0 = 32 * p;
        dbl4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            acc[v] = B[(size_t)(16 * qi + drow(lk, v)) * ldb + c0 + 16 * qj + lr];
        // minus the finished blocks X[:, 0:c0] times rows c0.. of L_JJ (transposed)
        acc = accum32<true, TK>(B, ldb, tk.L + (size_t)c0 * ldl, ldl, c0, acc, -1.0, As, Bs);
#pragma unroll
        for (int v = 0; v < 4; ++v) Sacc[16 * qi + drow(lk, v)][16 * qj + lr] = acc[v];
        __syncthreads();
        const double* dq = tk.Dinv + (size_t)(c0 + 16 * qj + lr) * ldd + c0 + lk;
        dbl4 o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 32; k += 4) o = mfma16(Sacc[16 * qi + lr][k + lk], dq[k], o);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * qi + drow(lk, v), col = c0 + 16 * qj + lr;
            B[(size_t)row * ldb + col] = o[v];
            if (B32) B32[(size_t)row * m + col] = (float)o[v];
        }
        __syncthreads();  // X_p stored (read by every wave next), Sacc free
    }
}

hipError_t launch_trsm_f64(const TrsmTask* d_tasks, int ntask, int m, hipStream_t s)
{
    if (ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_trsm_f64, dim3(ntask * (m / 32)), dim3(256), 0, s, d_tasks, m);
    return hipGetLastError();
}

}  // namespace gpr
