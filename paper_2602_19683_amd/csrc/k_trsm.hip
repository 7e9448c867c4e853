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
#include "k_trsm_dev.h"

namespace gpr {

__global__ __launch_bounds__(256) void k_trsm_f64(const TrsmTask* __restrict__ tasks, int m,
                                                  const int* __restrict__ abort_info)
{
    if (abort_info != nullptr && *abort_info > 0) return;  // the factorisation failed
    __shared__ TrsmLds sh;
    const int strips = m / 32;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lid / strips, s = lid - t * strips;
    trsm_strip(tasks[t], s, m, sh, threadIdx.x);
}

hipError_t launch_trsm_f64(const TrsmTask* d_tasks, int ntask, int m, const int* abort_info,
                           hipStream_t s)
{
    if (ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_trsm_f64, dim3(ntask * (m / 32)), dim3(256), 0, s, d_tasks, m,
                       abort_info);
    return hipGetLastError();
}

}  // namespace gpr
