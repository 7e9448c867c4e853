// k_update.hip -- batched FP64 tile updates C -= A B^T (the GEMM and SYRK
// tasks of Fig. 1, and the V / Sigma updates of the covariance solve).
//
// One launch runs a list of tile tasks; each m x m tile is cut into BM x BM
// blocks, one workgroup per block, and a symmetric (SYRK) task skips the
// blocks strictly above its diagonal. Workgroup ids are remapped so the
// blocks of one task stay on one XCD (shared L2 for A and B).
//
// Block kernel: WR x WC waves, each a (BM/WR) x (BM/WC) sub-block of 16 x 16
// FP64 MFMA tiles. A and B stream through LDS in k-slices of 16,
// double-buffered (global -> registers for slice k+1 while slice k feeds the
// MFMAs). LDS holds the slices k-major, so the 16 lanes that share a k read
// 16 consecutive doubles. The 128 x 128 block uses 16 waves of 32 x 32: with
// two workgroups per compute unit that is eight waves per SIMD, enough to
// hide the LDS and global latencies behind the other waves' MFMAs (measured
// faster than four waves of 64 x 64, which reuse operands more but leave
// two waves per SIMD).
#include "gpr_internal.h"
#include "k_common.h"
#include "k_update_dev.h"

namespace gpr {

template <int BM, int WR, int WC>
__global__ __launch_bounds__(WR * WC * 64, WR * WC / 2) void k_update_f64(
    const UpdateTask* __restrict__ tasks, int m, const int* __restrict__ abort_info)
{
    if (abort_info != nullptr && *abort_info > 0) return;  // the factorisation failed
    __shared__ UpdLds<BM> sh;
    const int nb = m / BM;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lid / (nb * nb);
    const int sub = lid - t * nb * nb;
    const int bi = sub / nb, bj = sub - bi * nb;
    const UpdateTask tk = tasks[t];
    if ((tk.flags & TASK_DIAG) && bj > bi) return;
    update_block<BM, WR, WC>(tk, bi, bj, m, sh, threadIdx.x);
}

// Block size (FP64 and the mixed kernels): the largest of 128, 64, 32 (dividing
// m) that still gives a launch at least UPD_MIN_WG workgroups. Launches of one
// or two tiles (the SYRK and the first GEMM of the next column, on the
// critical chain) thus use small blocks spread over many compute units and
// finish sooner; every block size accumulates each element over k in the same
// order (same bits).
constexpr long UPD_MIN_WG = 128;

int update_block_size(int ntask, int m)
{
    if (m % 128 == 0 && (long)ntask * (m / 128) * (m / 128) >= UPD_MIN_WG) return 128;
    if (m % 64 == 0 && (long)ntask * (m / 64) * (m / 64) >= UPD_MIN_WG) return 64;
    return 32;
}

// Sums of split updates: C -= part_0, then part_1, ... per element. One
// workgroup per 128 x 128 block (256 threads, 64 elements each); for a
// symmetric task only the lower 32 x 32 blocks (m a multiple of 128).
__global__ __launch_bounds__(256) void k_update_reduce(const ReduceTask* __restrict__ tasks, int m,
                                                       const int* __restrict__ abort_info)
{
    if (abort_info != nullptr && *abort_info > 0) return;
    constexpr int BM = 128;
    const int nb = m / BM;
    const int t = blockIdx.x / (nb * nb);
    const int sub = blockIdx.x - t * nb * nb;
    const int bi = sub / nb, bj = sub - bi * nb;
    const ReduceTask tk = tasks[t];
    if ((tk.flags & TASK_DIAG) && bj > bi) return;
    const size_t off = (size_t)bi * BM * m + (size_t)bj * BM;
    double* __restrict__ C = tk.C + (size_t)bi * BM * tk.ldc + (size_t)bj * BM;
    const bool diag = (tk.flags & TASK_DIAG) != 0;
    for (int e = threadIdx.x; e < BM * BM / 2; e += 256) {
        const int r = e / (BM / 2), c = (e % (BM / 2)) * 2;
        // a symmetric task's parts hold its lower 32 x 32 blocks (every update
        // block size computes those)
        if (diag && (bj * BM + c) / 32 > (bi * BM + r) / 32) continue;
        double2 v = gld2(C + (size_t)r * tk.ldc + c);
        for (int p = 0; p < tk.nparts; ++p) {
            const double2 q = gld2(tk.part + p * tk.stride + off + (size_t)r * m + c);
            v.x -= q.x;
            v.y -= q.y;
        }
        gst(C + (size_t)r * tk.ldc + c, v.x);
        gst(C + (size_t)r * tk.ldc + c + 1, v.y);
    }
}

hipError_t launch_update_reduce(const ReduceTask* d_tasks, int ntask, int m, const int* abort_info,
                                hipStream_t s)
{
    if (ntask <= 0) return hipSuccess;
    const int nb = m / 128;
    hipLaunchKernelGGL(k_update_reduce, dim3(ntask * nb * nb), dim3(256), 0, s, d_tasks, m,
                       abort_info);
    return hipGetLastError();
}

hipError_t launch_update_f64(const UpdateTask* d_tasks, int ntask, int m, const int* abort_info,
                             hipStream_t s)
{
    if (ntask <= 0) return hipSuccess;
    const int bm = update_block_size(ntask, m);
    if (bm == 128) {
        const int nb = m / 128;
        hipLaunchKernelGGL((k_update_f64<128, 4, 4>), dim3(ntask * nb * nb), dim3(1024), 0, s, d_tasks, m, abort_info);
    } else if (bm == 64) {
        const int nb = m / 64;
        hipLaunchKernelGGL((k_update_f64<64, 2, 2>), dim3(ntask * nb * nb), dim3(256), 0, s, d_tasks, m, abort_info);
    } else {
        const int nb = m / 32;
        hipLaunchKernelGGL((k_update_f64<32, 2, 2>), dim3(ntask * nb * nb), dim3(256), 0, s, d_tasks, m, abort_info);
    }
    return hipGetLastError();
}

}  // namespace gpr
