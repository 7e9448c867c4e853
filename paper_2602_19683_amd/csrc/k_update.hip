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

namespace gpr {

template <int BM, int WR, int WC>
__global__ __launch_bounds__(WR * WC * 64, WR * WC / 2) void k_update_f64(
    const UpdateTask* __restrict__ tasks, int m)
{
    constexpr int NT = WR * WC * 64;  // threads
    constexpr int KB = 16;
    constexpr int TR = BM / WR / 16;  // MFMA tiles per wave, rows
    constexpr int TC = BM / WC / 16;  // MFMA tiles per wave, columns
    constexpr int LD = BM + 4;        // padded LDS row (k-major slices)
    constexpr int NLD = BM * KB / 2 / NT;  // double2 loads per thread per operand
    static_assert(NLD >= 1 && TR >= 1 && TC >= 1, "block too small");
    __shared__ double As[2][KB][LD];
    __shared__ double Bs[2][KB][LD];

    const int nb = m / BM;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lid / (nb * nb);
    const int sub = lid - t * nb * nb;
    const int bi = sub / nb, bj = sub - bi * nb;
    const UpdateTask tk = tasks[t];
    if ((tk.flags & TASK_DIAG) && bj > bi) return;

    const double* __restrict__ A = tk.A + (size_t)bi * BM * tk.lda;
    const double* __restrict__ B = tk.B + (size_t)bj * BM * tk.ldb;
    double* __restrict__ C = tk.C + (size_t)bi * BM * tk.ldc + (size_t)bj * BM;
    const int lda = tk.lda, ldb = tk.ldb, ldc = tk.ldc;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = (wave / WC) * (BM / WR), wc = (wave % WC) * (BM / WC);
    const int lr = lane & 15, lk = lane >> 4;

    double2 ra[NLD], rb[NLD];
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + NT * q;
            const int r = e / (KB / 2), kk = (e % (KB / 2)) * 2;
            ra[q] = *reinterpret_cast<const double2*>(A + (size_t)r * lda + k0 + kk);
            rb[q] = *reinterpret_cast<const double2*>(B + (size_t)r * ldb + k0 + kk);
        }
    };
    auto swrite = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + NT * q;
            const int r = e / (KB / 2), kk = (e % (KB / 2)) * 2;
            As[buf][kk][r] = ra[q].x;
            As[buf][kk + 1][r] = ra[q].y;
            Bs[buf][kk][r] = rb[q].x;
            Bs[buf][kk + 1][r] = rb[q].y;
        }
    };

    dbl4 acc[TR][TC];
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    gload(0);
    swrite(0);
    __syncthreads();
    const int nk = m / KB;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * KB);
#pragma unroll
        for (int kk = 0; kk < KB; kk += 4) {
            double a[TR], b[TC];
#pragma unroll
            for (int i = 0; i < TR; ++i) a[i] = As[cur][kk + lk][wr + 16 * i + lr];
#pragma unroll
            for (int j = 0; j < TC; ++j) b[j] = Bs[cur][kk + lk][wc + 16 * j + lr];
#pragma unroll
            for (int i = 0; i < TR; ++i)
#pragma unroll
                for (int j = 0; j < TC; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
        }
        if (kt + 1 < nk) swrite(cur ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wr + 16 * i + drow(lk, v);
                const int col = wc + 16 * j + lr;
                C[(size_t)row * ldc + col] -= acc[i][j][v];
            }
}

hipError_t launch_update_f64(const UpdateTask* d_tasks, int ntask, int m, hipStream_t s)
{
    if (ntask <= 0) return hipSuccess;
    if (m % 128 == 0) {
        const int nb = m / 128;
        hipLaunchKernelGGL((k_update_f64<128, 4, 4>), dim3(ntask * nb * nb), dim3(1024), 0, s, d_tasks, m);
    } else if (m % 64 == 0) {
        const int nb = m / 64;
        hipLaunchKernelGGL((k_update_f64<64, 2, 2>), dim3(ntask * nb * nb), dim3(256), 0, s, d_tasks, m);
    } else {
        const int nb = m / 32;
        hipLaunchKernelGGL((k_update_f64<32, 2, 2>), dim3(ntask * nb * nb), dim3(256), 0, s, d_tasks, m);
    }
    return hipGetLastError();
}

}  // namespace gpr
