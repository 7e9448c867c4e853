// k_update_mixed.hip -- tile updates C -= A B^T with low-precision inputs
// (the mixed-precision form of the GEMM / SYRK tasks of Fig. 1): the FP64
// operand tiles are rounded to FP32 or BF16 as they are staged into LDS,
// multiplied on the matching MFMA with an FP32 accumulator, and the
// accumulator is subtracted from the FP64 tile. POTRF, TRSM and every solve
// stay FP64.
//
// Same blocking as the FP64 kernel: one workgroup per 128 x 128 block of a
// tile with 16 waves of 32 x 32 (64 x 64 and 32 x 32 blocks, for launches of
// few tiles: 4 waves), XCD-aware block order, LDS double buffering. FP32: v_mfma_f32_16x16x4_f32, k-slices of 16, LDS k-major.
// BF16: v_mfma_f32_16x16x32_bf16, k-slices of 32, LDS row-major (each lane
// reads 8 consecutive bf16 of one row). Both FP32-accumulator layouts put
// element v of lane l at row 4 (l / 16) + v, column l % 16. A task may hold
// several consecutive products (left-looking updates), accumulated in FP32
// before the one subtraction from the FP64 tile, or write its sum as an FP64
// part of a split update.
#include "gpr_internal.h"
#include "k_common.h"
#include "k_update_mixed_dev.h"

namespace gpr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));


template <int BM, int WR, int WC>
__global__ __launch_bounds__(WR * WC * 64, WR * WC / 2) void k_update_f32(
    const UpdateTask* __restrict__ tasks, int m, const int* __restrict__ abort_info)
{
    if (abort_info != nullptr && *abort_info > 0) return;  // the factorisation failed
    __shared__ UpdLdsF32<BM> sh;
    const int nb = m / BM;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lid / (nb * nb);
    const int sub = lid - t * nb * nb;
    const int bi = sub / nb, bj = sub - bi * nb;
    const UpdateTask tk = tasks[t];
    if ((tk.flags & TASK_DIAG) && bj > bi) return;
    update_block_f32<BM, WR, WC>(tk, bi, bj, m, sh, threadIdx.x);
}

template <int BM, int WR, int WC>
__global__ __launch_bounds__(WR * WC * 64, WR * WC / 2) void k_update_bf16(
    const UpdateTask* __restrict__ tasks, int m, const int* __restrict__ abort_info)
{
    if (abort_info != nullptr && *abort_info > 0) return;  // the factorisation failed
    constexpr int NT = WR * WC * 64;
    constexpr int KB = 32;
    constexpr int TR = BM / WR / 16, TC = BM / WC / 16;
    constexpr int LD = KB + 8;                      // bf16 per LDS row (padded)
    constexpr int NLD = BM * KB / 2 / NT;           // double2 loads per thread per operand
    __shared__ __bf16 As[2][BM][LD];
    __shared__ __bf16 Bs[2][BM][LD];

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
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave / WC) * (BM / WR), wc = (wave % WC) * (BM / WC);
    const int lr = lane & 15, lk = lane >> 4;

    const int spt = m / KB;
    const long long kstride = tk.kstride;
    double2 ra[NLD], rb[NLD];
    auto gload = [&](int kt) {
        const size_t k0 = (size_t)(kt / spt) * kstride + (size_t)(kt % spt) * KB;
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + NT * q;
            const int r = e / (KB / 2), kk = (e % (KB / 2)) * 2;
            ra[q] = gld2(A + (size_t)r * lda + k0 + kk);
            rb[q] = gld2(B + (size_t)r * ldb + k0 + kk);
        }
    };
    auto swrite = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + NT * q;
            const int r = e / (KB / 2), kk = (e % (KB / 2)) * 2;
            bf16x2 pa, pb;
            pa[0] = (__bf16)(float)ra[q].x;
            pa[1] = (__bf16)(float)ra[q].y;
            pb[0] = (__bf16)(float)rb[q].x;
            pb[1] = (__bf16)(float)rb[q].y;
            *reinterpret_cast<bf16x2*>(&As[buf][r][kk]) = pa;
            *reinterpret_cast<bf16x2*>(&Bs[buf][r][kk]) = pb;
        }
    };
    flt4 acc[TR][TC];
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

    gload(0);
    swrite(0);
    __syncthreads();
    const int nk = spt * tk.nk;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload(kt + 1);
        bf16x8 a[TR], b[TC];
#pragma unroll
        for (int i = 0; i < TR; ++i)
            a[i] = *reinterpret_cast<const bf16x8*>(&As[cur][wr + 16 * i + lr][8 * lk]);
#pragma unroll
        for (int j = 0; j < TC; ++j)
            b[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][wc + 16 * j + lr][8 * lk]);
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
            for (int j = 0; j < TC; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (kt + 1 < nk) swrite(cur ^ 1);
        __syncthreads();
    }
    if (tk.part != nullptr) {
        double* __restrict__ Pp = tk.part + (size_t)bi * BM * ldc + (size_t)bj * BM;
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
            for (int j = 0; j < TC; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = wr + 16 * i + frow(lk, v);
                    const int col = wc + 16 * j + lr;
                    gst(Pp + (size_t)row * ldc + col, (double)acc[i][j][v]);
                }
        return;
    }
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wr + 16 * i + frow(lk, v);
                const int col = wc + 16 * j + lr;
                double* c = C + (size_t)row * ldc + col;
                gst(c, gld(c) - (double)acc[i][j][v]);
            }
}

hipError_t launch_update_mixed(const UpdateTask* d_tasks, int ntask, int m, int prec,
                               const int* abort_info, hipStream_t s)
{
    if (ntask <= 0) return hipSuccess;
    const int bm = update_block_size(ntask, m);
    const dim3 grid(ntask * (m / bm) * (m / bm));
    if (prec == GPR_MIXED_FP32) {
        if (bm == 128) hipLaunchKernelGGL((k_update_f32<128, 4, 4>), grid, dim3(1024), 0, s, d_tasks, m, abort_info);
        else if (bm == 64) hipLaunchKernelGGL((k_update_f32<64, 2, 2>), grid, dim3(256), 0, s, d_tasks, m, abort_info);
        else hipLaunchKernelGGL((k_update_f32<32, 2, 2>), grid, dim3(256), 0, s, d_tasks, m, abort_info);
    } else {
        if (bm == 128) hipLaunchKernelGGL((k_update_bf16<128, 4, 4>), grid, dim3(1024), 0, s, d_tasks, m, abort_info);
        else if (bm == 64) hipLaunchKernelGGL((k_update_bf16<64, 2, 2>), grid, dim3(256), 0, s, d_tasks, m, abort_info);
        else hipLaunchKernelGGL((k_update_bf16<32, 2, 2>), grid, dim3(256), 0, s, d_tasks, m, abort_info);
    }
    return hipGetLastError();
}

}  // namespace gpr
