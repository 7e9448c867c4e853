// k_update_dev.h -- one block of a tile update C -= A B^T (GEMM / SYRK tasks of
// Fig. 1), shared by the stream kernel and the persistent executor; the
// blocking is described in k_update.hip.
#pragma once

#include "gpr_internal.h"
#include "k_common.h"

namespace gpr {

template <int BM>
struct UpdLds {
    double As[2][16][BM + 4];
    double Bs[2][16][BM + 4];
};

// Block (bi, bj) of the task, WR x WC waves (WR * WC * 64 threads, tid the
// thread's index).
template <int BM, int WR, int WC>
__device__ inline void update_block(const UpdateTask& tk, int bi, int bj, int m, UpdLds<BM>& sh,
                                    int tid)
{
    constexpr int NT = WR * WC * 64;  // threads
    constexpr int KB = 16;
    constexpr int TR = BM / WR / 16;  // MFMA tiles per wave, rows
    constexpr int TC = BM / WC / 16;  // MFMA tiles per wave, columns
    constexpr int LD = BM + 4;        // padded LDS row (k-major slices)
    constexpr int NLD = BM * KB / 2 / NT;  // double2 loads per thread per operand
    static_assert(NLD >= 1 && TR >= 1 && TC >= 1, "block too small");
    double (*As)[KB][LD] = sh.As;
    double (*Bs)[KB][LD] = sh.Bs;

    const double* __restrict__ A = tk.A + (size_t)bi * BM * tk.lda;
    const double* __restrict__ B = tk.B + (size_t)bj * BM * tk.ldb;
    double* __restrict__ C = tk.C + (size_t)bi * BM * tk.ldc + (size_t)bj * BM;
    const int lda = tk.lda, ldb = tk.ldb, ldc = tk.ldc;

    const int lane = tid & 63, wave = tid >> 6;
    const int wr = (wave / WC) * (BM / WR), wc = (wave % WC) * (BM / WC);
    const int lr = lane & 15, lk = lane >> 4;

    // slice kt of the k range: tile kt / spt of the run, columns 16 (kt % spt) ..
    const int spt = m / KB;
    const long long kstride = tk.kstride;
    auto koff = [&](int kt) { return (size_t)(kt / spt) * kstride + (size_t)(kt % spt) * KB; };
    double2 ra[NLD], rb[NLD];
    auto gload = [&](int kt) {
        const size_t k0 = koff(kt);
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
    const int nk = spt * tk.nk;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload(kt + 1);
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

    if (tk.part != nullptr) {
        double* __restrict__ Pp = tk.part + (size_t)bi * BM * ldc + (size_t)bj * BM;
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
            for (int j = 0; j < TC; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = wr + 16 * i + drow(lk, v);
                    const int col = wc + 16 * j + lr;
                    gst(Pp + (size_t)row * ldc + col, acc[i][j][v]);
                }
        return;
    }
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wr + 16 * i + drow(lk, v);
                const int col = wc + 16 * j + lr;
                double* c = C + (size_t)row * ldc + col;
                gst(c, gld(c) - acc[i][j][v]);
            }
}


}  // namespace gpr
