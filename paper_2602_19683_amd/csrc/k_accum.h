// k_accum.h -- the 32 x 32 block product used by the diagonal-tile kernels
// (POTRF, the tile inverse, TRSM): a 256-thread workgroup accumulates
//     acc += sign * sum_{k < K} A[i][k] B(k, j),   i, j < 32,
// each wave holding one 16 x 16 quadrant (qi, qj) = (wave / 2, wave % 2) in the
// FP64 MFMA 16x16x4 layout. A: 32 rows, row-major (lda). NT: B(k, j) =
// B[j * ldb + k] (32 rows of B); otherwise B(k, j) = B[k * ldb + j]. K is a
// multiple of KC. Chunks of KC columns go through LDS k-major (the 16 lanes
// sharing a k read consecutive words), double-buffered. All 256 threads must
// call it (tid: the thread's index, 0..255); As and Bs are LDS arrays
// [2][KC][32 + 4]. ONE_CHAIN: every product is added to acc in k order
// (one MFMA chain), the order of the tile-update kernels' blocks; otherwise
// two chains (even and odd groups of four k) are added at the end of each
// chunk.
#pragma once

#include "k_common.h"

namespace gpr {

template <bool NT, int KC, bool ONE_CHAIN = false>
__device__ inline dbl4 accum32(const double* __restrict__ A, int lda, const double* __restrict__ B,
                               int ldb, int K, dbl4 acc, double sign, double (*As)[KC][36],
                               double (*Bs)[KC][36], int tid)
{
    static_assert(KC % 16 == 0, "chunk must hold whole double2 loads");
    constexpr int NL = KC / 16;       // double2 loads per thread per operand
    constexpr int CPR = KC / 2;       // double2 per 32-row operand row (KC columns)
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int qi = wave >> 1, qj = wave & 1;
    double2 ra[NL], rb[NL];
    auto gload = [&](int k0) {
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int e = tid + 256 * u;
            const int r = e / CPR, c = (e % CPR) * 2;  // row r (< 32), columns c, c + 1
            ra[u] = gld2(A + (size_t)r * lda + k0 + c);
            if (NT) {
                rb[u] = gld2(B + (size_t)r * ldb + k0 + c);
            } else {
                const int kr = e >> 4, jc = (e & 15) * 2;  // k row (< KC), columns jc, jc + 1
                rb[u] = gld2(B + (size_t)(k0 + kr) * ldb + jc);
            }
        }
    };
    auto swrite = [&](int buf) {
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int e = tid + 256 * u;
            const int r = e / CPR, c = (e % CPR) * 2;
            As[buf][c][r] = sign * ra[u].x;
            As[buf][c + 1][r] = sign * ra[u].y;
            if (NT) {
                Bs[buf][c][r] = rb[u].x;
                Bs[buf][c + 1][r] = rb[u].y;
            } else {
                const int kr = e >> 4, jc = (e & 15) * 2;
                Bs[buf][kr][jc] = rb[u].x;
                Bs[buf][kr][jc + 1] = rb[u].y;
            }
        }
    };
    const int nk = K / KC;
    if (nk == 0) return acc;
    __syncthreads();  // LDS buffers free
    gload(0);
    swrite(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * KC);
        if (ONE_CHAIN) {
#pragma unroll
            for (int kk = 0; kk < KC; kk += 4)
                acc = mfma16(As[cur][kk + lk][16 * qi + lr], Bs[cur][kk + lk][16 * qj + lr], acc);
        } else {
            dbl4 acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < KC; kk += 8) {
                acc = mfma16(As[cur][kk + lk][16 * qi + lr], Bs[cur][kk + lk][16 * qj + lr], acc);
                acc2 = mfma16(As[cur][kk + 4 + lk][16 * qi + lr],
                              Bs[cur][kk + 4 + lk][16 * qj + lr], acc2);
            }
            acc += acc2;
        }
        if (kt + 1 < nk) swrite(cur ^ 1);
        __syncthreads();
    }
    return acc;
}

typedef float flt4a __attribute__((ext_vector_type(4)));

// The 32 x 32 block product of accum32<true, KC, true> (B(k, j) = B[j * ldb + k])
// with both operands rounded to FP32 and FP32-accumulator MFMAs
// (v_mfma_f32_16x16x4_f32), one chain in k order from zero: the arithmetic
// of an FP32 tile-update block. Element v of a lane is row 4 (lane / 16) + v
// of its quadrant (the FP32-accumulator layout).
template <int KC>
__device__ inline flt4a accum32_f32(const double* __restrict__ A, int lda,
                                    const double* __restrict__ B, int ldb, int K,
                                    double (*As)[KC][36], double (*Bs)[KC][36], int tid)
{
    static_assert(KC % 16 == 0, "chunk must hold whole double2 loads");
    constexpr int NL = KC / 16;
    constexpr int CPR = KC / 2;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int qi = wave >> 1, qj = wave & 1;
    double2 ra[NL], rb[NL];
    auto gload = [&](int k0) {
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int e = tid + 256 * u;
            const int r = e / CPR, c = (e % CPR) * 2;
            ra[u] = gld2(A + (size_t)r * lda + k0 + c);
            rb[u] = gld2(B + (size_t)r * ldb + k0 + c);
        }
    };
    auto swrite = [&](int buf) {
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int e = tid + 256 * u;
            const int r = e / CPR, c = (e % CPR) * 2;
            As[buf][c][r] = ra[u].x;
            As[buf][c + 1][r] = ra[u].y;
            Bs[buf][c][r] = rb[u].x;
            Bs[buf][c + 1][r] = rb[u].y;
        }
    };
    flt4a acc = {0.f, 0.f, 0.f, 0.f};
    const int nk = K / KC;
    if (nk == 0) return acc;
    __syncthreads();  // LDS buffers free
    gload(0);
    swrite(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * KC);
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)As[cur][kk + lk][16 * qi + lr],
                                                       (float)Bs[cur][kk + lk][16 * qj + lr], acc,
                                                       0, 0, 0);
        if (kt + 1 < nk) swrite(cur ^ 1);
        __syncthreads();
    }
    return acc;
}

}  // namespace gpr
