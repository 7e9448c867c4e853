// k_potrf.hip -- POTRF of a diagonal tile (Fig. 1, task 1) and the inverse
// of the resulting triangular factor, which turns every TRSM and triangular
// vector solve into a product.
//
// POTRF: one workgroup (8 waves) per m x m tile, blocked left-looking over
// 32-column panels. For panel p (columns c0 = 32 p .. c0 + 31) every wave
// takes 16-row blocks of the rows below c0 and accumulates
//     acc = K[rows, panel] - L[rows, 0:c0] L[panel, 0:c0]^T
// with FP64 MFMA; the 32 x 32 diagonal block is then factored by one wave in
// registers (unblocked right-looking Cholesky), its inverse Dinv_p is formed
// by column substitution, and the rows below become acc Dinv_p^T. Each panel
// is written once, so the tile makes one pass through L2 per panel.
//
// TRTRI: block column c of Tinv = L^{-1} is X_c = Dinv_c and
//     X_r = -Dinv_r sum_{s=c}^{r-1} L[r, s] X_s,   r > c,
// one workgroup per block column, sequential in r.
#include "gpr_internal.h"
#include "k_common.h"

namespace gpr {

namespace {
constexpr int NB = 32;      // panel width
constexpr int NW = 8;       // waves per POTRF workgroup
}  // namespace

// Unblocked Cholesky of the 32 x 32 block in S (lower triangle read), by one
// wave; lane i < 32 owns row i. On return S holds L (zeros above the
// diagonal) and Si holds L^{-1} (zeros above). Returns the first failing
// local column or -1.
__device__ static int factor_diag32(double (*S)[NB + 1], double (*Si)[NB + 1], int lane)
{
    const int i = lane & 31;
    double a[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) a[k] = S[i][k];
    int bad = -1;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const double d = lane_bcast(a[j], j);
        if (!(d > 0.0) && bad < 0) bad = j;
        const double ljj = sqrt(d);
        const double lij = (i == j) ? ljj : a[j] / ljj;
        a[j] = (i >= j) ? lij : 0.0;
#pragma unroll
        for (int k = j + 1; k < NB; ++k) {
            const double lkj = lane_bcast(a[j], k);
            if (i >= k) a[k] -= a[j] * lkj;
        }
    }
    wave_lds_sync();
    if (lane < 32) {
#pragma unroll
        for (int k = 0; k < NB; ++k) S[i][k] = (k <= i) ? a[k] : 0.0;
    }
    wave_lds_sync();
    // column c = lane of L^{-1}: forward substitution of L x = e_c
    double x[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        double s = (r == i) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < r; ++k) s -= S[r][k] * x[k];
        x[r] = s / S[r][r];
    }
    if (lane < 32) {
#pragma unroll
        for (int r = 0; r < NB; ++r) Si[r][i] = x[r];
    }
    return bad;
}

// MAXQ: 16-row blocks per wave, m <= 16 * NW * MAXQ.
template <int MAXQ>
__global__ __launch_bounds__(NW * 64, 1) void k_potrf_f64(double* __restrict__ A, int lda, int m,
                                                          double* __restrict__ Tinv, int ldt,
                                                          int* __restrict__ info, int64_t col_base)
{
    __shared__ double Sd[NB][NB + 1];
    __shared__ double Si[NB][NB + 1];
    __shared__ double Sw[NW][16][NB + 1];
    __shared__ int s_bad;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    if (tid == 0) s_bad = -1;

    const int P = m / NB;
    for (int p = 0; p < P; ++p) {
        const int c0 = p * NB;
        const int nrb = (m - c0) / 16;

        // 1. left-looking accumulation of the panel
        dbl4 acc[MAXQ][2];
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int rb = wave + NW * q;
            if (rb < nrb) {
                const int r0 = c0 + 16 * rb;
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        acc[q][t][v] = A[(size_t)(r0 + drow(lk, v)) * lda + c0 + 16 * t + lr];
                const double* arow = A + (size_t)(r0 + lr) * lda + lk;
                const double* b0 = A + (size_t)(c0 + lr) * lda + lk;
                const double* b1 = A + (size_t)(c0 + 16 + lr) * lda + lk;
                for (int k = 0; k < c0; k += 4) {
                    const double a = -arow[k];
                    acc[q][0] = mfma16(a, b0[k], acc[q][0]);
                    acc[q][1] = mfma16(a, b1[k], acc[q][1]);
                }
            }
        }
        // 2. diagonal block (row blocks 0 and 1 belong to waves 0 and 1, q = 0)
        if (wave < 2) {
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) Sd[16 * wave + drow(lk, v)][16 * t + lr] = acc[0][t][v];
        }
        __syncthreads();
        if (wave == 0) {
            const int bad = factor_diag32(Sd, Si, lane);
            if (lane == 0 && bad >= 0 && s_bad < 0) s_bad = c0 + bad;
        }
        __syncthreads();
        for (int e = tid; e < NB * NB; e += NW * 64) {
            const int r = e / NB, c = e % NB;
            A[(size_t)(c0 + r) * lda + c0 + c] = Sd[r][c];
            Tinv[(size_t)(c0 + r) * ldt + c0 + c] = Si[r][c];
        }
        // 3. rows below the diagonal block: L = acc Dinv^T
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int rb = wave + NW * q;
            if (rb >= 2 && rb < nrb) {
                const int r0 = c0 + 16 * rb;
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) Sw[wave][drow(lk, v)][16 * t + lr] = acc[q][t][v];
                wave_lds_sync();
                dbl4 o0 = {0.0, 0.0, 0.0, 0.0}, o1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k = 0; k < NB; k += 4) {
                    const double a = Sw[wave][lr][k + lk];
                    o0 = mfma16(a, Si[lr][k + lk], o0);
                    o1 = mfma16(a, Si[16 + lr][k + lk], o1);
                }
                wave_lds_sync();
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    A[(size_t)(r0 + drow(lk, v)) * lda + c0 + lr] = o0[v];
                    A[(size_t)(r0 + drow(lk, v)) * lda + c0 + 16 + lr] = o1[v];
                }
            }
        }
        __syncthreads();
    }
    // zero the strict upper triangle of the tile (outside the diagonal blocks,
    // which were written with zeros above their diagonal)
    for (int r = tid / 64; r < m; r += NW) {
        const int cstart = (r / NB + 1) * NB;
        for (int c = cstart + lane; c < m; c += 64) A[(size_t)r * lda + c] = 0.0;
    }
    if (tid == 0 && s_bad >= 0 && info != nullptr) {
        if (*info == 0) *info = (int)(col_base + s_bad + 1);
    }
}

__global__ __launch_bounds__(256) void k_trtri_f64(const double* __restrict__ L, int lda,
                                                   double* __restrict__ Tinv, int ldt, int m)
{
    __shared__ double Sacc[NB][NB + 1];
    const int c = blockIdx.x;
    const int P = m / NB;
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
        dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
        const double* arow = L + (size_t)(r * NB + 16 * qi + lr) * lda + lk;
        const double* bcol = Tinv + (size_t)lk * ldt + c * NB + 16 * qj + lr;
        for (int k = c * NB; k < r * NB; k += 8) {
            acc0 = mfma16(arow[k], bcol[(size_t)k * ldt], acc0);
            acc1 = mfma16(arow[k + 4], bcol[(size_t)(k + 4) * ldt], acc1);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Sacc[16 * qi + drow(lk, v)][16 * qj + lr] = acc0[v] + acc1[v];
        __syncthreads();
        dbl4 o = {0.0, 0.0, 0.0, 0.0};
        const double* dinv_row = Tinv + (size_t)(r * NB + 16 * qi + lr) * ldt + r * NB + lk;
#pragma unroll
        for (int k = 0; k < NB; k += 4) o = mfma16(-dinv_row[k], Sacc[k + lk][16 * qj + lr], o);
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Tinv[(size_t)(r * NB + 16 * qi + drow(lk, v)) * ldt + c * NB + 16 * qj + lr] = o[v];
        __syncthreads();
    }
}

hipError_t launch_potrf_f64(double* A, int lda, int m, double* Tinv, int ldt, int* info,
                            int64_t col_base, hipStream_t s)
{
    if (m <= 16 * NW * 4)
        hipLaunchKernelGGL(k_potrf_f64<4>, dim3(1), dim3(NW * 64), 0, s, A, lda, m, Tinv, ldt,
                           info, col_base);
    else
        hipLaunchKernelGGL(k_potrf_f64<8>, dim3(1), dim3(NW * 64), 0, s, A, lda, m, Tinv, ldt,
                           info, col_base);
    return hipGetLastError();
}

hipError_t launch_trtri_f64(const double* L, int lda, double* Tinv, int ldt, int m, hipStream_t s)
{
    hipLaunchKernelGGL(k_trtri_f64, dim3(m / NB), dim3(256), 0, s, L, lda, Tinv, ldt, m);
    return hipGetLastError();
}

}  // namespace gpr
