// k_assemble.hip -- covariance assembly (eq. (1), Sec. 4.1) straight into
// tiles, and conversions between tiles and dense row-major arrays.
//
// Assembly: only the tiles that are stored are computed (lower tiles of K and
// of K_{X*,X*}, Sec. 4.2). A workgroup fills 32 x 32 sub-blocks, grid-strided
// over all sub-blocks of the launch; its 32 row points and 32 column points
// are staged in LDS (column points transposed, so consecutive lanes read
// consecutive words), and every row of a sub-block is written as 256
// contiguous bytes.
#include "gpr_internal.h"
#include "k_common.h"

namespace gpr {

namespace {
constexpr int SB = 32;        // sub-block side
constexpr int MAXD = 64;      // feature dimensions staged in LDS
}

__device__ inline void lower_tile_coords(int64_t t, int& I, int& J)
{
    // t = I (I + 1) / 2 + J, 0 <= J <= I
    int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)(i + 1) * (i + 2) / 2 <= t) ++i;
    while ((int64_t)i * (i + 1) / 2 > t) --i;
    I = i;
    J = (int)(t - (int64_t)i * (i + 1) / 2);
}

// DT > 0: the feature count D equals DT (loops unrolled, the column point's
// features held in registers across the thread's four rows); DT = 0: any D.
// Both accumulate d2 = fma(q_d, q_d, d2) in feature order, written out so
// that the compiler cannot fuse a different product of an unrolled pair
// (same bits for every D).
template <int DT>
__global__ __launch_bounds__(256) void k_assemble(TileMat T, int tile_rows, int64_t ntiles,
                                                  const double* __restrict__ A, int64_t na,
                                                  const double* __restrict__ B, int64_t nb, int D,
                                                  double l, double v, double s2, int diag_noise,
                                                  int identity_pad, const double* __restrict__ hyp,
                                                  double* __restrict__ copy)
{
    if (hyp) {  // hyperparameters held on the device (l, v, sigma^2)
        l = hyp[0];
        v = hyp[1];
        s2 = hyp[2];
    }
    __shared__ double Sa[SB][MAXD + 1];
    __shared__ double Sb[MAXD][SB + 1];
    const int m = T.m;
    const int sbt = m / SB;                    // sub-blocks per tile side
    const int64_t per_tile = (int64_t)sbt * sbt;
    const int64_t total = ntiles * per_tile;
    const double inv2l = 1.0 / (2.0 * l);
    const int tid = threadIdx.x;
    const int Dl = D < MAXD ? D : MAXD;

    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int64_t t = w / per_tile;
        const int sub = (int)(w - t * per_tile);
        int I, J;
        if (T.layout == 0) lower_tile_coords(t, I, J);
        else { I = (int)(t / T.ncolt); J = (int)(t - (int64_t)I * T.ncolt); }
        const int si = sub / sbt, sj = sub - si * sbt;
        const int64_t i0 = (int64_t)I * m + si * SB;
        const int64_t j0 = (int64_t)J * m + sj * SB;
        double* out = tile_ptr(T, I, J) + (size_t)si * SB * m + sj * SB;
        double* cout = copy ? copy + (out - T.base) : nullptr;

        __syncthreads();
        for (int e = tid; e < SB * Dl; e += 256) {
            const int r = e / Dl, d = e - r * Dl;
            Sa[r][d] = (i0 + r < na) ? A[(i0 + r) * D + d] : 0.0;
            Sb[d][r] = (j0 + r < nb) ? B[(j0 + r) * D + d] : 0.0;
        }
        __syncthreads();
        const int c = tid & 31;
        const int64_t j = j0 + c;
        double bc[DT > 0 ? DT : 1];
        if constexpr (DT > 0) {
#pragma unroll
            for (int d = 0; d < DT; ++d) bc[d] = Sb[d][c];
        }
        for (int r = tid >> 5; r < SB; r += 8) {
            const int64_t i = i0 + r;
            double val;
            if (i < na && j < nb) {
                double d2 = 0.0;
                if constexpr (DT > 0) {
#pragma unroll
                    for (int d = 0; d < DT; ++d) {
                        const double q = Sa[r][d] - bc[d];
                        d2 = fma(q, q, d2);
                    }
                } else {
                    for (int d = 0; d < Dl; ++d) {
                        const double q = Sa[r][d] - Sb[d][c];
                        d2 = fma(q, q, d2);
                    }
                    for (int d = Dl; d < D; ++d) {  // dimensions beyond the LDS stage
                        const double q = A[i * D + d] - B[j * D + d];
                        d2 = fma(q, q, d2);
                    }
                }
                val = v * exp(-d2 * inv2l);
                if (diag_noise && i == j) val += s2;
            } else {
                val = (identity_pad && i == j) ? 1.0 : 0.0;
            }
            out[(size_t)r * m + c] = val;
            if (cout) cout[(size_t)r * m + c] = val;
        }
    }
}

// Assembly without LDS or barriers, for m a multiple of 64 and D = DT known:
// a workgroup fills a 64 x 64 block, wave w rows 16 w .. 16 w + 15 and lane l
// column l. The lane's column point stays in registers; a row point is the
// same for the whole wave, so its features come through scalar loads; every
// row is stored as 512 contiguous bytes. Same arithmetic as k_assemble.
template <int DT>
__global__ __launch_bounds__(256) void k_assemble_w(TileMat T, int64_t ntiles,
                                                    const double* __restrict__ A, int64_t na,
                                                    const double* __restrict__ B, int64_t nb,
                                                    double l, double v, double s2, int diag_noise,
                                                    int identity_pad, const double* __restrict__ hyp,
                                                    double* __restrict__ copy)
{
    if (hyp) {  // hyperparameters held on the device (l, v, sigma^2)
        l = hyp[0];
        v = hyp[1];
        s2 = hyp[2];
    }
    const int m = T.m;
    const int bt = m / 64;                     // 64 x 64 blocks per tile side
    const int64_t per_tile = (int64_t)bt * bt;
    const int64_t total = ntiles * per_tile;
    const double inv2l = 1.0 / (2.0 * l);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int64_t t = w / per_tile;
        const int sub = (int)(w - t * per_tile);
        int I, J;
        if (T.layout == 0) lower_tile_coords(t, I, J);
        else { I = (int)(t / T.ncolt); J = (int)(t - (int64_t)I * T.ncolt); }
        const int si = sub / bt, sj = sub - si * bt;
        const int r0 = si * 64 + wave * 16;    // first row of this wave, within the tile
        const int64_t j = (int64_t)J * m + sj * 64 + lane;
        double* out = tile_ptr(T, I, J) + (size_t)r0 * m + sj * 64 + lane;
        double* cout = copy ? copy + (out - T.base) : nullptr;
        const bool jin = j < nb;
        double bc[DT];
#pragma unroll
        for (int d = 0; d < DT; ++d) bc[d] = jin ? B[j * DT + d] : 0.0;
        for (int r = 0; r < 16; ++r) {
            const int64_t i = (int64_t)I * m + r0 + r;   // uniform across the wave
            double val;
            if (i < na && jin) {
                const double* ar = A + i * DT;
                double d2 = 0.0;
#pragma unroll
                for (int d = 0; d < DT; ++d) {
                    const double q = ar[d] - bc[d];
                    d2 = fma(q, q, d2);
                }
                val = v * exp(-d2 * inv2l);
                if (diag_noise && i == j) val += s2;
            } else {
                val = (identity_pad && i == j) ? 1.0 : 0.0;
            }
            out[(size_t)r * m] = val;
            if (cout) cout[(size_t)r * m] = val;
        }
    }
}

hipError_t launch_assemble(const TileMat& T, int tile_rows, const double* A, int64_t na,
                           const double* B, int64_t nb, int D, double l, double v, double s2,
                           bool diag_noise, bool identity_pad, hipStream_t s, const double* hyp,
                           double* copy)
{
    const int64_t ntiles = T.layout == 0 ? (int64_t)tile_rows * (tile_rows + 1) / 2
                                         : (int64_t)tile_rows * T.ncolt;
    if (ntiles <= 0) return hipSuccess;
    const int64_t subs = ntiles * (T.m / SB) * (T.m / SB);
    const int64_t grid = subs < 65536 ? subs : 65536;
    const int dn = diag_noise ? 1 : 0, ip = identity_pad ? 1 : 0;
    if (T.m % 64 == 0 && D >= 1 && D <= 8) {
        const int64_t items = ntiles * (T.m / 64) * (T.m / 64);
        const int64_t g = items < 65536 ? items : 65536;
#define GPR_ASMW(DT)                                                                             \
    hipLaunchKernelGGL(k_assemble_w<DT>, dim3((unsigned)g), dim3(256), 0, s, T, ntiles, A, na, B, \
                       nb, l, v, s2, dn, ip, hyp, copy)
        switch (D) {
        case 1: GPR_ASMW(1); break;
        case 2: GPR_ASMW(2); break;
        case 3: GPR_ASMW(3); break;
        case 4: GPR_ASMW(4); break;
        case 5: GPR_ASMW(5); break;
        case 6: GPR_ASMW(6); break;
        case 7: GPR_ASMW(7); break;
        default: GPR_ASMW(8); break;
        }
#undef GPR_ASMW
        return hipGetLastError();
    }
#define GPR_ASM(DT)                                                                              \
    hipLaunchKernelGGL(k_assemble<DT>, dim3((unsigned)grid), dim3(256), 0, s, T, tile_rows,     \
                       ntiles, A, na, B, nb, D, l, v, s2, dn, ip, hyp, copy)
    switch (D) {
    case 1: GPR_ASM(1); break;
    case 2: GPR_ASM(2); break;
    case 3: GPR_ASM(3); break;
    case 4: GPR_ASM(4); break;
    case 5: GPR_ASM(5); break;
    case 6: GPR_ASM(6); break;
    case 7: GPR_ASM(7); break;
    case 8: GPR_ASM(8); break;
    default: GPR_ASM(0); break;
    }
#undef GPR_ASM
    return hipGetLastError();
}

// Dense n x n (lower triangle read) -> lower tiles; padding gets the identity.
__global__ __launch_bounds__(256) void k_dense_to_tiled(const double* __restrict__ Ad, int64_t n,
                                                        int64_t lda, TileMat T, int64_t ntiles)
{
    const int m = T.m;
    const int sbt = m / SB;
    const int64_t per_tile = (int64_t)sbt * sbt;
    const int64_t total = ntiles * per_tile;
    const int tid = threadIdx.x;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int64_t t = w / per_tile;
        const int sub = (int)(w - t * per_tile);
        int I, J;
        lower_tile_coords(t, I, J);
        const int si = sub / sbt, sj = sub - si * sbt;
        const int64_t i0 = (int64_t)I * m + si * SB, j0 = (int64_t)J * m + sj * SB;
        double* out = tile_ptr(T, I, J) + (size_t)si * SB * m + sj * SB;
        const int c = tid & 31;
        for (int r = tid >> 5; r < SB; r += 8) {
            const int64_t i = i0 + r, j = j0 + c;
            double val;
            if (i < n && j < n) val = (j <= i) ? Ad[i * lda + j] : 0.0;
            else val = (i == j) ? 1.0 : 0.0;
            out[(size_t)r * m + c] = val;
        }
    }
}

hipError_t launch_dense_to_tiled(const double* A, int64_t n, int64_t lda, const TileMat& T,
                                 int tile_rows, hipStream_t s)
{
    const int64_t ntiles = (int64_t)tile_rows * (tile_rows + 1) / 2;
    const int64_t subs = ntiles * (T.m / SB) * (T.m / SB);
    const int64_t grid = subs < 65536 ? subs : 65536;
    hipLaunchKernelGGL(k_dense_to_tiled, dim3((unsigned)grid), dim3(256), 0, s, A, n, lda, T,
                       ntiles);
    return hipGetLastError();
}

// Lower tiles -> dense n x n. Output block (bi, bj) of 32 x 32: for bi >= bj
// read from tile storage directly; above the diagonal either mirror (read the
// transposed block through LDS) or write zeros.
__global__ __launch_bounds__(256) void k_tiled_to_dense(TileMat T, int64_t n, double* __restrict__ out,
                                                        int64_t ldo, int mirror)
{
    __shared__ double St[SB][SB + 1];
    const int m = T.m;
    const int64_t nbk = (n + SB - 1) / SB;
    const int64_t total = nbk * nbk;
    const int tid = threadIdx.x;
    const int c = tid & 31;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const int64_t bi = w / nbk, bj = w - bi * nbk;
        const int64_t i0 = bi * SB, j0 = bj * SB;
        if (bi >= bj) {
            for (int r = tid >> 5; r < SB; r += 8) {
                const int64_t i = i0 + r, j = j0 + c;
                if (i >= n || j >= n) continue;
                double val = 0.0;
                if (j <= i || mirror) {
                    // lower entries straight from storage; on a diagonal block
                    // the upper part is mirrored
                    const int64_t ii = j <= i ? i : j, jj = j <= i ? j : i;
                    val = tile_ptr(T, (int)(ii / m), (int)(jj / m))[(size_t)(ii % m) * m + jj % m];
                }
                out[i * ldo + j] = val;
            }
        } else if (mirror) {
            __syncthreads();
            // block (bj, bi) is below the diagonal: load it, write transposed
            for (int r = tid >> 5; r < SB; r += 8) {
                const int64_t i = j0 + r, j = i0 + c;   // element (i, j) with i > j
                St[r][c] = (i < n && j < n)
                               ? tile_ptr(T, (int)(i / m), (int)(j / m))[(size_t)(i % m) * m + j % m]
                               : 0.0;
            }
            __syncthreads();
            for (int r = tid >> 5; r < SB; r += 8) {
                const int64_t i = i0 + r, j = j0 + c;
                if (i < n && j < n) out[i * ldo + j] = St[c][r];
            }
        } else {
            for (int r = tid >> 5; r < SB; r += 8) {
                const int64_t i = i0 + r, j = j0 + c;
                if (i < n && j < n) out[i * ldo + j] = 0.0;
            }
        }
    }
}

hipError_t launch_tiled_to_dense(const TileMat& T, int64_t n, double* out, int64_t ldo,
                                 bool mirror, hipStream_t s)
{
    const int64_t nbk = (n + SB - 1) / SB;
    const int64_t total = nbk * nbk;
    if (total <= 0) return hipSuccess;
    const int64_t grid = total < 65536 ? total : 65536;
    hipLaunchKernelGGL(k_tiled_to_dense, dim3((unsigned)grid), dim3(256), 0, s, T, n, out, ldo,
                       mirror ? 1 : 0);
    return hipGetLastError();
}

}  // namespace gpr
