// k_trsv.hip -- the triangular vector solves of the prediction (Sec. 4.1,
// after eq. (2)): beta = L^{-1} b and alpha = L^{-T} beta by block
// substitution over the lower tiles of L with the inverses of its diagonal
// tiles. Forward, tile row by tile row (r = b on entry):
//     beta_J = Tinv_J r_J                       (one launch, m / 32 workgroups)
//     r_K -= L_KJ beta_J,  K > J                (one launch for all K)
// Backward over J = M-1 .. 0 with transposed tiles:
//     alpha_J = Tinv_J^T r_J,  r_K -= L_JK^T alpha_J,  K < J.
// The launch boundaries order the steps (a device-scope handoff between
// workgroups costs more than a launch here). Tile addresses are computed from
// the tile indices, so no task descriptors are needed. Every product sums in a
// fixed order: results are bitwise reproducible.
#include "gpr_internal.h"
#include "k_common.h"

namespace gpr {

namespace {

__device__ inline double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// y (-)= op(T) x on 32 outputs (block blk) of an m x m tile, 256 threads.
// Non-transposed: each wave owns 8 rows and walks their columns together
// (eight independent loads per step), then a fixed butterfly adds the lanes.
// Transposed: thread (g, c) sums column c over row group g (four chains); the
// groups are added in order.
template <bool TRANS>
__device__ inline void gemv_block(const double* __restrict__ T, const double* __restrict__ x,
                                  double* __restrict__ y, int blk, int m, bool set,
                                  double (*part)[32])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (!TRANS) {
        const int row0 = blk * 32 + wave * 8;
        const double* Tr = T + (size_t)row0 * m;
        double s[8];
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) s[rr] = 0.0;
        for (int c = lane; c < m; c += 64) {
            const double xc = x[c];
#pragma unroll
            for (int rr = 0; rr < 8; ++rr) s[rr] += Tr[(size_t)rr * m + c] * xc;
        }
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) s[rr] = wave_sum(s[rr]);
        if (lane < 8) {
            double v = s[0];
#pragma unroll
            for (int rr = 1; rr < 8; ++rr) v = (lane == rr) ? s[rr] : v;
            const int row = row0 + lane;
            y[row] = set ? v : y[row] - v;
        }
        return;
    }
    const int c = tid & 31, g = tid >> 5;
    const int col = blk * 32 + c;
    const int rows = m / 8;
    const double* Tc = T + (size_t)g * rows * m + col;
    const double* xg = x + g * rows;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int r = 0; r < rows; r += 4) {
        s0 += Tc[(size_t)r * m] * xg[r];
        s1 += Tc[(size_t)(r + 1) * m] * xg[r + 1];
        s2 += Tc[(size_t)(r + 2) * m] * xg[r + 2];
        s3 += Tc[(size_t)(r + 3) * m] * xg[r + 3];
    }
    part[g][c] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (tid < 32) {
        double tot = part[0][c];
#pragma unroll
        for (int q = 1; q < 8; ++q) tot += part[q][c];
        y[col] = set ? tot : y[col] - tot;
    }
}

}  // namespace

// x_J = op(Tinv_J) r_J, one workgroup per 32 outputs.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_trsv_diag(const double* __restrict__ Tinv, int J, int m,
                                                   const double* __restrict__ r,
                                                   double* __restrict__ x)
{
    __shared__ double part[8][32];
    const size_t off = (size_t)J * m;
    gemv_block<TRANS>(Tinv + off * m, r + off, x + off, blockIdx.x, m, true, part);
}

// r_K -= L_KJ x_J for K > J (forward) or r_K -= L_JK^T x_J for K < J
// (backward); workgroup b: tile row K = first + b / (m / 32), block b % (m / 32).
template <bool TRANS>
__global__ __launch_bounds__(256) void k_trsv_update(TileMat L, int J, int first,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ r)
{
    __shared__ double part[8][32];
    const int m = L.m;
    const int per = m / 32;
    const int K = first + blockIdx.x / per, blk = blockIdx.x % per;
    const double* T = TRANS ? tile_ptr(L, J, K) : tile_ptr(L, K, J);
    gemv_block<TRANS>(T, x + (size_t)J * m, r + (size_t)K * m, blk, m, false, part);
}

hipError_t launch_trsv(const TileMat& L, const double* Tinv, int M, const double* b, double* r,
                       double* x, bool trans, hipStream_t s)
{
    if (M <= 0) return hipSuccess;
    const int m = L.m, per = m / 32;
    const hipError_t e = hipMemcpyAsync(r, b, (size_t)M * m * sizeof(double),
                                        hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    for (int step = 0; step < M; ++step) {
        const int J = trans ? M - 1 - step : step;
        const int first = trans ? 0 : J + 1;
        const int count = trans ? J : M - 1 - J;
        if (trans) {
            hipLaunchKernelGGL(k_trsv_diag<true>, dim3(per), dim3(256), 0, s, Tinv, J, m, r, x);
            if (count > 0)
                hipLaunchKernelGGL(k_trsv_update<true>, dim3(count * per), dim3(256), 0, s, L, J,
                                   first, x, r);
        } else {
            hipLaunchKernelGGL(k_trsv_diag<false>, dim3(per), dim3(256), 0, s, Tinv, J, m, r, x);
            if (count > 0)
                hipLaunchKernelGGL(k_trsv_update<false>, dim3(count * per), dim3(256), 0, s, L, J,
                                   first, x, r);
        }
    }
    return hipGetLastError();
}

}  // namespace gpr
