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

// The products below are latency-bound: one step moves a few MB with a
// dependent launch on either side. Each lane therefore issues all of its
// loads before it adds anything (up to GV_LOADS in flight), and a workgroup
// covers a small slice of the tile, so that a tile is spread over many
// workgroups.
constexpr int GV_ROWS = 8;    // non-transposed: rows per workgroup (2 per wave)
constexpr int GV_COLS = 16;   // transposed: columns per workgroup
constexpr int GV_LOADS = 32;  // transposed: rows per lane per unrolled chunk

// y (-)= T x on rows GV_ROWS blk .. + GV_ROWS - 1 of an m x m tile, 256 threads.
// Wave w owns rows 2w, 2w + 1 of the slice; lane l takes columns l + 64 k
// (k < m / 64, at most 16). The lane sums in k order, then a fixed butterfly
// adds the lanes.
__device__ inline void gemv_rows(const double* __restrict__ T, const double* __restrict__ x,
                                 double* __restrict__ y, int blk, int m, bool set)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row0 = blk * GV_ROWS + 2 * wave;
    const double* T0 = T + (size_t)row0 * m;
    const double* T1 = T0 + m;
    double a0[16], a1[16], xv[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int c = lane + 64 * k;
        const bool in = c < m;
        a0[k] = in ? T0[c] : 0.0;
        a1[k] = in ? T1[c] : 0.0;
        xv[k] = in ? x[c] : 0.0;
    }
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        s0 = fma(a0[k], xv[k], s0);
        s1 = fma(a1[k], xv[k], s1);
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if (lane < 2) {
        const int row = row0 + lane;
        const double v = lane ? s1 : s0;
        y[row] = set ? v : y[row] - v;
    }
}

// y (-)= T^T x on columns GV_COLS blk .. + GV_COLS - 1 of an m x m tile, 256
// threads: thread (g, c), g < 16, sums column c over rows g, g + 16, ...
// (m / 16 of them, in chunks of GV_LOADS loads issued together); the 16
// partial sums of a column are added in g order.
__device__ inline void gemv_cols(const double* __restrict__ T, const double* __restrict__ x,
                                 double* __restrict__ y, int blk, int m, bool set,
                                 double (*part)[GV_COLS])
{
    const int tid = threadIdx.x, c = tid & (GV_COLS - 1), g = tid / GV_COLS;
    const int col = blk * GV_COLS + c;
    const int rows = m / 16;
    double s = 0.0;
    for (int r0 = 0; r0 < rows; r0 += GV_LOADS) {
        double a[GV_LOADS], xv[GV_LOADS];
#pragma unroll
        for (int q = 0; q < GV_LOADS; ++q) {
            const int r = 16 * (r0 + q) + g;
            const bool in = r0 + q < rows;
            a[q] = in ? T[(size_t)r * m + col] : 0.0;
            xv[q] = in ? x[r] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < GV_LOADS; ++q) s = fma(a[q], xv[q], s);
    }
    part[g][c] = s;
    __syncthreads();
    if (tid < GV_COLS) {
        double tot = part[0][c];
#pragma unroll
        for (int q = 1; q < 16; ++q) tot += part[q][c];
        y[col] = set ? tot : y[col] - tot;
    }
}

template <bool TRANS>
__device__ inline void gemv_block(const double* __restrict__ T, const double* __restrict__ x,
                                  double* __restrict__ y, int blk, int m, bool set,
                                  double (*part)[GV_COLS])
{
    if (TRANS) gemv_cols(T, x, y, blk, m, set, part);
    else gemv_rows(T, x, y, blk, m, set);
}

// workgroups per tile
template <bool TRANS>
__host__ __device__ inline int gv_per_tile(int m) { return TRANS ? m / GV_COLS : m / GV_ROWS; }

}  // namespace

// x_J = op(Tinv_J) r_J; workgroup b takes slice b of the outputs.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_trsv_diag(const double* __restrict__ Tinv, int J, int m,
                                                   const double* __restrict__ r,
                                                   double* __restrict__ x)
{
    __shared__ double part[16][GV_COLS];
    const size_t off = (size_t)J * m;
    gemv_block<TRANS>(Tinv + off * m, r + off, x + off, blockIdx.x, m, true, part);
}

// r_K -= L_KJ x_J for K > J (forward) or r_K -= L_JK^T x_J for K < J
// (backward); workgroup b: tile row K = first + b / per, slice b % per.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_trsv_update(TileMat L, int J, int first,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ r)
{
    __shared__ double part[16][GV_COLS];
    const int m = L.m;
    const int per = gv_per_tile<TRANS>(m);
    const int K = first + blockIdx.x / per, blk = blockIdx.x % per;
    const double* T = TRANS ? tile_ptr(L, J, K) : tile_ptr(L, K, J);
    gemv_block<TRANS>(T, x + (size_t)J * m, r + (size_t)K * m, blk, m, false, part);
}

hipError_t launch_trsv(const TileMat& L, const double* Tinv, int M, const double* b, double* r,
                       double* x, bool trans, hipStream_t s)
{
    if (M <= 0) return hipSuccess;
    const int m = L.m, per = trans ? gv_per_tile<true>(m) : gv_per_tile<false>(m);
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
