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

// Sums (T x)[row0] and (T x)[row0 + 1] of an m x m tile for the calling wave
// (every lane gets both). Lane l takes columns l + 64 k (k < m / 64, at most
// 16), issuing all of its loads first; it sums in k order, then a fixed
// butterfly adds the lanes.
__device__ inline void row_pair_dot(const double* __restrict__ T, const double* __restrict__ x,
                                    int row0, int m, int lane, double& s0, double& s1)
{
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
    s0 = 0.0;
    s1 = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        s0 = fma(a0[k], xv[k], s0);
        s1 = fma(a1[k], xv[k], s1);
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
}

// y (-)= T x on rows GV_ROWS blk .. + GV_ROWS - 1 of an m x m tile, 256 threads;
// wave w owns rows 2w, 2w + 1 of the slice.
__device__ inline void gemv_rows(const double* __restrict__ T, const double* __restrict__ x,
                                 double* __restrict__ y, int blk, int m, bool set)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row0 = blk * GV_ROWS + 2 * wave;
    double s0, s1;
    row_pair_dot(T, x, row0, m, lane, s0, s1);
    if (lane < 2) {
        const int row = row0 + lane;
        const double v = lane ? s1 : s0;
        y[row] = set ? v : y[row] - v;
    }
}

// (T^T x)[col] for the GV_COLS columns GV_COLS blk .. of an m x m tile, 256
// threads: thread (g, c), g < 16, sums column c over rows g, g + 16, ...
// (m / 16 of them, in chunks of GV_LOADS loads issued together); the 16
// partial sums of a column are added in g order. The result is valid in
// threads tid < GV_COLS (column GV_COLS blk + tid); part is free on return.
__device__ inline double col_dot(const double* __restrict__ T, const double* __restrict__ x,
                                 int blk, int m, double (*part)[GV_COLS])
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
    double tot = 0.0;
    if (tid < GV_COLS) {
        tot = part[0][c];
#pragma unroll
        for (int q = 1; q < 16; ++q) tot += part[q][c];
    }
    __syncthreads();
    return tot;
}

// y (-)= T^T x on the columns GV_COLS blk .. of an m x m tile, 256 threads.
__device__ inline void gemv_cols(const double* __restrict__ T, const double* __restrict__ x,
                                 double* __restrict__ y, int blk, int m, bool set,
                                 double (*part)[GV_COLS])
{
    const double tot = col_dot(T, x, blk, m, part);
    if (threadIdx.x < GV_COLS) {
        const int col = blk * GV_COLS + threadIdx.x;
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

// Two tile rows per step, with W_p = -Tinv_{J+1} L_{J+1,J} Tinv_J (J = 2 p),
// the off-diagonal block of the inverse of the pair's 2 x 2 block:
//   forward   x_J = Tinv_J r_J,             x_{J+1} = W_p r_J + Tinv_{J+1} r_{J+1}
//   backward  x_{J+1} = Tinv_{J+1}^T r_{J+1}, x_J = Tinv_J^T r_J + W_p^T r_{J+1}
// Workgroups [0, per) take x_J, [per, 2 per) take x_{J+1}.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_trsv_diag2(const double* __restrict__ Tinv,
                                                    const double* __restrict__ W, int J, int m,
                                                    const double* __restrict__ r,
                                                    double* __restrict__ x)
{
    __shared__ double part[16][GV_COLS];
    const int per = gv_per_tile<TRANS>(m);
    const int half = blockIdx.x / per, blk = blockIdx.x % per;
    const size_t mm = (size_t)m * m, o0 = (size_t)J * m;
    const double* T0 = Tinv + (size_t)J * mm;
    const double* T1 = T0 + mm;
    const double* r0 = r + o0;
    const double* r1 = r0 + m;
    double* x0 = x + o0;
    double* x1 = x0 + m;
    if (!TRANS) {
        if (half == 0) {
            gemv_rows(T0, r0, x0, blk, m, true);
        } else {
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            const int row0 = blk * GV_ROWS + 2 * wave;
            double a0, a1, b0, b1;
            row_pair_dot(W, r0, row0, m, lane, a0, a1);
            row_pair_dot(T1, r1, row0, m, lane, b0, b1);
            if (lane < 2) x1[row0 + lane] = lane ? a1 + b1 : a0 + b0;
        }
    } else {
        if (half == 1) {
            gemv_cols(T1, r1, x1, blk, m, true, part);
        } else {
            const double a = col_dot(T0, r0, blk, m, part);
            const double b = col_dot(W, r1, blk, m, part);
            if (threadIdx.x < GV_COLS) x0[blk * GV_COLS + threadIdx.x] = a + b;
        }
    }
}

// Forward: r_K -= L_{K,J} x_J, then r_K -= L_{K,J+1} x_{J+1}, for K >= J + 2.
// Backward: r_K -= L_{J+1,K}^T x_{J+1}, then r_K -= L_{J,K}^T x_J, for K < J
// (the order of the one-tile steps). Workgroup b: tile row K = first + b /
// per, slice b % per.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_trsv_update2(TileMat L, int J, int first,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ r)
{
    __shared__ double part[16][GV_COLS];
    const int m = L.m;
    const int per = gv_per_tile<TRANS>(m);
    const int K = first + blockIdx.x / per, blk = blockIdx.x % per;
    double* rk = r + (size_t)K * m;
    if (!TRANS) {
        gemv_rows(tile_ptr(L, K, J), x + (size_t)J * m, rk, blk, m, false);
        gemv_rows(tile_ptr(L, K, J + 1), x + (size_t)(J + 1) * m, rk, blk, m, false);
    } else {
        gemv_cols(tile_ptr(L, J + 1, K), x + (size_t)(J + 1) * m, rk, blk, m, false, part);
        gemv_cols(tile_ptr(L, J, K), x + (size_t)J * m, rk, blk, m, false, part);
    }
}

hipError_t launch_trsv(const TileMat& L, const double* Tinv, const double* W, int M,
                       const double* b, double* r, double* x, bool trans, hipStream_t s)
{
    if (M <= 0) return hipSuccess;
    const int m = L.m, per = trans ? gv_per_tile<true>(m) : gv_per_tile<false>(m);
    const hipError_t e = hipMemcpyAsync(r, b, (size_t)M * m * sizeof(double),
                                        hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    if (W && M >= 2) {
        const int P = M / 2;
        const bool odd = M % 2 != 0;
        const size_t mm = (size_t)m * m;
        if (!trans) {
            for (int p = 0; p < P; ++p) {
                const int J = 2 * p, count = M - J - 2;
                hipLaunchKernelGGL(k_trsv_diag2<false>, dim3(2 * per), dim3(256), 0, s, Tinv,
                                   W + p * mm, J, m, r, x);
                if (count > 0)
                    hipLaunchKernelGGL(k_trsv_update2<false>, dim3(count * per), dim3(256), 0, s,
                                       L, J, J + 2, x, r);
            }
            if (odd)
                hipLaunchKernelGGL(k_trsv_diag<false>, dim3(per), dim3(256), 0, s, Tinv, M - 1, m,
                                   r, x);
        } else {
            if (odd) {
                hipLaunchKernelGGL(k_trsv_diag<true>, dim3(per), dim3(256), 0, s, Tinv, M - 1, m,
                                   r, x);
                hipLaunchKernelGGL(k_trsv_update<true>, dim3((M - 1) * per), dim3(256), 0, s, L,
                                   M - 1, 0, x, r);
            }
            for (int p = P - 1; p >= 0; --p) {
                const int J = 2 * p;
                hipLaunchKernelGGL(k_trsv_diag2<true>, dim3(2 * per), dim3(256), 0, s, Tinv,
                                   W + p * mm, J, m, r, x);
                if (J > 0)
                    hipLaunchKernelGGL(k_trsv_update2<true>, dim3(J * per), dim3(256), 0, s, L, J,
                                       0, x, r);
            }
        }
        return hipGetLastError();
    }
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
