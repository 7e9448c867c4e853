// k_trsv.hip -- the triangular vector solves of the prediction (Sec. 4.1,
// after eq. (2)): beta = L^{-1} b and alpha = L^{-T} beta by block
// substitution over the lower tiles of L, a group of G consecutive tile rows
// per step (G = trsv_group(m, prec): 4 for tiles up to 256, and up to 512
// for a factor with mixed-precision updates, whose refinement runs many
// solves; else 2). The inverse of
// the group's G x G block of tiles is known: its diagonal tiles are the
// diagonal-tile inverses Tinv, its off-diagonal tiles Inv_ij (i > j) are built
// once per factor (the plan in solve_plan.cpp, run by api.hip). Forward,
// group g = tiles J0 .. J0 + ns - 1 (r = b on entry):
//     x_{J0+i} = sum_{j <= i} Inv_ij r_{J0+j}                  (one launch)
//     r_K -= sum_j L_{K,J0+j} x_{J0+j},  K >= J0 + ns          (one launch)
// Backward over the groups in reverse, with transposed tiles:
//     x_{J0+j} = sum_{i >= j} Inv_ij^T r_{J0+i},
//     r_K -= sum_i L_{J0+i,K}^T x_{J0+i},  K < J0.
// The launch boundaries order the steps (a device-scope handoff between
// workgroups costs more than a launch here), so a solve is 2 ceil(M / G) - 1
// launches. Tile addresses are computed from the tile indices, so no task
// descriptors are needed. Every product sums in a fixed order: results are
// bitwise reproducible.
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
// loads before it adds anything, and a workgroup covers a small slice of the
// tile rows, so that a step is spread over many workgroups.
constexpr int GV_ROWS = 8;    // non-transposed: rows per workgroup (2 per wave)
constexpr int GV_COLS = 16;   // transposed: columns per workgroup
constexpr int GV_LOADS = 32;  // transposed: operand loads per lane per chunk

// Offset (in tiles) of Inv_ij, i > j, within its group's block of slots.
__host__ __device__ inline int inv_slot(int i, int j) { return i * (i - 1) / 2 + j; }

// Rows row0, row0 + 1 of sum_{j < ns} T_j x_j for the calling wave (every lane
// gets both sums), T_j = seg.tile(j) an m x m tile, x_j = seg.vec(j). Lane l
// takes columns l + 64 q (q < Q) of every segment and issues all of its loads
// first; it sums segment by segment in column order, then a fixed butterfly
// adds the lanes. Needs m <= 64 Q and ns <= G.
template <int G, int Q, class Seg>
__device__ inline void rows_dot(const Seg& seg, int ns, int row0, int m, int lane, double& s0,
                                double& s1)
{
    double a0[G][Q], a1[G][Q], xv[G][Q];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const double* T0 = seg.tile(j) + (size_t)row0 * m;
        const double* T1 = T0 + m;
        const double* x = seg.vec(j);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int c = lane + 64 * q;
            const bool in = j < ns && c < m;
            a0[j][q] = in ? gld(T0 + c) : 0.0;
            a1[j][q] = in ? gld(T1 + c) : 0.0;
            xv[j][q] = in ? gld(x + c) : 0.0;
        }
    }
    s0 = 0.0;
    s1 = 0.0;
#pragma unroll
    for (int j = 0; j < G; ++j)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            s0 = fma(a0[j][q], xv[j][q], s0);
            s1 = fma(a1[j][q], xv[j][q], s1);
        }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
}

// Column col of sum_{i < ns} T_i^T x_i, 256 threads: thread (g, c), g < 16,
// c < GV_COLS, sums over the rows g, g + 16, ... of every segment in turn, in
// chunks of GV_LOADS loads issued together; the 16 partial sums of a column
// are then added in g order. The result is valid in threads tid < GV_COLS
// (column GV_COLS blk + tid); part is free on return.
template <class Seg>
__device__ inline double cols_dot(const Seg& seg, int ns, int blk, int m,
                                  double (*part)[GV_COLS])
{
    const int tid = threadIdx.x, c = tid & (GV_COLS - 1), g = tid / GV_COLS;
    const int col = blk * GV_COLS + c;
    const int rps = m / 16;          // rows per segment and thread
    const int total = ns * rps;
    int sg = 0, q = 0;               // position of the next load
    double s = 0.0;
    for (int base = 0; base < total; base += GV_LOADS) {
        double a[GV_LOADS], xv[GV_LOADS];
#pragma unroll
        for (int u = 0; u < GV_LOADS; ++u) {
            const bool in = base + u < total;
            const int r = 16 * q + g;
            a[u] = in ? gld(seg.tile(sg) + (size_t)r * m + col) : 0.0;
            xv[u] = in ? gld(seg.vec(sg) + r) : 0.0;
            if (++q == rps) {
                q = 0;
                ++sg;
            }
        }
#pragma unroll
        for (int u = 0; u < GV_LOADS; ++u) s = fma(a[u], xv[u], s);
    }
    part[g][c] = s;
    __syncthreads();
    double tot = 0.0;
    if (tid < GV_COLS) {
        tot = part[0][c];
#pragma unroll
        for (int k = 1; k < 16; ++k) tot += part[k][c];
    }
    __syncthreads();
    return tot;
}

// Segments of the group inverse: row i of the block (forward) or column j
// (backward, segments i = j + s). Inv_ii = Tinv_{J0+i}; the others sit at
// slot inv_slot(i, j) of the group's block Wg.
struct InvRow {
    const double *Tinv, *Wg, *r;
    size_t mm;
    int J0, i, m;
    __device__ const double* tile(int j) const
    {
        return j == i ? Tinv + (size_t)(J0 + i) * mm : Wg + (size_t)inv_slot(i, j) * mm;
    }
    __device__ const double* vec(int j) const { return r + (size_t)(J0 + j) * m; }
};
struct InvCol {
    const double *Tinv, *Wg, *r;
    size_t mm;
    int J0, j, m;
    __device__ const double* tile(int s) const
    {
        const int i = j + s;
        return s == 0 ? Tinv + (size_t)(J0 + j) * mm : Wg + (size_t)inv_slot(i, j) * mm;
    }
    __device__ const double* vec(int s) const { return r + (size_t)(J0 + j + s) * m; }
};
// Tiles (K, J0 + j) of L (forward) or (J0 + i, K) (backward).
struct LRow {
    TileMat L;
    const double* x;
    int K, J0;
    __device__ const double* tile(int j) const { return tile_ptr(L, K, J0 + j); }
    __device__ const double* vec(int j) const { return x + (size_t)(J0 + j) * L.m; }
};
struct LCol {
    TileMat L;
    const double* x;
    int K, J0;
    __device__ const double* tile(int i) const { return tile_ptr(L, J0 + i, K); }
    __device__ const double* vec(int i) const { return x + (size_t)(J0 + i) * L.m; }
};

}  // namespace

// Diagonal step of group J0 (ns tiles): x_{J0..J0+ns-1} from r. Workgroup b
// takes tile i = b / per of the group, slice b % per of its outputs.
template <bool TRANS, int G, int Q>
__global__ __launch_bounds__(256) void k_trsv_group_diag(const double* __restrict__ Tinv,
                                                         const double* __restrict__ Wg, int J0,
                                                         int ns, int m,
                                                         const double* __restrict__ r,
                                                         double* __restrict__ x)
{
    __shared__ double part[16][GV_COLS];
    const size_t mm = (size_t)m * m;
    if (!TRANS) {
        const int per = m / GV_ROWS;
        const int i = blockIdx.x / per, blk = blockIdx.x % per;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int row0 = blk * GV_ROWS + 2 * wave;
        const InvRow seg{Tinv, Wg, r, mm, J0, i, m};
        double s0, s1;
        rows_dot<G, Q>(seg, i + 1, row0, m, lane, s0, s1);
        if (lane < 2) gst(x + (size_t)(J0 + i) * m + row0 + lane, lane ? s1 : s0);
    } else {
        const int per = m / GV_COLS;
        const int j = blockIdx.x / per, blk = blockIdx.x % per;
        const InvCol seg{Tinv, Wg, r, mm, J0, j, m};
        const double tot = cols_dot(seg, ns - j, blk, m, part);
        if (threadIdx.x < GV_COLS)
            gst(x + (size_t)(J0 + j) * m + blk * GV_COLS + threadIdx.x, tot);
    }
}

// Update after group J0 (ns tiles): forward r_K -= sum_j L_{K,J0+j} x_{J0+j}
// for the tile rows K = first + b / per; backward r_K -= sum_i L_{J0+i,K}^T
// x_{J0+i}. Workgroup b: tile row first + b / per, slice b % per.
template <bool TRANS, int G, int Q>
__global__ __launch_bounds__(256) void k_trsv_group_update(TileMat L, int J0, int ns, int first,
                                                           const double* __restrict__ x,
                                                           double* __restrict__ r)
{
    __shared__ double part[16][GV_COLS];
    const int m = L.m;
    if (!TRANS) {
        const int per = m / GV_ROWS;
        const int K = first + blockIdx.x / per, blk = blockIdx.x % per;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int row0 = blk * GV_ROWS + 2 * wave;
        const LRow seg{L, x, K, J0};
        double s0, s1;
        rows_dot<G, Q>(seg, ns, row0, m, lane, s0, s1);
        if (lane < 2) {
            double* y = r + (size_t)K * m + row0 + lane;
            gst(y, gld(y) - (lane ? s1 : s0));
        }
    } else {
        const int per = m / GV_COLS;
        const int K = first + blockIdx.x / per, blk = blockIdx.x % per;
        const LCol seg{L, x, K, J0};
        const double tot = cols_dot(seg, ns, blk, m, part);
        if (threadIdx.x < GV_COLS) {
            double* y = r + (size_t)K * m + blk * GV_COLS + threadIdx.x;
            gst(y, gld(y) - tot);
        }
    }
}

int trsv_group(int m, int prec)
{
    return (m <= 256 || (prec != GPR_FP64 && m <= 512)) ? 4 : 2;
}

namespace {

template <int G, int Q>
void trsv_steps(const TileMat& L, const double* Tinv, const double* W, int M, double* r,
                double* x, bool trans, hipStream_t s)
{
    const int m = L.m;
    const size_t mm = (size_t)m * m;
    // without the off-diagonal inverse tiles: one tile row per step
    const int g = W ? G : 1;
    const int ng = (M + g - 1) / g;
    const size_t gslots = (size_t)G * (G - 1) / 2;   // slots per group
    const int per_f = m / GV_ROWS, per_b = m / GV_COLS;
    for (int step = 0; step < ng; ++step) {
        const int gi = trans ? ng - 1 - step : step;
        const int J0 = gi * g, ns = M - J0 < g ? M - J0 : g;
        const double* Wg = W ? W + gi * gslots * mm : nullptr;
        if (!trans) {
            hipLaunchKernelGGL((k_trsv_group_diag<false, G, Q>), dim3(ns * per_f), dim3(256), 0,
                               s, Tinv, Wg, J0, ns, m, r, x);
            const int rest = M - J0 - ns;
            if (rest > 0)
                hipLaunchKernelGGL((k_trsv_group_update<false, G, Q>), dim3(rest * per_f),
                                   dim3(256), 0, s, L, J0, ns, J0 + ns, x, r);
        } else {
            hipLaunchKernelGGL((k_trsv_group_diag<true, G, Q>), dim3(ns * per_b), dim3(256), 0,
                               s, Tinv, Wg, J0, ns, m, r, x);
            if (J0 > 0)
                hipLaunchKernelGGL((k_trsv_group_update<true, G, Q>), dim3(J0 * per_b),
                                   dim3(256), 0, s, L, J0, ns, 0, x, r);
        }
    }
}

}  // namespace

hipError_t launch_trsv(const TileMat& L, const double* Tinv, const double* W, int G, int M,
                       const double* b, double* r, double* x, bool trans, hipStream_t s)
{
    if (M <= 0) return hipSuccess;
    const int m = L.m;
    const hipError_t e = hipMemcpyAsync(r, b, (size_t)M * m * sizeof(double),
                                        hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    // group size of W, and loads per lane and tile row (m <= 64 Q)
    if (G == 4 && m <= 256) trsv_steps<4, 4>(L, Tinv, W, M, r, x, trans, s);
    else if (G == 4 && m <= 512) trsv_steps<4, 8>(L, Tinv, W, M, r, x, trans, s);
    else if (G == 2 && m <= 512) trsv_steps<2, 8>(L, Tinv, W, M, r, x, trans, s);
    else if (G == 2) trsv_steps<2, 16>(L, Tinv, W, M, r, x, trans, s);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}
}  // namespace gpr
