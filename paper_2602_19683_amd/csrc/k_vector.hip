// k_vector.hip -- vector kernels of the prediction (Sec. 4.1):
//   * tile GEMVs for the triangular solves L beta = y and L^T alpha = beta,
//     run tile row by tile row with the inverted diagonal tiles;
//   * the matrix-free kernel matvec sum_j k(a_i, b_j) x_j that gives the
//     predictive mean (eq. (2)) from alpha without storing K_{X*,X}, and the
//     residual y - K alpha of the iterative refinement.
// All reductions run in a fixed order, so results are bitwise reproducible.
#include "gpr_internal.h"
#include "k_common.h"

namespace gpr {

__device__ inline double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// y (-)= op(T) x for each task, in blocks of 32 output entries.
// Non-transposed: each wave owns 8 rows, the lanes stride over the columns
// and a fixed butterfly adds them. Transposed: thread (g, c) sums column c
// over row group g of 8; the groups are added in order.
__global__ __launch_bounds__(256) void k_gemv_f64(const GemvTask* __restrict__ tasks, int m)
{
    __shared__ double part[8][32];
    const int per = m / 32;
    const int t = blockIdx.x / per, blk = blockIdx.x - t * per;
    const GemvTask tk = tasks[t];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (!tk.trans) {
        for (int rr = 0; rr < 8; ++rr) {
            const int row = blk * 32 + wave * 8 + rr;
            const double* Tr = tk.T + (size_t)row * tk.ld;
            double s = 0.0;
            for (int c = lane; c < m; c += 64) s += Tr[c] * tk.x[c];
            s = wave_sum(s);
            if (lane == 0) tk.y[row] = tk.set ? s : tk.y[row] - s;
        }
    } else {
        const int c = tid & 31, g = tid >> 5;
        const int col = blk * 32 + c;
        const int rows = m / 8;
        double s = 0.0;
        for (int r = g * rows; r < (g + 1) * rows; ++r) s += tk.T[(size_t)r * tk.ld + col] * tk.x[r];
        part[g][c] = s;
        __syncthreads();
        if (tid < 32) {
            double tot = part[0][c];
#pragma unroll
            for (int q = 1; q < 8; ++q) tot += part[q][c];
            tk.y[col] = tk.set ? tot : tk.y[col] - tot;
        }
    }
}

hipError_t launch_gemv_f64(const GemvTask* d_tasks, int ntask, int m, hipStream_t s)
{
    if (ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gemv_f64, dim3(ntask * (m / 32)), dim3(256), 0, s, d_tasks, m);
    return hipGetLastError();
}

// out_i = [base_i -] (sum_{j < nb} v exp(-|a_i - b_j|^2 / (2 l)) x_j + [noise] s2 x_i)
// A workgroup owns 32 rows of A, 8 lanes per row striding over j; the 8
// partial sums are combined by a fixed butterfly.
__global__ __launch_bounds__(256) void k_kernel_matvec(const double* __restrict__ A, int64_t na,
                                                       const double* __restrict__ B, int64_t nb,
                                                       int D, double l, double v, double s2,
                                                       int noise, const double* __restrict__ x,
                                                       const double* __restrict__ base,
                                                       double* __restrict__ out)
{
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 32 + tid / 8;
    const int sub = tid & 7;
    const double inv2l = 1.0 / (2.0 * l);
    double s = 0.0;
    if (i < na) {
        const double* a = A + i * D;
        for (int64_t j = sub; j < nb; j += 8) {
            const double* b = B + j * D;
            double d2 = 0.0;
            for (int d = 0; d < D; ++d) {
                const double t = a[d] - b[d];
                d2 += t * t;
            }
            s += v * exp(-d2 * inv2l) * x[j];
        }
    }
    s += __shfl_xor(s, 4, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 1, 64);
    if (i < na && sub == 0) {
        if (noise && i < nb) s += s2 * x[i];
        out[i] = base ? base[i] - s : s;
    }
}

hipError_t launch_kernel_matvec(const double* A, int64_t na, const double* B, int64_t nb, int D,
                                double l, double v, double s2, bool noise, const double* x,
                                const double* base, double* out, hipStream_t s)
{
    if (na <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((na + 31) / 32);
    hipLaunchKernelGGL(k_kernel_matvec, dim3(grid), dim3(256), 0, s, A, na, B, nb, D, l, v, s2,
                       noise ? 1 : 0, x, base, out);
    return hipGetLastError();
}

__global__ void k_set_int(int* p, int value) { *p = value; }

hipError_t launch_set_int(int* p, int value, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, value);
    return hipGetLastError();
}

// dst[0:n] = src[0:n], dst[n:n_pad] = 0
__global__ void k_copy_pad(const double* __restrict__ src, double* __restrict__ dst, int64_t n,
                           int64_t n_pad)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = i < n ? src[i] : 0.0;
}

hipError_t launch_copy_f64(const double* src, double* dst, int64_t n, int64_t n_pad, hipStream_t s)
{
    if (n_pad <= 0) return hipSuccess;
    int64_t blocks = (n_pad + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_copy_pad, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n, n_pad);
    return hipGetLastError();
}

}  // namespace gpr
