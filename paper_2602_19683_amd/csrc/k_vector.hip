// k_vector.hip -- vector kernels of the prediction (Sec. 4.1):
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


// Matrix-free kernel matvec out_i = base_i - sum_j k(a_i, b_j) x_j (or without
// base, the plain sum), for the predictive mean (eq. (2)): the cross
// covariance is never stored. Workgroup (row block, column chunk) takes 64
// rows (4 per thread, features in registers) against one chunk of the columns;
// the points of B are staged in LDS 256 at a time with their x_j, and the 16
// lanes of a row group take every 16th point. Each workgroup writes its
// partial sums; a second kernel adds the chunks in order (fixed-order sums:
// bitwise reproducible), so the launch has enough workgroups for the whole
// chip even for a few thousand rows.
namespace {
constexpr int MV_ROWS = 64;   // rows per workgroup
constexpr int MV_R = 4;       // rows per thread
constexpr int MV_CH = 256;    // training points per LDS chunk
}

int matvec_chunks(int64_t na, int64_t nb)
{
    const int64_t rb = (na + MV_ROWS - 1) / MV_ROWS;
    const int64_t maxc = (nb + MV_CH - 1) / MV_CH;
    int64_t c = (1024 + rb - 1) / rb;
    if (c > maxc) c = maxc;
    if (c > 64) c = 64;
    return (int)(c < 1 ? 1 : c);
}

template <int MAXD>
__global__ __launch_bounds__(256) void k_kernel_matvec(const double* __restrict__ A, int64_t na,
                                                       const double* __restrict__ B, int64_t nb,
                                                       int D, double l, double v,
                                                       const double* __restrict__ x,
                                                       int64_t cw, double* __restrict__ part)
{
    __shared__ double Sb[MAXD][MV_CH + 1];
    __shared__ double Sx[MV_CH];
    const int tid = threadIdx.x;
    const int sub = tid & 15, grp = tid >> 4;  // 16 groups of 16 lanes
    const int64_t i0 = (int64_t)blockIdx.x * MV_ROWS + grp * MV_R;
    const int64_t jb = (int64_t)blockIdx.y * cw;
    const int64_t je = jb + cw < nb ? jb + cw : nb;
    const double inv2l = 1.0 / (2.0 * l);
    double a[MV_R][MAXD];
#pragma unroll
    for (int r = 0; r < MV_R; ++r)
#pragma unroll
        for (int d = 0; d < MAXD; ++d)
            a[r][d] = (i0 + r < na && d < D) ? A[(i0 + r) * D + d] : 0.0;
    double acc[MV_R];
#pragma unroll
    for (int r = 0; r < MV_R; ++r) acc[r] = 0.0;

    for (int64_t j0 = jb; j0 < je; j0 += MV_CH) {
        __syncthreads();
        for (int e = tid; e < MV_CH * MAXD; e += 256) {
            const int jj = e / MAXD, d = e % MAXD;
            Sb[d][jj] = (j0 + jj < je && d < D) ? B[(j0 + jj) * D + d] : 0.0;
        }
        if (tid < MV_CH) Sx[tid] = (j0 + tid < je) ? x[j0 + tid] : 0.0;
        __syncthreads();
        for (int jj = sub; jj < MV_CH; jj += 16) {
            const double xj = Sx[jj];
            double d2[MV_R];
#pragma unroll
            for (int r = 0; r < MV_R; ++r) d2[r] = 0.0;
#pragma unroll
            for (int d = 0; d < MAXD; ++d) {
                const double bd = Sb[d][jj];
#pragma unroll
                for (int r = 0; r < MV_R; ++r) {
                    const double q = a[r][d] - bd;
                    d2[r] += q * q;
                }
            }
#pragma unroll
            for (int r = 0; r < MV_R; ++r) acc[r] += v * exp(-d2[r] * inv2l) * xj;
        }
    }
    // features beyond MAXD (rare): recompute those rows' sums exactly
    if (D > MAXD) {
#pragma unroll
        for (int r = 0; r < MV_R; ++r) {
            acc[r] = 0.0;
            if (i0 + r >= na) continue;
            for (int64_t j = jb + sub; j < je; j += 16) {
                double d2 = 0.0;
                for (int d = 0; d < D; ++d) {
                    const double q = A[(i0 + r) * D + d] - B[j * D + d];
                    d2 += q * q;
                }
                acc[r] += v * exp(-d2 * inv2l) * x[j];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < MV_R; ++r) {
        double sr = acc[r];
        sr += __shfl_xor(sr, 8, 64);
        sr += __shfl_xor(sr, 4, 64);
        sr += __shfl_xor(sr, 2, 64);
        sr += __shfl_xor(sr, 1, 64);
        const int64_t i = i0 + r;
        if (sub == 0 && i < na) part[(int64_t)blockIdx.y * na + i] = sr;
    }
}

__global__ __launch_bounds__(256) void k_matvec_finish(const double* __restrict__ part, int nch,
                                                       int64_t na, int64_t nb, double s2, int noise,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ base,
                                                       double* __restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < na;
         i += (int64_t)gridDim.x * 256) {
        double sr = 0.0;
        for (int c = 0; c < nch; ++c) sr += part[(int64_t)c * na + i];
        if (noise && i < nb) sr += s2 * x[i];
        out[i] = base ? base[i] - sr : sr;
    }
}

hipError_t launch_kernel_matvec(const double* A, int64_t na, const double* B, int64_t nb, int D,
                                double l, double v, double s2, bool noise, const double* x,
                                const double* base, double* out, double* work, hipStream_t s)
{
    if (na <= 0) return hipSuccess;
    const int nch = matvec_chunks(na, nb);
    const int64_t per = (nb + nch - 1) / nch;
    const int64_t cw = (per + MV_CH - 1) / MV_CH * MV_CH;
    const dim3 grid((unsigned)((na + MV_ROWS - 1) / MV_ROWS), (unsigned)nch);
    if (D <= 8)
        hipLaunchKernelGGL(k_kernel_matvec<8>, grid, dim3(256), 0, s, A, na, B, nb, D, l, v, x, cw,
                           work);
    else
        hipLaunchKernelGGL(k_kernel_matvec<16>, grid, dim3(256), 0, s, A, na, B, nb, D, l, v, x, cw,
                           work);
    const int64_t fb = (na + 255) / 256;
    hipLaunchKernelGGL(k_matvec_finish, dim3((unsigned)(fb < 1024 ? fb : 1024)), dim3(256), 0, s,
                       work, nch, na, nb, s2, noise ? 1 : 0, x, base, out);
    return hipGetLastError();
}

// out[0] = sum_i x_i^2 (one workgroup, fixed order: strided per thread, then
// a tree over the 256 partial sums).
__global__ __launch_bounds__(256) void k_sumsq(const double* __restrict__ x, int64_t n,
                                               double* __restrict__ out)
{
    __shared__ double part[256];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int64_t i = tid; i < n; i += 256) s += x[i] * x[i];
    part[tid] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w) part[tid] += part[tid + w];
        __syncthreads();
    }
    if (tid == 0) out[0] = part[0];
}

hipError_t launch_sumsq(const double* x, int64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(256), 0, s, x, n, out);
    return hipGetLastError();
}

// out[0] = sum x_i y_i, in the same fixed order as k_sumsq.
__global__ __launch_bounds__(256) void k_dot(const double* __restrict__ x,
                                            const double* __restrict__ y, int64_t n,
                                            double* __restrict__ out)
{
    __shared__ double part[256];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int64_t i = tid; i < n; i += 256) s += x[i] * y[i];
    part[tid] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w) part[tid] += part[tid + w];
        __syncthreads();
    }
    if (tid == 0) out[0] = part[0];
}

hipError_t launch_dot(const double* x, const double* y, int64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot, dim3(1), dim3(256), 0, s, x, y, n, out);
    return hipGetLastError();
}

// Conjugate-gradient vector updates with the scalars kept in device memory
// (no host round trip inside an iteration). With w = -K p:
//   a = rz / (p^T K p) = rz / (-pw);  x += a p;  r += a w   (r -= a K p)
__global__ void k_cg_xr(double* __restrict__ x, double* __restrict__ r,
                        const double* __restrict__ p, const double* __restrict__ w,
                        const double* __restrict__ rz, const double* __restrict__ pw, int64_t n)
{
    const double a = rz[0] / -pw[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += a * p[i];
        r[i] += a * w[i];
    }
}

//   p = z + (rz_new / rz_old) p
__global__ void k_cg_p(double* __restrict__ p, const double* __restrict__ z,
                       const double* __restrict__ rz_new, const double* __restrict__ rz_old,
                       int64_t n)
{
    const double b = rz_new[0] / rz_old[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + b * p[i];
}

namespace {
unsigned vec_blocks(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)(b > 2048 ? 2048 : b);
}
}  // namespace

hipError_t launch_cg_xr(double* x, double* r, const double* p, const double* w,
                        const double* rz, const double* pw, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cg_xr, dim3(vec_blocks(n)), dim3(256), 0, s, x, r, p, w, rz, pw, n);
    return hipGetLastError();
}

hipError_t launch_cg_p(double* p, const double* z, const double* rz_new, const double* rz_old,
                       int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cg_p, dim3(vec_blocks(n)), dim3(256), 0, s, p, z, rz_new, rz_old, n);
    return hipGetLastError();
}

// y[i] += x[i]
__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] += x[i];
}

hipError_t launch_axpy(double* y, const double* x, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)blocks), dim3(256), 0, s, y, x, n);
    return hipGetLastError();
}

// out_i = base_i - (K x)_i (base may be null: out = -K x) for the symmetric
// matrix stored as lower tiles
// (diagonal tiles hold both triangles). Workgroup (I, b) owns rows
// I m + 32 b .. + 31: it adds the tile-row part sum_{J <= I} K_IJ x_J and the
// transposed tile-column part sum_{I' > I} K_{I'I}^T x_{I'} in a fixed order
// (no atomics), reading each off-diagonal tile twice over the whole launch.
__global__ __launch_bounds__(256) void k_symv_tiled(TileMat K, int M, const double* __restrict__ x,
                                                    const double* __restrict__ base,
                                                    double* __restrict__ out, int64_t n)
{
    __shared__ double part[8][32];
    const int m = K.m;
    const int per = m / 32;
    const int I = blockIdx.x / per, b = blockIdx.x % per;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // row part: wave w takes rows 8w .. 8w+7 of the block, lanes stride columns
    double s[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) s[r] = 0.0;
    for (int J = 0; J <= I; ++J) {
        const double* T = tile_ptr(K, I, J) + (size_t)(32 * b + 8 * wave) * m;
        const double* xj = x + (size_t)J * m;
        for (int c = lane; c < m; c += 64) {
            const double xc = xj[c];
#pragma unroll
            for (int r = 0; r < 8; ++r) s[r] += T[(size_t)r * m + c] * xc;
        }
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        double v = s[r];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        s[r] = v;
    }
    // transposed part: thread (g, c) sums column 32 b + c over row group g of
    // every tile below the diagonal in tile column I
    const int c = tid & 31, g = tid >> 5;
    double t = 0.0;
    for (int Ip = I + 1; Ip < M; ++Ip) {
        const double* T = tile_ptr(K, Ip, I) + 32 * b + c;
        const double* xi = x + (size_t)Ip * m;
        const int rows = m / 8;
        for (int r = g * rows; r < (g + 1) * rows; ++r) t += T[(size_t)r * m] * xi[r];
    }
    part[g][c] = t;
    __syncthreads();
    if (lane < 8) {
        const int row = 32 * b + 8 * wave + lane;     // row within the tile row
        double tot = s[0];
#pragma unroll
        for (int r = 1; r < 8; ++r) tot = (lane == r) ? s[r] : tot;
        double tr = part[0][8 * wave + lane];
#pragma unroll
        for (int q = 1; q < 8; ++q) tr += part[q][8 * wave + lane];
        const int64_t gi = (int64_t)I * m + row;
        if (gi < n) out[gi] = (base ? base[gi] : 0.0) - (tot + tr);
    }
}

hipError_t launch_symv_tiled(const TileMat& K, int M, const double* x, const double* base,
                             double* out, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_symv_tiled, dim3(M * (K.m / 32)), dim3(256), 0, s, K, M, x, base, out, n);
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

// Predictive variances without the covariance matrix (eq. (3), diagonal):
// var_i = k(x*_i, x*_i) - sum_j (V^T)_{ij}^2 with k(x, x) = v (the test block
// is noise-free). One wave per test row; each lane sums its columns of every
// tile in order, then a fixed butterfly: bitwise reproducible.
__global__ __launch_bounds__(256) void k_rowsq_var(TileMat V, int M, int64_t n_test, double v,
                                                   double* __restrict__ var)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n_test) return;
    const int m = V.m;
    const int I = (int)(i / m), r = (int)(i % m);
    double acc = 0.0;
    for (int J = 0; J < M; ++J) {
        const double* row = tile_ptr(V, I, J) + (size_t)r * m;
        for (int c = lane; c < m; c += 64) acc = fma(row[c], row[c], acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) var[i] = v - acc;
}

// The diagonal of a lower-tiled matrix (the predictive variances when the
// full covariance is formed): out_i = S_ii, i < n.
__global__ void k_tile_diag(TileMat S, int64_t n, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int m = S.m;
    const int I = (int)(i / m), r = (int)(i % m);
    out[i] = tile_ptr(S, I, I)[(size_t)r * m + r];
}

hipError_t launch_rowsq_var(const TileMat& V, int M, int64_t n_test, double v, double* var,
                            hipStream_t s)
{
    if (n_test <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rowsq_var, dim3((unsigned)((n_test + 3) / 4)), dim3(256), 0, s, V, M,
                       n_test, v, var);
    return hipGetLastError();
}

hipError_t launch_tile_diag(const TileMat& S, int64_t n, double* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, n, out);
    return hipGetLastError();
}

}  // namespace gpr
