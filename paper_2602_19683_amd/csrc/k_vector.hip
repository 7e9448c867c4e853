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
// matrix stored as M lower tiles (layout 0, diagonal tiles full):
//   (K x)_I = sum_{J <= I} K_IJ x_J + sum_{I' > I} K_{I'I}^T x_{I'}.
// Pass 1 reads every stored tile once: workgroup (t, s) takes rows
// 32 s .. 32 s + 31 of lower tile t = (I, J) and writes those rows of K_IJ x_J
// (complete) to prow[t], and, for I > J, the part of K_IJ^T x_I over its 32
// rows (a length-m partial) to pcol[t][s]. Pass 2 adds, for each output row,
// its I + 1 row products and (M - 1 - I) m / 32 column partials in a fixed
// order. No atomics: the result is bitwise reproducible.
namespace {
constexpr int SV_R = 32;   // rows per pass-1 workgroup (8 per wave)
constexpr int SV_KC = 4;   // column groups of 64 per load chunk (32 loads in flight)
}

size_t symv_work_doubles(int M, int m)
{
    const size_t T = (size_t)M * (M + 1) / 2;
    return T * m + T * (size_t)(m / SV_R) * m;
}

__global__ __launch_bounds__(256) void k_symv_part(TileMat K, const double* __restrict__ x,
                                                   double* __restrict__ prow,
                                                   double* __restrict__ pcol)
{
    __shared__ double part[4][1024];
    const int m = K.m, S = m / SV_R;
    const int t = blockIdx.x / S, s = blockIdx.x % S;
    int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int J = t - I * (I + 1) / 2;
    const bool offd = I > J;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row0 = SV_R * s + 8 * wave;  // this wave's 8 rows, within the tile
    const double* T = tile_ptr(K, I, J) + (size_t)row0 * m;
    const double* xJ = x + (size_t)J * m;
    const double* xI = x + (size_t)I * m + row0;
    double xr[8], rs[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        xr[r] = xI[r];
        rs[r] = 0.0;
    }
    const int G = (m + 63) / 64;  // column groups of 64
    for (int k0 = 0; k0 < G; k0 += SV_KC) {
        double a[8][SV_KC], xc[SV_KC];
#pragma unroll
        for (int kk = 0; kk < SV_KC; ++kk) {
            const int c = lane + 64 * (k0 + kk);
            const bool in = k0 + kk < G && c < m;
            xc[kk] = in ? xJ[c] : 0.0;
#pragma unroll
            for (int r = 0; r < 8; ++r) a[r][kk] = in ? T[(size_t)r * m + c] : 0.0;
        }
#pragma unroll
        for (int kk = 0; kk < SV_KC; ++kk) {
#pragma unroll
            for (int r = 0; r < 8; ++r) rs[r] = fma(a[r][kk], xc[kk], rs[r]);
            const int c = lane + 64 * (k0 + kk);
            if (offd && k0 + kk < G && c < m) {
                double cs = 0.0;
#pragma unroll
                for (int r = 0; r < 8; ++r) cs = fma(a[r][kk], xr[r], cs);
                part[wave][c] = cs;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) rs[r] = wave_sum(rs[r]);
    if (lane < 8) {
        double v = rs[0];
#pragma unroll
        for (int r = 1; r < 8; ++r) v = (lane == r) ? rs[r] : v;
        prow[(size_t)t * m + row0 + lane] = v;
    }
    if (offd) {
        __syncthreads();
        double* pc = pcol + ((size_t)t * S + s) * m;
        for (int c = tid; c < m; c += 256)
            pc[c] = ((part[0][c] + part[1][c]) + part[2][c]) + part[3][c];
    }
}

// Pass 2: workgroup b takes output rows 32 b .. 32 b + 31 (one tile row I,
// since m is a multiple of 32); thread (g, e), g < 8, adds entries g, g + 8,
// ... of row e's list (the row products of tiles (I, 0..I), then the column
// partials of tiles (I + 1.., I) slice by slice); the 8 sums are added in g
// order.
__global__ __launch_bounds__(256) void k_symv_sum(int M, int m, const double* __restrict__ prow,
                                                  const double* __restrict__ pcol,
                                                  const double* __restrict__ base,
                                                  double* __restrict__ out, int64_t n)
{
    __shared__ double part[8][32];
    const int S = m / SV_R;
    const int tid = threadIdx.x, e = tid & 31, g = tid >> 5;
    const int64_t i = (int64_t)blockIdx.x * 32 + e;
    const int I = (int)(i / m), li = (int)(i % m);
    const int nrow = I + 1, ntot = nrow + (M - 1 - I) * S;
    double acc = 0.0;
    for (int q0 = g; q0 < ntot; q0 += 8 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + 8 * u;
            const double* p = nullptr;
            if (q < nrow) {
                p = prow + (size_t)(I * (I + 1) / 2 + q) * m;
            } else if (q < ntot) {
                const int w = q - nrow, Ip = I + 1 + w / S, sp = w % S;
                p = pcol + ((size_t)(Ip * (Ip + 1) / 2 + I) * S + sp) * m;
            }
            v[u] = p ? p[li] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    part[g][e] = acc;
    __syncthreads();
    if (tid < 32 && i < n) {
        double tot = part[0][e];
#pragma unroll
        for (int q = 1; q < 8; ++q) tot += part[q][e];
        out[i] = (base ? base[i] : 0.0) - tot;
    }
}

hipError_t launch_symv_tiled(const TileMat& K, int M, const double* x, const double* base,
                             double* out, int64_t n, double* work, hipStream_t s)
{
    const int m = K.m;
    if (M <= 0 || m % SV_R || m > 1024) return hipErrorInvalidValue;
    const size_t T = (size_t)M * (M + 1) / 2;
    double* prow = work;
    double* pcol = work + T * m;
    hipLaunchKernelGGL(k_symv_part, dim3((unsigned)(T * (m / SV_R))), dim3(256), 0, s, K, x, prow,
                       pcol);
    hipLaunchKernelGGL(k_symv_sum, dim3((unsigned)((size_t)M * m / 32)), dim3(256), 0, s, M, m,
                       prow, pcol, base, out, n);
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

// Predictive mean from the test rows (eqs. (2) and (3) share V = L^{-1}
// K_{X,X*}): mean = K_{X*,X} L^{-T} L^{-1} y = V^T beta with beta = L^{-1} y,
// so no backward solve is needed once V^T is formed. One wave per test row;
// each lane sums its columns of every tile in order, then a fixed butterfly:
// bitwise reproducible. beta has M m entries (zero padding).
__global__ __launch_bounds__(256) void k_rowdot_mean(TileMat V, int M, int64_t n_test,
                                                     const double* __restrict__ beta,
                                                     double* __restrict__ mean)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n_test) return;
    const int m = V.m;
    const int I = (int)(i / m), r = (int)(i % m);
    double acc = 0.0;
    for (int J = 0; J < M; ++J) {
        const double* row = tile_ptr(V, I, J) + (size_t)r * m;
        const double* b = beta + (size_t)J * m;
#pragma unroll 4
        for (int c = lane; c < m; c += 64) acc = fma(gld(row + c), gld(b + c), acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) mean[i] = acc;
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

hipError_t launch_rowdot_mean(const TileMat& V, int M, int64_t n_test, const double* beta,
                              double* mean, hipStream_t s)
{
    if (n_test <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rowdot_mean, dim3((unsigned)((n_test + 3) / 4)), dim3(256), 0, s, V, M,
                       n_test, beta, mean);
    return hipGetLastError();
}

hipError_t launch_tile_diag(const TileMat& S, int64_t n, double* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, n, out);
    return hipGetLastError();
}

}  // namespace gpr
