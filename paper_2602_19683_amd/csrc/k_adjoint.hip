// k_adjoint.hip -- the elementwise ends of the NLML gradient:
//   * the seed of the reverse sweep: the adjoint of the factor for
//     NLML = 1/2 beta^T beta + sum_i log L_ii + n/2 log(2 pi), beta = L^{-1} y:
//       Lbar = -tril(alpha beta^T) + diag(1 / L_ii),  alpha = L^{-T} beta
//     (the solve adjoint: d(1/2 beta^T beta) = -alpha^T dL beta);
//   * the kernel-gradient reduction g_theta = sum_{i >= j} Abar_ij dK_ij/dtheta
//     for the squared-exponential kernel of eq. (1) read as
//     k = v exp(-s / (2 l)), s = |x_i - x_j|^2:
//       dK/dl = v e s / (2 l^2),  dK/dv = e,  dK/dsigma^2 = delta_ij;
//   * the NLML value and the final fixed-order sums.
// All sums run in a fixed order (per-workgroup partials, then one workgroup),
// so results are bitwise reproducible.
#include "gpr_internal.h"
#include "k_common.h"

namespace gpr {

namespace {

// Tile (I, J) of the lower-tiled layout from its index t = I (I + 1) / 2 + J.
__device__ inline void lower_tile_coords(int t, int& I, int& J)
{
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
}

constexpr int GR_B = 32;      // square block of a tile per workgroup
constexpr int GR_DC = 32;     // feature dimensions staged per pass
constexpr int GR_MAXWG = 4096;

}  // namespace

// grid (ceil(m^2 / 1024), tiles): 4 entries per thread
__global__ __launch_bounds__(256) void k_lbar_init(TileMat W, TileMat L, const double* __restrict__ alpha,
                                                   const double* __restrict__ beta)
{
    int I, J;
    lower_tile_coords(blockIdx.y, I, J);
    const int m = W.m;
    double* __restrict__ Wt = tile_ptr(W, I, J);
    const double* __restrict__ Lt = tile_ptr(L, I, I);
    for (int u = 0; u < 4; ++u) {
        const int e = blockIdx.x * 1024 + u * 256 + threadIdx.x;
        if (e >= m * m) break;
        const int r = e / m, c = e - r * m;
        double val = 0.0;
        if (I > J || c <= r) {
            val = -alpha[(size_t)I * m + r] * beta[(size_t)J * m + c];
            if (I == J && r == c) val += 1.0 / Lt[(size_t)r * m + r];
        }
        Wt[e] = val;
    }
}

hipError_t launch_lbar_init(const TileMat& W, const TileMat& L, int M, const double* alpha,
                            const double* beta, hipStream_t s)
{
    const int m = W.m;
    const dim3 grid((m * m + 1023) / 1024, M * (M + 1) / 2);
    hipLaunchKernelGGL(k_lbar_init, grid, dim3(256), 0, s, W, L, alpha, beta);
    return hipGetLastError();
}

int grad_reduce_parts(int M, int m)
{
    const long nb = (long)(m / GR_B) * (m / GR_B) * M * (M + 1) / 2;
    return (int)(nb < GR_MAXWG ? nb : GR_MAXWG);
}

// Workgroup w takes blocks w, w + grid, ... of the lower tiles (32 x 32 blocks,
// those above the diagonal of a diagonal tile skipped). Thread (ty, tx) owns
// rows 4 ty .. 4 ty + 3 and column tx of a block. Points of the block's rows and
// columns are staged in LDS GR_DC dimensions at a time.
__global__ __launch_bounds__(256) void k_grad_reduce(TileMat A, int M, const double* __restrict__ X,
                                                     int64_t n, int D, double l,
                                                     double* __restrict__ parts,
                                                     const double* __restrict__ hyp)
{
    if (hyp) l = hyp[0];  // lengthscale held on the device
    __shared__ double Xr[GR_B][GR_DC + 1];
    __shared__ double Xc[GR_B][GR_DC + 1];
    __shared__ double red[3][256];
    const int m = A.m;
    const int nbt = m / GR_B;
    const long nblocks = (long)nbt * nbt * M * (M + 1) / 2;
    const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
    const double inv2l = 1.0 / (2.0 * l);
    double gls = 0.0, gv = 0.0, gs = 0.0;
    for (long b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const int t = (int)(b / (nbt * nbt));
        const int sb = (int)(b - (long)t * nbt * nbt);
        const int bi = sb / nbt, bj = sb - bi * nbt;
        int I, J;
        lower_tile_coords(t, I, J);
        if (I == J && bj > bi) continue;  // uniform across the workgroup
        const int64_t r0 = (int64_t)I * m + bi * GR_B, c0 = (int64_t)J * m + bj * GR_B;
        if (r0 >= n || c0 >= n) continue;
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (int d0 = 0; d0 < D; d0 += GR_DC) {
            __syncthreads();
            for (int e = tid; e < GR_B * GR_DC; e += 256) {
                const int p = e / GR_DC, d = e - p * GR_DC;
                const bool okd = d0 + d < D;
                Xr[p][d] = (okd && r0 + p < n) ? X[(r0 + p) * D + d0 + d] : 0.0;
                Xc[p][d] = (okd && c0 + p < n) ? X[(c0 + p) * D + d0 + d] : 0.0;
            }
            __syncthreads();
            const int dn = D - d0 < GR_DC ? D - d0 : GR_DC;
            for (int d = 0; d < dn; ++d) {
                const double xc = Xc[tx][d];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double z = Xr[4 * ty + q][d] - xc;
                    s[q] += z * z;
                }
            }
        }
        const double* __restrict__ At = tile_ptr(A, I, J);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int rr = bi * GR_B + 4 * ty + q, cc = bj * GR_B + tx;
            const int64_t gi = (int64_t)I * m + rr, gj = (int64_t)J * m + cc;
            if (gi >= n || gj >= n || gj > gi) continue;
            const double a = At[(size_t)rr * m + cc];
            const double e = exp(-s[q] * inv2l);
            gv += a * e;
            gls += a * e * s[q];
            if (gi == gj) gs += a;
        }
    }
    red[0][tid] = gls;
    red[1][tid] = gv;
    red[2][tid] = gs;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w)
            for (int k = 0; k < 3; ++k) red[k][tid] += red[k][tid + w];
        __syncthreads();
    }
    if (tid < 3) parts[3 * (size_t)blockIdx.x + tid] = red[tid][0];
}

hipError_t launch_grad_reduce(const TileMat& A, int M, const double* X, int64_t n, int D,
                              double l, double* parts, hipStream_t s, const double* hyp)
{
    hipLaunchKernelGGL(k_grad_reduce, dim3(grad_reduce_parts(M, A.m)), dim3(256), 0, s, A, M, X, n,
                       D, l, parts, hyp);
    return hipGetLastError();
}

// Thread per output column of a 256-column strip; rows strided over grid y.
__global__ __launch_bounds__(256) void k_kbar_export(TileMat A, int64_t n, double* __restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int m = A.m;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        const int64_t r = i > j ? i : j, c = i > j ? j : i;
        const int I = (int)(r / m), J = (int)(c / m);
        const double a = tile_ptr(A, I, J)[(size_t)(r - (int64_t)I * m) * m + (c - (int64_t)J * m)];
        out[i * n + j] = (i == j) ? a : 0.5 * a;
    }
}

hipError_t launch_kbar_export(const TileMat& A, int64_t n, double* out, hipStream_t s)
{
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)(n < 4096 ? n : 4096));
    hipLaunchKernelGGL(k_kbar_export, grid, dim3(256), 0, s, A, n, out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_nlml_finish(TileMat L, const double* __restrict__ beta,
                                                     int64_t n, const double* __restrict__ parts,
                                                     int nparts, double l, double v,
                                                     const int* __restrict__ info,
                                                     double* __restrict__ out_nlml,
                                                     double* __restrict__ out_grad3,
                                                     const double* __restrict__ hyp)
{
    if (hyp) {  // hyperparameters held on the device
        l = hyp[0];
        v = hyp[1];
    }
    __shared__ double red[5][256];
    const int tid = threadIdx.x;
    const int m = L.m;
    double sl = 0.0, sb = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int64_t i = tid; i < n; i += 256) {
        const int I = (int)(i / m), r = (int)(i - (int64_t)I * m);
        sl += log(tile_ptr(L, I, I)[(size_t)r * m + r]);
        sb += beta[i] * beta[i];
    }
    for (int p = tid; p < nparts; p += 256) {
        g0 += parts[3 * (size_t)p];
        g1 += parts[3 * (size_t)p + 1];
        g2 += parts[3 * (size_t)p + 2];
    }
    red[0][tid] = sl;
    red[1][tid] = sb;
    red[2][tid] = g0;
    red[3][tid] = g1;
    red[4][tid] = g2;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w)
            for (int k = 0; k < 5; ++k) red[k][tid] += red[k][tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        const bool bad = info[0] > 0;
        const double nan = __builtin_nan("");
        const double two_pi = 6.283185307179586476925286766559;
        out_nlml[0] = bad ? nan : 0.5 * red[1][0] + red[0][0] + 0.5 * (double)n * log(two_pi);
        if (out_grad3) {
            out_grad3[0] = bad ? nan : red[2][0] * v / (2.0 * l * l);
            out_grad3[1] = bad ? nan : red[3][0];
            out_grad3[2] = bad ? nan : red[4][0];
        }
    }
}

hipError_t launch_nlml_finish(const TileMat& L, const double* beta, int64_t n, const double* parts,
                              int nparts, double l, double v, const int* info, double* out_nlml,
                              double* out_grad3, hipStream_t s, const double* hyp)
{
    hipLaunchKernelGGL(k_nlml_finish, dim3(1), dim3(256), 0, s, L, beta, n, parts, nparts, l, v,
                       info, out_nlml, out_grad3, hyp);
    return hipGetLastError();
}

// Adam on log theta, one thread: the state lives in device memory between
// the evaluations, so the fit needs no host round trip per step.
__global__ void k_adam_init(AdamState* st, double z0, double z1, double z2)
{
    const double z[3] = {z0, z1, z2};
    for (int k = 0; k < 3; ++k) {
        st->z[k] = z[k];
        st->m[k] = 0.0;
        st->s[k] = 0.0;
        st->theta[k] = exp(z[k]);
    }
    st->b1t = 1.0;
    st->b2t = 1.0;
    st->prev = 0.0;
    st->t = 0;
    st->stop = 0;
}

__global__ void k_adam_step(AdamState* st, const double* __restrict__ fit,
                            double* __restrict__ trace, int max_steps, double lr, double beta1,
                            double beta2, double eps, double tol)
{
    if (st->stop) return;
    const double f = fit[0];
    if (!isfinite(f)) {
        st->stop = 2;
        return;
    }
    if (trace) trace[st->t] = f;
    const int t = ++st->t;
    st->b1t *= beta1;
    st->b2t *= beta2;
    for (int k = 0; k < 3; ++k) {
        const double gz = fit[1 + k] * st->theta[k];   // d/dlog(theta) = theta d/dtheta
        st->m[k] = beta1 * st->m[k] + (1.0 - beta1) * gz;
        st->s[k] = beta2 * st->s[k] + (1.0 - beta2) * gz * gz;
        const double mh = st->m[k] / (1.0 - st->b1t), sh = st->s[k] / (1.0 - st->b2t);
        st->z[k] -= lr * mh / (sqrt(sh) + eps);
        st->theta[k] = exp(st->z[k]);
    }
    if ((t > 1 && tol > 0 && fabs(f - st->prev) <= tol * fabs(st->prev)) || t >= max_steps)
        st->stop = 1;
    st->prev = f;
}

hipError_t launch_adam_init(AdamState* st, double z0, double z1, double z2, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam_init, dim3(1), dim3(1), 0, s, st, z0, z1, z2);
    return hipGetLastError();
}

hipError_t launch_adam_step(AdamState* st, const double* fit, double* trace, int max_steps,
                            double lr, double beta1, double beta2, double eps, double tol,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_adam_step, dim3(1), dim3(1), 0, s, st, fit, trace, max_steps, lr, beta1,
                       beta2, eps, tol);
    return hipGetLastError();
}

}  // namespace gpr
