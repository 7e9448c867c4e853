// k_trsm.hip -- batched TRSM tasks of Fig. 1, B := B L_JJ^{-T} (the reading
// L_IJ = K_IJ L_JJ^{-T}), by blocked substitution.
//
// One workgroup owns a strip of R rows of one tile and keeps it in LDS. For
// each 32-column block p of the diagonal factor, left to right:
//     X_p = B_p Dinv_p^T                      (Dinv_p = inverse of the 32 x 32
//                                              diagonal block p of L_JJ, made
//                                              by POTRF)
//     B_q -= X_p L_JJ[q, p]^T   for q > p     (right-looking strip update)
// X_p is final when computed and is written out (and, in a mixed precision,
// also as a low-precision copy for the tile updates that consume it). Only
// the 32 x 32 diagonal-block inverses are needed, so no full inverse of L_JJ
// sits on the critical path.
#include "gpr_internal.h"
#include "k_common.h"

namespace gpr {

template <int R, int NW>
__global__ __launch_bounds__(NW * 64) void k_trsm_f64(const TrsmTask* __restrict__ tasks, int m)
{
    constexpr int RT = R / 16;  // row tiles per strip
    extern __shared__ double S[];  // R x (m + 1)
    const int ld = m + 1;
    const int strips = m / R;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lid / strips, s = lid - t * strips;
    const TrsmTask tk = tasks[t];
    double* __restrict__ B = tk.B + (size_t)s * R * tk.ldb;
    const int ldb = tk.ldb, ldl = tk.ldl, ldd = tk.ldd;
    const double* __restrict__ Lj = tk.L;
    const double* __restrict__ Dv = tk.Dinv;
    float* __restrict__ B32 = tk.B32 ? tk.B32 + (size_t)s * R * m : nullptr;

    const int tid = threadIdx.x;
    for (int e = 2 * tid; e < R * m; e += 2 * NW * 64) {
        const int r = e / m, c = e - r * m;
        const double2 v = *reinterpret_cast<const double2*>(B + (size_t)r * ldb + c);
        S[r * ld + c] = v.x;
        S[r * ld + c + 1] = v.y;
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int P = m / 32;
    for (int p = 0; p < P; ++p) {
        const int c0 = 32 * p;
        // X_p = B_p Dinv_p^T: 2 RT output tiles of 16 x 16, waves 0 .. 2 RT - 1
        dbl4 o = {0.0, 0.0, 0.0, 0.0};
        const int rt = wave >> 1, ct = wave & 1;
        if (wave < 2 * RT) {
            const double* a = S + (16 * rt + lr) * ld + c0 + lk;
            const double* b = Dv + (size_t)(c0 + 16 * ct + lr) * ldd + c0 + lk;
#pragma unroll
            for (int k = 0; k < 32; k += 4) o = mfma16(a[k], b[k], o);
        }
        __syncthreads();  // every read of block p done before it is overwritten
        if (wave < 2 * RT) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * rt + drow(lk, v), col = c0 + 16 * ct + lr;
                S[row * ld + col] = o[v];
                B[(size_t)row * ldb + col] = o[v];
                if (B32) B32[(size_t)row * m + col] = (float)o[v];
            }
        }
        __syncthreads();
        // B_q -= X_p L[q, p]^T for q > p: tiles (q, rt, ct) spread over the waves
        const int ntile = (P - p - 1) * 2 * RT;
        for (int tt = wave; tt < ntile; tt += NW) {
            const int q = p + 1 + tt / (2 * RT);
            const int rr = (tt % (2 * RT)) >> 1, cc = tt & 1;
            const int col0 = 32 * q + 16 * cc;
            dbl4 acc;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] = S[(16 * rr + drow(lk, v)) * ld + col0 + lr];
            const double* a = S + (16 * rr + lr) * ld + c0 + lk;
            const double* b = Lj + (size_t)(col0 + lr) * ldl + c0 + lk;
            double bv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) bv[u] = b[4 * u];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = mfma16(-a[4 * u], bv[u], acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) S[(16 * rr + drow(lk, v)) * ld + col0 + lr] = acc[v];
        }
        __syncthreads();
    }
}

template <int R, int NW>
static hipError_t launch_trsm_cfg(const TrsmTask* d_tasks, int ntask, int m, hipStream_t s)
{
    const size_t lds = (size_t)R * (m + 1) * sizeof(double);
    static size_t lds_set = 0;
    if (lds > 65536 && lds > lds_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_trsm_f64<R, NW>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set = lds;
    }
    hipLaunchKernelGGL((k_trsm_f64<R, NW>), dim3(ntask * (m / R)), dim3(NW * 64), lds, s, d_tasks, m);
    return hipGetLastError();
}

hipError_t launch_trsm_f64(const TrsmTask* d_tasks, int ntask, int m, hipStream_t s)
{
    if (ntask <= 0) return hipSuccess;
    if (m <= 512) return launch_trsm_cfg<32, 8>(d_tasks, ntask, m, s);
    return launch_trsm_cfg<16, 8>(d_tasks, ntask, m, s);
}

}  // namespace gpr
