// k_trsm.hip -- batched TRSM tasks of Fig. 1, B := B L_JJ^{-T}, applied as
// B Tinv^T with Tinv = L_JJ^{-1} (lower triangular, from k_trtri).
//
// One workgroup owns a strip of R rows of one tile: it stages the strip in
// LDS (so the product can overwrite it in place), then each wave computes
// R x 16 output blocks, interleaved across waves so that the triangular
// work (output column j needs k <= j only) is balanced. Each Tinv fragment
// read from L2 feeds R / 16 MFMAs; the k loop issues eight fragments' loads
// before their MFMAs.
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
    const int ldb = tk.ldb, ldt = tk.ldt;
    const double* __restrict__ Ti = tk.Tinv;

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
    const int nct = m / 16;
    for (int ct = wave; ct < nct; ct += NW) {
        const int c0 = 16 * ct;
        dbl4 acc[RT][2];
#pragma unroll
        for (int i = 0; i < RT; ++i) acc[i][0] = acc[i][1] = dbl4{0.0, 0.0, 0.0, 0.0};
        const double* trow = Ti + (size_t)(c0 + lr) * ldt + lk;  // B[k][j] = Tinv[c0+j][k]
        const double* srow = S + lr * ld + lk;                    // A[i][k] = strip[i][k]
        const int kend = c0 + 16;                                 // Tinv[j][k] = 0 for k > j
        int k = 0;
        for (; k + 32 <= kend; k += 32) {
            double b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) b[u] = trow[k + 4 * u];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int i = 0; i < RT; ++i)
                    acc[i][u & 1] = mfma16(srow[16 * i * ld + k + 4 * u], b[u], acc[i][u & 1]);
        }
        if (k < kend) {  // remaining 16 columns
            double b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) b[u] = trow[k + 4 * u];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int i = 0; i < RT; ++i)
                    acc[i][u & 1] = mfma16(srow[16 * i * ld + k + 4 * u], b[u], acc[i][u & 1]);
        }
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                B[(size_t)(16 * i + drow(lk, v)) * ldb + c0 + lr] = acc[i][0][v] + acc[i][1][v];
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
