// k_trsm.hip -- batched TRSM tasks of Fig. 1, B := B L_JJ^{-T}, applied as
// B Tinv^T with Tinv = L_JJ^{-1} (lower triangular, from k_trtri).
//
// One workgroup owns a strip of 16 rows of one tile: it stages the strip in
// LDS (so the product can overwrite it in place), then each wave computes
// 16 x 16 output blocks, interleaved across waves so that the triangular
// work (output column j needs k <= j only) is balanced.
#include "gpr_internal.h"
#include "k_common.h"

namespace gpr {

namespace {
constexpr int R = 16;
}

__global__ __launch_bounds__(256) void k_trsm_f64(const TrsmTask* __restrict__ tasks, int m)
{
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
    for (int e = tid; e < R * m; e += 256) {
        const int r = e / m, c = e - r * m;
        S[r * ld + c] = B[(size_t)r * ldb + c];
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int nct = m / 16;
    for (int ct = wave; ct < nct; ct += 4) {
        const int c0 = 16 * ct;
        dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
        const double* trow = Ti + (size_t)(c0 + lr) * ldt + lk;   // B[k][j] = Tinv[c0+j][k]
        const double* srow = S + lr * ld + lk;                     // A[i][k] = strip[i][k]
        const int kend = c0 + 16;                                  // Tinv[j][k] = 0 for k > j
        int k = 0;
        for (; k + 8 <= kend; k += 8) {
            acc0 = mfma16(srow[k], trow[k], acc0);
            acc1 = mfma16(srow[k + 4], trow[k + 4], acc1);
        }
        for (; k < kend; k += 4) acc0 = mfma16(srow[k], trow[k], acc0);
#pragma unroll
        for (int v = 0; v < 4; ++v) B[(size_t)(drow(lk, v)) * ldb + c0 + lr] = acc0[v] + acc1[v];
    }
}

hipError_t launch_trsm_f64(const TrsmTask* d_tasks, int ntask, int m, hipStream_t s)
{
    if (ntask <= 0) return hipSuccess;
    const size_t lds = (size_t)R * (m + 1) * sizeof(double);
    static size_t lds_set = 0;
    if (lds > 65536 && lds > lds_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_trsm_f64),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set = lds;
    }
    hipLaunchKernelGGL(k_trsm_f64, dim3(ntask * (m / R)), dim3(256), lds, s, d_tasks, m);
    return hipGetLastError();
}

}  // namespace gpr
