// k_trsm_dev.h -- one TRSM strip task (32 rows of B := B L_JJ^{-T}), shared by
// the stream kernel and the persistent executor; the algorithm is described
// in k_trsm.hip.
#pragma once

#include "gpr_internal.h"
#include "k_accum.h"
#include "k_common.h"

namespace gpr {

namespace trsm_detail {
constexpr int TK = 16;  // k-chunk of the block product
}
using trsm_detail::TK;

struct TrsmLds {
    double As[2][TK][36];
    double Bs[2][TK][36];
    double Sacc[32][33];
};

// No wait before a column block: the diagonal tile is complete at the start.
struct TrsmNoWait {
    __device__ void operator()(int) const {}
};

// Strip s (rows 32 s .. 32 s + 31) of the task; 256 threads, tid = 0..255.
// before_block(p), called by every thread before column block p is read, can
// wait until rows 32 p .. 32 p + 31 of the diagonal tile and their block
// inverse are final (a POTRF still running beside the strip).
template <class Wait = TrsmNoWait>
__device__ inline void trsm_strip(const TrsmTask& tk, int s, int m, TrsmLds& sh, int tid,
                                  Wait before_block = Wait())
{
    double (*As)[TK][36] = sh.As;
    double (*Bs)[TK][36] = sh.Bs;
    double (*Sacc)[33] = sh.Sacc;
    double* __restrict__ B = tk.B + (size_t)s * 32 * tk.ldb;
    const int ldb = tk.ldb, ldl = tk.ldl, ldd = tk.ldd;
    float* __restrict__ B32 = tk.B32 ? tk.B32 + (size_t)s * 32 * m : nullptr;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int qi = wave >> 1, qj = wave & 1;
    const int P = m / 32;
    for (int p = 0; p < P; ++p) {
        before_block(p);
        const int c0 = 32 * p;
        dbl4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            acc[v] = gld(B + (size_t)(16 * qi + drow(lk, v)) * ldb + c0 + 16 * qj + lr);
        // minus the finished blocks X[:, 0:c0] times rows c0.. of L_JJ (transposed)
        acc = accum32<true, TK>(B, ldb, tk.L + (size_t)c0 * ldl, ldl, c0, acc, -1.0, As, Bs, tid);
#pragma unroll
        for (int v = 0; v < 4; ++v) Sacc[16 * qi + drow(lk, v)][16 * qj + lr] = acc[v];
        __syncthreads();
        const double* dq = tk.Dinv + (size_t)(c0 + 16 * qj + lr) * ldd + c0 + lk;
        dbl4 o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 32; k += 4) o = mfma16(Sacc[16 * qi + lr][k + lk], gld(dq + k), o);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * qi + drow(lk, v), col = c0 + 16 * qj + lr;
            gst(B + (size_t)row * ldb + col, o[v]);
            if (B32) gst(B32 + (size_t)row * m + col, (float)o[v]);
        }
        __syncthreads();  // X_p stored (read by every wave next), Sacc free
    }
}


}  // namespace gpr
