// k_tgemm.hip -- batched tile products for the reverse (adjoint) sweep of the
// tiled Cholesky:
//     C = beta Cin + sum_t alpha_t op(A_t) op(B_t) + sum_p Part_p,
// op = identity or transpose, every operand an m x m row-major tile, with an
// optional epilogue (Phi: lower triangle with the diagonal halved; or the
// symmetric matrix whose lower triangle is the result). One workgroup per
// BM x BM block of an output tile accumulates all terms of its task in
// registers (FP64 MFMA 16x16x4), so each output block is written once by one
// workgroup: deterministic, no atomics. Operands are staged through LDS in
// k-major slices of 16, double buffered across the (term, slice) sequence.
// The 128 x 128 block uses 8 waves of 64 x 32 (four waves per SIMD at two
// workgroups per compute unit, without register spills).
#include "gpr_internal.h"
#include "k_common.h"

namespace gpr {

template <int BM, int WR, int WC>
__global__ __launch_bounds__(WR * WC * 64, WR * WC / 2) void k_tgemm_f64(
    const TGemmTask* __restrict__ tasks, const TGemmTerm* __restrict__ terms, int m)
{
    constexpr int NT = WR * WC * 64;
    constexpr int KB = 16;
    constexpr int TR = BM / WR / 16, TC = BM / WC / 16;
    constexpr int LD = BM + 4;
    constexpr int NLD = BM * KB / 2 / NT;
    __shared__ double As[2][KB][LD];
    __shared__ double Bs[2][KB][LD];

    const int nb = m / BM;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int t = lid / (nb * nb);
    const int sub = lid - t * nb * nb;
    const int bi = sub / nb, bj = sub - bi * nb;
    const TGemmTask tk = tasks[t];
    if (tk.epi == TG_EPI_SYM && bj > bi) return;  // mirrored from block (bj, bi)
    const int i0 = bi * BM, j0 = bj * BM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave / WC) * (BM / WR), wc = (wave % WC) * (BM / WC);
    const int lr = lane & 15, lk = lane >> 4;

    dbl4 acc[TR][TC];
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    const int nks = m / KB;
    const int total = tk.nterm * nks;
    double2 ra[NLD], rb[NLD];
    double alpha = 0.0;
    int flags = 0;

    // Global -> registers for slice s. Element (r, kk) of op(A) restricted to
    // rows i0.., and (kk, c) of op(B) restricted to columns j0..; a masked
    // operand reads zero above the diagonal of its stored tile.
    auto gload = [&](int s) {
        const TGemmTerm tm = terms[tk.first_term + s / nks];
        const int k0 = (s % nks) * KB;
        alpha = tm.alpha;
        flags = tm.flags;
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const int e = tid + NT * u;
            int srow, scol;
            if (!(tm.flags & TG_TRANS_A)) {
                const int r = e / (KB / 2), kk = (e % (KB / 2)) * 2;
                srow = i0 + r;
                scol = k0 + kk;
                ra[u] = gld2(tm.A + (size_t)srow * tm.lda + scol);
                if (tm.flags & TG_TRI_A) {
                    if (scol > srow) ra[u].x = 0.0;
                    if (scol + 1 > srow) ra[u].y = 0.0;
                }
            } else {
                const int kk = e / (BM / 2), r = (e % (BM / 2)) * 2;
                srow = k0 + kk;
                scol = i0 + r;
                ra[u] = gld2(tm.A + (size_t)srow * tm.lda + scol);
                if (tm.flags & TG_TRI_A) {
                    if (scol > srow) ra[u].x = 0.0;
                    if (scol + 1 > srow) ra[u].y = 0.0;
                }
            }
            if (tm.flags & TG_TRANS_B) {
                const int c = e / (KB / 2), kk = (e % (KB / 2)) * 2;
                srow = j0 + c;
                scol = k0 + kk;
                rb[u] = gld2(tm.B + (size_t)srow * tm.ldb + scol);
                if (tm.flags & TG_TRI_B) {
                    if (scol > srow) rb[u].x = 0.0;
                    if (scol + 1 > srow) rb[u].y = 0.0;
                }
            } else {
                const int kk = e / (BM / 2), c = (e % (BM / 2)) * 2;
                srow = k0 + kk;
                scol = j0 + c;
                rb[u] = gld2(tm.B + (size_t)srow * tm.ldb + scol);
                if (tm.flags & TG_TRI_B) {
                    if (scol > srow) rb[u].x = 0.0;
                    if (scol + 1 > srow) rb[u].y = 0.0;
                }
            }
        }
    };
    // Registers -> LDS buffer, k-major; alpha is folded into op(A).
    auto swrite = [&](int buf) {
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const int e = tid + NT * u;
            if (!(flags & TG_TRANS_A)) {
                const int r = e / (KB / 2), kk = (e % (KB / 2)) * 2;
                As[buf][kk][r] = alpha * ra[u].x;
                As[buf][kk + 1][r] = alpha * ra[u].y;
            } else {
                const int kk = e / (BM / 2), r = (e % (BM / 2)) * 2;
                As[buf][kk][r] = alpha * ra[u].x;
                As[buf][kk][r + 1] = alpha * ra[u].y;
            }
            if (flags & TG_TRANS_B) {
                const int c = e / (KB / 2), kk = (e % (KB / 2)) * 2;
                Bs[buf][kk][c] = rb[u].x;
                Bs[buf][kk + 1][c] = rb[u].y;
            } else {
                const int kk = e / (BM / 2), c = (e % (BM / 2)) * 2;
                Bs[buf][kk][c] = rb[u].x;
                Bs[buf][kk][c + 1] = rb[u].y;
            }
        }
    };

    if (total > 0) {
        gload(0);
        swrite(0);
        __syncthreads();
        for (int s = 0; s < total; ++s) {
            const int cur = s & 1;
            if (s + 1 < total) gload(s + 1);
#pragma unroll
            for (int kk = 0; kk < KB; kk += 4) {
                double a[TR], b[TC];
#pragma unroll
                for (int i = 0; i < TR; ++i) a[i] = As[cur][kk + lk][wr + 16 * i + lr];
#pragma unroll
                for (int j = 0; j < TC; ++j) b[j] = Bs[cur][kk + lk][wc + 16 * j + lr];
#pragma unroll
                for (int i = 0; i < TR; ++i)
#pragma unroll
                    for (int j = 0; j < TC; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
            }
            if (s + 1 < total) swrite(cur ^ 1);
            __syncthreads();
        }
    }

    // Epilogue: each input tile (Cin, then the partial tiles) is read for all
    // of this lane's elements before anything is added or written (C may be
    // Cin, so per-element load-add-store sequences would serialise); every
    // element still sums acc + beta Cin + part 0 + part 1 + ... in that order.
    double val[TR][TC][4];
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) val[i][j][v] = acc[i][j][v];
    auto addtile = [&](const double* T, int ld, double f) {
        double t[TR][TC][4];
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
            for (int j = 0; j < TC; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    t[i][j][v] = gld(T + (size_t)(i0 + wr + 16 * i + drow(lk, v)) * ld + j0 + wc +
                                     16 * j + lr);
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
            for (int j = 0; j < TC; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) val[i][j][v] += f * t[i][j][v];
    };
    if (tk.beta != 0.0) addtile(tk.Cin, tk.ldcin, tk.beta);
    for (int p = 0; p < tk.npart; ++p) addtile(tk.part + (size_t)p * tk.part_stride, m, 1.0);
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = i0 + wr + 16 * i + drow(lk, v);
                const int gj = j0 + wc + 16 * j + lr;
                const double x = val[i][j][v];
                if (tk.epi == TG_EPI_PHI) {
                    gst(tk.C + (size_t)gi * tk.ldc + gj, gj > gi ? 0.0 : (gj == gi ? 0.5 * x : x));
                } else if (tk.epi == TG_EPI_SYM) {
                    if (gi >= gj) gst(tk.C + (size_t)gi * tk.ldc + gj, x);
                    if (gi > gj) gst(tk.C + (size_t)gj * tk.ldc + gi, x);
                } else {
                    gst(tk.C + (size_t)gi * tk.ldc + gj, x);
                }
            }
}

int tgemm_block(int ntask, int m)
{
    // the largest block that still gives a launch about two workgroups per
    // CU (128-row blocks) or four (64-row blocks): measured best for 8 to 128
    // tasks per launch of 256 and 512 tiles
    if (m % 128 == 0 && (long)ntask * (m / 128) * (m / 128) >= 512) return 128;
    if (m % 64 == 0 && (long)ntask * (m / 64) * (m / 64) >= 1024) return 64;
    return 32;
}

hipError_t launch_tgemm_f64(const TGemmTask* d_tasks, int ntask, const TGemmTerm* d_terms, int m,
                            int bm, hipStream_t s)
{
    if (ntask <= 0) return hipSuccess;
    const int nb = m / bm;
    const dim3 grid(ntask * nb * nb);
    if (bm == 128)
        hipLaunchKernelGGL((k_tgemm_f64<128, 2, 4>), grid, dim3(512), 0, s, d_tasks, d_terms, m);
    else if (bm == 64)
        hipLaunchKernelGGL((k_tgemm_f64<64, 2, 2>), grid, dim3(256), 0, s, d_tasks, d_terms, m);
    else
        hipLaunchKernelGGL((k_tgemm_f64<32, 2, 2>), grid, dim3(256), 0, s, d_tasks, d_terms, m);
    return hipGetLastError();
}

}  // namespace gpr
