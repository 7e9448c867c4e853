// k_potrf_dev.h -- the POTRF row-panel routine and its 32 x 32 diagonal
// factorisation, shared by the stream kernel (one workgroup per panel) and the
// persistent executor (one task per panel). The algorithm is described in
// k_potrf.hip.
#pragma once

#include "gpr_internal.h"
#include "k_accum.h"
#include "k_common.h"

namespace gpr {

namespace potrf_detail {
constexpr int NB = 32;       // panel width
constexpr int KC = 32;       // k-chunk staged in LDS
constexpr int SP = NB + 4;   // padded LDS row
constexpr unsigned SPIN_LIMIT = 1u << 22;
}  // namespace potrf_detail
using potrf_detail::NB;
using potrf_detail::KC;
using potrf_detail::SP;
using potrf_detail::SPIN_LIMIT;

// 1 / sqrt(d) to about one ulp: the hardware estimate and two Newton steps
// y <- y (3/2 - d y^2 / 2). A pivot d <= 0 gives NaN or infinity, and the
// caller reports it.
__device__ inline double rsqrt_refined(double d)
{
    double y = __builtin_amdgcn_rsq(d);
    const double h = 0.5 * d;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// Cholesky factor and inverse of the 16 x 16 block S[r0.., r0..] (lower
// triangle read), by one wave, right-looking over four blocks of four
// columns with one reciprocal square root per pivot. Lane (g, i) =
// (lane / 16, lane % 16) holds row i, columns 4 g .. 4 g + 3, so the four
// columns of block b are held by group b. Per block: group b puts its rows
// of the block in the LDS panel; every lane of the group factors the 4 x 4
// diagonal block (redundantly) and solves its own row against it; the group
// puts the finished rows in the panel, and the lanes of later groups apply
// the four columns to their entries. Every entry receives the same fused
// multiply-adds in the same column order as a column-by-column factorisation
// (so the bits are those of that order), with three wave-level LDS
// handoffs per four columns instead of two per column. The inverse is formed
// one column per lane by forward substitution with the stored pivot
// reciprocals. On return the block of S holds L (zeros above the diagonal)
// and the block of Si holds L^{-1}. Returns the first failing local column
// or -1. dv: 16 pivot reciprocals; scratch: 80 doubles of LDS (the 16 x 4
// panel and the 16 pivots).
__device__ inline int chol_inv16(double (*S)[NB + 1], double (*Si)[NB + 1], int r0, double* dv,
                                 double* scratch, int lane)
{
    const int i = lane & 15, g = lane >> 4;
    double (*pan)[4] = reinterpret_cast<double (*)[4]>(scratch);
    double* piv = scratch + 64;
    double a[4];  // a[q] = row i, column 4 g + q
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = S[r0 + i][r0 + 4 * g + q];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int c0 = 4 * b;
        if (g == b) {
#pragma unroll
            for (int c = 0; c < 4; ++c) pan[i][c] = a[c];
        }
        wave_lds_sync();
        if (g == b) {
            // the 4 x 4 diagonal block, right-looking, column by column
            double d[4][4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c <= r; ++c) d[r][c] = pan[c0 + r][c];
            double inv[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double p = d[c][c];
                inv[c] = rsqrt_refined(p);
                if (i == 0) {
                    piv[c0 + c] = p;
                    dv[c0 + c] = inv[c];
                }
                d[c][c] = p * inv[c];
#pragma unroll
                for (int r = c + 1; r < 4; ++r) d[r][c] *= inv[c];
#pragma unroll
                for (int r = c + 1; r < 4; ++r)
#pragma unroll
                    for (int k = c + 1; k <= r; ++k) d[r][k] = fma(-d[r][c], d[k][c], d[r][k]);
            }
            if (i >= c0 + 4) {
                // a row below the block: solve it against the block
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    a[c] *= inv[c];
#pragma unroll
                    for (int k = c + 1; k < 4; ++k) a[k] = fma(-a[c], d[k][c], a[k]);
                }
            } else {
                // a row of the block (its factor, zeros above the diagonal), or
                // a row above it (upper triangle: zeros)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    double v = 0.0;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (i == c0 + r && c <= r) v = d[r][c];
                    a[c] = v;
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) pan[i][c] = a[c];
        }
        wave_lds_sync();
        if (g > b) {
            double li[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) li[c] = pan[i][c];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // a[q] -= L[i][c0 + c] L[k][c0 + c], c = 0..3 in order, in rows i >= k
                const int k = 4 * g + q;
                if (i >= k) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) a[q] = fma(-li[c], pan[k][c], a[q]);
                }
            }
        }
        wave_lds_sync();
    }
    int bad = -1;
#pragma unroll
    for (int j = 15; j >= 0; --j)
        if (!(piv[j] > 0.0)) bad = j;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = 4 * g + q;
        S[r0 + i][r0 + k] = (k <= i) ? a[q] : 0.0;
    }
    wave_lds_sync();
    double x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        double s0 = (r == i) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < r; ++k) {
            const double t = S[r0 + r][r0 + k] * x[k];
            if (k & 1) s1 -= t;
            else s0 -= t;
        }
        x[r] = (s0 + s1) * dv[r];
    }
    if (lane < 16) {
#pragma unroll
        for (int r = 0; r < 16; ++r) Si[r0 + r][r0 + i] = x[r];
    }
    wave_lds_sync();
    return bad;
}

// Cholesky factor and inverse of the 32 x 32 block in S (lower triangle read),
// by one wave, as a 2 x 2 block recursion over 16 x 16 blocks:
//     L11 = chol(A11), Y11 = L11^{-1}
//     L21 = A21 Y11^T,  S22 = A22 - L21 L21^T                (FP64 MFMA)
//     L22 = chol(S22),  Y22 = L22^{-1}
//     Y21 = -Y22 (L21 Y11)                                  (FP64 MFMA)
// which halves the sequential depth of the 32-column factorisation and its
// inverse. On return S holds L (zeros above the diagonal) and Si holds L^{-1}
// (zeros above). Returns the first failing local column or -1. dv: 32 doubles
// and col: 80 doubles of LDS scratch.
__device__ inline int factor_diag32(double (*S)[NB + 1], double (*Si)[NB + 1], double* dv,
                                    double* col, int lane)
{
    const int lr = lane & 15, lk = lane >> 4;
    int bad = chol_inv16(S, Si, 0, dv, col, lane);
    // L21 = A21 Y11^T
    dbl4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 16; k += 4) t = mfma16(S[16 + lr][k + lk], Si[lr][k + lk], t);
    wave_lds_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) S[16 + drow(lk, v)][lr] = t[v];
    wave_lds_sync();
    // S22 = A22 - L21 L21^T
    dbl4 u;
#pragma unroll
    for (int v = 0; v < 4; ++v) u[v] = S[16 + drow(lk, v)][16 + lr];
#pragma unroll
    for (int k = 0; k < 16; k += 4) u = mfma16(-S[16 + lr][k + lk], S[16 + lr][k + lk], u);
    wave_lds_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) S[16 + drow(lk, v)][16 + lr] = u[v];
    wave_lds_sync();
    const int bad2 = chol_inv16(S, Si, 16, dv + 16, col, lane);
    if (bad < 0 && bad2 >= 0) bad = 16 + bad2;
    // Y21 = -Y22 W, W = L21 Y11 (W held in the Y21 block until it is replaced)
    dbl4 w = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 16; k += 4) w = mfma16(S[16 + lr][k + lk], Si[k + lk][lr], w);
#pragma unroll
    for (int v = 0; v < 4; ++v) Si[16 + drow(lk, v)][lr] = w[v];
    wave_lds_sync();
    dbl4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 16; k += 4)
        z = mfma16(-Si[16 + lr][16 + k + lk], Si[16 + k + lk][lr], z);
    wave_lds_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) Si[16 + drow(lk, v)][lr] = z[v];
    for (int e = lane; e < 256; e += 64) {
        S[e >> 4][16 + (e & 15)] = 0.0;
        Si[e >> 4][16 + (e & 15)] = 0.0;
    }
    wave_lds_sync();
    return bad;
}

// Polls with relaxed loads (no cache invalidation per poll) and acquires once
// the flag holds the epoch. Gives up at the spin limit, or early once *err
// reports that another wait has already given up.
__device__ inline bool wait_flag(const unsigned* f, unsigned epoch, const int* err)
{
    unsigned it = 0;
    bool ok = true;
    while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
        __builtin_amdgcn_s_sleep(2);
        if (++it > SPIN_LIMIT ||
            ((it & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            ok = false;
            break;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}

__device__ inline void flag_error(int* err)
{
    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// LDS of one panel task.
struct PotrfLds {
    double As[2][KC][SP];
    double Bs[2][KC][SP];
    double Sacc[NB][NB + 1];
    double Si[NB][NB + 1];
    double dv[NB];
    double col[80];  // panel and pivots of the diagonal-block factorisation
};

// Row panel w of the POTRF of the m x m tile A (see k_potrf.hip). 256 threads;
// tid is the thread's index (0..255). syrk (nullable): an m x m tile S
// (leading dimension m) whose product S S^T is first subtracted from the
// panel's blocks (the tile's last SYRK update, run by the panel itself). Each
// element's products are summed in k order from zero and the sum subtracted
// once, as the tile-update kernels do, so the result is bitwise theirs; with
// syrk_f32 the operands are rounded to FP32 and summed by FP32-accumulator
// MFMAs, as in an FP32 tile update.
__device__ inline void potrf_panel(double* __restrict__ A, int lda, int m, double* __restrict__ Tinv,
                                   int ldt, int* __restrict__ info, int64_t col_base,
                                   unsigned* __restrict__ flags, unsigned epoch,
                                   int* __restrict__ err, int w, PotrfLds& sh, int tid,
                                   const double* __restrict__ syrk = nullptr,
                                   bool syrk_f32 = false)
{
    double (*As)[KC][SP] = sh.As;
    double (*Bs)[KC][SP] = sh.Bs;
    double (*Sacc)[NB + 1] = sh.Sacc;
    double (*Si)[NB + 1] = sh.Si;
    double* dv = sh.dv;
    const int P = m / NB;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int qi = wave >> 1, qj = wave & 1;
    const int row0 = NB * w;
    double* Aw = A + (size_t)row0 * lda;  // row panel w
    // flags[q]: off-diagonal blocks L[q, 0:q] stored; flags[P + q]: L[q, q]
    // and its inverse stored (row panel q complete)
    unsigned* off_done = flags;
    unsigned* diag_done = flags + P;

    if (syrk != nullptr) {
        // K[w, q] -= S[w rows] S[q rows]^T for q <= w; the panel owns these blocks
        for (int q = 0; q <= w; ++q) {
            if (syrk_f32) {
                const flt4a acc = accum32_f32<KC>(syrk + (size_t)row0 * m, m,
                                                  syrk + (size_t)NB * q * m, m, m, As, Bs, tid);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double* c = Aw + (size_t)(16 * qi + 4 * lk + v) * lda + NB * q + 16 * qj + lr;
                    gst(c, gld(c) - (double)acc[v]);
                }
                continue;
            }
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
            acc = accum32<true, KC, true>(syrk + (size_t)row0 * m, m, syrk + (size_t)NB * q * m, m,
                                          m, acc, 1.0, As, Bs, tid);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double* c = Aw + (size_t)(16 * qi + drow(lk, v)) * lda + NB * q + 16 * qj + lr;
                gst(c, gld(c) - acc[v]);
            }
        }
        __syncthreads();  // the updated blocks are read by every wave below
    }
    // running sum of L[w, p] L[w, p]^T over the finished blocks p < q, this
    // wave's 16 x 16 quadrant of the diagonal block
    dbl4 dacc = {0.0, 0.0, 0.0, 0.0};
    for (int q = 0; q < w; ++q) {
        // acc = K[w, q] - L[w, 0:q] L[q, 0:q]^T needs the off-diagonal blocks of
        // row panel q; the product with Dinv_q then needs its diagonal block
        if (tid == 0 && !wait_flag(off_done + q, epoch, err)) flag_error(err);
        __syncthreads();
        dbl4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            acc[v] = Aw[(size_t)(16 * qi + drow(lk, v)) * lda + NB * q + 16 * qj + lr];
        acc = accum32<true, KC>(Aw, lda, A + (size_t)NB * q * lda, lda, NB * q, acc, -1.0, As, Bs,
                                tid);
#pragma unroll
        for (int v = 0; v < 4; ++v) Sacc[16 * qi + drow(lk, v)][16 * qj + lr] = acc[v];
        if (tid == 0 && !wait_flag(diag_done + q, epoch, err)) flag_error(err);
        __syncthreads();
        // L[w, q] = acc Dinv_q^T; Dinv_q is the diagonal block q of Tinv
        const double* dq = Tinv + (size_t)(NB * q + 16 * qj + lr) * ldt + NB * q + lk;
        dbl4 o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < NB; k += 4) o = mfma16(Sacc[16 * qi + lr][k + lk], dq[k], o);
        __syncthreads();  // every read of Sacc done
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 16 * qi + drow(lk, v), c = 16 * qj + lr;
            Aw[(size_t)r * lda + NB * q + c] = o[v];
            Sacc[r][c] = o[v];
        }
        __syncthreads();
        // dacc += L[w, q] L[w, q]^T
#pragma unroll
        for (int k = 0; k < NB; k += 4)
            dacc = mfma16(Sacc[16 * qi + lr][k + lk], Sacc[16 * qj + lr][k + lk], dacc);
    }
    __syncthreads();  // Sacc reads done; L[w, 0:w] stored by every wave
    // row panel w's off-diagonal blocks are final: published by the last wave,
    // so that the release does not delay the factorisation in wave 0
    if (tid == 192) __hip_atomic_store(off_done + w, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = 16 * qi + drow(lk, v), c = 16 * qj + lr;
        Sacc[r][c] = Aw[(size_t)r * lda + row0 + c] - dacc[v];
    }
    __syncthreads();
    int bad = -1;
    if (wave == 0) bad = factor_diag32(Sacc, Si, dv, sh.col, lane);
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 256) {
        const int r = e / NB, c = e % NB;
        Aw[(size_t)r * lda + row0 + c] = Sacc[r][c];
        Tinv[(size_t)(row0 + r) * ldt + row0 + c] = Si[r][c];
    }
    // every earlier panel is complete (flags acquired), so the first failure
    // seen here in column order is the first overall
    if (tid == 0 && bad >= 0 && info != nullptr && *info == 0)
        *info = (int)(col_base + row0 + bad + 1);
    __syncthreads();
    if (tid == 0) __hip_atomic_store(diag_done + w, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    // strict upper triangle of the tile in this row panel: no other panel
    // reads it, so it is written after the handoff, off the dependency chain
    const int rest = m - row0 - NB;
    for (int e = tid; e < NB * rest; e += 256) {
        const int r = e / rest, c = e % rest;
        Aw[(size_t)r * lda + row0 + NB + c] = 0.0;
    }
}
}  // namespace gpr
