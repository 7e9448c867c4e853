/*
 * gpr_oracle.c -- plain CPU reference ("oracle") for exact Gaussian-process
 * prediction with the squared-exponential kernel.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the GPU library links, includes or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it. It shares no code with the GPU path.
 *
 * It computes the plain definitions, untiled, in textbook loop order:
 *   - kernel and covariance matrices: Sec. 4.1, eq. (1);
 *   - Cholesky K = L L^T, forward/backward substitution, mean: Sec. 4.1,
 *     eq. (2) and the solve recipe that follows it;
 *   - posterior covariance via L V = K_{X,X*}, W = V^T V: Sec. 4.1, eq. (3);
 *   - negative log marginal likelihood and its gradient (not stated in the
 *     paper; the textbook GP formulas for the kernel the paper cites);
 *   - Gauss-Jordan inversion as an independent route for small n.
 *
 * Readings of the paper taken here (listed with reasons in the design notes):
 *   - eq. (1) divides the squared distance by 2*l (not 2*l^2), as printed;
 *   - the noise term sigma^2 is an index Kronecker delta on the training set:
 *     K = k(X,X) + sigma^2 I, while k(X*,X) and k(X*,X*) carry no noise;
 *   - the third hyperparameter is the noise *variance* sigma^2;
 *   - all matrices are row-major and 0-based (Sec. 4.3).
 *
 * The arithmetic type is OR_REAL (double by default). Building with
 * -DOR_REAL="long double" gives an extended-precision copy used to measure
 * how much of any disagreement is the double oracle's own rounding. The
 * interface always takes and returns double.
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared (no -ffast-math: it changes
 * rounding and the order of sums).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>

#ifndef OR_REAL
#define OR_REAL double
#endif
typedef OR_REAL real;

#define OR_PI 3.14159265358979323846264338327950288L

/* sizeof the arithmetic type, so a caller can tell the two builds apart. */
int orc_real_bytes(void) { return (int)sizeof(real); }

/* Threads an OpenMP parallel region of this library runs with. */
int orc_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
}

/* ---------------------------------------------------------------------- */
/* Kernel, eq. (1)                                                         */
/* ---------------------------------------------------------------------- */

/* Squared Euclidean distance sum_{d=0}^{D-1} (a_d - b_d)^2, summed in
 * ascending d (eq. (1), the sum inside the exponential). */
static real sqdist(const double* a, const double* b, int D)
{
    real s = 0;
    for (int d = 0; d < D; ++d) {
        real t = (real)a[d] - (real)b[d];
        s += t * t;
    }
    return s;
}

/* Squared-exponential part of eq. (1): v * exp(-s / (2 l)). */
static real kse(const double* a, const double* b, int D, real l, real v)
{
    return v * exp(-sqdist(a, b, D) / (2 * l));
}

/* out[i*nb + j] = v exp(-|a_i - b_j|^2 / (2 l)) for the rows a_i of A
 * (na x D) and b_j of B (nb x D): the squared-exponential part of eq. (1),
 * no noise term (the cross covariance K_{X*,X} and the test block K_{X*,X*}
 * carry none under the index reading of eq. (1)'s Kronecker delta). */
void orc_kernel_matrix(const double* A, int64_t na, const double* B, int64_t nb,
                       int D, double l, double v, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < na; ++i)
        for (int64_t j = 0; j < nb; ++j)
            out[i * nb + j] = (double)kse(A + i * D, B + j * D, D, (real)l, (real)v);
}

/* Training covariance K = k(X, X) + sigma^2 I: entries with i >= j are
 * computed, then mirrored, so K is exactly symmetric. */
void orc_assemble_K(const double* X, int64_t n, int D, double l, double v,
                    double s2, double* K)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            real k = kse(X + i * D, X + j * D, D, (real)l, (real)v);
            if (i == j) k += (real)s2;
            K[i * n + j] = (double)k;
            K[j * n + i] = (double)k;
        }
}

/* ---------------------------------------------------------------------- */
/* Dense linear algebra in plain loops (working precision `real`)          */
/* ---------------------------------------------------------------------- */

/* Cholesky-Crout of the n x n SPD matrix K (only the lower triangle read):
 * for j = 0..n-1: d = K_jj - sum_{k<j} L_jk^2; stop if not d > 0;
 * L_jj = sqrt(d); L_ij = (K_ij - sum_{k<j} L_ik L_jk) / L_jj for i > j.
 * L is row-major lower triangular with zeros above the diagonal.
 * Returns 0, or the 1-based column of the first non-positive pivot. */
static int chol_real(const real* K, int64_t n, real* L)
{
    memset(L, 0, sizeof(real) * (size_t)(n * n));
    for (int64_t j = 0; j < n; ++j) {
        const real* Lj = L + j * n;
        real d = K[j * n + j];
        for (int64_t k = 0; k < j; ++k) d -= Lj[k] * Lj[k];
        if (!(d > 0)) return (int)(j + 1);
        real ljj = sqrt(d);
        L[j * n + j] = ljj;
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            const real* Li = L + i * n;
            real s = K[i * n + j];
            for (int64_t k = 0; k < j; ++k) s -= Li[k] * Lj[k];
            L[i * n + j] = s / ljj;
        }
    }
    return 0;
}

/* Forward substitution L x = b. */
static void forward_real(const real* L, int64_t n, const real* b, real* x)
{
    for (int64_t i = 0; i < n; ++i) {
        real s = b[i];
        for (int64_t k = 0; k < i; ++k) s -= L[i * n + k] * x[k];
        x[i] = s / L[i * n + i];
    }
}

/* Backward substitution L^T x = b. */
static void backward_real(const real* L, int64_t n, const real* b, real* x)
{
    for (int64_t i = n - 1; i >= 0; --i) {
        real s = b[i];
        for (int64_t k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
        x[i] = s / L[i * n + i];
    }
}

static real* to_real(const double* a, int64_t cnt)
{
    real* r = (real*)malloc(sizeof(real) * (size_t)(cnt > 0 ? cnt : 1));
    if (!r) return NULL;
    for (int64_t i = 0; i < cnt; ++i) r[i] = (real)a[i];
    return r;
}

static void to_double(const real* a, int64_t cnt, double* out)
{
    for (int64_t i = 0; i < cnt; ++i) out[i] = (double)a[i];
}

/* Public wrappers over the working-precision routines. */

int orc_cholesky(const double* K, int64_t n, double* L)
{
    real* Kr = to_real(K, n * n);
    real* Lr = (real*)malloc(sizeof(real) * (size_t)(n * n > 0 ? n * n : 1));
    if (!Kr || !Lr) { free(Kr); free(Lr); return -1; }
    int info = chol_real(Kr, n, Lr);
    to_double(Lr, n * n, L);
    free(Kr); free(Lr);
    return info;
}

void orc_forward(const double* L, int64_t n, const double* b, double* x)
{
    real* Lr = to_real(L, n * n);
    real* br = to_real(b, n);
    real* xr = to_real(b, n);
    forward_real(Lr, n, br, xr);
    to_double(xr, n, x);
    free(Lr); free(br); free(xr);
}

void orc_backward(const double* L, int64_t n, const double* b, double* x)
{
    real* Lr = to_real(L, n * n);
    real* br = to_real(b, n);
    real* xr = to_real(b, n);
    backward_real(Lr, n, br, xr);
    to_double(xr, n, x);
    free(Lr); free(br); free(xr);
}

/* ---------------------------------------------------------------------- */
/* Prediction, eqs. (2) and (3)                                            */
/* ---------------------------------------------------------------------- */

/* Full exact-GP prediction from the plain definitions.
 *   K   = k(X,X) + sigma^2 I       (eq. (1), noise by index)
 *   Ks  = k(X*, X)   (n* x n)      (no noise)
 *   Kss = k(X*, X*)  (n* x n*)     (no noise)
 *   K = L L^T; L beta = y; L^T alpha = beta          (eq. (2) recipe)
 *   mean_i = sum_j Ks_ij alpha_j                      (eq. (2))
 *   V^T row c = forward solve of L v = Ks[c, :]^T      (L V = K_{X,X*})
 *   cov_ij = Kss_ij - sum_k Vt_ik Vt_jk, i >= j, mirrored (eq. (3))
 * Outputs (any may be NULL): L (n x n, zeros above the diagonal), alpha (n),
 * beta (n), mean (n*), cov (n* x n*, both triangles).
 * Returns 0, the 1-based column of a failed pivot, or -1 on allocation
 * failure. */
int orc_predict(const double* X, const double* y, int64_t n,
                const double* Xs, int64_t ns, int D,
                double l, double v, double s2,
                double* L_out, double* beta_out, double* alpha_out,
                double* mean_out, double* cov_out)
{
    real lr = (real)l, vr = (real)v, s2r = (real)s2;
    real* K = (real*)malloc(sizeof(real) * (size_t)(n * n));
    real* L = (real*)malloc(sizeof(real) * (size_t)(n * n));
    real* yr = to_real(y, n);
    real* beta = (real*)malloc(sizeof(real) * (size_t)n);
    real* alpha = (real*)malloc(sizeof(real) * (size_t)n);
    real* Ks = (real*)malloc(sizeof(real) * (size_t)(ns * n > 0 ? ns * n : 1));
    if (!K || !L || !yr || !beta || !alpha || !Ks) {
        free(K); free(L); free(yr); free(beta); free(alpha); free(Ks);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            real k = kse(X + i * D, X + j * D, D, lr, vr);
            if (i == j) k += s2r;
            K[i * n + j] = k;
            K[j * n + i] = k;
        }
    int info = chol_real(K, n, L);
    free(K);
    if (info) {
        if (L_out) to_double(L, n * n, L_out);
        free(L); free(yr); free(beta); free(alpha); free(Ks);
        return info;
    }
    forward_real(L, n, yr, beta);
    backward_real(L, n, beta, alpha);

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ns; ++i)
        for (int64_t j = 0; j < n; ++j)
            Ks[i * n + j] = kse(Xs + i * D, X + j * D, D, lr, vr);

    if (mean_out) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < ns; ++i) {
            real s = 0;
            for (int64_t j = 0; j < n; ++j) s += Ks[i * n + j] * alpha[j];
            mean_out[i] = (double)s;
        }
    }
    if (cov_out) {
        real* Vt = (real*)malloc(sizeof(real) * (size_t)(ns * n > 0 ? ns * n : 1));
        if (!Vt) { free(L); free(yr); free(beta); free(alpha); free(Ks); return -1; }
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < ns; ++c)
            forward_real(L, n, Ks + c * n, Vt + c * n);
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t i = 0; i < ns; ++i)
            for (int64_t j = 0; j <= i; ++j) {
                real s = kse(Xs + i * D, Xs + j * D, D, lr, vr);
                const real* vi = Vt + i * n;
                const real* vj = Vt + j * n;
                for (int64_t k = 0; k < n; ++k) s -= vi[k] * vj[k];
                cov_out[i * ns + j] = (double)s;
                cov_out[j * ns + i] = (double)s;
            }
        free(Vt);
    }
    if (L_out) to_double(L, n * n, L_out);
    if (beta_out) to_double(beta, n, beta_out);
    if (alpha_out) to_double(alpha, n, alpha_out);
    free(L); free(yr); free(beta); free(alpha); free(Ks);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Negative log marginal likelihood and gradient                           */
/* ---------------------------------------------------------------------- */

/* NLML = 1/2 y^T alpha + sum_i log L_ii + (n/2) log(2 pi), and its gradient
 * with respect to (l, v, sigma^2) from the trace formula
 *   dNLML/dtheta = 1/2 tr((K^{-1} - alpha alpha^T) dK/dtheta),
 * computed through the explicit inverse: Linv column j by forward
 * substitution of L x = e_j, then K^{-1} = Linv^T Linv. With
 * e_ij = exp(-s_ij / (2 l)) and A = K^{-1} - alpha alpha^T:
 *   dK/dv = e, dK/dsigma^2 = I, dK/dl = v e s / (2 l^2)   (eq. (1) as printed).
 * Either output pointer may be NULL. Returns 0, a pivot column, or -1. */
int orc_nlml_grad(const double* X, const double* y, int64_t n, int D,
                  double l, double v, double s2, double* nlml_out, double* grad3)
{
    real lr = (real)l, vr = (real)v, s2r = (real)s2;
    size_t nn = (size_t)(n * n);
    real* K = (real*)malloc(sizeof(real) * nn);
    real* L = (real*)malloc(sizeof(real) * nn);
    real* yr = to_real(y, n);
    real* beta = (real*)malloc(sizeof(real) * (size_t)n);
    real* alpha = (real*)malloc(sizeof(real) * (size_t)n);
    if (!K || !L || !yr || !beta || !alpha) {
        free(K); free(L); free(yr); free(beta); free(alpha);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            real k = kse(X + i * D, X + j * D, D, lr, vr);
            if (i == j) k += s2r;
            K[i * n + j] = k;
            K[j * n + i] = k;
        }
    int info = chol_real(K, n, L);
    if (info) { free(K); free(L); free(yr); free(beta); free(alpha); return info; }
    forward_real(L, n, yr, beta);
    backward_real(L, n, beta, alpha);

    if (nlml_out) {
        real quad = 0, logdet = 0;
        for (int64_t i = 0; i < n; ++i) quad += yr[i] * alpha[i];
        for (int64_t i = 0; i < n; ++i) logdet += log(L[i * n + i]);
        *nlml_out = (double)(quad / 2 + logdet + (real)n / 2 * log(2 * (real)OR_PI));
    }
    if (grad3) {
        /* LinvT[j][i] = (L^{-1})_{ij}; row j of LinvT is column j of L^{-1}. */
        real* LinvT = K; /* reuse storage: K is no longer needed */
        memset(LinvT, 0, sizeof(real) * nn);
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t j = 0; j < n; ++j) {
            real* x = LinvT + j * n;
            for (int64_t i = j; i < n; ++i) {
                real s = (i == j) ? 1 : 0;
                for (int64_t k = j; k < i; ++k) s -= L[i * n + k] * x[k];
                x[i] = s / L[i * n + i];
            }
        }
        /* A_ij = (K^{-1})_ij - alpha_i alpha_j, with
         * (K^{-1})_ij = sum_k (L^{-1})_{ki} (L^{-1})_{kj} = sum_k LinvT[i][k] LinvT[j][k]. */
        real gv = 0, gs = 0, gl = 0;
        real* rowv = (real*)calloc((size_t)n, sizeof(real));
        real* rowl = (real*)calloc((size_t)n, sizeof(real));
        real* rows = (real*)calloc((size_t)n, sizeof(real));
        if (!rowv || !rowl || !rows) {
            free(rowv); free(rowl); free(rows);
            free(K); free(L); free(yr); free(beta); free(alpha);
            return -1;
        }
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t i = 0; i < n; ++i) {
            real sv = 0, sl = 0;
            for (int64_t j = 0; j < n; ++j) {
                int64_t k0 = i > j ? i : j;
                real kinv = 0;
                for (int64_t k = k0; k < n; ++k) kinv += LinvT[i * n + k] * LinvT[j * n + k];
                real a = kinv - alpha[i] * alpha[j];
                real s = sqdist(X + i * D, X + j * D, D);
                real e = exp(-s / (2 * lr));
                sv += a * e;
                sl += a * vr * e * s / (2 * lr * lr);
                if (i == j) rows[i] = a;
            }
            rowv[i] = sv;
            rowl[i] = sl;
        }
        for (int64_t i = 0; i < n; ++i) { gv += rowv[i]; gl += rowl[i]; gs += rows[i]; }
        grad3[0] = (double)(gl / 2);
        grad3[1] = (double)(gv / 2);
        grad3[2] = (double)(gs / 2);
        free(rowv); free(rowl); free(rows);
    }
    free(K); free(L); free(yr); free(beta); free(alpha);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Independent route: Gauss-Jordan inversion with partial pivoting         */
/* ---------------------------------------------------------------------- */

/* Ainv = A^{-1} for a general n x n matrix by Gauss-Jordan elimination on
 * [A | I] with partial (row) pivoting. Meant for n <= 64. Returns 0, or 1 if
 * a pivot is exactly zero. */
int orc_gauss_jordan_inverse(const double* A, int64_t n, double* Ainv)
{
    int64_t w = 2 * n;
    real* M = (real*)calloc((size_t)(n * w > 0 ? n * w : 1), sizeof(real));
    if (!M) return -1;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) M[i * w + j] = (real)A[i * n + j];
        M[i * w + n + i] = 1;
    }
    for (int64_t c = 0; c < n; ++c) {
        int64_t p = c;
        real best = fabs(M[c * w + c]);
        for (int64_t r = c + 1; r < n; ++r)
            if (fabs(M[r * w + c]) > best) { best = fabs(M[r * w + c]); p = r; }
        if (best == 0) { free(M); return 1; }
        if (p != c)
            for (int64_t j = 0; j < w; ++j) {
                real t = M[c * w + j]; M[c * w + j] = M[p * w + j]; M[p * w + j] = t;
            }
        real piv = M[c * w + c];
        for (int64_t j = 0; j < w; ++j) M[c * w + j] /= piv;
        for (int64_t r = 0; r < n; ++r) {
            if (r == c) continue;
            real f = M[r * w + c];
            if (f == 0) continue;
            for (int64_t j = 0; j < w; ++j) M[r * w + j] -= f * M[c * w + j];
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) Ainv[i * n + j] = (double)M[i * w + n + j];
    free(M);
    return 0;
}
