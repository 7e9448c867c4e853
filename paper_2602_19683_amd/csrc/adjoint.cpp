// adjoint.cpp -- task plan of the reverse (adjoint) sweep of the tiled
// Cholesky of Fig. 1, for the NLML gradient.
//
// Reverse-mode differentiation of the right-looking tile algorithm
//   POTRF  L_JJ = chol(A_JJ)
//   TRSM   L_IJ = A_IJ L_JJ^{-T}                       (I > J)
//   update A_IK -= L_IJ L_KJ^T                         (J < K <= I)
// visits the steps in reverse. Given the adjoint Lbar of the factor (lower
// tiles), it produces Abar, the adjoint of the lower triangle of K: for every
// perturbation dK, d f = sum_{i >= j} Abar_ij dK_ij. With B = Abar + Abar^T
// (the symmetric matrix; diagonal entries doubled) and Tinv_K = L_KK^{-1},
// step K (K = M-1 down to 0) is:
//   TRSM adjoint   Abar_IK = Lbar_IK Tinv_K                         (I > K)
//   diagonal sum   Lbar_KK -= tril(sum_{R>K} Abar_RK^T L_RK)
//   POTRF adjoint  G = the symmetric matrix with lower triangle L_KK^T tril(Lbar_KK),
//                  Abar_KK = Phi(Tinv_K^T G Tinv_K)   (Phi: lower, diagonal halved)
//   push           Lbar_RJ -= B_RK L_KJ   for every J < K and R > J, i.e.
//                    row K:   Lbar_KJ -= sum_{R>K} Abar_RK^T L_RJ + (Abar_KK + Abar_KK^T) L_KJ
//                    R > K:   Lbar_RJ -= Abar_RK L_KJ.
// (POTRF adjoint: from dK = dL L^T + L dL^T, L^{-1} dL = Phi(L^{-1} dK L^{-T}), so
// <Lbar, dL> = <L^{-T} Phi(L^T Lbar) L^{-1}, dK>; summed over the two triangles
// this is Phi(S + S^T) with S + S^T = Tinv^T G Tinv.)
//
// The row-K sums over R are long and feed few output tiles, so they run
// split-K: chunks of G consecutive R go to separate partial tiles (one task
// each, many workgroups), and the task that consumes them adds the partials in
// chunk order (fixed order: the result is deterministic).
#include <algorithm>

#include "gpr_internal.h"

namespace gpr {

namespace {

struct PB {
    AdjPlan P;
    int launch_begin(int kind, int step)
    {
        P.launches.push_back({kind, step, (int)P.tasks.size(), 0});
        return (int)P.launches.size() - 1;
    }
    void task(AdjRef out, AdjRef cin, int part0, int npart, int epi,
              std::initializer_list<AdjTerm> terms)
    {
        AdjTask t{out, cin, part0, npart, (int)P.terms.size(), (int)terms.size(), epi};
        for (const auto& x : terms) P.terms.push_back(x);
        P.tasks.push_back(t);
        P.launches.back().count += 1;
    }
    void task_terms(AdjRef out, AdjRef cin, int part0, int npart, int epi,
                    const std::vector<AdjTerm>& terms)
    {
        AdjTask t{out, cin, part0, npart, (int)P.terms.size(), (int)terms.size(), epi};
        P.terms.insert(P.terms.end(), terms.begin(), terms.end());
        P.tasks.push_back(t);
        P.launches.back().count += 1;
    }
};

constexpr AdjRef NONE{AM_NONE, 0, 0};
AdjRef R_(int mat, int I, int J) { return AdjRef{mat, I, J}; }

}  // namespace

AdjPlan build_adjoint(int M, int G)
{
    PB b;
    if (G < 1) G = 1;
    for (int K = M - 1; K >= 0; --K) {
        const int nt = M - K - 1;          // tile rows below the diagonal tile
        const int C = (nt + G - 1) / G;    // chunks of the row-K sums
        if (nt > 0) {
            // TRSM adjoint
            b.launch_begin(AK_TRSM, K);
            for (int I = K + 1; I < M; ++I)
                b.task(R_(AM_ABAR, I, K), NONE, 0, 0, TG_EPI_NONE,
                       {AdjTerm{R_(AM_LBAR, I, K), R_(AM_TINV, K, K), 1, TG_TRI_B}});
            // partial sums -sum_{R in chunk} Abar_RK^T L_RJ for J = 0 .. K
            b.launch_begin(AK_PART, K);
            for (int J = K; J >= 0; --J)  // the diagonal tile's partials first
                for (int c = 0; c < C; ++c) {
                    std::vector<AdjTerm> t;
                    for (int R = K + 1 + c * G; R < std::min(M, K + 1 + (c + 1) * G); ++R)
                        t.push_back({R_(AM_ABAR, R, K), R_(AM_L, R, J), -1, TG_TRANS_A});
                    b.task_terms(R_(AM_PART, J * C + c, 0), NONE, 0, 0, TG_EPI_NONE, t);
                }
            b.P.max_part = std::max(b.P.max_part, (K + 1) * C);
            // Q = Lbar_KK + sum of its partials
            b.launch_begin(AK_DIAG_SUM, K);
            b.task(R_(AM_Q, 0, 0), R_(AM_LBAR, K, K), K * C, C, TG_EPI_NONE, {});
        }
        const AdjRef Q = nt > 0 ? R_(AM_Q, 0, 0) : R_(AM_LBAR, K, K);
        // POTRF adjoint: three products on single tiles
        b.launch_begin(AK_POTRF, K);
        b.task(R_(AM_G, 0, 0), NONE, 0, 0, TG_EPI_SYM,
               {AdjTerm{R_(AM_L, K, K), Q, 1, TG_TRANS_A | TG_TRI_A | TG_TRI_B}});
        b.launch_begin(AK_POTRF, K);
        b.task(R_(AM_X, 0, 0), NONE, 0, 0, TG_EPI_NONE,
               {AdjTerm{R_(AM_G, 0, 0), R_(AM_TINV, K, K), 1, TG_TRI_B}});
        b.launch_begin(AK_POTRF, K);
        b.task(R_(AM_ABAR, K, K), NONE, 0, 0, TG_EPI_PHI,
               {AdjTerm{R_(AM_TINV, K, K), R_(AM_X, 0, 0), 1, TG_TRANS_A | TG_TRI_A}});
        // push into the columns J < K
        if (K > 0) {
            b.launch_begin(AK_PUSH, K);
            for (int J = K - 1; J >= 0; --J) {  // column K-1 (needed next) first
                b.task(R_(AM_LBAR, K, J), R_(AM_LBAR, K, J), nt > 0 ? J * C : 0, nt > 0 ? C : 0,
                       TG_EPI_NONE,
                       {AdjTerm{R_(AM_ABAR, K, K), R_(AM_L, K, J), -1, 0},
                        AdjTerm{R_(AM_ABAR, K, K), R_(AM_L, K, J), -1, TG_TRANS_A}});
                for (int R = K + 1; R < M; ++R)
                    b.task(R_(AM_LBAR, R, J), R_(AM_LBAR, R, J), 0, 0, TG_EPI_NONE,
                           {AdjTerm{R_(AM_ABAR, R, K), R_(AM_L, K, J), -1, 0}});
            }
        }
    }
    return b.P;
}

}  // namespace gpr

// Flattened export for host-side checks (see gpr.h).
extern "C" int gpr_adjoint_describe(int32_t M, int32_t G, int32_t* tasks, int64_t task_cap,
                                    int64_t* n_tasks, int32_t* terms, int64_t term_cap,
                                    int64_t* n_terms, int32_t* launches, int64_t launch_cap,
                                    int64_t* n_launches)
{
    if (M < 1 || G < 1 || !n_tasks || !n_terms || !n_launches) return GPR_EINVAL;
    gpr::AdjPlan P = gpr::build_adjoint(M, G);
    *n_tasks = (int64_t)P.tasks.size();
    *n_terms = (int64_t)P.terms.size();
    *n_launches = (int64_t)P.launches.size();
    if (*n_tasks > task_cap || *n_terms > term_cap || *n_launches > launch_cap) return GPR_EINVAL;
    if (tasks)
        for (size_t i = 0; i < P.tasks.size(); ++i) {
            const auto& t = P.tasks[i];
            int32_t* o = tasks + 12 * i;
            o[0] = t.out.mat; o[1] = t.out.I; o[2] = t.out.J;
            o[3] = t.cin.mat; o[4] = t.cin.I; o[5] = t.cin.J;
            o[6] = t.part0; o[7] = t.npart; o[8] = t.first_term; o[9] = t.nterm;
            o[10] = t.epi; o[11] = 0;
        }
    if (terms)
        for (size_t i = 0; i < P.terms.size(); ++i) {
            const auto& t = P.terms[i];
            int32_t* o = terms + 8 * i;
            o[0] = t.A.mat; o[1] = t.A.I; o[2] = t.A.J;
            o[3] = t.B.mat; o[4] = t.B.I; o[5] = t.B.J;
            o[6] = t.alpha; o[7] = t.flags;
        }
    if (launches)
        for (size_t i = 0; i < P.launches.size(); ++i) {
            const auto& L = P.launches[i];
            int32_t* o = launches + 4 * i;
            o[0] = L.kind; o[1] = L.step; o[2] = L.first; o[3] = L.count;
        }
    return GPR_OK;
}
