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
// The sweep is run left-looking ("pull"): no step pushes into later columns.
// Collecting the pushes that tile (I, J), I > J, receives from the steps
// K > J gives its final value just before step J needs it:
//   Lbar_IJ -= sum_{R>I} Abar_RI^T L_RJ + (Abar_II + Abar_II^T) L_IJ
//              + sum_{J<K<I} Abar_IK L_KJ                        (M - J terms)
// and the diagonal tile only receives the row sum of its own step:
//   Q = Lbar_JJ - sum_{R>J} Abar_RJ^T L_RJ.
// Step J (J = M-1 down to 0) therefore runs: the pulls of column J (deep
// products, M - J terms each), the TRSM adjoint of column J, the diagonal
// row sum, and the POTRF adjoint. The long sums run split-K: chunks of G
// consecutive terms go to separate partial tiles (one task each, many
// workgroups), and the task that consumes them adds the partials in chunk
// order (fixed order: the result is deterministic).
//
// Look-ahead on two streams: the pull terms of column J that involve only
// the columns >= J + 2 ("early": all but the terms with column J + 1) are
// final once step J + 2 is done, so they run on a second stream while step
// J + 1 runs its chain (TRSM adjoint, row sum, POTRF adjoint) on the caller's
// stream; the terms with column J + 1 ("late") follow on the caller's stream.
// Partial tiles alternate between two sets by the parity of J, so the early
// pulls of one step never overwrite partials another step still reads.
#include <algorithm>

#include "gpr_internal.h"

namespace gpr {

namespace {

struct PB {
    AdjPlan P;
    int launch_begin(int kind, int step, int stream = 0, int wait = -1)
    {
        P.launches.push_back({kind, step, (int)P.tasks.size(), 0, stream, wait});
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
    // drops an empty launch just begun (no tasks)
    void drop_if_empty()
    {
        if (!P.launches.empty() && P.launches.back().count == 0) P.launches.pop_back();
    }
};

constexpr AdjRef NONE{AM_NONE, 0, 0};
AdjRef R_(int mat, int I, int J) { return AdjRef{mat, I, J}; }

}  // namespace

namespace {

// The pull terms of tile (I, J), I > J, split by whether they involve column
// J + 1 (late) or only columns >= J + 2 (early).
void pull_terms(int M, int I, int J, std::vector<AdjTerm>& early, std::vector<AdjTerm>& late)
{
    early.clear();
    late.clear();
    std::vector<AdjTerm>& colI = (I == J + 1) ? late : early;
    for (int R = I + 1; R < M; ++R)
        colI.push_back({R_(AM_ABAR, R, I), R_(AM_L, R, J), -1, TG_TRANS_A});
    colI.push_back({R_(AM_ABAR, I, I), R_(AM_L, I, J), -1, 0});
    colI.push_back({R_(AM_ABAR, I, I), R_(AM_L, I, J), -1, TG_TRANS_A});
    for (int K = J + 1; K < I; ++K)
        (K == J + 1 ? late : early).push_back({R_(AM_ABAR, I, K), R_(AM_L, K, J), -1, 0});
}

int chunks(size_t n, int G) { return (int)((n + (size_t)G - 1) / (size_t)G); }

}  // namespace

AdjPlan build_adjoint(int M, int G)
{
    PB b;
    if (G < 1) G = 1;
    // partial tiles per step: the pulls (early chunks, then late chunks, tile
    // by tile), or the diagonal row sum; two sets, by the parity of the step
    std::vector<AdjTerm> e, l;
    int per_step = 1;
    for (int J = 0; J < M; ++J) {
        int p = 0;
        for (int I = J + 1; I < M; ++I) {
            pull_terms(M, I, J, e, l);
            p += chunks(e.size(), G) + chunks(l.size(), G);
        }
        per_step = std::max({per_step, p, chunks((size_t)(M - J - 1), G)});
    }
    b.P.max_part = 2 * per_step;
    auto set0 = [&](int J) { return (J & 1) * per_step; };
    // partial-tile layout of step J: tile I's early chunks at early0[I], its
    // late chunks right after them
    auto layout = [&](int J, std::vector<int>& early0, std::vector<int>& ne, std::vector<int>& nl) {
        early0.assign(M, 0);
        ne.assign(M, 0);
        nl.assign(M, 0);
        int p = set0(J);
        for (int I = J + 1; I < M; ++I) {
            pull_terms(M, I, J, e, l);
            early0[I] = p;
            ne[I] = chunks(e.size(), G);
            nl[I] = chunks(l.size(), G);
            p += ne[I] + nl[I];
        }
    };
    auto emit_chunks = [&](const std::vector<AdjTerm>& t, int p0) {
        for (size_t c = 0; c < t.size(); c += (size_t)G) {
            const std::vector<AdjTerm> chunk(t.begin() + c, t.begin() + std::min(t.size(), c + G));
            b.task_terms(R_(AM_PART, p0++, 0), NONE, 0, 0, TG_EPI_NONE, chunk);
        }
    };
    // the early pulls of column J, on the second stream after `after`
    std::vector<int> early_launch(M, -1);
    auto emit_early = [&](int J, int after) {
        if (J < 0) return;
        std::vector<int> e0, ne, nl;
        layout(J, e0, ne, nl);
        b.launch_begin(AK_PART, J, 1, after);
        for (int I = J + 1; I < M; ++I) {
            pull_terms(M, I, J, e, l);
            emit_chunks(e, e0[I]);
        }
        if (b.P.launches.back().count == 0) b.drop_if_empty();
        else early_launch[J] = (int)b.P.launches.size() - 1;
    };
    // column M - 2 has no early terms (its only tile row is M - 1 = J + 1)
    for (int J = M - 1; J >= 0; --J) {
        const int nt = M - J - 1;  // tile rows below the diagonal tile
        if (nt > 0) {
            std::vector<int> e0, ne, nl;
            layout(J, e0, ne, nl);
            // late pulls (the terms with column J + 1)
            b.launch_begin(AK_PART, J);
            for (int I = J + 1; I < M; ++I) {
                pull_terms(M, I, J, e, l);
                emit_chunks(l, e0[I] + ne[I]);
            }
            b.drop_if_empty();
            // Lbar_IJ += its partials (early, then late), in place
            b.launch_begin(AK_PUSH, J, 0, early_launch[J]);
            for (int I = J + 1; I < M; ++I)
                b.task(R_(AM_LBAR, I, J), R_(AM_LBAR, I, J), e0[I], ne[I] + nl[I], TG_EPI_NONE,
                       {});
            // TRSM adjoint
            b.launch_begin(AK_TRSM, J);
            for (int I = J + 1; I < M; ++I)
                b.task(R_(AM_ABAR, I, J), NONE, 0, 0, TG_EPI_NONE,
                       {AdjTerm{R_(AM_LBAR, I, J), R_(AM_TINV, J, J), 1, TG_TRI_B}});
            // the diagonal tile's row sum -sum_{R>J} Abar_RJ^T L_RJ, in chunks
            b.launch_begin(AK_PART, J);
            const int C = chunks((size_t)nt, G);
            for (int c = 0; c < C; ++c) {
                std::vector<AdjTerm> t;
                for (int R = J + 1 + c * G; R < std::min(M, J + 1 + (c + 1) * G); ++R)
                    t.push_back({R_(AM_ABAR, R, J), R_(AM_L, R, J), -1, TG_TRANS_A});
                b.task_terms(R_(AM_PART, set0(J) + c, 0), NONE, 0, 0, TG_EPI_NONE, t);
            }
            // Q = Lbar_JJ + its partials
            b.launch_begin(AK_DIAG_SUM, J);
            b.task(R_(AM_Q, 0, 0), R_(AM_LBAR, J, J), set0(J), C, TG_EPI_NONE, {});
        }
        const AdjRef Q = nt > 0 ? R_(AM_Q, 0, 0) : R_(AM_LBAR, J, J);
        // POTRF adjoint: three products on single tiles
        b.launch_begin(AK_POTRF, J);
        b.task(R_(AM_G, 0, 0), NONE, 0, 0, TG_EPI_SYM,
               {AdjTerm{R_(AM_L, J, J), Q, 1, TG_TRANS_A | TG_TRI_A | TG_TRI_B}});
        b.launch_begin(AK_POTRF, J);
        b.task(R_(AM_X, 0, 0), NONE, 0, 0, TG_EPI_NONE,
               {AdjTerm{R_(AM_G, 0, 0), R_(AM_TINV, J, J), 1, TG_TRI_B}});
        const int potrf3 = b.launch_begin(AK_POTRF, J);
        b.task(R_(AM_ABAR, J, J), NONE, 0, 0, TG_EPI_PHI,
               {AdjTerm{R_(AM_TINV, J, J), R_(AM_X, 0, 0), 1, TG_TRANS_A | TG_TRI_A}});
        // column J - 2's early pulls need the columns >= J: now final
        emit_early(J - 2, potrf3);
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
            int32_t* o = launches + 6 * i;
            o[0] = L.kind; o[1] = L.step; o[2] = L.first; o[3] = L.count;
            o[4] = L.stream; o[5] = L.wait;
        }
    return GPR_OK;
}
