// schedule.cpp -- turns the tile task graph of the right-looking tiled
// Cholesky (Sec. 4.2, Fig. 1) and of the covariance solve (Sec. 4.1: L V =
// K_{X,X*}, Sigma = K_{X*,X*} - V^T V) into batched launches on three
// streams.
//
// The test rows are appended below the training rows: with
//   A = [[K, .], [K_{X*,X}, K_{X*,X*}]]
// the right-looking sweep over the first M tile columns turns the rows below
// into V^T = K_{X*,X} L^{-T} (TRSM, then GEMM updates) and the lower-right
// block into K_{X*,X*} - V^T V (SYRK / GEMM updates). Every task is one of
// the four tile operations of Fig. 1 acting on the extended lower-tiled
// matrix, so one dependency rule covers both.
//
// Dependencies (tile (I, K) updated at step J with the panel of column J):
//   POTRF(J)      after the last update of (J, J)           -- SYRK(J, J, J-1)
//   TRSM(I, J)    after POTRF(J) and the last update of (I, J)
//   update(I,K,J) after TRSM(I, J), TRSM(K, J) and update(I, K, J-1).
//
// When the training block is factored (modes 0 and 2), only three tile tasks
// separate POTRF(J) from POTRF(J+1): TRSM(J+1, J) and SYRK(J+1, J+1, J).
// They run on the critical stream C; everything else of step J goes to a
// panel stream P (the other TRSMs of column J, then the GEMMs of column J+1,
// GEMM(J+2, J+1, J) first because the next step's critical TRSM needs it) or
// to the bulk stream B (all updates of columns >= J+2):
//   C: POTRF(J); [wait G1(J-1)] TRSM(J+1, J); [wait R(J-1)] SYRK(J+1, J+1, J)
//   P: [wait POTRF(J)] TRSM(rest of column J);
//      [wait TRSM(J+1, J), R(J-1)] G1(J) = GEMM(J+2, J+1, J); N(J) = the other
//      GEMMs of column J+1
//   B: [wait TRSM(J+1, J), TRSM(rest of J)] R(J)
// Tiles of column J+1 get their updates of steps < J in R (waited for), of
// step J on P; tiles of columns >= J+2 get all their updates on B in step
// order. The covariance solve with a given factor (mode 1) has no POTRF and
// uses C (TRSM of the test rows, then the updates of column J+1) and B.
// Modes 3 and 4 are modes 1 and 2 without the updates of the test block
// (columns K >= M): only V^T is formed, for the predictive variances.
#include <algorithm>

#include "gpr_internal.h"

namespace gpr {

namespace {

struct Builder {
    Schedule S;
    int add(int stream, std::vector<int> waits, int kind, const std::vector<SchedTask>& tasks,
            int step)
    {
        if (tasks.empty()) return -1;
        SchedLaunch L;
        L.stream = stream;
        L.nwait = 0;
        for (int w : waits)
            if (w >= 0 && S.launches[w].stream != stream && L.nwait < 3) L.wait[L.nwait++] = w;
        for (int k = L.nwait; k < 3; ++k) L.wait[k] = -1;
        L.kind = kind;
        L.first = (int)S.tasks.size();
        L.count = (int)tasks.size();
        L.step = step;
        S.tasks.insert(S.tasks.end(), tasks.begin(), tasks.end());
        S.launches.push_back(L);
        return (int)S.launches.size() - 1;
    }
};

SchedTask upd(int I, int K, int J) { return SchedTask{I == K ? K_SYRK : K_GEMM, I, K, J}; }

}  // namespace

Schedule build_schedule(int M, int Mhat, int mode)
{
    Builder b;
    const bool factor = sweep_factors(mode);
    const bool predict = sweep_test_rows(mode);
    const bool block = sweep_test_block(mode);  // updates of the test block too
    const int T = M + (predict ? Mhat : 0);  // tile rows of the extended matrix
    // columns K of the updates: all, or only the training columns (V only)
    auto keep = [&](int K) { return block || K < M; };
    enum { C = 0, P = 1, B = 2 };

    if (!factor) {
        // covariance rows with a given factor: C runs TRSM(column J) and the
        // updates of column J+1, B the rest
        int last_R = -1;
        for (int J = 0; J < M; ++J) {
            std::vector<SchedTask> tr, N, R;
            for (int I = M; I < T; ++I) tr.push_back({K_TRSM, I, J, J});
            for (int I = M; I < T; ++I)
                for (int K = J + 1; K <= I; ++K) {
                    if (!keep(K)) continue;
                    if (K == J + 1 && K < M) N.push_back(upd(I, K, J));
                    else R.push_back(upd(I, K, J));
                }
            const int t = b.add(C, {}, LK_TRSM, tr, J);
            b.add(C, {last_R}, LK_UPDATE, N, J);
            const int r = b.add(B, {t}, LK_UPDATE, R, J);
            if (r >= 0) last_R = r;
        }
        return b.S;
    }

    int last_R = -1, last_G1 = -1;
    for (int J = 0; J < M; ++J) {
        const int potrf = b.add(C, {}, LK_POTRF, {SchedTask{K_POTRF, J, J, J}}, J);
        const bool next = J + 1 < M;  // is there a next factored column?
        // critical TRSM and SYRK
        int t1 = -1;
        if (next) {
            t1 = b.add(C, {last_G1}, LK_TRSM, {SchedTask{K_TRSM, J + 1, J, J}}, J);
            b.add(C, {last_R}, LK_UPDATE, {upd(J + 1, J + 1, J)}, J);
        }
        // the other TRSMs of column J
        std::vector<SchedTask> trest;
        for (int I = J + (next ? 2 : 1); I < T; ++I) trest.push_back({K_TRSM, I, J, J});
        const int tr = b.add(P, {potrf}, LK_TRSM, trest, J);
        // GEMMs of column J+1: G1 = (J+2, J+1) first, then the rest
        last_G1 = -1;
        if (next) {
            if (J + 2 < M) last_G1 = b.add(P, {t1, last_R}, LK_UPDATE, {upd(J + 2, J + 1, J)}, J);
            std::vector<SchedTask> N;
            for (int I = J + 2; I < T; ++I)
                if (!(I == J + 2 && J + 2 < M) && keep(J + 1)) N.push_back(upd(I, J + 1, J));
            b.add(P, {t1, last_R}, LK_UPDATE, N, J);
        }
        // everything else of step J
        std::vector<SchedTask> R;
        for (int I = J + 1; I < T; ++I)
            for (int K = (next ? J + 2 : J + 1); K <= I; ++K)
                if (keep(K)) R.push_back(upd(I, K, J));
        const int r = b.add(B, {t1, tr}, LK_UPDATE, R, J);
        if (r >= 0) last_R = r;
    }
    return b.S;
}

// Left-looking variant (Sec. 4.2 names it beside the right-looking Fig. 1):
// tile column K receives the products L_IJ L_KJ^T of all earlier columns
// J < K just before it is factored, instead of one rank-m update per step.
// Its terms 0 .. K-2 come as one multi-term task per tile (Ub(K), on the bulk
// stream, issued at step K-1 once column K-2 is final, so it runs beside the
// factorisation of column K-1); its last term K-1 follows once column K-1 is
// final, split like the right-looking step: the diagonal tile's SYRK on the
// critical stream, GEMM(K+1, K, K-1) first on the panel stream (the next
// critical TRSM needs it), then the rest. The test block of the covariance
// solve takes all M terms in one task per tile after the last column.
//   C: [wait Ub(J)] SYRK(J, J, J-1); POTRF(J); [wait G1(J)] TRSM(J+1, J)
//   P: [wait Ub(J), TRSM(J, J-1)] G1(J) = GEMM(J+1, J, J-1); the other last-term
//      GEMMs of column J; [wait POTRF(J)] TRSM(rest of column J)
//   B: [wait the TRSMs of rows >= J+1 in column J-1] Ub(J+1) = terms 0 .. J-1
//      of column J+1
// With a given factor (modes 1, 3) only the test rows are swept: C runs the
// last-term updates and the TRSMs of each column, B the Ub launches.
Schedule build_schedule_left(int M, int Mhat, int mode)
{
    Builder b;
    const bool factor = sweep_factors(mode);
    const bool predict = sweep_test_rows(mode);
    const bool block = sweep_test_block(mode);
    const int T = M + (predict ? Mhat : 0);
    const int I0 = factor ? 0 : M;  // first swept tile row
    enum { C = 0, P = 1, B = 2 };
    auto upd = [](int I, int K, int k0, int nk) {
        SchedTask t{I == K ? K_SYRK : K_GEMM, I, K, k0};
        t.nk = nk;
        return t;
    };
    int bulk = -1;                     // Ub(J), issued at step J - 1
    int col_crit = -1, col_rest = -1;  // the TRSMs of column J - 1
    for (int J = 0; J < M; ++J) {
        const bool next = factor && J + 1 < M;
        int g1 = -1;
        if (J >= 1) {
            std::vector<SchedTask> N;
            for (int I = std::max(J, I0); I < T; ++I) {
                if (factor && (I == J || (next && I == J + 1))) continue;
                N.push_back(upd(I, J, J - 1, 1));
            }
            if (factor) b.add(C, {bulk}, LK_UPDATE, {upd(J, J, J - 1, 1)}, J);
            if (next) g1 = b.add(P, {bulk, col_crit}, LK_UPDATE, {upd(J + 1, J, J - 1, 1)}, J);
            // after G1 on the same stream, which already waited for the same launches
            if (g1 >= 0) b.add(P, {}, LK_UPDATE, N, J);
            else b.add(factor ? P : C, {bulk, col_crit}, LK_UPDATE, N, J);
        }
        int crit = -1, rest = -1;
        if (factor) {
            const int potrf = b.add(C, {}, LK_POTRF, {SchedTask{K_POTRF, J, J, J}}, J);
            if (next) crit = b.add(C, {g1}, LK_TRSM, {SchedTask{K_TRSM, J + 1, J, J}}, J);
            std::vector<SchedTask> tr;
            for (int I = J + (next ? 2 : 1); I < T; ++I) tr.push_back({K_TRSM, I, J, J});
            rest = b.add(P, {potrf}, LK_TRSM, tr, J);
        } else {
            std::vector<SchedTask> tr;
            for (int I = M; I < T; ++I) tr.push_back({K_TRSM, I, J, J});
            rest = b.add(C, {}, LK_TRSM, tr, J);
        }
        int nbulk = -1;
        if (J >= 1 && J + 1 < M) {
            std::vector<SchedTask> U;
            for (int I = std::max(J + 1, I0); I < T; ++I) U.push_back(upd(I, J + 1, 0, J));
            // reads rows >= J + 1 of columns < J: the TRSMs of column J - 1
            // other than the critical one (row J)
            nbulk = b.add(B, {col_rest}, LK_UPDATE, U, J);
        }
        bulk = nbulk;
        col_crit = crit;
        col_rest = rest;
    }
    if (block) {
        std::vector<SchedTask> W;
        for (int I = M; I < T; ++I)
            for (int K = M; K <= I; ++K) W.push_back(upd(I, K, 0, M));
        b.add(B, {col_crit, col_rest}, LK_UPDATE, W, M);
    }
    return b.S;
}

Schedule build_schedule_variant(int M, int Mhat, int mode, int variant)
{
    return variant == GPR_LEFT_LOOKING ? build_schedule_left(M, Mhat, mode)
                                       : build_schedule(M, Mhat, mode);
}

}  // namespace gpr

extern "C" int gpr_schedule_describe_variant(int32_t M, int32_t Mhat, int32_t mode,
                                             int32_t variant, int32_t* tasks, int64_t task_cap,
                                             int64_t* n_tasks, int32_t* launches,
                                             int64_t launch_cap, int64_t* n_launches)
{
    if (M < 1 || Mhat < 0 || mode < 0 || mode > 4 || !n_tasks || !n_launches) return GPR_EINVAL;
    if (variant != GPR_RIGHT_LOOKING && variant != GPR_LEFT_LOOKING) return GPR_EINVAL;
    if (mode != gpr::SWEEP_CHOLESKY && Mhat < 1) return GPR_EINVAL;
    gpr::Schedule S = gpr::build_schedule_variant(M, Mhat, mode, variant);
    *n_tasks = (int64_t)S.tasks.size();
    *n_launches = (int64_t)S.launches.size();
    if ((int64_t)S.tasks.size() > task_cap || (int64_t)S.launches.size() > launch_cap)
        return GPR_EINVAL;
    if (tasks) {
        for (size_t li = 0; li < S.launches.size(); ++li) {
            const auto& L = S.launches[li];
            for (int t = L.first; t < L.first + L.count; ++t) {
                const auto& k = S.tasks[t];
                int32_t* o = tasks + 6 * (size_t)t;
                o[0] = k.kind; o[1] = k.I; o[2] = k.K; o[3] = k.J; o[4] = k.nk;
                o[5] = (int32_t)li;
            }
        }
    }
    if (launches) {
        for (size_t li = 0; li < S.launches.size(); ++li) {
            int32_t* o = launches + 5 * li;
            o[0] = S.launches[li].stream;
            o[1] = S.launches[li].wait[0];
            o[2] = S.launches[li].wait[1];
            o[3] = S.launches[li].wait[2];
            o[4] = S.launches[li].kind;
        }
    }
    return GPR_OK;
}

extern "C" int gpr_schedule_describe(int32_t M, int32_t Mhat, int32_t mode, int32_t* tasks,
                                     int64_t task_cap, int64_t* n_tasks, int32_t* launches,
                                     int64_t launch_cap, int64_t* n_launches)
{
    if (M < 1 || Mhat < 0 || mode < 0 || mode > 4 || !n_tasks || !n_launches) return GPR_EINVAL;
    if (mode != gpr::SWEEP_CHOLESKY && Mhat < 1) return GPR_EINVAL;
    gpr::Schedule S = gpr::build_schedule(M, Mhat, mode);
    *n_tasks = (int64_t)S.tasks.size();
    *n_launches = (int64_t)S.launches.size();
    if ((int64_t)S.tasks.size() > task_cap || (int64_t)S.launches.size() > launch_cap)
        return GPR_EINVAL;
    if (tasks) {
        for (size_t li = 0; li < S.launches.size(); ++li) {
            const auto& L = S.launches[li];
            for (int t = L.first; t < L.first + L.count; ++t) {
                const auto& k = S.tasks[t];
                int32_t* o = tasks + 5 * (size_t)t;
                o[0] = k.kind; o[1] = k.I; o[2] = k.K; o[3] = k.J; o[4] = (int32_t)li;
            }
        }
    }
    if (launches) {
        for (size_t li = 0; li < S.launches.size(); ++li) {
            int32_t* o = launches + 5 * li;
            o[0] = S.launches[li].stream;
            o[1] = S.launches[li].wait[0];
            o[2] = S.launches[li].wait[1];
            o[3] = S.launches[li].wait[2];
            o[4] = S.launches[li].kind;
        }
    }
    return GPR_OK;
}
