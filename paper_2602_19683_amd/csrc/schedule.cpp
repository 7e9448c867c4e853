// schedule.cpp -- turns the tile task graph of the right-looking tiled
// Cholesky (Sec. 4.2, Fig. 1) and of the covariance solve (Sec. 4.1: L V =
// K_{X,X*}, Sigma = K_{X*,X*} - V^T V) into batched launches on two streams.
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
//   POTRF(J)      after the last update of (J, J)           -- SYRK(J, J-1)
//   TRSM(I, J)    after POTRF(J) and the last update of (I, J)
//   update(I,K,J) after TRSM(I, J), TRSM(K, J) and update(I, K, J-1).
//
// Execution with one step of look-ahead on a critical stream C and a bulk
// stream B. At step J:
//   C: POTRF(J); TRSM(column J); [wait for R(J-1)]; N(J)
//   B: [wait for TRSM(J)]; R(J)
// where N(J) are the updates of tile column J+1 (the next panel) and R(J)
// all other updates of step J. Tiles of column J+1 get their step-J' < J
// updates in R(J'), which N(J) waits for; tiles of columns >= J+2 get all
// their updates on B in step order. So POTRF(J+1) and TRSM(J+1) run on C
// while R(J) still runs on B.
#include <algorithm>

#include "gpr_internal.h"

namespace gpr {

Schedule build_schedule(int M, int Mhat, int mode)
{
    Schedule S;
    const bool factor = (mode == SWEEP_CHOLESKY || mode == SWEEP_FUSED);
    const bool predict = (mode == SWEEP_PREDICT || mode == SWEEP_FUSED);
    const int T = M + (predict ? Mhat : 0);  // tile rows of the extended matrix
    const int row_lo = factor ? 0 : M;       // first row that is written

    int last_R = -1;  // index of R(J-1) launch, or -1
    for (int J = 0; J < M; ++J) {
        // ---- critical stream: POTRF(J)
        if (factor) {
            SchedLaunch L{0, -1, LK_POTRF, (int)S.tasks.size(), 1, J};
            S.tasks.push_back({K_POTRF, J, J, J});
            S.launches.push_back(L);
        }
        // ---- critical stream: TRSM of column J (rows below the diagonal)
        int trsm_launch = -1;
        {
            SchedLaunch L{0, -1, LK_TRSM, (int)S.tasks.size(), 0, J};
            for (int I = std::max(J + 1, row_lo); I < T; ++I) {
                if (I < M && !factor) continue;
                S.tasks.push_back({K_TRSM, I, J, J});
            }
            L.count = (int)S.tasks.size() - L.first;
            if (L.count > 0) {
                trsm_launch = (int)S.launches.size();
                S.launches.push_back(L);
            }
        }
        if (trsm_launch < 0) continue;  // nothing below: no updates at this step

        // ---- updates of step J, split into N(J) (column J+1) and R(J).
        std::vector<SchedTask> N, R;
        for (int I = J + 1; I < T; ++I) {
            if (I < M && !factor) continue;
            for (int K = J + 1; K <= I; ++K) {
                if (K < M && I < M && !factor) continue;
                // training tiles (I, K < M) exist only when factoring; test rows
                // always pair with training columns K < M (V) or test columns (Sigma)
                const SchedTask t{I == K ? K_SYRK : K_GEMM, I, K, J};
                if (K == J + 1 && K < M) N.push_back(t);
                else R.push_back(t);
            }
        }
        if (!N.empty()) {
            SchedLaunch L{0, last_R, LK_UPDATE, (int)S.tasks.size(), (int)N.size(), J};
            S.tasks.insert(S.tasks.end(), N.begin(), N.end());
            S.launches.push_back(L);
        }
        if (!R.empty()) {
            SchedLaunch L{1, trsm_launch, LK_UPDATE, (int)S.tasks.size(), (int)R.size(), J};
            S.tasks.insert(S.tasks.end(), R.begin(), R.end());
            last_R = (int)S.launches.size();
            S.launches.push_back(L);
        }
    }
    return S;
}

}  // namespace gpr

extern "C" int gpr_schedule_describe(int32_t M, int32_t Mhat, int32_t mode, int32_t* tasks,
                                     int64_t task_cap, int64_t* n_tasks, int32_t* launches,
                                     int64_t launch_cap, int64_t* n_launches)
{
    if (M < 1 || Mhat < 0 || mode < 0 || mode > 2 || !n_tasks || !n_launches) return GPR_EINVAL;
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
            int32_t* o = launches + 3 * li;
            o[0] = S.launches[li].stream;
            o[1] = S.launches[li].wait;
            o[2] = S.launches[li].kind;
        }
    }
    return GPR_OK;
}
