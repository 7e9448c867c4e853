// solve_plan.cpp -- the batched tile products that build the group inverses
// of the vector solves (Sec. 4.1, the two triangular solves after eq. (2)),
// planned on the host with symbolic operands.
//
// The solves take G consecutive tile rows per step (G = trsv_group(m, prec)); a step
// applies the inverse of the group's G x G block of tiles of L. Its diagonal
// tiles are the inverses of the diagonal tiles of L; its off-diagonal tiles
// Inv_ij (i > j, indices relative to the group's first tile J0) are built by
// doubling: with the inverses of the blocks B1 = [s0, s0 + H) and
// B2 = [s0 + H, s0 + 2H) of a group known, the block of the inverse of B1 + B2
// below its diagonal is -Inv(B2) Q Inv(B1), Q the tiles of L between them:
//   Y_cb                  = sum_{d = b}^{H-1} L_{J0+s0+H+c, J0+s0+d} Inv(B1)_db
//   Inv_{s0+H+c, s0+b}    = -sum_{e = 0}^{c} Inv(B2)_ce Y_eb
// (H = 1, 2, ..., G / 2; for H = 1 this is W = -Tinv_{J+1} L_{J+1,J} Tinv_J).
// Each product is one launch of the batched tile-product kernel, all tasks of
// a level side by side: 2 log2 G launches, each reading only what earlier
// launches wrote. Slots: Inv_ij of group g at W slot g S + i (i - 1) / 2 + j,
// S = G (G - 1) / 2; Y_cb at the Y slot of the Inv tile it becomes.
#include <algorithm>

#include "gpr_internal.h"

namespace gpr {

TinvPlan plan_tinv_groups(int M, int G)
{
    TinvPlan P;
    P.G = G;
    const int ng = (M + G - 1) / G;
    const int S = G * (G - 1) / 2;
    P.nslot = (long long)ng * S;
    if (M < 2 || G < 2) return P;
    auto slot = [&](int g, int i, int j) { return g * S + i * (i - 1) / 2 + j; };
    // Inv_ij of group g (relative indices), i >= j
    auto inv = [&](int g, int i, int j) {
        return i == j ? TinvRef{TR_TINV, g * G + i, 0} : TinvRef{TR_W, slot(g, i, j), 0};
    };
    for (int H = 1; H < G; H *= 2) {
        for (int pass = 0; pass < 2; ++pass) {
            TinvLaunchPlan lp;
            lp.first_task = (int)P.tasks.size();
            lp.first_term = (int)P.terms.size();
            auto add_task = [&](TinvRef out) {
                // first_term counts from the launch's first term
                P.tasks.push_back(TinvTaskPlan{out, (int)P.terms.size() - lp.first_term, 0});
            };
            auto add_term = [&](TinvRef A, TinvRef B, double alpha) {
                P.terms.push_back(TinvTermPlan{A, B, alpha});
                ++P.tasks.back().nterm;
            };
            for (int g = 0; g < ng; ++g) {
                const int J0 = g * G, ns = std::min(G, M - J0);
                for (int s0 = 0; s0 + H < ns; s0 += 2 * H) {
                    const int h2 = std::min(H, ns - s0 - H);
                    for (int c = 0; c < h2; ++c)
                        for (int b = 0; b < H; ++b) {
                            const int row = s0 + H + c, col = s0 + b;
                            if (pass == 0) {
                                add_task(TinvRef{TR_Y, slot(g, row, col), 0});
                                for (int d = b; d < H; ++d)
                                    add_term(TinvRef{TR_L, J0 + row, J0 + s0 + d},
                                             inv(g, s0 + d, col), 1.0);
                            } else {
                                add_task(TinvRef{TR_W, slot(g, row, col), 0});
                                for (int e = 0; e <= c; ++e)
                                    add_term(inv(g, row, s0 + H + e),
                                             TinvRef{TR_Y, slot(g, s0 + H + e, col), 0}, -1.0);
                            }
                        }
                }
            }
            lp.ntask = (int)P.tasks.size() - lp.first_task;
            lp.nterm = (int)P.terms.size() - lp.first_term;
            P.launches.push_back(lp);
        }
    }
    return P;
}

bool tinv_plan_valid(const TinvPlan& P)
{
    for (const TinvLaunchPlan& lp : P.launches)
        for (int t = lp.first_task; t < lp.first_task + lp.ntask; ++t) {
            const TinvTaskPlan& k = P.tasks[t];
            if (k.first_term < 0 || k.nterm < 1 || k.first_term + k.nterm > lp.nterm) return false;
        }
    return true;
}

}  // namespace gpr

extern "C" int gpr_solve_plan_describe(int32_t M, int32_t tile, int32_t* group, int32_t* tasks,
                                       int64_t task_cap, int64_t* n_tasks, int32_t* terms,
                                       int64_t term_cap, int64_t* n_terms)
{
    using namespace gpr;
    if (M < 1 || tile < 32 || tile > 1024 || tile % 32 != 0 || !n_tasks || !n_terms)
        return GPR_EINVAL;
    const TinvPlan P = plan_tinv_groups(M, trsv_group(tile, GPR_FP64));
    if (group) *group = P.G;
    *n_tasks = (int64_t)P.tasks.size();
    *n_terms = (int64_t)P.terms.size();
    if ((tasks && task_cap < *n_tasks) || (terms && term_cap < *n_terms)) return GPR_EINVAL;
    if (tasks)
        for (size_t l = 0; l < P.launches.size(); ++l)
            for (int t = P.launches[l].first_task;
                 t < P.launches[l].first_task + P.launches[l].ntask; ++t) {
                const TinvTaskPlan& k = P.tasks[t];
                int32_t* o = tasks + 6 * (size_t)t;
                o[0] = (int32_t)l;
                o[1] = k.out.kind;
                o[2] = k.out.a;
                o[3] = k.out.b;
                o[4] = k.first_term;
                o[5] = k.nterm;
            }
    if (terms)
        for (size_t u = 0; u < P.terms.size(); ++u) {
            const TinvTermPlan& v = P.terms[u];
            int32_t* o = terms + 7 * u;
            o[0] = v.A.kind;
            o[1] = v.A.a;
            o[2] = v.A.b;
            o[3] = v.B.kind;
            o[4] = v.B.a;
            o[5] = v.B.b;
            o[6] = v.alpha > 0 ? 1 : -1;
        }
    return GPR_OK;
}
