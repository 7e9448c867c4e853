// persist.cpp -- the ticket order of the persistent sweep executor (host).
//
// The tile tasks of the sweep (the same task graph as schedule.cpp) are
// ranked by their upward rank -- the estimated time from the task's start to
// the end of the sweep along its longest chain of dependent tasks -- and the
// order is made by a list-scheduling simulation of W workgroups: whenever a
// simulated workgroup is free it takes the next item of the highest-ranked
// task whose inputs are (estimated to be) final, or, if none is, of the task
// that becomes ready first. A task is released to the simulation only when
// every item of every task it waits for has been handed out, so the order is
// topological (the precondition of the deadlock-freedom argument in
// persist.h), and items are mostly ready when a real workgroup takes them.
// Estimated durations (per item, microseconds, from kernel timings at m = 512
// on the target) only steer the order; correctness never depends on them.
#include <algorithm>
#include <queue>
#include <unordered_map>
#include <vector>

#include "gpr_internal.h"
#include "persist.h"

namespace gpr {

namespace {

struct PTaskNode {
    int kind, I, K, J;
    int nitem;
    double dur;   // per item
    double rank;
    std::vector<int> succ;
    int npred = 0;
};

}  // namespace

PGeom persist_geom(int M, int Mhat, int mode, int m, int bm)
{
    PGeom g;
    g.M = M;
    g.factor = sweep_factors(mode) ? 1 : 0;
    g.T = M + (sweep_test_rows(mode) ? Mhat : 0);
    g.P = m / 32;
    g.nb = m / bm;
    return g;
}

std::vector<PItem> build_persist_order(int M, int Mhat, int mode, int m, int bm, int workers)
{
    const PGeom g = persist_geom(M, Mhat, mode, m, bm);
    const int T = g.T;
    std::vector<PTaskNode> tasks;
    std::unordered_map<int64_t, int> index;
    auto key = [&](int kind, int I, int K, int J) {
        return (((int64_t)kind * T + I) * T + K) * T + J;
    };
    auto find = [&](int kind, int I, int K, int J) -> int {
        auto it = index.find(key(kind, I, K, J));
        return it == index.end() ? -1 : it->second;
    };
    // per-item durations (microseconds); a workgroup of the update blocks
    // runs at about 52 TFLOP/s shared over `workers`
    const double rate = 52.0e6 / std::max(workers, 1);  // flop per microsecond
    const double t_upd = 2.0 * bm * bm * (double)m / rate;
    const double t_strip = 1.6 * 32.0 * m * (double)m / rate;
    const double t_panel = 261.0 * ((double)m / 512) * ((double)m / 512);
    auto add = [&](int kind, int I, int K, int J) {
        PTaskNode t;
        t.kind = kind;
        t.I = I;
        t.K = K;
        t.J = J;
        if (kind == PI_POTRF) {
            t.nitem = g.P;
            t.dur = t_panel;
        } else if (kind == PI_TRSM) {
            t.nitem = g.P;
            t.dur = t_strip;
        } else {
            t.nitem = (int)pnblk(g, I, K);
            t.dur = t_upd;
        }
        t.rank = 0.0;
        index[key(kind, I, K, J)] = (int)tasks.size();
        tasks.push_back(t);
    };
    // creation order is topological: step J ascending; in a step POTRF,
    // TRSMs, then updates
    const bool block = sweep_test_block(mode);  // updates of the test block too
    for (int J = 0; J < M; ++J) {
        if (g.factor) add(PI_POTRF, J, J, J);
        for (int I = (g.factor ? J + 1 : M); I < T; ++I) add(PI_TRSM, I, J, J);
        for (int I = (g.factor ? J + 1 : M); I < T; ++I)
            for (int K = J + 1; K <= I; ++K)
                if (block || K < M) add(PI_UPDATE, I, K, J);
    }
    // predecessors (the tasks whose items an item waits for, persist.h)
    auto link = [&](int pred, int succ) {
        if (pred < 0) return;
        tasks[pred].succ.push_back(succ);
        tasks[succ].npred += 1;
    };
    for (int t = 0; t < (int)tasks.size(); ++t) {
        const PTaskNode n = tasks[t];
        if (n.kind == PI_POTRF) {
            if (n.J > 0) link(find(PI_UPDATE, n.J, n.J, n.J - 1), t);
        } else if (n.kind == PI_TRSM) {
            if (n.J > 0) link(find(PI_UPDATE, n.I, n.J, n.J - 1), t);
            if (g.factor) link(find(PI_POTRF, n.J, n.J, n.J), t);
        } else {
            link(find(PI_TRSM, n.I, n.J, n.J), t);
            if (!pgiven(g, n.K) && n.K != n.I) link(find(PI_TRSM, n.K, n.J, n.J), t);
            if (n.J > 0) link(find(PI_UPDATE, n.I, n.K, n.J - 1), t);
        }
    }
    for (int t = (int)tasks.size() - 1; t >= 0; --t) {
        double best = 0.0;
        for (int s : tasks[t].succ) best = std::max(best, tasks[s].rank);
        tasks[t].rank = tasks[t].dur + best;
    }

    // list-scheduling simulation
    std::vector<PItem> order;
    size_t total = 0;
    for (const auto& t : tasks) total += (size_t)t.nitem;
    order.reserve(total);
    std::vector<int> next_item(tasks.size(), 0);
    std::vector<double> ready_at(tasks.size(), 0.0), finish(tasks.size(), 0.0);
    auto by_rank = [&](int a, int b) {
        if (tasks[a].rank != tasks[b].rank) return tasks[a].rank < tasks[b].rank;
        return a > b;  // earlier-created first among equal ranks
    };
    auto by_ready = [&](int a, int b) {
        if (ready_at[a] != ready_at[b]) return ready_at[a] > ready_at[b];
        return by_rank(a, b);
    };
    std::priority_queue<int, std::vector<int>, decltype(by_rank)> ready(by_rank);
    std::priority_queue<int, std::vector<int>, decltype(by_ready)> future(by_ready);
    std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
    for (int w = 0; w < std::max(workers, 1); ++w) free_at.push(0.0);
    for (int t = 0; t < (int)tasks.size(); ++t)
        if (tasks[t].npred == 0) future.push(t);
    while (order.size() < total) {
        const double now = free_at.top();
        free_at.pop();
        while (!future.empty() && ready_at[future.top()] <= now) {
            ready.push(future.top());
            future.pop();
        }
        int t;
        if (!ready.empty()) {
            t = ready.top();
        } else {
            t = future.top();
            future.pop();
            ready.push(t);
        }
        PTaskNode& n = tasks[t];
        const double start = std::max(now, ready_at[t]);
        const double end = start + n.dur;
        finish[t] = std::max(finish[t], end);
        free_at.push(end);
        order.push_back(PItem{n.kind | (next_item[t] << 4), n.I, n.K, n.J});
        if (++next_item[t] == n.nitem) {
            ready.pop();  // t is on top of `ready` here
            for (int s : n.succ) {
                ready_at[s] = std::max(ready_at[s], finish[t]);
                if (--tasks[s].npred == 0) future.push(s);
            }
        }
    }
    return order;
}

}  // namespace gpr

// Describe the ticket order (tests and tooling): per item 5 int32
// (kind, sub, I, K, J) and 8 int64 (number of waits, then (counter, value)
// x 3, then the counter the item increments).
extern "C" int gpr_persist_describe(int32_t M, int32_t Mhat, int32_t mode, int32_t tile,
                                    int32_t block, int32_t workers, int32_t* items,
                                    int64_t* waits, int64_t cap, int64_t* n_items)
{
    if (M < 1 || Mhat < 0 || mode < 0 || mode > 4 || !n_items) return GPR_EINVAL;
    if (mode != gpr::SWEEP_CHOLESKY && Mhat < 1) return GPR_EINVAL;
    if (tile < 32 || tile % 32 != 0 || block < 32 || tile % block != 0 || workers < 1)
        return GPR_EINVAL;
    const std::vector<gpr::PItem> order =
        gpr::build_persist_order(M, Mhat, mode, tile, block, workers);
    *n_items = (int64_t)order.size();
    if ((int64_t)order.size() > cap) return GPR_EINVAL;
    const gpr::PGeom g = gpr::persist_geom(M, Mhat, mode, tile, block);
    for (size_t i = 0; i < order.size(); ++i) {
        const gpr::PItem& it = order[i];
        if (items) {
            int32_t* o = items + 5 * i;
            o[0] = it.kind_sub & 15;
            o[1] = it.kind_sub >> 4;
            o[2] = it.I;
            o[3] = it.K;
            o[4] = it.J;
        }
        if (waits) {
            const gpr::PWaits w = gpr::pitem_waits(g, it);
            int64_t* o = waits + 8 * i;
            int n = 0;
            for (int k = 0; k < 3; ++k)
                if (w.val[k] != 0u) {
                    o[1 + 2 * n] = w.cnt[k];
                    o[2 + 2 * n] = (int64_t)w.val[k];
                    ++n;
                }
            for (int k = n; k < 3; ++k) {
                o[1 + 2 * k] = -1;
                o[2 + 2 * k] = 0;
            }
            o[0] = n;
            o[7] = w.sig;
        }
    }
    return GPR_OK;
}
