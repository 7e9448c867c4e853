// persist.h -- work items of the persistent sweep executor and the rule that
// orders them (shared by the host planner and the device kernel).
//
// The persistent executor runs the tile task graph of the extended sweep
// (schedule.cpp: the tiled Cholesky of Fig. 1 with the test rows appended,
// or the covariance solve with a given factor) in ONE kernel launch. Each
// tile task is cut into work items of one workgroup each:
//   POTRF(J)       m / 32 row panels w (k_potrf_dev.h);
//   TRSM(I, J)     m / 32 strips of 32 rows (k_trsm_dev.h);
//   update(I,K,J)  the BM x BM blocks of C -= A B^T (k_update_dev.h; a SYRK
//                  task has only the blocks on or below its diagonal).
// The host lists the items in one order (a ticket order); each workgroup
// takes the next ticket with an atomic increment, waits until the item's
// inputs are final, runs it, and counts it done.
//
// Progress counter of tile (I, K): the number of finished items that wrote
// it. Its items come in a fixed sequence -- the update blocks of steps 0, 1,
// .., then (when the tile is in column K < M) the TRSM strips or POTRF
// panels -- so one counter per tile says how far the tile is:
//   >= J nblk(I, K)         all updates of steps < J done;
//   >= J nblk(I, J) + P     for a tile of column J: factored / solved (final).
// Waits of an item (a tile of the given factor, in the covariance solve, is
// final from the start and is not waited for):
//   POTRF(J) panel   cnt(J, J) >= J nblk(J, J)
//   TRSM(I, J)       cnt(I, J) >= J nblk(I, J);  cnt(J, J) final
//   update(I, K, J)  cnt(I, J) final;  cnt(K, J) final;  cnt(I, K) >= J nblk(I, K)
// Within a POTRF, panel w also waits for panels q < w (flags, as in the
// stream kernel). Every wait therefore targets items of tasks that come
// earlier in any topological order; the planner emits the items of a task
// only after all items of the tasks it waits for, and the panels of a POTRF
// in increasing w. Then the holder of the lowest unfinished ticket always
// has its inputs ready, so every wait ends -- for any number of resident
// workgroups.
#pragma once

#include <cstdint>

namespace gpr {

enum : int { PI_POTRF = 0, PI_TRSM = 1, PI_UPDATE = 2 };

// One ticket. kind_sub = kind | sub << 4 (sub: panel, strip or block index
// bi * nb + bj). For POTRF, I = K = J; for TRSM, K = J.
struct PItem {
    int kind_sub, I, K, J;
};

struct PGeom {
    int M;       // factored (or given) tile columns
    int T;       // tile rows of the extended matrix
    int factor;  // 1: the factor is computed here; 0: given (covariance solve)
    int P;       // m / 32: TRSM strips and POTRF panels per tile
    int nb;      // m / BM: update blocks per tile row
};

// Three wait slots; an unused slot has value 0 (always satisfied). The slots
// have fixed roles so that device code indexes them with constants.
struct PWaits {
    int64_t cnt[3];
    unsigned val[3];
    int64_t sig;  // counter this item increments
};

__host__ __device__ inline int64_t ptile(int I, int K) { return (int64_t)I * (I + 1) / 2 + K; }

__host__ __device__ inline unsigned pnblk(const PGeom& g, int I, int K)
{
    return I == K ? (unsigned)(g.nb * (g.nb + 1) / 2) : (unsigned)(g.nb * g.nb);
}

// Counter value at which tile (I, J) of column J < M is final.
__host__ __device__ inline unsigned pfinal(const PGeom& g, int I, int J)
{
    return (unsigned)J * pnblk(g, I, J) + (unsigned)g.P;
}

__host__ __device__ inline bool pgiven(const PGeom& g, int I) { return !g.factor && I < g.M; }

__host__ __device__ inline PWaits pitem_waits(const PGeom& g, const PItem& it)
{
    const int kind = it.kind_sub & 15;
    const int I = it.I, K = it.K, J = it.J;
    PWaits w;
    if (kind == PI_POTRF) {
        w.sig = ptile(J, J);
        w.cnt[0] = ptile(J, J);
        w.val[0] = (unsigned)J * pnblk(g, J, J);
        w.cnt[1] = w.cnt[2] = w.sig;
        w.val[1] = w.val[2] = 0u;
    } else if (kind == PI_TRSM) {
        w.sig = ptile(I, J);
        w.cnt[0] = ptile(I, J);
        w.val[0] = (unsigned)J * pnblk(g, I, J);
        w.cnt[1] = ptile(J, J);
        w.val[1] = pgiven(g, J) ? 0u : pfinal(g, J, J);
        w.cnt[2] = w.sig;
        w.val[2] = 0u;
    } else {
        w.sig = ptile(I, K);
        w.cnt[0] = ptile(I, J);
        w.val[0] = pgiven(g, I) ? 0u : pfinal(g, I, J);
        w.cnt[1] = ptile(K, J);
        w.val[1] = (pgiven(g, K) || K == I) ? 0u : pfinal(g, K, J);
        w.cnt[2] = ptile(I, K);
        w.val[2] = (unsigned)J * pnblk(g, I, K);
    }
    return w;
}

}  // namespace gpr
