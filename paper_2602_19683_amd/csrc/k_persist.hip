// k_persist.hip -- the persistent sweep executor: the whole tile task graph of
// a sweep (Fig. 1 on the extended matrix, see persist.h) in one launch.
//
// A grid of as many 256-thread workgroups as fit on the chip at once loops:
// take the next ticket (one atomic increment), wait until the item's input
// tiles are final (relaxed polling of per-tile progress counters, then one
// device-scope acquire), run the item with the same device routine the
// stream kernels use (POTRF panel, TRSM strip, update block), and count it
// done with a device-scope release. Each output element is computed by the
// same instructions in the same order as under the stream executor, so the
// two executors agree bit for bit.
//
// Counters and the ticket are cleared by a fill kernel on the same stream
// before the launch. A wait that exceeds its spin limit sets *err; after
// that every wait returns at once, so the grid still drains.
#include "gpr_internal.h"
#include "k_common.h"
#include "k_potrf_dev.h"
#include "k_trsm_dev.h"
#include "k_update_dev.h"
#include "k_update_mixed_dev.h"
#include "persist.h"

namespace gpr {

namespace {

constexpr unsigned PSPIN_LIMIT = 1u << 22;  // a few seconds of polling

struct PersistArgs {
    const PItem* items;
    int64_t nitems;
    TileMat K;     // training lower tiles (the factor)
    double* tinv;  // inverses of the diagonal tiles of the factor
    TileMat V;     // test rows x M tiles
    TileMat S;     // test lower tiles
    PGeom g;
    int m;
    unsigned* cnt;     // progress counter per tile of the extended matrix
    unsigned* ticket;
    unsigned* flags;   // POTRF panel flags (2 m / 32)
    unsigned epoch0;   // POTRF(J) publishes epoch0 + J
    int* info;
    int* err;
};

__device__ inline double* ext_tile(const PersistArgs& a, int I, int K)
{
    if (I < a.g.M) return tile_ptr(a.K, I, K);
    if (K < a.g.M) return tile_ptr(a.V, I - a.g.M, K);
    return tile_ptr(a.S, I - a.g.M, K - a.g.M);
}

__device__ inline bool wait_count(const unsigned* c, unsigned v, int* err)
{
    unsigned it = 0;
    while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) {
        if ((it & 255) == 255 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return false;
        __builtin_amdgcn_s_sleep(2);
        if (++it > PSPIN_LIMIT) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

template <int BM>
union PersistLds {
    UpdLds<BM> u;
    UpdLdsF32<BM> uf;
    PotrfLds p;
    TrsmLds t;
};

}  // namespace

// F32: the update items round their operands to FP32 (the mixed-precision
// sweep); POTRF and TRSM items stay FP64.
template <int BM, bool F32>
__global__ __launch_bounds__(256, 2) void k_persist(PersistArgs a)
{
    __shared__ PersistLds<BM> sh;
    __shared__ unsigned s_ticket;
    const int tid = threadIdx.x;
    const int m = a.m;
    // The loop has one exit, at its head, on a workgroup-uniform value, and
    // the only divergent regions (thread 0's waits, counter increment and
    // next ticket) sit between two barriers. (A "for (;;)" with the ticket
    // taken at the top and a break after the barrier let the compiler split
    // the loop so that the other lanes of thread 0's wave re-ran the barrier
    // and the body with a stale ticket while thread 0 waited to take the next
    // one, which never ends.)
    if (tid == 0) s_ticket = __hip_atomic_fetch_add(a.ticket, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    // uniform across the workgroup: keeps the item and every address derived
    // from it in scalar registers
    unsigned t = __builtin_amdgcn_readfirstlane(s_ticket);
    while ((int64_t)t < a.nitems) {
        const PItem it = a.items[t];
        const PWaits w = pitem_waits(a.g, it);
        if (tid == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (w.val[k] != 0u) (void)wait_count(a.cnt + w.cnt[k], w.val[k], a.err);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        // the thread index, opaque to the compiler from here on: index
        // arithmetic of the three routines is then not hoisted out of the
        // loop, where it would stay live in registers across every item
        int ltid = tid;
        __asm__ volatile("" : "+v"(ltid));
        const int kind = it.kind_sub & 15, sub = it.kind_sub >> 4;
        if (kind == PI_UPDATE) {
            const int nb = a.g.nb;
            int bi, bj;
            if (it.I == it.K) {  // lower blocks in row order: sub = bi (bi + 1) / 2 + bj
                bi = 0;
                while ((bi + 1) * (bi + 2) / 2 <= sub) ++bi;
                bj = sub - bi * (bi + 1) / 2;
            } else {
                bi = sub / nb;
                bj = sub - bi * nb;
            }
            const UpdateTask tk{ext_tile(a, it.I, it.K), ext_tile(a, it.I, it.J),
                                ext_tile(a, it.K, it.J), m, m, m, it.I == it.K ? TASK_DIAG : 0};
            if (F32)
                update_block_f32<BM, 2, 2>(tk, bi, bj, m, sh.uf, ltid);
            else
                update_block<BM, 2, 2>(tk, bi, bj, m, sh.u, ltid);
        } else if (kind == PI_TRSM) {
            const TrsmTask tk{ext_tile(a, it.I, it.J), ext_tile(a, it.J, it.J),
                              a.tinv + (size_t)it.J * m * m, nullptr, m, m, m, 0};
            trsm_strip(tk, sub, m, sh.t, ltid);
        } else {
            potrf_panel(ext_tile(a, it.J, it.J), m, m, a.tinv + (size_t)it.J * m * m, m, a.info,
                        (int64_t)it.J * m, a.flags, a.epoch0 + (unsigned)it.J, a.err, sub, sh.p,
                        ltid);
        }
        __syncthreads();
        if (tid == 0) {
            __hip_atomic_fetch_add(a.cnt + w.sig, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            s_ticket = __hip_atomic_fetch_add(a.ticket, 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        t = __builtin_amdgcn_readfirstlane(s_ticket);
    }
}

__global__ void k_zero_u32(unsigned* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Update blocks of 128 x 128 (four waves of 64 x 64) where the tile allows:
// fewer, larger items reuse each loaded operand twice as often as 64 x 64
// blocks (measured 1.4x faster for the whole sweep at m = 512).
int persist_block(int m) { return m % 128 == 0 ? 128 : (m % 64 == 0 ? 64 : 32); }

namespace {

template <bool F32>
hipError_t occupancy(int* per, int bm)
{
    if (bm == 128) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_persist<128, F32>, 256, 0);
    if (bm == 64) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_persist<64, F32>, 256, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_persist<32, F32>, 256, 0);
}

template <bool F32>
void launch(int bm, dim3 grid, hipStream_t s, const PersistArgs& a)
{
    if (bm == 128)
        hipLaunchKernelGGL((k_persist<128, F32>), grid, dim3(256), 0, s, a);
    else if (bm == 64)
        hipLaunchKernelGGL((k_persist<64, F32>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_persist<32, F32>), grid, dim3(256), 0, s, a);
}

}  // namespace

int persist_workers(int bm, int prec)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const hipError_t e = prec == GPR_MIXED_FP32 ? occupancy<true>(&per, bm)
                                                : occupancy<false>(&per, bm);
    if (e != hipSuccess) return 0;
    return per * cus;
}

hipError_t launch_persist(const PItem* d_items, int64_t nitems, const PGeom& g, int m, int bm,
                          int prec, int workers, const TileMat& K, double* tinv, const TileMat& V,
                          const TileMat& S, unsigned* d_cnt, int64_t ncnt, unsigned* flags,
                          unsigned epoch0, int* info, int* err, hipStream_t s)
{
    // counters and the ticket (d_cnt[ncnt]) start at zero
    const int64_t nz = ncnt + 1;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, d_cnt, nz);
    if (nitems <= 0) return hipGetLastError();
    PersistArgs a{d_items, nitems, K, tinv, V, S, g, m, d_cnt, d_cnt + ncnt, flags, epoch0,
                  info, err};
    const dim3 grid((unsigned)std::min<int64_t>(workers, nitems));
    if (prec == GPR_MIXED_FP32)
        launch<true>(bm, grid, s, a);
    else
        launch<false>(bm, grid, s, a);
    return hipGetLastError();
}

}  // namespace gpr
