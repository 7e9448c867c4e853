// api.hip -- C entry points of libgpr: context, tiled handles, and the
// executor that runs the tile schedule (schedule.cpp) on two HIP streams.
//
// Memory layout in HBM (n padded up to M m, test size up to Mhat m):
//   K / L      lower tiles, M (M + 1) / 2 tiles of m x m, tile-contiguous
//              row-major (Sec. 4.2: only the lower tiles are stored);
//   Tinv       M tiles, the inverses of the diagonal tiles of L;
//   V^T        Mhat x M tiles of K_{X*,X} solved in place into K_{X*,X} L^{-T};
//   Sigma      Mhat (Mhat + 1) / 2 lower tiles, exported to the caller's
//              dense row-major n_test x n_test array with both triangles;
//   vectors    y, beta, alpha padded to M m.
// Task descriptors for every launch of a call are built on the host, copied
// to the device in one transfer, and the launches index into them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "gpr_internal.h"

using namespace gpr;

// Work vectors of gpr_solve_noalloc: the right-hand side padded to whole
// tiles, the forward result and the solves' copy of their right-hand side,
// GPR_NOALLOC_MAX_N doubles each (3 MiB). Every GPU the library runs on holds
// one copy until the process ends. Host code never passes this name to a
// kernel: it is a host-side stand-in; the device address of each GPU's copy
// is taken once per device, at context creation, and kept below.
static __device__ __align__(256) double scratch[3 * GPR_NOALLOC_MAX_N];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Records the device address of `scratch` on the current device (`device`).
int scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return GPR_ENODEV;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return GPR_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return GPR_EHIP;
    g_scratch_dev[device] = static_cast<double*>(p);
    return GPR_OK;
}

double* scratch_device_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[device];
}
}  // namespace

// Device bytes held by a context's workspace and by the handles it created,
// against the cap read from the environment variable GPR_MAX_DEVICE_BYTES
// when the context was created (none if unset or 0). Handles keep the
// counter alive after their context is destroyed.
struct DevBudget {
    std::atomic<uint64_t> used{0};
    uint64_t cap = UINT64_MAX;
};
using Budget = std::shared_ptr<DevBudget>;

// Device flag words of a context: [0, 64) the POTRF row-panel flags (two per
// 32-row panel of a tile of up to 1024 rows), SIGNAL_FLAG the flag stored
// after an update launch that a fused POTRF + TRSM launch waits for.
constexpr int SIGNAL_FLAG = 64;
constexpr int FLAG_WORDS = 128;

struct gpr_ctx {
    int device = 0;
    Budget budget;                // device bytes held and their cap
    int n_streams = 3;            // 1: every launch on the caller's stream
    hipStream_t panel = nullptr;  // panel TRSMs and next-column GEMMs
    hipStream_t bulk = nullptr;   // trailing updates
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_last = nullptr, ev_desc = nullptr;
    bool last_valid = false, desc_valid = false;
    std::vector<hipEvent_t> evpool;
    int* d_info = nullptr;        // [0]: this factorisation, [1]: sticky since gpr_sync,
                                  // [2]: a device-side wait hit its limit
    unsigned* d_flags = nullptr;  // POTRF row-panel flags
    unsigned epoch = 0;
    unsigned sigseq = 0;          // values stored by launch_signal (d_flags[SIGNAL_FLAG])
    int variant = GPR_RIGHT_LOOKING;  // task order of the sweeps
    char* d_part = nullptr;       // part tiles of split (left-looking) updates
    size_t part_cap = 0;
    char* d_desc = nullptr;
    size_t desc_cap = 0;
    char* h_desc = nullptr;       // pinned staging
    size_t hdesc_cap = 0;
    char* d_ws = nullptr;         // prediction workspace
    size_t ws_cap = 0;
    gpr_tiled* scratch = nullptr; // for gpr_cholesky_dense
    gpr_tiled* nlml_K = nullptr;  // factor kept by gpr_nlml_grad
    char* d_fit = nullptr;        // gpr_fit_hyper: NLML and gradient, Adam state, NLML trace
    size_t fit_cap = 0;
    char* d_adj = nullptr;        // adjoint workspace (Lbar, Abar, partial tiles)
    size_t adj_cap = 0;
    // persistent executor: ticket order of the last sweep shape (device copy)
    int executor = GPR_EXEC_STREAMS;
    char* d_pitems = nullptr;
    size_t pitems_cap = 0;
    int64_t pkey[6] = {-1, -1, -1, -1, -1, -1};
    int64_t p_nitems = 0;
    int p_workers = 0, p_bm = 0, p_prec = -1;
    char* d_pcnt = nullptr;       // progress counters + ticket
    size_t pcnt_cap = 0;
    // instrumentation
    bool prof_on = false;
    std::vector<hipEvent_t> tpool;  // timing events, reused after each read
    size_t tpool_used = 0;
    struct ProfRec {
        int kind;
        hipEvent_t a, b;
        double flops, bytes;
    };
    std::vector<ProfRec> pending;
    int64_t p_launches[11] = {};
    double p_ms[11] = {}, p_flops[11] = {}, p_bytes[11] = {};
};

// One launch of the group-inverse build: byte offsets of its tasks and terms
// in the handle's descriptor buffer, and its task count.
struct TinvLaunch {
    size_t task_off, term_off;
    int ntask;
};

struct gpr_tiled {
    int device = 0;
    Budget budget;                // the creating context's counter
    size_t dev_bytes = 0;         // device bytes this handle holds
    int64_t n = 0;
    int m = 0;
    int M = 0;
    double* data = nullptr;
    double* tinv = nullptr;
    double* kcopy = nullptr;      // FP64 copy of K kept by a mixed-precision factorisation
    double* tpair = nullptr;      // off-diagonal tiles of the solves' group inverses, then scratch
    char* tpair_desc = nullptr;   // device descriptors of the launches that build them (fixed per handle)
    char* tpair_host = nullptr;   // their pinned host copy
    std::vector<TinvLaunch> tg_launches;  // those launches: descriptor offsets, task counts
    double tg_flops = 0.0;
    int tgroup = 0;               // tile rows per step of the vector solves (G)
    size_t tpair_bytes = 0;       // sizes of tpair and tpair_desc
    size_t tdesc_bytes = 0;
    int state = GPR_STATE_EMPTY;
    int prec = GPR_FP64;
};

namespace {

#define HIP_TRY(expr)                                 \
    do {                                              \
        if ((expr) != hipSuccess) return GPR_EHIP;    \
    } while (0)

// The number of devices is read once per process (the query costs far more
// than a launch, and every entry point checks its device); the device is made
// current only when it is not already.
int check_device(int device)
{
    static int count = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int c = 0;
        count = hipGetDeviceCount(&c) == hipSuccess ? c : 0;
    });
    if (count <= 0) return GPR_ENODEV;
    if (device < 0 || device >= count) return GPR_ENODEV;
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur == device) return GPR_OK;
    if (hipSetDevice(device) != hipSuccess) return GPR_EHIP;
    return GPR_OK;
}

bool valid_tile(int32_t tile) { return tile >= 32 && tile <= 1024 && tile % 32 == 0; }

bool valid_hyper(const gpr_hyper& h)
{
    return std::isfinite(h.lengthscale) && std::isfinite(h.vertical_variance) &&
           std::isfinite(h.noise_variance) && h.lengthscale > 0 && h.vertical_variance > 0;
}

// hipMalloc counted against the budget: GPR_ENOMEM if it would exceed the
// cap or the allocation fails.
int budget_malloc(const Budget& b, void** p, size_t bytes)
{
    *p = nullptr;
    if (b) {
        uint64_t cur = b->used.load();
        do {
            if (bytes > b->cap || cur > b->cap - bytes) return GPR_ENOMEM;
        } while (!b->used.compare_exchange_weak(cur, cur + bytes));
    }
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        if (b) b->used -= bytes;
        return GPR_ENOMEM;
    }
    return GPR_OK;
}

void budget_free(const Budget& b, void* p, size_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    if (b) b->used -= bytes;
}

// Device memory of a handle, counted against its context's budget.
int handle_malloc(gpr_tiled* T, void** p, size_t bytes)
{
    const int rc = budget_malloc(T->budget, p, bytes);
    if (rc == GPR_OK) T->dev_bytes += bytes;
    return rc;
}

int ensure_device_bytes(const Budget& b, char** p, size_t* cap, size_t need)
{
    if (need <= *cap) return GPR_OK;
    if (*p) {
        if (hipDeviceSynchronize() != hipSuccess) return GPR_EHIP;
        budget_free(b, *p, *cap);
        *p = nullptr;
        *cap = 0;
    }
    size_t want = need + need / 4;
    const int rc = budget_malloc(b, reinterpret_cast<void**>(p), want);
    if (rc) return rc;
    *cap = want;
    return GPR_OK;
}

// Host-side builder for the task descriptors of one call. Each segment is
// 64-byte aligned; `upload` copies everything to the device in one transfer.
struct DescBuffer {
    std::vector<char> host;
    size_t add(const void* data, size_t bytes)
    {
        size_t off = (host.size() + 63) & ~size_t(63);
        host.resize(off + bytes);
        if (bytes) std::memcpy(host.data() + off, data, bytes);
        return off;
    }
    int upload(gpr_ctx* ctx, hipStream_t s)
    {
        if (host.empty()) return GPR_OK;
        const size_t bytes = host.size();
        if (ctx->desc_valid) HIP_TRY(hipEventSynchronize(ctx->ev_desc));
        if (bytes > ctx->hdesc_cap) {
            if (ctx->h_desc) (void)hipHostFree(ctx->h_desc);
            ctx->h_desc = nullptr;
            ctx->hdesc_cap = 0;
            if (hipHostMalloc(reinterpret_cast<void**>(&ctx->h_desc), bytes * 2) != hipSuccess)
                return GPR_ENOMEM;
            ctx->hdesc_cap = bytes * 2;
        }
        int rc = ensure_device_bytes(ctx->budget, &ctx->d_desc, &ctx->desc_cap, bytes);
        if (rc) return rc;
        std::memcpy(ctx->h_desc, host.data(), bytes);
        HIP_TRY(hipMemcpyAsync(ctx->d_desc, ctx->h_desc, bytes, hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(ctx->ev_desc, s));
        ctx->desc_valid = true;
        return GPR_OK;
    }
    template <class T>
    const T* dev(gpr_ctx* ctx, size_t off) const
    {
        return reinterpret_cast<const T*>(ctx->d_desc + off);
    }
};

int ensure_events(gpr_ctx* ctx, size_t n)
{
    while (ctx->evpool.size() < n) {
        hipEvent_t e;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->evpool.push_back(e);
    }
    return GPR_OK;
}

enum ProfKind { PK_POTRF = 0, PK_TRTRI = 1, PK_TRSM = 2, PK_UPDATE = 3, PK_ASSEMBLE = 4,
                PK_TRSV = 5, PK_MATVEC = 6, PK_EXPORT = 7, PK_ADJOINT = 8, PK_REDUCE = 9,
                PK_PERSIST = 10, PK_COUNT = 11 };

hipEvent_t timing_event(gpr_ctx* ctx)
{
    if (ctx->tpool_used == ctx->tpool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->tpool.push_back(e);
    }
    return ctx->tpool[ctx->tpool_used++];
}

const char* const kProfName[PK_COUNT] = {"potrf", "trtri", "trsm", "update", "assemble", "trsv",
                                         "matvec", "export", "adjoint", "reduce", "persist"};

// A host-side range in a tool's marker trace (roctx; no cost without a tool):
// one per entry point and one per launch group (ProfScope), so a trace shows
// the phases of a call.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

// Brackets one launch with timing events while profiling is on, and with a
// marker range named for its kind.
struct ProfScope {
    gpr_ctx* c;
    hipStream_t s;
    int kind;
    double flops, bytes;
    hipEvent_t a = nullptr;
    Range range;
    ProfScope(gpr_ctx* c_, hipStream_t s_, int k, double f, double b)
        : c(c_), s(s_), kind(k), flops(f), bytes(b), range(kProfName[k])
    {
        if (c->prof_on && (a = timing_event(c)) != nullptr) (void)hipEventRecord(a, s);
    }
    ~ProfScope()
    {
        if (!a) return;
        hipEvent_t b = timing_event(c);
        if (!b) return;
        (void)hipEventRecord(b, s);
        c->pending.push_back({kind, a, b, flops, bytes});
    }
};

int resolve_profile(gpr_ctx* ctx)
{
    for (const auto& r : ctx->pending) {
        HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        ctx->p_launches[r.kind] += 1;
        ctx->p_ms[r.kind] += ms;
        ctx->p_flops[r.kind] += r.flops;
        ctx->p_bytes[r.kind] += r.bytes;
    }
    ctx->pending.clear();
    ctx->tpool_used = 0;
    return GPR_OK;
}

// Start of every call: order after the previous call of this context.
int begin_call(gpr_ctx* ctx, hipStream_t s)
{
    int rc = check_device(ctx->device);
    if (rc) return rc;
    if (ctx->last_valid) HIP_TRY(hipStreamWaitEvent(s, ctx->ev_last, 0));
    return GPR_OK;
}

int end_call(gpr_ctx* ctx, hipStream_t s)
{
    HIP_TRY(hipEventRecord(ctx->ev_last, s));
    ctx->last_valid = true;
    return GPR_OK;
}

// Pointers of the extended lower-tiled matrix used by the sweep.
struct SweepMats {
    TileMat K;        // training lower tiles
    double* tinv;     // M tiles
    TileMat V;        // Mhat x M
    TileMat S;        // Mhat lower tiles
    int M, Mhat, m;
    int prec;         // precision of the tile updates
    double* at(int I, int K_) const
    {
        if (I < M) return tile_ptr(K, I, K_);
        if (K_ < M) return tile_ptr(V, I - M, K_);
        return tile_ptr(S, I - M, K_ - M);
    }
};

struct SweepPlan {
    int mode = SWEEP_CHOLESKY;
    bool persistent = false;  // run by the persistent executor (no descriptors)
    Schedule sched;
    std::vector<size_t> off;  // descriptor offset per launch
    std::vector<int> nt;      // update launches: kernel tasks (split parts included)
    std::vector<size_t> roff; // update launches: ReduceTask descriptors
    std::vector<int> nred;    // update launches: tasks of the part sums (0: not split)
    int err = GPR_OK;         // the part buffer could not be allocated
};

// A long multi-term update launch (left-looking) with few 128 x 128 blocks is
// split along k so that it fills the chip: each task is cut into up to
// SPLIT_MAX runs of consecutive terms, whose sums go to part tiles, added to
// the tile in run order by a second kernel. Only bulk-stream launches split
// (they run one after the other, so one part buffer serves them all).
constexpr long SPLIT_TARGET = 1024;  // workgroups to aim for
constexpr int SPLIT_MAX = 8;

// The persistent executor runs FP64 and FP32-update sweeps; a context created
// for it runs the BF16 sweeps (whose updates have no persistent form) on the
// streams. GPR_EXEC_AUTO takes it for sweeps of small tiles over a small
// matrix, where the streams' per-step launches dominate.
bool use_persistent(const gpr_ctx* ctx, const SweepMats& X)
{
    const bool chosen =
        ctx->executor == GPR_EXEC_PERSISTENT ||
        (ctx->executor == GPR_EXEC_AUTO && X.m <= GPR_AUTO_PERSIST_TILE &&
         (int64_t)(X.M + X.Mhat) * X.m <= GPR_AUTO_PERSIST_ROWS);
    return chosen && ctx->variant == GPR_RIGHT_LOOKING &&
           (X.prec == GPR_FP64 || X.prec == GPR_MIXED_FP32);
}

// Builds the descriptors of a sweep into `db` (and sizes the part buffer of
// split updates).
SweepPlan plan_sweep(gpr_ctx* ctx, const SweepMats& X, int mode, DescBuffer& db)
{
    SweepPlan P;
    P.mode = mode;
    P.persistent = use_persistent(ctx, X);
    if (P.persistent) return P;
    P.sched = build_schedule_variant(X.M, X.Mhat, mode, ctx->variant);
    const size_t nl = P.sched.launches.size();
    P.off.assign(nl, 0);
    P.nt.assign(nl, 0);
    P.roff.assign(nl, 0);
    P.nred.assign(nl, 0);
    const int m = X.m;
    const size_t m2 = (size_t)m * m;
    // runs per task of each update launch, and the part tiles it needs
    std::vector<int> split(nl, 1);
    size_t parts_max = 0;
    for (size_t li = 0; li < nl; ++li) {
        const SchedLaunch& L = P.sched.launches[li];
        if (L.kind != LK_UPDATE || L.stream != 2 || m % 128 != 0) continue;
        const long nb = m / 128;
        long blocks = 0;
        int maxnk = 1;
        for (int t = L.first; t < L.first + L.count; ++t) {
            const SchedTask& k = P.sched.tasks[t];
            blocks += k.kind == K_SYRK ? nb * (nb + 1) / 2 : nb * nb;
            maxnk = std::max(maxnk, k.nk);
        }
        if (maxnk < 2 || blocks >= SPLIT_TARGET) continue;
        const int S = (int)std::min<long>({(long)maxnk, (SPLIT_TARGET + blocks - 1) / blocks,
                                          (long)SPLIT_MAX});
        if (S < 2) continue;
        split[li] = S;
        size_t parts = 0;
        for (int t = L.first; t < L.first + L.count; ++t)
            if (P.sched.tasks[t].nk >= 2) parts += std::min(S, P.sched.tasks[t].nk);
        parts_max = std::max(parts_max, parts);
    }
    double* part_base = nullptr;
    if (parts_max) {
        P.err = ensure_device_bytes(ctx->budget, &ctx->d_part, &ctx->part_cap,
                                    parts_max * m2 * sizeof(double));
        if (P.err) return P;
        part_base = reinterpret_cast<double*>(ctx->d_part);
    }
    for (size_t li = 0; li < nl; ++li) {
        const SchedLaunch& L = P.sched.launches[li];
        if (L.kind == LK_TRSM) {
            std::vector<TrsmTask> v;
            for (int t = L.first; t < L.first + L.count; ++t) {
                const SchedTask& k = P.sched.tasks[t];
                v.push_back({X.at(k.I, k.J), X.at(k.J, k.J), X.tinv + (size_t)k.J * m * m,
                             nullptr, m, m, m, 0});
            }
            P.off[li] = db.add(v.data(), v.size() * sizeof(TrsmTask));
        } else if (L.kind == LK_UPDATE) {
            std::vector<UpdateTask> v;
            std::vector<ReduceTask> red;
            size_t used = 0;  // part tiles handed out in this launch
            for (int t = L.first; t < L.first + L.count; ++t) {
                const SchedTask& k = P.sched.tasks[t];
                UpdateTask u{X.at(k.I, k.K), X.at(k.I, k.J), X.at(k.K, k.J), m, m, m,
                             k.kind == K_SYRK ? TASK_DIAG : 0};
                u.nk = k.nk;
                u.kstride = (long long)m2;  // tiles (I, k), k = J.. are adjacent
                const int runs = k.nk >= 2 ? std::min(split[li], k.nk) : 1;
                if (runs == 1) {
                    v.push_back(u);
                    continue;
                }
                ReduceTask r{u.C, part_base + used * m2, (long long)m2, m, runs, u.flags, 0};
                red.push_back(r);
                for (int c = 0; c < runs; ++c) {
                    const int k0 = c * k.nk / runs, k1 = (c + 1) * k.nk / runs;
                    UpdateTask w = u;
                    w.A = X.at(k.I, k.J + k0);
                    w.B = X.at(k.K, k.J + k0);
                    w.nk = k1 - k0;
                    w.part = part_base + (used + c) * m2;
                    v.push_back(w);
                }
                used += runs;
            }
            P.off[li] = db.add(v.data(), v.size() * sizeof(UpdateTask));
            P.nt[li] = (int)v.size();
            if (!red.empty()) {
                P.roff[li] = db.add(red.data(), red.size() * sizeof(ReduceTask));
                P.nred[li] = (int)red.size();
            }
        }
    }
    return P;
}

// The whole sweep as one persistent launch on s (k_persist.hip). The ticket
// order depends only on the shape and is kept in the context.
int run_persist(gpr_ctx* ctx, const SweepMats& X, int mode, hipStream_t s)
{
    const int m = X.m, M = X.M, bm = persist_block(m);
    const int Mhat = sweep_test_rows(mode) ? X.Mhat : 0;
    if (ctx->p_workers <= 0 || ctx->p_bm != bm || ctx->p_prec != X.prec) {
        ctx->p_workers = persist_workers(bm, X.prec);
        ctx->p_bm = bm;
        ctx->p_prec = X.prec;
        if (ctx->p_workers <= 0) return GPR_EHIP;
    }
    const int64_t key[6] = {M, Mhat, mode, m, bm, ctx->p_workers};
    if (!std::equal(key, key + 6, ctx->pkey)) {
        const std::vector<PItem> order = build_persist_order(M, Mhat, mode, m, bm, ctx->p_workers);
        const size_t bytes = order.size() * sizeof(PItem);
        // the previous order may still be read by a running sweep
        HIP_TRY(hipStreamSynchronize(s));
        int rc = ensure_device_bytes(ctx->budget, &ctx->d_pitems, &ctx->pitems_cap, bytes > 0 ? bytes : 64);
        if (rc) return rc;
        if (bytes) HIP_TRY(hipMemcpy(ctx->d_pitems, order.data(), bytes, hipMemcpyHostToDevice));
        std::copy(key, key + 6, ctx->pkey);
        ctx->p_nitems = (int64_t)order.size();
    }
    const PGeom g = persist_geom(M, Mhat, mode, m, bm);
    const int64_t ncnt = (int64_t)g.T * (g.T + 1) / 2;
    int rc = ensure_device_bytes(ctx->budget, &ctx->d_pcnt, &ctx->pcnt_cap, (size_t)(ncnt + 1) * sizeof(unsigned));
    if (rc) return rc;
    // flops of the tile tasks (Fig. 1 counts: POTRF m^3/3, TRSM m^3, SYRK m^3,
    // GEMM 2 m^3)
    const bool block = sweep_test_block(mode);
    double tasks = 0.0;
    for (int J = 0; J < M; ++J) {
        const int I0 = g.factor ? J + 1 : M;
        const double rows = g.T - I0;  // TRSM tasks of column J
        double upd = 0.0;              // update flops of step J in units of m^3
        for (int I = I0; I < g.T; ++I)
            for (int K = J + 1; K <= I; ++K)
                if (block || K < M) upd += K == I ? 1.0 : 2.0;  // SYRK 1, GEMM 2
        tasks += (g.factor ? 1.0 / 3.0 : 0.0) + rows + upd;
    }
    const unsigned epoch0 = ctx->epoch + 1;
    ctx->epoch += (unsigned)M;
    ProfScope ps(ctx, s, PK_PERSIST, tasks * (double)m * m * m, 0.0);
    HIP_TRY(launch_persist(reinterpret_cast<const PItem*>(ctx->d_pitems), ctx->p_nitems, g, m, bm,
                           X.prec, ctx->p_workers, X.K, X.tinv, X.V, X.S,
                           reinterpret_cast<unsigned*>(ctx->d_pcnt), ncnt, ctx->d_flags, epoch0,
                           ctx->d_info, ctx->d_info + 2, s));
    return GPR_OK;
}

// Issues the launches of a planned sweep. Logical streams: 0 critical (the
// caller's stream s), 1 panel, 2 bulk; with fewer streams in the context
// they fold onto s. The extra streams fork from s and join back into it.
// The extra streams join back into s: s waits for everything issued on them.
int join_sweep(gpr_ctx* ctx, hipStream_t s)
{
    hipStream_t phys[3] = {s, ctx->n_streams >= 3 ? ctx->panel : s,
                           ctx->n_streams >= 2 ? ctx->bulk : s};
    for (int q = 1; q < 3; ++q) {
        if (phys[q] == s || (q == 2 && phys[2] == phys[1])) continue;
        HIP_TRY(hipEventRecord(ctx->ev_join, phys[q]));
        HIP_TRY(hipStreamWaitEvent(s, ctx->ev_join, 0));
    }
    return GPR_OK;
}

// With join false the caller joins later (join_sweep): work issued on s in
// between runs after the sweep's launches on s only, beside the rest.
int run_sweep(gpr_ctx* ctx, const SweepMats& X, const SweepPlan& P, const DescBuffer& db,
              hipStream_t s, bool join = true)
{
    if (P.err) return P.err;
    if (P.persistent) return run_persist(ctx, X, P.mode, s);
    const auto& Ls = P.sched.launches;
    int rc = ensure_events(ctx, Ls.size());
    if (rc) return rc;
    hipStream_t phys[3] = {s, ctx->n_streams >= 3 ? ctx->panel : s,
                           ctx->n_streams >= 2 ? ctx->bulk : s};
    std::vector<char> waited(Ls.size(), 0);
    for (const auto& L : Ls)
        for (int k = 0; k < L.nwait; ++k)
            if (phys[Ls[L.wait[k]].stream] != phys[L.stream]) waited[L.wait[k]] = 1;
    // A POTRF followed on its stream by the one-tile TRSM of the next tile row
    // (the critical TRSM) runs as one launch, the TRSM strips following the
    // POTRF's row panels. The TRSM's wait for an update on another stream
    // becomes a device flag: that update launch is followed by a signal.
    std::vector<char> fused(Ls.size(), 0);      // TRSM launch run inside the POTRF before it
    std::vector<unsigned> signal(Ls.size(), 0); // value to signal after this launch (0: none)
    std::vector<unsigned> ready(Ls.size(), 0);  // POTRF launch: value its TRSM strips wait for
    // In FP64 and FP32-update sweeps, the one-tile SYRK that precedes a POTRF
    // on its stream (the last update of the diagonal tile) is applied by the
    // POTRF's own workgroups, in the sweep's update arithmetic.
    std::vector<int> syrk_of(Ls.size(), -1);    // POTRF launch: the SYRK launch it absorbs
    std::vector<char> absorbed(Ls.size(), 0);   // SYRK launch issued with a later POTRF
    {
        std::vector<int> last_on(3, -1);
        for (size_t li = 0; li < Ls.size(); ++li) {
            const SchedLaunch& L = Ls[li];
            const int pv = last_on[L.stream];
            last_on[L.stream] = (int)li;
            if (L.kind != LK_POTRF || pv < 0) continue;
            if (X.prec != GPR_FP64 && X.prec != GPR_MIXED_FP32) continue;
            const SchedLaunch& S = Ls[pv];
            if (S.kind != LK_UPDATE || S.count != 1) continue;
            const SchedTask& t = P.sched.tasks[S.first];
            if (t.kind != K_SYRK || t.I != L.step || t.K != L.step || t.nk != 1) continue;
            syrk_of[li] = pv;
            absorbed[pv] = 1;
        }
    }
    for (size_t li = 0; li + 1 < Ls.size(); ++li) {
        const SchedLaunch &Lp = Ls[li], &Lt = Ls[li + 1];
        if (Lp.kind != LK_POTRF || Lt.kind != LK_TRSM || Lt.count != 1 || Lp.stream != Lt.stream)
            continue;
        int cross = -1, ncross = 0;
        for (int k = 0; k < Lt.nwait; ++k)
            if (phys[Ls[Lt.wait[k]].stream] != phys[Lt.stream]) {
                cross = Lt.wait[k];
                ++ncross;
            }
        if (ncross > 1) continue;
        fused[li + 1] = 1;
        if (cross >= 0) {
            if (!signal[cross]) signal[cross] = ++ctx->sigseq;
            ready[li] = signal[cross];
        }
    }
    HIP_TRY(hipEventRecord(ctx->ev_fork, s));
    for (int q = 1; q < 3; ++q) {
        if (phys[q] == s || (q == 2 && phys[2] == phys[1])) continue;
        HIP_TRY(hipStreamWaitEvent(phys[q], ctx->ev_fork, 0));
    }
    const int m = X.m;
    // after a failed pivot the rest of a factorising sweep is skipped (the
    // record was reset before this sweep; a sweep with a given factor has none)
    const int* abort_info = sweep_factors(P.mode) ? ctx->d_info : nullptr;
    unsigned* sigflag = ctx->d_flags + SIGNAL_FLAG;
    for (size_t li = 0; li < Ls.size(); ++li) {
        const SchedLaunch& L = Ls[li];
        hipStream_t st = phys[L.stream];
        if (fused[li]) {  // issued with the POTRF before it
            if (waited[li]) HIP_TRY(hipEventRecord(ctx->evpool[li], st));
            continue;
        }
        if (absorbed[li]) continue;  // issued with the POTRF after it
        auto wait_for = [&](const SchedLaunch& W) -> int {
            for (int k = 0; k < W.nwait; ++k)
                if (phys[Ls[W.wait[k]].stream] != st)
                    HIP_TRY(hipStreamWaitEvent(st, ctx->evpool[W.wait[k]], 0));
            return GPR_OK;
        };
        if (L.kind == LK_POTRF && syrk_of[li] >= 0) {
            rc = wait_for(Ls[syrk_of[li]]);
            if (rc) return rc;
        }
        rc = wait_for(L);
        if (rc) return rc;
        const double m3 = (double)m * m * m;
        if (L.kind == LK_POTRF) {
            const int J = L.step;
            double* A = X.at(J, J);
            double* Ti = X.tinv + (size_t)J * m * m;
            const double* syrk =
                syrk_of[li] >= 0 ? X.at(J, P.sched.tasks[Ls[syrk_of[li]].first].J) : nullptr;
            const double fs = syrk ? m3 : 0.0;
            if (li + 1 < Ls.size() && fused[li + 1]) {
                ProfScope ps(ctx, st, PK_POTRF, m3 / 3.0 + m3 + fs, 0.0);
                HIP_TRY(launch_potrf_trsm_f64(A, m, m, Ti, m, ctx->d_info, (int64_t)J * m,
                                              ctx->d_flags, ++ctx->epoch, ctx->d_info + 2,
                                              db.dev<TrsmTask>(ctx, P.off[li + 1]),
                                              ready[li] ? sigflag : nullptr, ready[li], st, syrk,
                                              X.prec == GPR_MIXED_FP32));
            } else {
                ProfScope ps(ctx, st, PK_POTRF, m3 / 3.0 + fs, 0.0);
                HIP_TRY(launch_potrf_f64(A, m, m, Ti, m, ctx->d_info, (int64_t)J * m,
                                         ctx->d_flags, ++ctx->epoch, ctx->d_info + 2, st, syrk,
                                         X.prec == GPR_MIXED_FP32));
            }
            if (syrk_of[li] >= 0 && waited[syrk_of[li]])
                HIP_TRY(hipEventRecord(ctx->evpool[syrk_of[li]], st));
        } else if (L.kind == LK_TRSM) {
            ProfScope ps(ctx, st, PK_TRSM, L.count * m3, 0.0);
            HIP_TRY(launch_trsm_f64(db.dev<TrsmTask>(ctx, P.off[li]), L.count, m, abort_info, st));
        } else {
            double f = 0.0;
            for (int t = L.first; t < L.first + L.count; ++t)
                f += (P.sched.tasks[t].kind == K_SYRK ? m3 : 2.0 * m3) * P.sched.tasks[t].nk;
            ProfScope ps(ctx, st, PK_UPDATE, f, 0.0);
            if (X.prec == GPR_FP64)
                HIP_TRY(launch_update_f64(db.dev<UpdateTask>(ctx, P.off[li]), P.nt[li], m,
                                          abort_info, st));
            else
                HIP_TRY(launch_update_mixed(db.dev<UpdateTask>(ctx, P.off[li]), P.nt[li], m,
                                            X.prec, abort_info, st));
            if (P.nred[li])
                HIP_TRY(launch_update_reduce(db.dev<ReduceTask>(ctx, P.roff[li]), P.nred[li], m,
                                             abort_info, st));
        }
        if (signal[li]) HIP_TRY(launch_signal(sigflag, signal[li], st));
        if (waited[li]) HIP_TRY(hipEventRecord(ctx->evpool[li], st));
    }
    return join ? join_sweep(ctx, s) : GPR_OK;
}

int alloc_tiled(gpr_ctx* ctx, int64_t n, int m, gpr_tiled** out)
{
    gpr_tiled* T = new (std::nothrow) gpr_tiled;
    if (!T) return GPR_ENOMEM;
    T->device = ctx->device;
    T->n = n;
    T->m = m;
    T->M = (int)((n + m - 1) / m);
    T->budget = ctx->budget;
    const size_t tiles = (size_t)T->M * (T->M + 1) / 2;
    const int rc = handle_malloc(T, reinterpret_cast<void**>(&T->data), tiles * m * m * sizeof(double));
    if (rc) {
        delete T;
        return rc;
    }
    *out = T;
    return GPR_OK;
}

TileMat kmat(const gpr_tiled* T) { return TileMat{T->data, T->m, 0, 0}; }

size_t tiled_bytes(const gpr_tiled* T)
{
    return (size_t)T->M * (T->M + 1) / 2 * T->m * T->m * sizeof(double);
}

// A mixed-precision factorisation keeps an FP64 copy of K for the residual
// of the iterative refinement.
int save_kcopy(gpr_tiled* K, hipStream_t s)
{
    if (!K->kcopy) {
        const int rc = handle_malloc(K, reinterpret_cast<void**>(&K->kcopy), tiled_bytes(K));
        if (rc) return rc;
    }
    HIP_TRY(hipMemcpyAsync(K->kcopy, K->data, tiled_bytes(K), hipMemcpyDeviceToDevice, s));
    return GPR_OK;
}

bool valid_prec(int prec, int m)
{
    if (prec == GPR_FP64) return true;
    return (prec == GPR_MIXED_FP32 || prec == GPR_MIXED_BF16) && m % 64 == 0;
}

// Off-diagonal tiles of the inverses of the G x G blocks of tiles that the
// vector solves take in one step (k_trsv.hip; G = trsv_group(m, prec)), built
// by the batched tile-product launches of plan_tinv_groups (solve_plan.cpp):
// W slots in the first half of tpair, the scratch products Y in the second.
// Needs the diagonal-tile inverses; the handle's data and tinv buffers are
// allocated before and never move, so the descriptors are written once per
// handle and group size (a factorisation in another precision may change G).
int build_tinv_pairs(gpr_ctx* ctx, gpr_tiled* L, int prec, hipStream_t s)
{
    const int M = L->M, m = L->m;
    const int G = trsv_group(m, prec);
    if (L->tpair && L->tgroup != G) {
        // earlier solves on any stream may still read the old tiles
        if (hipDeviceSynchronize() != hipSuccess) return GPR_EHIP;
        budget_free(L->budget, L->tpair, L->tpair_bytes);
        budget_free(L->budget, L->tpair_desc, L->tdesc_bytes);
        L->dev_bytes -= L->tpair_bytes + L->tdesc_bytes;
        (void)hipHostFree(L->tpair_host);
        L->tpair = nullptr;
        L->tpair_desc = nullptr;
        L->tpair_host = nullptr;
        L->tpair_bytes = L->tdesc_bytes = 0;
        L->tg_launches.clear();
    }
    L->tgroup = G;
    if (M < 2) return GPR_OK;
    const size_t mm = (size_t)m * m;
    if (!L->tpair) {
        const TinvPlan P = plan_tinv_groups(M, G);
        if (!tinv_plan_valid(P)) return GPR_EINVAL;
        const size_t wbytes = 2 * (size_t)P.nslot * mm * sizeof(double);
        const size_t tb = (P.tasks.size() * sizeof(TGemmTask) + 63) & ~size_t(63);
        const size_t ub = P.terms.size() * sizeof(TGemmTerm);
        double* W = nullptr;
        char* desc = nullptr;
        char* host = nullptr;
        int rc = handle_malloc(L, reinterpret_cast<void**>(&W), wbytes);
        if (rc == GPR_OK) rc = handle_malloc(L, reinterpret_cast<void**>(&desc), tb + ub);
        if (rc == GPR_OK && hipHostMalloc(reinterpret_cast<void**>(&host), tb + ub) != hipSuccess) {
            (void)hipGetLastError();
            host = nullptr;
            rc = GPR_ENOMEM;
        }
        auto drop = [&](int code) {   // nothing kept: the next call plans again
            if (W) {
                budget_free(L->budget, W, wbytes);
                L->dev_bytes -= wbytes;
            }
            if (desc) {
                budget_free(L->budget, desc, tb + ub);
                L->dev_bytes -= tb + ub;
            }
            if (host) (void)hipHostFree(host);
            return code;
        };
        if (rc) return drop(rc);
        double* Y = W + (size_t)P.nslot * mm;
        const TileMat Lm = kmat(L);
        auto ptr = [&](const TinvRef& r) -> const double* {
            switch (r.kind) {
            case TR_L: return tile_ptr(Lm, r.a, r.b);
            case TR_TINV: return L->tinv + (size_t)r.a * mm;
            case TR_W: return W + (size_t)r.a * mm;
            default: return Y + (size_t)r.a * mm;
            }
        };
        TGemmTask* tk = reinterpret_cast<TGemmTask*>(host);
        TGemmTerm* tm = reinterpret_cast<TGemmTerm*>(host + tb);
        for (size_t t = 0; t < P.tasks.size(); ++t) {
            const TinvTaskPlan& k = P.tasks[t];
            tk[t] = TGemmTask{const_cast<double*>(ptr(k.out)), nullptr, nullptr, 0, 0.0, m, m, 0,
                              k.first_term, k.nterm, TG_EPI_NONE};
        }
        for (size_t u = 0; u < P.terms.size(); ++u)
            tm[u] = TGemmTerm{ptr(P.terms[u].A), ptr(P.terms[u].B), P.terms[u].alpha, m, m, 0, 0};
        if (hipMemcpyAsync(desc, host, tb + ub, hipMemcpyHostToDevice, s) != hipSuccess) {
            (void)hipGetLastError();
            return drop(GPR_EHIP);
        }
        L->tpair_desc = desc;
        L->tpair_host = host;
        L->tg_launches.clear();
        for (const TinvLaunchPlan& lp : P.launches)
            L->tg_launches.push_back(TinvLaunch{lp.first_task * sizeof(TGemmTask),
                                                tb + lp.first_term * sizeof(TGemmTerm),
                                                lp.ntask});
        L->tg_flops = 2.0 * (double)P.terms.size() * m * mm;
        L->tpair = W;
        L->tpair_bytes = wbytes;
        L->tdesc_bytes = tb + ub;
    }
    ProfScope ps(ctx, s, PK_TRTRI, L->tg_flops, 0.0);
    for (const TinvLaunch& t : L->tg_launches) {
        if (t.ntask == 0) continue;
        HIP_TRY(launch_tgemm_f64(reinterpret_cast<const TGemmTask*>(L->tpair_desc + t.task_off),
                                 t.ntask,
                                 reinterpret_cast<const TGemmTerm*>(L->tpair_desc + t.term_off),
                                 m, tgemm_block(t.ntask, m), s));
    }
    return GPR_OK;
}

// Vector solves with the factor: beta = L^{-1} rhs, alpha = L^{-T} beta
// (k_trsv.hip; the second is skipped when alpha is null); tmp is scratch. All
// vectors have length M m.
int run_trsv_pair(gpr_ctx* ctx, const gpr_tiled* L, const double* rhs, double* tmp,
                  double* beta, double* alpha, hipStream_t s)
{
    const int M = L->M, m = L->m;
    const double f = 2.0 * (double)m * m * ((double)M * (M - 1) / 2 + M);
    {
        ProfScope ps(ctx, s, PK_TRSV, f, 0.0);
        HIP_TRY(launch_trsv(kmat(L), L->tinv, L->tpair, L->tgroup, M, rhs, tmp, beta, false, s));
    }
    if (alpha) {
        ProfScope ps(ctx, s, PK_TRSV, f, 0.0);
        HIP_TRY(launch_trsv(kmat(L), L->tinv, L->tpair, L->tgroup, M, beta, tmp, alpha, true, s));
    }
    return GPR_OK;
}

// Buffers of the reverse sweep (symbolic operands of an AdjPlan resolve here).
struct AdjBufs {
    TileMat L, Lbar, Abar;
    double* tinv;
    double* part;
    double *q, *g, *x;
    int m;
    double* at(const AdjRef& r) const
    {
        const size_t m2 = (size_t)m * m;
        switch (r.mat) {
        case AM_L: return tile_ptr(L, r.I, r.J);
        case AM_LBAR: return tile_ptr(Lbar, r.I, r.J);
        case AM_ABAR: return tile_ptr(Abar, r.I, r.J);
        case AM_TINV: return tinv + (size_t)r.I * m2;
        case AM_PART: return part + (size_t)r.I * m2;
        case AM_Q: return q;
        case AM_G: return g;
        case AM_X: return x;
        default: return nullptr;
        }
    }
};

struct AdjExec {
    std::vector<size_t> task_off, term_off;
    std::vector<int> bm;
    std::vector<double> flops;
};

AdjExec plan_adjoint_exec(const AdjPlan& P, const AdjBufs& B, DescBuffer& db)
{
    AdjExec E;
    const int m = B.m;
    const double m3 = (double)m * m * m;
    for (const AdjLaunch& L : P.launches) {
        std::vector<TGemmTask> tv;
        std::vector<TGemmTerm> rv;
        const int term0 = L.count ? P.tasks[L.first].first_term : 0;
        double f = 0.0;
        for (int t = L.first; t < L.first + L.count; ++t) {
            const AdjTask& a = P.tasks[t];
            TGemmTask k;
            k.C = B.at(a.out);
            k.Cin = a.cin.mat == AM_NONE ? nullptr : B.at(a.cin);
            k.beta = a.cin.mat == AM_NONE ? 0.0 : 1.0;
            k.part = a.npart ? B.part + (size_t)a.part0 * m * m : nullptr;
            k.part_stride = (long long)m * m;
            k.ldc = k.ldcin = m;
            k.npart = a.npart;
            k.first_term = a.first_term - term0;
            k.nterm = a.nterm;
            k.epi = a.epi;
            tv.push_back(k);
            for (int q = a.first_term; q < a.first_term + a.nterm; ++q) {
                const AdjTerm& x = P.terms[q];
                rv.push_back({B.at(x.A), B.at(x.B), (double)x.alpha, m, m, x.flags, 0});
                f += (a.epi == TG_EPI_SYM ? 1.0 : 2.0) * m3;
            }
        }
        E.task_off.push_back(db.add(tv.data(), tv.size() * sizeof(TGemmTask)));
        E.term_off.push_back(db.add(rv.data(), rv.size() * sizeof(TGemmTerm)));
        E.bm.push_back(tgemm_block(L.count, m));
        E.flops.push_back(f);
    }
    return E;
}

// The reverse sweep on two streams: the chain of each step on the caller's
// stream s, the early pulls on a second stream (the bulk stream of the
// context; with one stream everything runs on s in list order, which the
// plan also allows). Waits across the streams are events.
int run_adjoint(gpr_ctx* ctx, const AdjPlan& P, const AdjExec& E, int m, const DescBuffer& db,
                hipStream_t s)
{
    const auto& Ls = P.launches;
    int rc = ensure_events(ctx, Ls.size());
    if (rc) return rc;
    const hipStream_t phys[2] = {s, ctx->n_streams >= 2 ? ctx->bulk : s};
    const bool two = phys[1] != s;
    std::vector<char> waited(Ls.size(), 0);
    for (const auto& L : Ls)
        if (L.wait >= 0 && phys[Ls[L.wait].stream] != phys[L.stream]) waited[L.wait] = 1;
    if (two) {
        HIP_TRY(hipEventRecord(ctx->ev_fork, s));
        HIP_TRY(hipStreamWaitEvent(phys[1], ctx->ev_fork, 0));
    }
    for (size_t i = 0; i < Ls.size(); ++i) {
        const AdjLaunch& L = Ls[i];
        hipStream_t st = phys[L.stream];
        if (L.wait >= 0 && phys[Ls[L.wait].stream] != st)
            HIP_TRY(hipStreamWaitEvent(st, ctx->evpool[L.wait], 0));
        {
            ProfScope ps(ctx, st, PK_ADJOINT, E.flops[i], 0.0);
            HIP_TRY(launch_tgemm_f64(db.dev<TGemmTask>(ctx, E.task_off[i]), L.count,
                                     db.dev<TGemmTerm>(ctx, E.term_off[i]), m, E.bm[i], st));
        }
        if (waited[i]) HIP_TRY(hipEventRecord(ctx->evpool[i], st));
    }
    if (two) {
        HIP_TRY(hipEventRecord(ctx->ev_join, phys[1]));
        HIP_TRY(hipStreamWaitEvent(s, ctx->ev_join, 0));
    }
    return GPR_OK;
}

// Split of the row sums of the reverse sweep into partial tiles: chunks of
// this many terms.
constexpr int ADJ_CHUNK = 2;

int finish_info(gpr_ctx* ctx, int32_t* info_dev, hipStream_t s);

}  // namespace

// ---------------------------------------------------------------------------

__global__ void k_info_finish(int* info, int32_t* out)
{
    if (info[0] > 0 && info[1] == 0) info[1] = info[0];
    if (out) *out = info[0];
}

namespace {
int finish_info(gpr_ctx* ctx, int32_t* info_dev, hipStream_t s)
{
    hipLaunchKernelGGL(k_info_finish, dim3(1), dim3(1), 0, s, ctx->d_info, info_dev);
    return hipGetLastError() == hipSuccess ? GPR_OK : GPR_EHIP;
}
}  // namespace

namespace {
// gpr_assemble; with_copy: the same launch also writes the FP64 copy of K that
// a mixed-precision factorisation keeps for its refinement (K->kcopy), so
// that no separate copy of the matrix is needed.
int assemble_impl(gpr_ctx* ctx, const double* X, int64_t n, int32_t D, gpr_hyper h,
                  int32_t tile, gpr_tiled** K_inout, hipStream_t s, bool with_copy)
{
    Range range("gpr_assemble");
    int rc = begin_call(ctx, s);
    if (rc) return rc;
    gpr_tiled* K = *K_inout;
    if (!K) {
        rc = alloc_tiled(ctx, n, tile, &K);
        if (rc) return rc;
    }
    if (with_copy && !K->kcopy) {
        rc = handle_malloc(K, reinterpret_cast<void**>(&K->kcopy), tiled_bytes(K));
        if (rc) {
            if (!*K_inout) gpr_tiled_free(K);
            return rc;
        }
    }
    hipError_t e;
    {
        ProfScope ps(ctx, s, PK_ASSEMBLE, 0.0, (with_copy ? 2.0 : 1.0) * (double)tiled_bytes(K));
        e = launch_assemble(kmat(K), K->M, X, n, X, n, D, h.lengthscale, h.vertical_variance,
                            h.noise_variance, true, true, s, nullptr,
                            with_copy ? K->kcopy : nullptr);
    }
    if (e != hipSuccess) {
        if (!*K_inout) gpr_tiled_free(K);
        return GPR_EHIP;
    }
    K->state = GPR_STATE_K;
    K->prec = GPR_FP64;
    *K_inout = K;
    return end_call(ctx, s);
}
}  // namespace

extern "C" {

int gpr_abi_version(void) { return GPR_ABI_VERSION; }

#ifndef GPR_SOURCE_HASH
#define GPR_SOURCE_HASH "unknown"
#endif
const char* gpr_source_hash(void) { return GPR_SOURCE_HASH; }

const char* gpr_strerror(int status)
{
    switch (status) {
    case GPR_OK: return "success";
    case GPR_ENOTPD: return "matrix is not positive definite (non-positive Cholesky pivot)";
    case GPR_EINVAL: return "invalid argument";
    case GPR_ENOMEM: return "device allocation failed";
    case GPR_EHIP: return "HIP runtime error";
    case GPR_ENODEV: return "no usable GPU device";
    case GPR_ENOTSUP: return "not supported by this library";
    default: return "unknown status";
    }
}

int gpr_ctx_create(gpr_ctx** out, int device, int n_streams, gpr_executor ex)
{
    if (!out || n_streams < 1) return GPR_EINVAL;
    *out = nullptr;
    if (ex != GPR_EXEC_STREAMS && ex != GPR_EXEC_PERSISTENT && ex != GPR_EXEC_AUTO)
        return GPR_EINVAL;
    int rc = check_device(device);
    if (rc) return rc;
    gpr_ctx* c = new (std::nothrow) gpr_ctx;
    if (!c) return GPR_ENOMEM;
    c->device = device;
    c->budget = std::make_shared<DevBudget>();
    if (const char* cap = std::getenv("GPR_MAX_DEVICE_BYTES")) {
        const unsigned long long v = std::strtoull(cap, nullptr, 10);
        if (v > 0) c->budget->cap = v;
    }
    c->executor = ex;
    c->n_streams = n_streams >= 3 ? 3 : n_streams;
    bool ok = hipStreamCreateWithFlags(&c->bulk, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&c->panel, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_last, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_desc, hipEventDisableTiming) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&c->d_info), 4 * sizeof(int)) == hipSuccess &&
              hipMemset(c->d_info, 0, 4 * sizeof(int)) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&c->d_flags), FLAG_WORDS * sizeof(unsigned)) == hipSuccess &&
              hipMemset(c->d_flags, 0, FLAG_WORDS * sizeof(unsigned)) == hipSuccess &&
              hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        gpr_ctx_destroy(c);
        return GPR_EHIP;
    }
    rc = scratch_setup(device);
    if (rc) {
        gpr_ctx_destroy(c);
        return rc;
    }

    *out = c;
    return GPR_OK;
}

int gpr_ctx_set_variant(gpr_ctx* ctx, gpr_variant v)
{
    if (!ctx || (v != GPR_RIGHT_LOOKING && v != GPR_LEFT_LOOKING)) return GPR_EINVAL;
    ctx->variant = (int)v;
    return GPR_OK;
}

int gpr_ctx_destroy(gpr_ctx* c)
{
    if (!c) return GPR_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (c->scratch) gpr_tiled_free(c->scratch);
    if (c->nlml_K) gpr_tiled_free(c->nlml_K);
    budget_free(c->budget, c->d_fit, c->fit_cap);
    budget_free(c->budget, c->d_adj, c->adj_cap);
    budget_free(c->budget, c->d_part, c->part_cap);
    for (auto e : c->evpool) (void)hipEventDestroy(e);
    for (auto e : c->tpool) (void)hipEventDestroy(e);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ev_last) (void)hipEventDestroy(c->ev_last);
    if (c->ev_desc) (void)hipEventDestroy(c->ev_desc);
    if (c->bulk) (void)hipStreamDestroy(c->bulk);
    if (c->panel) (void)hipStreamDestroy(c->panel);
    if (c->d_info) (void)hipFree(c->d_info);
    if (c->d_flags) (void)hipFree(c->d_flags);
    budget_free(c->budget, c->d_desc, c->desc_cap);
    if (c->h_desc) (void)hipHostFree(c->h_desc);
    budget_free(c->budget, c->d_ws, c->ws_cap);
    budget_free(c->budget, c->d_pitems, c->pitems_cap);
    budget_free(c->budget, c->d_pcnt, c->pcnt_cap);
    delete c;
    return GPR_OK;
}

int gpr_assemble(gpr_ctx* ctx, const double* X, int64_t n, int32_t D, gpr_hyper h, int32_t tile,
                 gpr_tiled** K_inout, void* stream)
{
    if (!ctx || !X || !K_inout || n < 1 || D < 1 || !valid_tile(tile) || !valid_hyper(h))
        return GPR_EINVAL;
    if (*K_inout && ((*K_inout)->n != n || (*K_inout)->m != tile)) return GPR_EINVAL;
    return assemble_impl(ctx, X, n, D, h, tile, K_inout, static_cast<hipStream_t>(stream), false);
}

int gpr_cholesky(gpr_ctx* ctx, gpr_tiled* K, gpr_precision prec, int32_t* info_dev, void* stream)
{
    Range range("gpr_cholesky");
    if (!ctx || !K || K->state != GPR_STATE_K || K->device != ctx->device) return GPR_EINVAL;
    if (!valid_prec(prec, K->m)) return GPR_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = begin_call(ctx, s);
    if (rc) return rc;
    const int m = K->m, M = K->M;
    if (prec != GPR_FP64) {
        rc = save_kcopy(K, s);
        if (rc) return rc;
    }
    if (!K->tinv) {
        const int arc = handle_malloc(K, reinterpret_cast<void**>(&K->tinv),
                                      (size_t)M * m * m * sizeof(double));
        if (arc) return arc;
    }
    SweepMats X{kmat(K), K->tinv, TileMat{nullptr, m, 1, M}, TileMat{nullptr, m, 0, 0}, M, 0, m,
                (int)prec};
    DescBuffer db;
    SweepPlan P = plan_sweep(ctx, X, SWEEP_CHOLESKY, db);
    rc = db.upload(ctx, s);
    if (rc) return rc;
    HIP_TRY(launch_set_int(ctx->d_info, 0, s));
    rc = run_sweep(ctx, X, P, db, s);
    if (rc) return rc;
    {
        // full inverses of the diagonal tiles for the vector solves, all at once
        ProfScope ps(ctx, s, PK_TRTRI, M * (double)m * m * m / 3.0, 0.0);
        HIP_TRY(launch_trtri_f64(kmat(K), M, K->tinv, s));
    }
    rc = build_tinv_pairs(ctx, K, prec, s);
    if (rc) return rc;
    rc = finish_info(ctx, info_dev, s);
    if (rc) return rc;
    K->state = GPR_STATE_L;
    K->prec = prec;
    return end_call(ctx, s);
}

int gpr_cholesky_dense(gpr_ctx* ctx, double* A, int64_t n, int32_t tile, gpr_precision prec,
                       int32_t* info_dev, void* stream)
{
    Range range("gpr_cholesky_dense");
    if (!ctx || !A || n < 1 || !valid_tile(tile) || !valid_prec(prec, tile)) return GPR_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = begin_call(ctx, s);
    if (rc) return rc;
    gpr_tiled* T = ctx->scratch;
    if (T && (T->n != n || T->m != tile)) {
        gpr_tiled_free(T);
        T = ctx->scratch = nullptr;
    }
    if (!T) {
        rc = alloc_tiled(ctx, n, tile, &T);
        if (rc) return rc;
        ctx->scratch = T;
    }
    HIP_TRY(launch_dense_to_tiled(A, n, n, kmat(T), T->M, s));
    T->state = GPR_STATE_K;
    rc = end_call(ctx, s);
    if (rc) return rc;
    rc = gpr_cholesky(ctx, T, prec, info_dev, stream);
    if (rc) return rc;
    rc = begin_call(ctx, s);
    if (rc) return rc;
    HIP_TRY(launch_tiled_to_dense(kmat(T), n, A, n, false, s));
    return end_call(ctx, s);
}

}  // extern "C"

namespace {

// Internal status: the mixed factorisation failed (pivot, or refinement did
// not converge); the caller may retry in a higher precision.
constexpr int RETRY_HIGHER = 100;

// Mean (and covariance) with the factor in L. fused: L holds K (assembled),
// and the factorisation runs in the same sweep as the covariance rows, in
// precision prec. With a mixed-precision factor, alpha is refined in FP64:
//   r = y - K alpha (K from the saved FP64 copy), d = L^{-T} L^{-1} r,
//   alpha += d,
// until ||r|| / ||y|| <= 1e-14, stagnation, or 50 steps; if a step gains
// less than a factor 4 while ||r|| / ||y|| > 1e-12, the remaining steps are
// conjugate gradients preconditioned by the same factor. This synchronises
// the stream once per step.
int predict_impl(gpr_ctx* ctx, gpr_tiled* L, const double* X, const double* y, int64_t n,
                 const double* Xs, int64_t n_test, int32_t D, const gpr_hyper& h, double* mean,
                 double* cov, double* var, int32_t* info_dev, hipStream_t s, bool fused,
                 int prec, gpr_ir_stats* ir, bool kcopy_written = false)
{
    const int m = L->m, M = L->M;
    const int Mhat = (int)((n_test + m - 1) / m);
    const size_t npad = (size_t)M * m;
    const size_t vec_bytes = 8 * npad * sizeof(double) + 256;
    const bool rows = cov || var;  // the test rows V^T are needed
    const size_t v_bytes = rows ? (size_t)Mhat * M * m * m * sizeof(double) : 0;
    const size_t s_bytes = cov ? (size_t)Mhat * (Mhat + 1) / 2 * m * m * sizeof(double) : 0;
    const size_t mv_bytes = (size_t)matvec_chunks(n_test, n) * n_test * sizeof(double);
    const int fprec = fused ? prec : L->prec;
    // partial products of the refinement's K x (mixed precision only)
    const size_t sv_bytes = fprec != GPR_FP64 ? symv_work_doubles(M, m) * sizeof(double) : 0;
    int rc = ensure_device_bytes(ctx->budget, &ctx->d_ws, &ctx->ws_cap,
                                 vec_bytes + v_bytes + s_bytes + mv_bytes + sv_bytes);
    if (rc) return rc;
    if (fused && !L->tinv) {
        const int arc = handle_malloc(L, reinterpret_cast<void**>(&L->tinv),
                                      (size_t)M * m * m * sizeof(double));
        if (arc) return arc;
    }
    double* r = reinterpret_cast<double*>(ctx->d_ws);
    double* beta = r + npad;
    double* alpha = beta + npad;
    double* acc = alpha + npad;     // refined alpha
    double* scal = acc + npad;      // small scalars (norms)
    double* tmp = scal + npad;      // scratch of the triangular solves
    double* pv = tmp + npad;        // conjugate-gradient direction p
    double* wv = pv + npad;         // -K p
    double* Vb = wv + npad;
    double* Sb = reinterpret_cast<double*>(reinterpret_cast<char*>(Vb) + v_bytes);
    double* mvw = reinterpret_cast<double*>(reinterpret_cast<char*>(Sb) + s_bytes);
    double* svw = reinterpret_cast<double*>(reinterpret_cast<char*>(mvw) + mv_bytes);

    DescBuffer db;
    SweepMats SM{kmat(L), L->tinv, TileMat{Vb, m, 1, M}, TileMat{Sb, m, 0, 0}, M,
                 rows ? Mhat : 0, m, fprec};
    SweepPlan PP;
    // the full covariance needs the test block; variances alone only V^T
    const int mode = fused ? (cov ? SWEEP_FUSED : (var ? SWEEP_FUSED_V : SWEEP_CHOLESKY))
                           : (cov ? SWEEP_PREDICT : SWEEP_PREDICT_V);
    if (fused || rows) PP = plan_sweep(ctx, SM, mode, db);
    rc = db.upload(ctx, s);
    if (rc) return rc;

    if (fused && prec != GPR_FP64 && !kcopy_written) {
        rc = save_kcopy(L, s);
        if (rc) return rc;
    }
    if (rows) {
        // K_{X*,X} tiles (to become V^T) and lower tiles of K_{X*,X*}; no noise
        ProfScope ps(ctx, s, PK_ASSEMBLE, 0.0, (double)(v_bytes + s_bytes));
        HIP_TRY(launch_assemble(SM.V, Mhat, Xs, n_test, X, n, D, h.lengthscale,
                                h.vertical_variance, h.noise_variance, false, false, s));
        if (cov)
            HIP_TRY(launch_assemble(SM.S, Mhat, Xs, n_test, Xs, n_test, D, h.lengthscale,
                                    h.vertical_variance, h.noise_variance, false, false, s));
    }
    if (fused) HIP_TRY(launch_set_int(ctx->d_info, 0, s));
    // In a factorising sweep with test rows, the critical stream's last launch
    // (POTRF of the last tile column) completes the training factor: every
    // training tile was final before it (its own updates waited for them).
    // What the other streams still run touches only the test rows (V^T and
    // the test block), so the inverses, the solves and the mean go on s
    // beside it, and s joins them before the covariance or variances are
    // read. Every return below joins first.
    struct DeferredJoin {
        gpr_ctx* c;
        hipStream_t st;
        bool pending;
        int now()
        {
            pending = false;
            return join_sweep(c, st);
        }
        ~DeferredJoin()
        {
            if (pending) (void)join_sweep(c, st);
        }
    } dj{ctx, s, false};
    if (fused || rows) {
        const bool defer = fused && rows && !PP.persistent;
        rc = run_sweep(ctx, SM, PP, db, s, !defer);
        if (rc) return rc;
        dj.pending = defer;
    }
    if (fused) {
        {
            ProfScope ps(ctx, s, PK_TRTRI, M * (double)m * m * m / 3.0, 0.0);
            HIP_TRY(launch_trtri_f64(kmat(L), M, L->tinv, s));
        }
        rc = build_tinv_pairs(ctx, L, prec, s);
        if (rc) return rc;
    }
    // a mixed factorisation made by this call: its pivot record is read on the
    // host (a failed pivot makes the caller retry one precision higher, and
    // the failure is not reported: no finish_info for this attempt), in the
    // same round trip as the norms of y and of the first residual below
    const bool check_pivot = fused && prec != GPR_FP64;
    if (fused) {
        L->state = GPR_STATE_L;
        L->prec = prec;
        if (!check_pivot) {
            rc = finish_info(ctx, info_dev, s);
            if (rc) return rc;
        }
    }
    // With the test rows formed and an FP64 factor the mean is V^T beta
    // (eqs. (2), (3): K_{X*,X} K^{-1} y = (L^{-1} K_{X,X*})^T L^{-1} y), so only
    // the forward solve runs; otherwise alpha = K^{-1} y via both triangular
    // solves (Sec. 4.1), refined for a mixed-precision factor.
    const bool mean_from_v = rows && L->prec == GPR_FP64;
    HIP_TRY(launch_copy_f64(y, r, n, (int64_t)npad, s));
    rc = run_trsv_pair(ctx, L, r, tmp, beta, mean_from_v ? nullptr : alpha, s);
    if (rc) return rc;
    const double* alpha_used = alpha;
    if (ir) {
        ir->iters = 0;
        ir->rel_residual = -1.0;
        ir->fallback_precision = L->prec;
        ir->method = GPR_REFINE_IR;
    }
    if (L->prec != GPR_FP64) {
        if (!L->kcopy) return GPR_EINVAL;
        const TileMat Kc{L->kcopy, m, 0, 0};
        HIP_TRY(launch_copy_f64(alpha, acc, (int64_t)npad, (int64_t)npad, s));
        // ||y||^2 in scal[1]; r = y - K acc (FP64, padding of r stays zero)
        // and ||r||^2 in scal[0]; one host round trip for both (and the pivot)
        HIP_TRY(launch_sumsq(y, n, scal + 1, s));
        HIP_TRY(launch_symv_tiled(Kc, M, acc, y, r, n, svw, s));
        HIP_TRY(launch_sumsq(r, n, scal, s));
        double sq[2] = {0.0, 0.0};
        int info = 0;
        HIP_TRY(hipMemcpyAsync(sq, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        if (check_pivot)
            HIP_TRY(hipMemcpyAsync(&info, ctx->d_info, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (info > 0) return RETRY_HIGHER;
        if (check_pivot) {
            rc = finish_info(ctx, info_dev, s);
            if (rc) return rc;
        }
        const double yn = std::sqrt(sq[1]);
        auto rel_of = [&](double rr) { return yn > 0 ? std::sqrt(rr) / yn : std::sqrt(rr); };
        // ||r|| / ||y|| of the residual held in r (host round trip)
        auto residual = [&](double* out_rel) -> int {
            HIP_TRY(launch_sumsq(r, n, scal, s));
            double rr = 0.0;
            HIP_TRY(hipMemcpyAsync(&rr, scal, sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            *out_rel = rel_of(rr);
            return GPR_OK;
        };
        constexpr int max_steps = 50;
        double prev = -1.0, rel = rel_of(sq[0]);
        int it = 0;
        bool to_cg = false;
        for (; it <= max_steps; ++it) {
            if (it > 0) {
                // r = y - K acc (FP64), padding of r stays zero
                HIP_TRY(launch_symv_tiled(Kc, M, acc, y, r, n, svw, s));
                rc = residual(&rel);
                if (rc) return rc;
            }
            if (rel <= 1e-14 || it == max_steps) break;
            // a step that gains less than a factor 4 far above the rounding
            // floor: the iteration matrix I - (L~ L~^T)^{-1} K contracts slowly
            // or not at all (kappa(K) u too large); go on with CG
            if (prev >= 0 && rel > 1e-12 && rel > 0.25 * prev) {
                to_cg = true;
                break;
            }
            if (prev >= 0 && rel > 0.9 * prev) break;   // stagnation at the floor
            prev = rel;
            rc = run_trsv_pair(ctx, L, r, tmp, beta, alpha, s);  // alpha = L^{-T} L^{-1} r
            if (rc) return rc;
            HIP_TRY(launch_axpy(acc, alpha, (int64_t)npad, s));
        }
        if (to_cg) {
            // Conjugate gradients on K x = y from x = acc, preconditioned by
            // the mixed factor (z = L~^{-T} L~^{-1} r): converges to the same
            // FP64 solution as long as L~ L~^T is positive definite, which a
            // successful factorisation guarantees. Vectors are updated over
            // the first n entries only, so the padding of r, acc and p stays
            // zero. The loop stops on the updated residual; the true
            // residual of the last iterate is reported.
            double* z = alpha;
            double* pw = scal + 1;
            rc = run_trsv_pair(ctx, L, r, tmp, beta, z, s);
            if (rc) return rc;
            HIP_TRY(launch_dot(r, z, n, scal + 2, s));
            HIP_TRY(launch_copy_f64(z, pv, n, (int64_t)npad, s));
            for (int k = 0; it < max_steps; ++k) {
                ++it;
                double* rz = scal + 2 + (k & 1);
                double* rz_next = scal + 2 + ((k + 1) & 1);
                HIP_TRY(launch_symv_tiled(Kc, M, pv, nullptr, wv, n, svw, s));  // w = -K p
                HIP_TRY(launch_dot(pv, wv, n, pw, s));
                HIP_TRY(launch_cg_xr(acc, r, pv, wv, rz, pw, n, s));
                rc = residual(&rel);
                if (rc) return rc;
                if (!(rel > 1e-14)) break;   // converged, or not finite
                rc = run_trsv_pair(ctx, L, r, tmp, beta, z, s);
                if (rc) return rc;
                HIP_TRY(launch_dot(r, z, n, rz_next, s));
                HIP_TRY(launch_cg_p(pv, z, rz_next, rz, n, s));
            }
            HIP_TRY(launch_symv_tiled(Kc, M, acc, y, r, n, svw, s));
            rc = residual(&rel);
            if (rc) return rc;
        }
        if (ir) {
            ir->iters = it;
            ir->rel_residual = rel;
            ir->method = to_cg ? GPR_REFINE_PCG : GPR_REFINE_IR;
        }
        // not converged to where the mean can be trusted: let a fused caller retry
        if (fused && !(rel <= 1e-10)) return RETRY_HIGHER;
        alpha_used = acc;
    }
    // mean = K_{X*,X} alpha, eq. (2), without storing K_{X*,X}
    if (!mean_from_v) {
        ProfScope ps(ctx, s, PK_MATVEC, 2.0 * (double)n_test * (double)n, 0.0);
        HIP_TRY(launch_kernel_matvec(Xs, n_test, X, n, D, h.lengthscale, h.vertical_variance,
                                     h.noise_variance, false, alpha_used, nullptr, mean, mvw,
                                     s));
    }
    if (dj.pending) {
        rc = dj.now();
        if (rc) return rc;
    }
    if (mean_from_v) {
        // V^T is complete once the sweep's streams have joined
        ProfScope ps(ctx, s, PK_MATVEC, 2.0 * (double)n_test * (double)n, 0.0);
        HIP_TRY(launch_rowdot_mean(SM.V, M, n_test, beta, mean, s));
    }
    if (cov) {
        ProfScope ps(ctx, s, PK_EXPORT, 0.0, (double)n_test * n_test * sizeof(double));
        HIP_TRY(launch_tiled_to_dense(SM.S, n_test, cov, n_test, true, s));
    }
    if (var) {
        // the diagonal of the covariance when it was formed, else from V^T
        ProfScope ps(ctx, s, PK_EXPORT, 0.0,
                     cov ? 16.0 * n_test : (double)n_test * M * m * sizeof(double));
        if (cov)
            HIP_TRY(launch_tile_diag(SM.S, n_test, var, s));
        else
            HIP_TRY(launch_rowsq_var(SM.V, M, n_test, h.vertical_variance, var, s));
    }
    return GPR_OK;
}

// One NLML (and gradient) evaluation, split into the part that depends only
// on the shape (buffers and launch descriptors, uploaded once) and the
// launches, so that a loop of evaluations (the hyperparameter fit) plans once.
struct NlmlRun {
    gpr_tiled* K = nullptr;
    bool grad = false;
    int nparts = 0;
    double *r = nullptr, *beta = nullptr, *alpha = nullptr, *tmp = nullptr, *parts = nullptr;
    SweepMats SM{};
    SweepPlan PP;
    AdjPlan AP;
    AdjExec AE;
    AdjBufs AB{};
    DescBuffer db;
};

int nlml_prepare(gpr_ctx* ctx, int64_t n, int32_t tile, bool grad, NlmlRun& R, hipStream_t s)
{
    gpr_tiled* K = ctx->nlml_K;
    if (K && (K->n != n || K->m != tile)) {
        gpr_tiled_free(K);
        K = ctx->nlml_K = nullptr;
    }
    if (!K) {
        int rc = alloc_tiled(ctx, n, tile, &K);
        if (rc) return rc;
        ctx->nlml_K = K;
    }
    const int m = K->m, M = K->M;
    if (!K->tinv) {
        const int arc = handle_malloc(K, reinterpret_cast<void**>(&K->tinv),
                                      (size_t)M * m * m * sizeof(double));
        if (arc) return arc;
    }
    R.K = K;
    R.grad = grad;
    const size_t npad = (size_t)M * m;
    R.nparts = grad ? grad_reduce_parts(M, m) : 0;
    int rc = ensure_device_bytes(ctx->budget, &ctx->d_ws, &ctx->ws_cap,
                                 (4 * npad + 3 * (size_t)(R.nparts + 1)) * sizeof(double) + 256);
    if (rc) return rc;
    R.r = reinterpret_cast<double*>(ctx->d_ws);
    R.beta = R.r + npad;
    R.alpha = R.beta + npad;
    R.tmp = R.alpha + npad;     // scratch of the triangular solves
    R.parts = R.tmp + npad;
    R.SM = SweepMats{kmat(K), K->tinv, TileMat{nullptr, m, 1, M}, TileMat{nullptr, m, 0, 0}, M,
                     0, m, GPR_FP64};
    R.PP = plan_sweep(ctx, R.SM, SWEEP_CHOLESKY, R.db);
    if (grad) {
        R.AP = build_adjoint(M, ADJ_CHUNK);
        const size_t tb = tiled_bytes(K);
        const size_t m2b = (size_t)m * m * sizeof(double);
        rc = ensure_device_bytes(ctx->budget, &ctx->d_adj, &ctx->adj_cap,
                                 2 * tb + (size_t)(R.AP.max_part + 3) * m2b);
        if (rc) return rc;
        double* base = reinterpret_cast<double*>(ctx->d_adj);
        R.AB.L = kmat(K);
        R.AB.Lbar = TileMat{base, m, 0, 0};
        R.AB.Abar = TileMat{base + tb / sizeof(double), m, 0, 0};
        R.AB.part = base + 2 * tb / sizeof(double);
        R.AB.q = R.AB.part + (size_t)R.AP.max_part * m * m;
        R.AB.g = R.AB.q + (size_t)m * m;
        R.AB.x = R.AB.g + (size_t)m * m;
        R.AB.tinv = K->tinv;
        R.AB.m = m;
        R.AE = plan_adjoint_exec(R.AP, R.AB, R.db);
    }
    return R.db.upload(ctx, s);
}

// The launches of one evaluation at (l, v, sigma^2) = h, or at the device
// array hyp (3 doubles) when it is given.
int nlml_launch(gpr_ctx* ctx, NlmlRun& R, const double* X, const double* y, int64_t n, int32_t D,
                const gpr_hyper& h, const double* hyp, double* out_nlml, double* out_grad3,
                double* out_Kbar, hipStream_t s)
{
    gpr_tiled* K = R.K;
    const int m = K->m, M = K->M;
    const size_t npad = (size_t)M * m;
    // K (with noise), its factor, and the diagonal-tile inverses
    {
        ProfScope ps(ctx, s, PK_ASSEMBLE, 0.0, (double)tiled_bytes(K));
        HIP_TRY(launch_assemble(kmat(K), M, X, n, X, n, D, h.lengthscale, h.vertical_variance,
                                h.noise_variance, true, true, s, hyp));
    }
    K->state = GPR_STATE_K;
    HIP_TRY(launch_set_int(ctx->d_info, 0, s));
    int rc = run_sweep(ctx, R.SM, R.PP, R.db, s);
    if (rc) return rc;
    {
        ProfScope ps(ctx, s, PK_TRTRI, M * (double)m * m * m / 3.0, 0.0);
        HIP_TRY(launch_trtri_f64(kmat(K), M, K->tinv, s));
    }
    rc = build_tinv_pairs(ctx, K, GPR_FP64, s);
    if (rc) return rc;
    K->state = GPR_STATE_L;
    K->prec = GPR_FP64;
    rc = finish_info(ctx, nullptr, s);
    if (rc) return rc;
    // beta = L^{-1} y (kept), and for the gradient alpha = L^{-T} beta
    HIP_TRY(launch_copy_f64(y, R.r, n, (int64_t)npad, s));
    rc = run_trsv_pair(ctx, K, R.r, R.tmp, R.beta, R.grad ? R.alpha : nullptr, s);
    if (rc) return rc;
    if (R.grad) {
        {
            ProfScope ps(ctx, s, PK_REDUCE, 0.0, (double)tiled_bytes(K));
            HIP_TRY(launch_lbar_init(R.AB.Lbar, R.AB.L, M, R.alpha, R.beta, s));
        }
        rc = run_adjoint(ctx, R.AP, R.AE, m, R.db, s);
        if (rc) return rc;
        {
            ProfScope ps(ctx, s, PK_REDUCE, 0.0, (double)tiled_bytes(K));
            HIP_TRY(launch_grad_reduce(R.AB.Abar, M, X, n, D, h.lengthscale, R.parts, s, hyp));
        }
        if (out_Kbar) HIP_TRY(launch_kbar_export(R.AB.Abar, n, out_Kbar, s));
    }
    HIP_TRY(launch_nlml_finish(kmat(K), R.beta, n, R.parts, out_grad3 ? R.nparts : 0,
                               h.lengthscale, h.vertical_variance, ctx->d_info, out_nlml,
                               out_grad3, s, hyp));
    return GPR_OK;
}

}  // namespace

extern "C" {

int gpr_predict_var(gpr_ctx* ctx, gpr_tiled* L, const double* X, const double* y, int64_t n,
                    const double* Xs, int64_t n_test, int32_t D, gpr_hyper h, double* mean,
                    double* cov, double* var, gpr_ir_stats* ir, void* stream)
{
    Range range("gpr_predict_var");
    if (!ctx || !L || !X || !y || n < 1 || D < 1 || n_test < 0 || !valid_hyper(h))
        return GPR_EINVAL;
    if (L->state != GPR_STATE_L || L->n != n || L->device != ctx->device) return GPR_EINVAL;
    if (n_test > 0 && (!Xs || !mean)) return GPR_EINVAL;
    if (n_test == 0) return GPR_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = begin_call(ctx, s);
    if (rc) return rc;
    rc = predict_impl(ctx, L, X, y, n, Xs, n_test, D, h, mean, cov, var, nullptr, s, false,
                      L->prec, ir);
    if (rc) return rc;
    return end_call(ctx, s);
}

int gpr_predict(gpr_ctx* ctx, gpr_tiled* L, const double* X, const double* y, int64_t n,
                const double* Xs, int64_t n_test, int32_t D, gpr_hyper h, double* mean,
                double* cov, gpr_ir_stats* ir, void* stream)
{
    Range range("gpr_predict");
    return gpr_predict_var(ctx, L, X, y, n, Xs, n_test, D, h, mean, cov, nullptr, ir, stream);
}

int gpr_fit_predict_var(gpr_ctx* ctx, const double* X, const double* y, int64_t n,
                        const double* Xs, int64_t n_test, int32_t D, gpr_hyper h, int32_t tile,
                        gpr_precision prec, gpr_tiled** K_inout, double* mean, double* cov,
                        double* var, int32_t* info_dev, gpr_ir_stats* ir, void* stream)
{
    Range range("gpr_fit_predict_var");
    if (!ctx || !X || !y || !K_inout || n < 1 || D < 1 || n_test < 1 || !Xs || !mean ||
        !valid_tile(tile) || !valid_hyper(h) || !valid_prec(prec, tile))
        return GPR_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // a mixed factorisation that fails (pivot, or refinement) is redone one
    // precision step higher: BF16 -> FP32 -> FP64
    if (*K_inout && ((*K_inout)->n != n || (*K_inout)->m != tile)) return GPR_EINVAL;
    for (int p = (int)prec;; p = (p == GPR_MIXED_BF16) ? GPR_MIXED_FP32 : GPR_FP64) {
        // a mixed factorisation's FP64 copy of K is written by the assembly
        const bool copy = p != GPR_FP64;
        int rc = assemble_impl(ctx, X, n, D, h, tile, K_inout, s, copy);
        if (rc) return rc;
        rc = begin_call(ctx, s);
        if (rc) return rc;
        gpr_tiled* K = *K_inout;
        rc = predict_impl(ctx, K, X, y, n, Xs, n_test, D, h, mean, cov, var, info_dev, s, true, p,
                          ir, copy);
        if (rc == RETRY_HIGHER && p != GPR_FP64) {
            rc = end_call(ctx, s);
            if (rc) return rc;
            continue;
        }
        if (rc) return rc;
        if (ir) ir->fallback_precision = p;
        return end_call(ctx, s);
    }
}

int gpr_fit_predict(gpr_ctx* ctx, const double* X, const double* y, int64_t n, const double* Xs,
                    int64_t n_test, int32_t D, gpr_hyper h, int32_t tile, gpr_precision prec,
                    gpr_tiled** K_inout, double* mean, double* cov, int32_t* info_dev,
                    gpr_ir_stats* ir, void* stream)
{
    Range range("gpr_fit_predict");
    return gpr_fit_predict_var(ctx, X, y, n, Xs, n_test, D, h, tile, prec, K_inout, mean, cov,
                               nullptr, info_dev, ir, stream);
}

int gpr_solve(gpr_ctx* ctx, gpr_tiled* L, const double* b, double* x, void* stream)
{
    Range range("gpr_solve");
    if (!ctx || !L || !b || !x || L->state != GPR_STATE_L || L->device != ctx->device)
        return GPR_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = begin_call(ctx, s);
    if (rc) return rc;
    const size_t npad = (size_t)L->M * L->m;
    rc = ensure_device_bytes(ctx->budget, &ctx->d_ws, &ctx->ws_cap, 4 * npad * sizeof(double) + 256);
    if (rc) return rc;
    double* r = reinterpret_cast<double*>(ctx->d_ws);
    double* beta = r + npad;
    double* alpha = beta + npad;
    double* tmp = alpha + npad;
    HIP_TRY(launch_copy_f64(b, r, L->n, (int64_t)npad, s));
    rc = run_trsv_pair(ctx, L, r, tmp, beta, alpha, s);
    if (rc) return rc;
    HIP_TRY(launch_copy_f64(alpha, x, L->n, L->n, s));
    return end_call(ctx, s);
}

int gpr_solve_noalloc(gpr_ctx* ctx, gpr_tiled* L, const double* b, double* x, void* stream)
{
    if (!ctx || !L || !b || !x || L->state != GPR_STATE_L || L->device != ctx->device)
        return GPR_EINVAL;
    const size_t npad = (size_t)L->M * L->m;
    if (npad > (size_t)GPR_NOALLOC_MAX_N) return GPR_EINVAL;
    double* base = scratch_device_ptr(ctx->device);
    if (!base) return GPR_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = begin_call(ctx, s);
    if (rc) return rc;
    // The same launches as gpr_solve; the right-hand side's buffer takes the
    // result of the backward solve (it is no longer read by then).
    double* r = base;
    double* beta = r + npad;
    double* tmp = beta + npad;
    HIP_TRY(launch_copy_f64(b, r, L->n, (int64_t)npad, s));
    HIP_TRY(launch_trsv(kmat(L), L->tinv, L->tpair, L->tgroup, L->M, r, tmp, beta, false, s));
    HIP_TRY(launch_trsv(kmat(L), L->tinv, L->tpair, L->tgroup, L->M, beta, tmp, r, true, s));
    HIP_TRY(launch_copy_f64(r, x, L->n, L->n, s));
    return end_call(ctx, s);
}

int gpr_nlml_grad(gpr_ctx* ctx, const double* X, const double* y, int64_t n, int32_t D,
                  gpr_hyper h, int32_t tile, gpr_precision prec, double* out_nlml,
                  double* out_grad3, double* out_Kbar, void* stream)
{
    Range range("gpr_nlml_grad");
    if (!ctx || !X || !y || n < 1 || D < 1 || !valid_tile(tile) || !valid_hyper(h) || !out_nlml)
        return GPR_EINVAL;
    if (!valid_prec(prec, tile)) return GPR_EINVAL;
    if (prec != GPR_FP64) return GPR_ENOTSUP;  // log det needs the FP64 factor
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = begin_call(ctx, s);
    if (rc) return rc;
    NlmlRun R;
    rc = nlml_prepare(ctx, n, tile, out_grad3 || out_Kbar, R, s);
    if (rc) return rc;
    rc = nlml_launch(ctx, R, X, y, n, D, h, nullptr, out_nlml, out_grad3, out_Kbar, s);
    if (rc) return rc;
    return end_call(ctx, s);
}

int gpr_profile_enable(gpr_ctx* ctx, int on)
{
    if (!ctx) return GPR_EINVAL;
    ctx->prof_on = on != 0;
    return GPR_OK;
}

int gpr_profile_read(gpr_ctx* ctx, int kind, int64_t* launches, double* total_ms, double* flops,
                     double* bytes, int reset)
{
    if (!ctx || kind < 0 || kind >= PK_COUNT) return GPR_EINVAL;
    int rc = check_device(ctx->device);
    if (rc) return rc;
    rc = resolve_profile(ctx);
    if (rc) return rc;
    if (launches) *launches = ctx->p_launches[kind];
    if (total_ms) *total_ms = ctx->p_ms[kind];
    if (flops) *flops = ctx->p_flops[kind];
    if (bytes) *bytes = ctx->p_bytes[kind];
    if (reset) {
        for (int k = 0; k < PK_COUNT; ++k) {
            ctx->p_launches[k] = 0;
            ctx->p_ms[k] = ctx->p_flops[k] = ctx->p_bytes[k] = 0.0;
        }
    }
    return GPR_OK;
}

int gpr_tiled_info(const gpr_tiled* T, int64_t* n, int32_t* tile, int32_t* state)
{
    if (!T) return GPR_EINVAL;
    if (n) *n = T->n;
    if (tile) *tile = T->m;
    if (state) *state = T->state;
    return GPR_OK;
}

int gpr_tiled_to_dense(gpr_ctx* ctx, const gpr_tiled* T, double* out, void* stream)
{
    Range range("gpr_tiled_to_dense");
    if (!ctx || !T || !out || T->state == GPR_STATE_EMPTY || T->device != ctx->device)
        return GPR_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = begin_call(ctx, s);
    if (rc) return rc;
    HIP_TRY(launch_tiled_to_dense(kmat(T), T->n, out, T->n, T->state == GPR_STATE_K, s));
    return end_call(ctx, s);
}

int gpr_tiled_free(gpr_tiled* T)
{
    if (!T) return GPR_EINVAL;
    (void)hipSetDevice(T->device);
    (void)hipDeviceSynchronize();
    if (T->data) (void)hipFree(T->data);
    if (T->tinv) (void)hipFree(T->tinv);
    if (T->kcopy) (void)hipFree(T->kcopy);
    if (T->tpair) (void)hipFree(T->tpair);
    if (T->tpair_desc) (void)hipFree(T->tpair_desc);
    if (T->budget) T->budget->used -= T->dev_bytes;
    if (T->tpair_host) (void)hipHostFree(T->tpair_host);
    delete T;
    return GPR_OK;
}

int gpr_fit_hyper(gpr_ctx* ctx, const double* X, const double* y, int64_t n, int32_t D,
                  int32_t tile, const double* theta0, int32_t max_steps, double lr, double beta1,
                  double beta2, double eps, double tol, double* theta_out, double* nlml_trace,
                  int32_t* steps_done, void* stream)
{
    Range range("gpr_fit_hyper");
    if (!ctx || !X || !y || n < 1 || D < 1 || !valid_tile(tile) || !theta0 || !theta_out ||
        max_steps < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) ||
        !(eps >= 0) || !(tol >= 0))
        return GPR_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!(theta0[k] > 0) || !std::isfinite(theta0[k])) return GPR_EINVAL;
    if (steps_done) *steps_done = 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = begin_call(ctx, s);
    if (rc) return rc;
    // device buffer: NLML and gradient of the current step (4 doubles), the
    // Adam state, then the NLML trace (max_steps doubles)
    const size_t st_off = 64, tr_off = 64 + ((sizeof(AdamState) + 63) / 64) * 64;
    rc = ensure_device_bytes(ctx->budget, &ctx->d_fit, &ctx->fit_cap, tr_off + (size_t)max_steps * sizeof(double));
    if (rc) return rc;
    double* fit = reinterpret_cast<double*>(ctx->d_fit);
    AdamState* st = reinterpret_cast<AdamState*>(ctx->d_fit + st_off);
    double* trace = reinterpret_cast<double*>(ctx->d_fit + tr_off);
    const double* theta_dev =
        reinterpret_cast<const double*>(ctx->d_fit + st_off + offsetof(AdamState, theta));
    static_assert(offsetof(AdamState, stop) == offsetof(AdamState, t) + sizeof(int),
                  "t and stop are read together");
    NlmlRun R;
    rc = nlml_prepare(ctx, n, tile, true, R, s);
    if (rc) return rc;
    // Adam on z = log theta, entirely on the device: each evaluation reads
    // theta = exp(z) from the state, and the step kernel updates it; the host
    // only reads the stop flag every few steps (the evaluations issued after
    // a stop leave the state as it is)
    HIP_TRY(launch_adam_init(st, std::log(theta0[0]), std::log(theta0[1]), std::log(theta0[2]), s));
    const gpr_hyper h0{theta0[0], theta0[1], theta0[2]};  // unused: the kernels read theta
    constexpr int CHECK_EVERY = 4;
    int issued = 0, t = 0, stop = 0;
    while (issued < max_steps) {
        const int chunk = std::min(CHECK_EVERY, max_steps - issued);
        for (int c = 0; c < chunk; ++c) {
            rc = nlml_launch(ctx, R, X, y, n, D, h0, theta_dev, fit, fit + 1, nullptr, s);
            if (rc) return rc;
            HIP_TRY(launch_adam_step(st, fit, trace, max_steps, lr, beta1, beta2, eps, tol, s));
        }
        issued += chunk;
        int ts[2] = {0, 0};   // AdamState::t and ::stop are adjacent
        HIP_TRY(hipMemcpyAsync(ts, ctx->d_fit + st_off + offsetof(AdamState, t), sizeof(ts),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        t = ts[0];
        stop = ts[1];
        if (stop) break;
    }
    double th[3];
    HIP_TRY(hipMemcpyAsync(th, theta_dev, sizeof(th), hipMemcpyDeviceToHost, s));
    if (nlml_trace && t > 0)
        HIP_TRY(hipMemcpyAsync(nlml_trace, trace, (size_t)t * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    rc = end_call(ctx, s);
    if (rc) return rc;
    rc = gpr_sync(ctx, stream, nullptr);
    if (steps_done) *steps_done = t;
    if (rc) return rc;   // GPR_ENOTPD: K(theta) lost positive definiteness
    if (stop == 2) return GPR_ENOTPD;
    for (int k = 0; k < 3; ++k) theta_out[k] = th[k];
    return GPR_OK;
}

int gpr_sync(gpr_ctx* ctx, void* stream, int64_t* column)
{
    if (!ctx) return GPR_EINVAL;
    if (column) *column = 0;
    int rc = check_device(ctx->device);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamSynchronize(s));
    if (ctx->last_valid) HIP_TRY(hipEventSynchronize(ctx->ev_last));
    int info[3] = {0, 0, 0};
    HIP_TRY(hipMemcpy(info, ctx->d_info, sizeof(info), hipMemcpyDeviceToHost));
    if (info[2] != 0) {
        // a device-side wait timed out: the results of the calls queued since
        // the previous gpr_sync are invalid; clear the record (and a pivot
        // failure recorded with it) so that later calls wait normally again
        const int zero[2] = {0, 0};
        HIP_TRY(hipMemcpy(ctx->d_info + 1, zero, sizeof(zero), hipMemcpyHostToDevice));
        return GPR_EHIP;
    }
    if (info[1] > 0) {
        if (column) *column = info[1];
        const int zero = 0;
        HIP_TRY(hipMemcpy(ctx->d_info + 1, &zero, sizeof(int), hipMemcpyHostToDevice));
        return GPR_ENOTPD;
    }
    return GPR_OK;
}

}  // extern "C"
