// Host runtime of libcoop: the C ABI declared in include/coop.h.
//
// Responsibilities: sizing a cooperative launch to the device, the launch
// itself (context initialisation, scratch buffers, the persistent kernel),
// the host side of the scheduler (the target word the resizing barrier
// queries, joiner grids that supply forks), the co-task injector that
// periodically claims workgroups for a non-cooperative task (the paper's
// multitasking experiment), and statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <condition_variable>
#include <deque>
#include <thread>
#include <vector>

#include "coop.h"
#include "coop_device.hpp"
#include "coop_internal.h"

using coop::Ctx;
using coop::CtxCore;
using coop::HostCtl;
using coop::Work;

// Scratch of coop_bfs_noalloc: one array per GPU, for callers that cannot
// allocate. Host code never uses this name as an address (it is a host-side
// stand-in): coop_init looks up the device address with
// hipGetSymbolAddress and keeps it in the runtime.
static __device__ __align__(256) unsigned char scratch[COOP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr uint32_t kDefaultLds = 96 * 1024;       // > half a CU's 160 KiB: one workgroup per CU
constexpr uint32_t kDefaultHeavy = 512;          // measured on R-MAT 22: 1% faster than 128 (2048: as 128; 8192+: slower)
// BFS direction rule: a top-down level is followed by a bottom-up one when
// the frontier's arcs x alpha exceed the arcs not yet visited. Beamer et
// al. use 14 on CPUs; here a top-down claim is a random atomic, and on 60
// R-MAT 22 sources 45..70 ran 6% faster than 14 (100: 2% slower than 48).
constexpr uint32_t kDefaultAlpha = 48;
constexpr uint32_t kDefaultStrip = 512;          // one wave walk step (64 lanes x 8 arcs)
constexpr uint64_t kDefaultWatchdogNs = 10ull * 1000 * 1000 * 1000;
// The query server stays off the GPU: its launch has ended a GPU machine with a
// memory fault or hung queue twice, and no cause has been shown yet.
constexpr bool kServerEnabled = false;
constexpr uint32_t kDefaultStartupNs = 20 * 1000;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    double pos = q * (double)(v.size() - 1);
    size_t i = (size_t)pos;
    double f = pos - (double)i;
    if (i + 1 >= v.size()) return v.back();
    return v[i] * (1.0 - f) + v[i + 1] * f;
}

}  // namespace

struct coop_graph {
    coop_rt* rt;
    const uint32_t* row_ptr;
    const uint32_t* col;
    const uint32_t* w;
    uint32_t n;
    uint64_t arcs;
    uint32_t max_deg;
    uint32_t* deg0 = nullptr;                            // device bitmap: vertices without arcs
    uint32_t* col_bu = nullptr;                          // bottom-up probe order (arcs + 4 words)
    uint2* first2 = nullptr;                             // skewed graphs: first two neighbours of every vertex in that order
    uint32_t words = 0;                                  // bitmap words (multiple of 64)
    std::vector<uint32_t> deg;                           // host copy of the degrees
    std::map<std::pair<uint32_t, uint32_t>, uint64_t> strips;   // (threshold, strip) -> capacity

    uint64_t heavy_strips(uint32_t th, uint32_t strip) {
        auto key = std::make_pair(th, strip);
        auto it = strips.find(key);
        if (it != strips.end()) return it->second;
        uint64_t s = 0;
        for (uint32_t d : deg)
            if (d > th) s += (d + strip - 1) / strip;
        strips[key] = s;
        return s;
    }
    // the same count without caching it (no allocation)
    uint64_t heavy_strips_lookup(uint32_t th, uint32_t strip) const {
        auto it = strips.find(std::make_pair(th, strip));
        if (it != strips.end()) return it->second;
        uint64_t s = 0;
        for (uint32_t d : deg)
            if (d > th) s += (d + strip - 1) / strip;
        return s;
    }
};

struct coop_handle {
    coop_rt* rt = nullptr;
    int kind = 0;
    bool coop = false;
    coop::Cfg cfg{};
    uint32_t* slots = nullptr;           // per-workgroup statistics (device)
    uint32_t grid = 0, block = 0, lds = 0;
    Ctx* ctx = nullptr;
    Work* work = nullptr;
    HostCtl* host = nullptr;             // pinned, fine-grained
    std::vector<std::pair<void*, size_t>> scratch;
    hipStream_t stream = nullptr;
    hipEvent_t ev_init = nullptr, ev_start = nullptr, ev_end = nullptr, ev_join = nullptr;
    bool joined = false;
    uint32_t forked = 0;                 // joiner-grid workgroups launched
    coop::BfsArgs bfs{};
    coop::SsspArgs sssp{};
    coop::ColorArgs color{};
    coop::BarrierBenchArgs bb{};
    // batched launch
    coop::BatchArgs batch{};
    std::vector<coop::BatchInst> batch_inst;   // descriptors in ticket order (host copy)
    std::vector<uint32_t> batch_first, batch_roots;
    coop::TeamState* teams = nullptr;
    coop::BatchCtl* bctl = nullptr;
    uint32_t* bslots = nullptr;
    size_t bslot_words = 0;
    // serving launch
    coop::ServeArgs serve{};
    // work-stealing octree
    coop::OctreeArgs octree{};
    // connected components
    coop::CcArgs cc{};
};

struct coop_rt {
    int device = 0;
    hipDeviceProp_t props{};
    uint32_t wall_khz = 100000;
    uint32_t xcds = 1;                         // XCDs workgroups are dealt over
    uint32_t ses = 1;                          // shader engines per XCD
    hipStream_t joiner_stream = nullptr;
    hipStream_t cotask_stream = nullptr;
    std::recursive_mutex mu;
    int last_hip = 0;
    std::multimap<size_t, void*> pool;         // free device buffers by size
    std::vector<HostCtl*> host_pool;           // free pinned control blocks
    std::vector<coop_handle*> detached;        // handles the caller did not keep
    // co-task state (counters on the device, stamps in pinned host memory)
    uint32_t* d_cot = nullptr;                 // [0] started, [1] finished (cumulative)
    uint32_t* d_check = nullptr;               // graph check: column indices outside [0, n)
    void* noalloc = nullptr;                   // device address of `scratch` on this GPU
    uint32_t cot_launched = 0;                 // co-task workgroups launched so far
    uint64_t* h_stamp = nullptr;               // [0] all started, [1] all finished
    // injector
    std::thread injector;
    std::atomic<bool> inj_stop{false};
    std::atomic<coop_handle*> inj_handle{nullptr};
    std::atomic<uint32_t> inj_busy{0};         // 1 while the injector touches inj_handle
    coop_cotask_cfg inj_cfg{};
    std::vector<double> inj_lat, inj_gather, inj_busy_ms;
    double inj_setup_max = 0, inj_restore_max = 0;
    uint32_t inj_late = 0;
    int inj_error = 0;
    // sharing the GPU between cooperative launches
    struct Shared {
        coop_handle* h = nullptr;
        uint32_t weight = 1, share = 0;
        double t_add = 0, t_end = 0;
        bool ended = false;
    };
    std::thread sharer;
    std::atomic<bool> share_stop{false};
    std::mutex share_mu;                       // guards `shared` and the handles in it
    std::vector<Shared> shared;
    uint32_t share_period_us = 200;
    uint32_t share_updates = 0, share_forks = 0;
    int share_error = 0;
};

namespace {

int hip_fail(coop_rt* rt, hipError_t e) {
    if (rt) rt->last_hip = (int)e;
    return COOP_E_HIP;
}

#define HIP_TRY(rt, expr)                         \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) return hip_fail((rt), _e); \
    } while (0)

void* pool_get(coop_rt* rt, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    auto it = rt->pool.find(bytes);
    if (it != rt->pool.end()) {
        void* p = it->second;
        rt->pool.erase(it);
        return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        // free cached buffers and try again
        for (auto& kv : rt->pool) (void)hipFree(kv.second);
        rt->pool.clear();
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    }
    return p;
}

void pool_put(coop_rt* rt, void* p, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    rt->pool.emplace(bytes, p);
}

HostCtl* host_get(coop_rt* rt) {
    if (!rt->host_pool.empty()) {
        HostCtl* h = rt->host_pool.back();
        rt->host_pool.pop_back();
        return h;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(HostCtl), hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
        return nullptr;
    std::memset(p, 0, sizeof(HostCtl));
    return static_cast<HostCtl*>(p);
}

void handle_free(coop_handle* h) {
    coop_rt* rt = h->rt;
    for (auto& s : h->scratch) pool_put(rt, s.first, s.second);
    h->scratch.clear();
    if (h->host) rt->host_pool.push_back(h->host);
    for (hipEvent_t e : {h->ev_init, h->ev_start, h->ev_end, h->ev_join})
        if (e) (void)hipEventDestroy(e);
    delete h;
}

bool handle_done(coop_handle* h) {
    if (hipEventQuery(h->ev_end) != hipSuccess) return false;
    if (h->joined && hipEventQuery(h->ev_join) != hipSuccess) return false;
    return true;
}

void reap(coop_rt* rt) {
    auto& d = rt->detached;
    for (size_t i = 0; i < d.size();) {
        if (rt->inj_handle.load() != d[i] && handle_done(d[i])) {
            handle_free(d[i]);
            d[i] = d.back();
            d.pop_back();
        } else {
            ++i;
        }
    }
}

void* scratch_buf(coop_handle* h, size_t bytes) {
    void* p = pool_get(h->rt, bytes);
    if (p) h->scratch.emplace_back(p, bytes);
    return p;
}

struct Sizing {
    uint32_t grid, block, lds, mode;
    uint32_t resident;                         // workgroups of this size the device holds at once
    uint64_t watchdog_ticks;
    uint32_t startup_ticks, sched_p16;
    bool coop;
};

int size_launch(coop_rt* rt, const coop_launch_opts* o, Sizing* s, uint32_t min_lds = 0,
                uint32_t (*occupancy)(bool, uint32_t, uint32_t) = nullptr) {
    coop_launch_opts d;
    coop_launch_opts_default(&d);
    if (!o) o = &d;
    if (o->mode != COOP_MODE_PLAIN && o->mode != COOP_MODE_COOP) return COOP_E_INVALID;
    s->coop = o->mode == COOP_MODE_COOP;
    s->block = o->group_size ? o->group_size : 1024;
    if (s->block % 64 || s->block > coop::kMaxThreads || s->block == 0) return COOP_E_INVALID;
    s->lds = min_lds ? std::max<uint32_t>(o->lds_bytes, min_lds)
                     : std::max<uint32_t>(o->lds_bytes ? o->lds_bytes : kDefaultLds, coop::kernel_lds_bytes());
    if (s->lds > (uint32_t)rt->props.maxSharedMemoryPerMultiProcessor) return COOP_E_INVALID;
    const uint32_t cus = (uint32_t)rt->props.multiProcessorCount;
    // residency per CU from the LDS request (the binding resource here) and
    // the wave slots (32 per CU on CDNA)
    uint32_t by_lds = (uint32_t)rt->props.maxSharedMemoryPerMultiProcessor / s->lds;
    uint32_t by_waves = 32 / (s->block / 64);
    uint32_t per_cu = std::max<uint32_t>(1, std::min(by_lds, by_waves));
    if (occupancy) per_cu = std::max<uint32_t>(1, std::min(per_cu, occupancy(s->coop, s->block, s->lds)));
    const uint32_t resident = cus * per_cu;
    s->resident = resident;
    // the launch context holds per-id tables of kMaxGroups entries
    s->grid = o->num_groups ? o->num_groups : std::min<uint32_t>(resident, coop::kMaxGroups);
    if (s->grid == 0 || s->grid > coop::kMaxGroups) return COOP_E_INVALID;
    if (!s->coop && s->grid > resident) return COOP_E_INVALID;   // a plain barrier needs residency
    if (s->coop && (o->flags & COOP_F_RANDOM_SCHEDULE) && (o->sched_p < 0 || o->sched_p > 1))
        return COOP_E_INVALID;
    s->mode = 0;
    if (s->coop) {
        s->mode |= coop::kModeCoop;
        if (o->flags & COOP_F_PARK_KILLED) s->mode |= coop::kModePark;
        if (o->flags & COOP_F_RANDOM_SCHEDULE) s->mode |= coop::kModeRandomSched;
        if (o->flags & COOP_F_REGULAR_BARRIER) s->mode |= coop::kModeRegular;
    }
    if (o->flags & COOP_F_TEST_LOSE_ONE) s->mode |= coop::kModeLoseOne;
    s->sched_p16 = (uint32_t)std::lround(std::min(1.0, std::max(0.0, o->sched_p)) * 65536.0);
    const uint64_t wd = o->watchdog_ns ? o->watchdog_ns : kDefaultWatchdogNs;
    s->watchdog_ticks = wd * (uint64_t)rt->wall_khz / 1000000ull;
    if (s->watchdog_ticks == 0) s->watchdog_ticks = 1;
    const uint64_t su = o->startup_wait_ns ? o->startup_wait_ns : kDefaultStartupNs;
    s->startup_ticks = (uint32_t)std::min<uint64_t>(0xFFFFFFFFu, su * (uint64_t)rt->wall_khz / 1000000ull);
    return COOP_OK;
}

// Launch constants of a sized launch (`host`: the pinned target word of a
// host-driven schedule, or null).
void fill_cfg(coop_rt* rt, const coop_launch_opts* o, const Sizing& sz, HostCtl* host, coop::Cfg& cfg) {
    cfg = coop::Cfg{};
    cfg.N = sz.grid;
    cfg.mode = sz.mode;
    cfg.sched_p16 = sz.sched_p16;
    cfg.sched_seed = o ? o->sched_seed : 0;
    cfg.watchdog_ticks = sz.watchdog_ticks;
    cfg.host = host;
    cfg.trace = o ? o->d_trace : nullptr;
    cfg.trace_cap = (o && o->d_trace) ? o->trace_cap : 0u;
    cfg.epoch0_wait = sz.startup_ticks;
    cfg.wgtrace = o ? o->d_wgtrace : nullptr;
    cfg.wgtrace_cap = (o && o->d_wgtrace) ? o->trace_cap : 0u;
    cfg.ses = rt->ses;
    cfg.engines = rt->xcds * rt->ses;
    cfg.slots_per_engine = std::max<uint32_t>(1, sz.resident / std::max<uint32_t>(1, cfg.engines));
    cfg.join_window = coop::kJoinCap - sz.grid;
    if (o && o->join_window) cfg.join_window = std::min(cfg.join_window, std::max(o->join_window, sz.grid));
}

// Common launch preamble: handle, context, pinned control block, events.
int begin_launch(coop_rt* rt, const coop_launch_opts* o, const Sizing& sz, int kind, hipStream_t stream,
                 coop_handle** hout) {
    coop_handle* h = new (std::nothrow) coop_handle();
    if (!h) return COOP_E_OOM;
    h->rt = rt;
    h->kind = kind;
    h->coop = sz.coop;
    h->grid = sz.grid;
    h->block = sz.block;
    h->lds = sz.lds;
    h->stream = stream;
    const size_t cbytes = sizeof(Ctx) + sizeof(Work);
    char* cw = static_cast<char*>(scratch_buf(h, cbytes));
    if (!cw) { handle_free(h); return COOP_E_OOM; }
    h->ctx = reinterpret_cast<Ctx*>(cw);
    h->work = reinterpret_cast<Work*>(cw + sizeof(Ctx));
    HostCtl* host = nullptr;
    const bool host_sched = sz.coop && o && (o->flags & COOP_F_HOST_SCHEDULE);
    h->host = host_get(rt);
    if (!h->host) { handle_free(h); return COOP_E_OOM; }
    __atomic_store_n(&h->host->target, sz.grid, __ATOMIC_RELEASE);
    if (host_sched) host = h->host;
    for (hipEvent_t* e : {&h->ev_init, &h->ev_start, &h->ev_end, &h->ev_join}) {
        if (hipEventCreate(e) != hipSuccess) { handle_free(h); return hip_fail(rt, hipErrorOutOfMemory); }
    }
    fill_cfg(rt, o, sz, host, h->cfg);
    hipError_t e = coop::launch_init_ctx(h->ctx, h->work, stream);
    if (e != hipSuccess) { handle_free(h); return hip_fail(rt, e); }
    *hout = h;
    return COOP_OK;
}

int finish_launch(coop_rt* rt, coop_handle* h, hipError_t launch_err, coop_handle** out) {
    if (launch_err != hipSuccess) {
        (void)hipStreamSynchronize(h->stream);
        handle_free(h);
        return hip_fail(rt, launch_err);
    }
    (void)hipEventRecord(h->ev_end, h->stream);
    if (out) *out = h;
    else rt->detached.push_back(h);
    return COOP_OK;
}

hipError_t relaunch(coop_handle* h, bool joiner, uint32_t grid, hipStream_t s) {
    switch (h->kind) {
        case COOP_KERNEL_BFS: return coop::launch_bfs(h->bfs, h->coop, joiner, grid, h->block, h->lds, s);
        case COOP_KERNEL_SSSP: return coop::launch_sssp(h->sssp, h->coop, joiner, grid, h->block, h->lds, s);
        case COOP_KERNEL_COLOR:
        case COOP_KERNEL_MIS: return coop::launch_color(h->color, h->coop, joiner, grid, h->block, h->lds, s);
        case COOP_KERNEL_BARRIER:
            return coop::launch_barrier_bench(h->bb, h->coop, joiner, grid, h->block, h->lds, s);
        case COOP_KERNEL_BATCH: return coop::launch_batch(h->batch, h->coop, joiner, grid, h->block, h->lds, s);
        case COOP_KERNEL_SERVE: return coop::launch_serve(h->serve, h->coop, joiner, grid, h->block, h->lds, s);
        case COOP_KERNEL_OCTREE:
            return coop::launch_octree(h->octree, h->coop, joiner, grid, h->block, h->lds, s);
        case COOP_KERNEL_CC: return coop::launch_cc(h->cc, h->coop, joiner, grid, h->block, h->lds, s);
    }
    return hipErrorInvalidValue;
}

int fill_traversal(coop_handle* h, const coop_graph* g, const uint32_t* roots, uint32_t nroots,
                   uint64_t out_stride, const coop_launch_opts* o, coop::TraversalArgs* t, bool heavy,
                   bool queues) {
    t->cfg = h->cfg;
    t->ctx = h->ctx;
    t->work = h->work;
    t->row_ptr = g->row_ptr;
    t->col = g->col;
    t->w = g->w;
    t->n = g->n;
    t->N = h->grid;
    t->heavy_th = (o && o->heavy_threshold) ? o->heavy_threshold : kDefaultHeavy;
    t->strip = (o && o->strip) ? o->strip : kDefaultStrip;
    t->roots = roots;
    t->nroots = nroots;
    t->out_stride = (uint32_t)out_stride;
    const uint64_t hs = heavy ? const_cast<coop_graph*>(g)->heavy_strips(t->heavy_th, t->strip) : 0;
    if (hs > 0xFFFFFFFFull) return COOP_E_INVALID;
    t->heavy_cap = (uint32_t)hs;
    t->heavy = nullptr;
    if (hs) {
        t->heavy = static_cast<uint4*>(scratch_buf(h, hs * sizeof(uint4)));
        if (!t->heavy) return COOP_E_OOM;
    }
    t->frontier[0] = t->frontier[1] = nullptr;
    if (queues) {
        for (int i = 0; i < 2; ++i) {
            t->frontier[i] = static_cast<uint32_t*>(scratch_buf(h, (size_t)g->n * 4 + 4));
            if (!t->frontier[i]) return COOP_E_OOM;
        }
    }
    const size_t slot_words = (size_t)h->grid * coop::kSlotWords;
    t->slots = static_cast<uint32_t*>(scratch_buf(h, slot_words * 4));
    if (!t->slots) return COOP_E_OOM;
    h->slots = t->slots;
    hipError_t e = coop::launch_fill_u32(t->slots, slot_words, 0u, h->stream);
    if (e != hipSuccess) return hip_fail(h->rt, e);
    return COOP_OK;
}

// The bitmap of vertices without arcs (bottom-up BFS skips them), built on
// first use and kept with the graph.
int ensure_deg0(coop_rt* rt, coop_graph* g, hipStream_t s) {
    if (g->deg0) return COOP_OK;
    hipError_t e = hipMalloc(&g->deg0, (size_t)g->words * 4);
    if (e == hipSuccess) e = coop::launch_deg0_bitmap(g->row_ptr, g->n, g->deg0, g->words, s);
    if (e != hipSuccess) {
        if (g->deg0) (void)hipFree(g->deg0);
        g->deg0 = nullptr;
        return hip_fail(rt, e);
    }
    return COOP_OK;
}

int check_traversal_args(coop_rt* rt, const coop_graph* g, const uint32_t* roots, uint32_t nroots,
                         const void* out, uint64_t out_stride) {
    if (!rt || !g || !roots || !out || nroots == 0) return COOP_E_INVALID;
    if (g->rt != rt || g->n == 0) return COOP_E_INVALID;
    if (nroots > 1 && out_stride != 0 && out_stride < g->n) return COOP_E_INVALID;
    if (out_stride > 0xFFFFFFFFull) return COOP_E_INVALID;
    return COOP_OK;
}

}  // namespace

// =================================================================== C ABI

extern "C" {

const char* coop_strerror(int code) {
    switch (code) {
        case COOP_OK: return "ok";
        case COOP_E_INVALID: return "invalid argument";
        case COOP_E_OOM: return "out of memory";
        case COOP_E_HIP: return "HIP runtime error";
        case COOP_E_TIMEOUT: return "barrier watchdog expired (workgroups not resident or deadlock)";
        case COOP_E_BUSY: return "request can never fit";
        case COOP_E_OVERFLOW: return "distance overflows int32";
        case COOP_E_INTERNAL: return "internal capacity error";
        case COOP_E_TOO_BIG: return "request exceeds a fixed capacity (the no-allocation scratch)";
    }
    return "unknown error";
}

void coop_launch_opts_default(coop_launch_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mode = COOP_MODE_PLAIN;
}

int coop_init(int device, coop_rt** out) {
    if (!out) return COOP_E_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return COOP_E_INVALID;
    coop_rt* rt = new (std::nothrow) coop_rt();
    if (!rt) return COOP_E_OOM;
    rt->device = device;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipGetDeviceProperties(&rt->props, device);
    int khz = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device);
    if (e == hipSuccess) rt->wall_khz = khz > 0 ? (uint32_t)khz : 100000u;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&rt->joiner_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&rt->cotask_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&rt->d_cot, 256);
    if (e == hipSuccess) e = hipMemset(rt->d_cot, 0, 256);
    if (e == hipSuccess) e = hipMalloc(&rt->d_check, 256);
    // the allocation-free entry point's array, at its address on this GPU
    if (e == hipSuccess) e = hipGetSymbolAddress(&rt->noalloc, HIP_SYMBOL(scratch));
    if (e == hipSuccess && !rt->noalloc) e = hipErrorInvalidSymbol;
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&rt->h_stamp), 64,
                                           hipHostMallocCoherent | hipHostMallocMapped);
    if (e == hipSuccess) {
        // count the XCDs and the shader engines per XCD from where the
        // workgroups of a 2x oversubscribed grid land, one per CU at a time,
        // each holding its CU for 50 us
        const uint32_t groups = 2u * (uint32_t)std::max(1, rt->props.multiProcessorCount);
        const uint32_t lds = (uint32_t)rt->props.maxSharedMemoryPerMultiProcessor / 2 + 1024;
        uint32_t* d = nullptr;
        e = hipMalloc(&d, (size_t)groups * 8);
        if (e == hipSuccess)
            e = coop::launch_place_probe(d, groups, lds, 50ull * rt->wall_khz / 1000ull + 1, nullptr);
        std::vector<uint32_t> h((size_t)groups * 2, 0);
        if (e == hipSuccess) e = hipMemcpy(h.data(), d, (size_t)groups * 8, hipMemcpyDeviceToHost);
        if (d) (void)hipFree(d);
        uint32_t mx = 0, ms = 0;
        for (uint32_t g = 0; g < groups; ++g) {
            mx = std::max(mx, h[2 * g]);
            ms = std::max(ms, h[2 * g + 1]);
        }
        rt->xcds = mx + 1;
        rt->ses = ms + 1;
    }

    if (e != hipSuccess) {
        int rc = hip_fail(rt, e);
        coop_shutdown(rt);
        return rc;
    }
    *out = rt;
    return COOP_OK;
}

int coop_shutdown(coop_rt* rt) {
    if (!rt) return COOP_E_INVALID;
    if (rt->injector.joinable()) {
        rt->inj_stop = true;
        rt->injector.join();
    }
    if (rt->sharer.joinable()) {
        rt->share_stop = true;
        rt->sharer.join();
    }
    (void)hipDeviceSynchronize();
    for (coop_handle* h : rt->detached) handle_free(h);
    rt->detached.clear();
    for (auto& kv : rt->pool) (void)hipFree(kv.second);
    rt->pool.clear();
    for (HostCtl* h : rt->host_pool) (void)hipHostFree(h);
    rt->host_pool.clear();
    if (rt->d_cot) (void)hipFree(rt->d_cot);
    if (rt->d_check) (void)hipFree(rt->d_check);
    if (rt->h_stamp) (void)hipHostFree(rt->h_stamp);
    if (rt->joiner_stream) (void)hipStreamDestroy(rt->joiner_stream);
    if (rt->cotask_stream) (void)hipStreamDestroy(rt->cotask_stream);
    delete rt;
    return COOP_OK;
}

int coop_device_query(coop_rt* rt, coop_device_info* out) {
    if (!rt || !out) return COOP_E_INVALID;
    std::memset(out, 0, sizeof(*out));
    out->device = rt->device;
    out->compute_units = (uint32_t)rt->props.multiProcessorCount;
    out->lds_per_cu = (uint32_t)rt->props.maxSharedMemoryPerMultiProcessor;
    out->max_lds_per_group = (uint32_t)rt->props.sharedMemPerBlock;
    out->wall_clock_khz = rt->wall_khz;
    out->hbm_bytes = (uint64_t)rt->props.totalGlobalMem;
    std::snprintf(out->arch, sizeof(out->arch), "%s", rt->props.gcnArchName);
    out->xcds = rt->xcds;
    out->shader_engines = rt->ses;
    return COOP_OK;
}

int coop_last_hip_error(coop_rt* rt) { return rt ? rt->last_hip : 0; }

int coop_graph_wrap(coop_rt* rt, const uint32_t* d_row_ptr, const uint32_t* d_col, const uint32_t* d_w,
                    uint32_t n, uint64_t arcs, coop_graph** out) {
    if (!rt || !d_row_ptr || !out || n == 0) return COOP_E_INVALID;
    if (arcs > 0 && !d_col) return COOP_E_INVALID;
    if (arcs > 0xFFFFFFFFull) return COOP_E_INVALID;
    *out = nullptr;
    std::vector<uint32_t> rp((size_t)n + 1);
    HIP_TRY(rt, hipMemcpy(rp.data(), d_row_ptr, ((size_t)n + 1) * 4, hipMemcpyDeviceToHost));
    if (rp[0] != 0 || rp[n] != arcs) return COOP_E_INVALID;
    for (uint32_t v = 0; v < n; ++v)
        if (rp[v + 1] < rp[v]) return COOP_E_INVALID;
    if (arcs > 0) {
        // every column index must name a vertex: the kernels index their
        // per-vertex arrays with it unchecked
        std::lock_guard<std::recursive_mutex> lk(rt->mu);
        uint32_t bad = 0;
        hipError_t e = coop::launch_check_cols(d_col, arcs, n, rt->d_check, rt->cotask_stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&bad, rt->d_check, 4, hipMemcpyDeviceToHost, rt->cotask_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(rt->cotask_stream);
        if (e != hipSuccess) return hip_fail(rt, e);
        if (bad) return COOP_E_INVALID;
    }
    coop_graph* g = new (std::nothrow) coop_graph();
    if (!g) return COOP_E_OOM;
    g->rt = rt;
    g->row_ptr = d_row_ptr;
    g->col = d_col;
    g->w = d_w;
    g->n = n;
    g->arcs = arcs;
    g->deg.resize(n);
    g->max_deg = 0;
    g->words = (uint32_t)((((uint64_t)n + 31) / 32 + 63) / 64 * 64);
    for (uint32_t v = 0; v < n; ++v) {
        g->deg[v] = rp[v + 1] - rp[v];
        g->max_deg = std::max(g->max_deg, g->deg[v]);
    }
    {
        // the bitmap of vertices without arcs is built here, so that no
        // traversal launch has to allocate it
        std::lock_guard<std::recursive_mutex> lk(rt->mu);
        int rc = ensure_deg0(rt, g, rt->cotask_stream);
        if (rc == COOP_OK && hipStreamSynchronize(rt->cotask_stream) != hipSuccess) rc = COOP_E_HIP;
        // and the bottom-up probe order: every list by decreasing neighbour
        // degree (the first arc mostly decides a bottom-up probe)
        if (rc == COOP_OK) {
            hipError_t e = hipMalloc(&g->col_bu, (size_t)(arcs + 4) * 4);
            // a graph whose maximum degree exceeds 16 x its average has hubs
            // that decide most bottom-up probes on the first arcs
            const bool skewed = arcs > 0 && (uint64_t)g->max_deg * n > 16ull * arcs;
            if (e == hipSuccess && skewed) e = hipMalloc(&g->first2, (size_t)n * sizeof(uint2));
            if (e == hipSuccess)
                e = coop::build_degree_order(d_row_ptr, d_col, n, arcs, g->max_deg, g->col_bu, rt->cotask_stream);
            if (e == hipSuccess && skewed)
                e = coop::build_first_two(d_row_ptr, g->col_bu, n, g->first2, rt->cotask_stream);
            if (e != hipSuccess) rc = e == hipErrorOutOfMemory ? COOP_E_OOM : hip_fail(rt, e);
        }
        if (rc != COOP_OK) {
            if (g->first2) (void)hipFree(g->first2);
            if (g->col_bu) (void)hipFree(g->col_bu);
            if (g->deg0) (void)hipFree(g->deg0);
            delete g;
            return rc;
        }
    }
    *out = g;
    return COOP_OK;
}

int coop_graph_release(coop_graph* g) {
    if (!g) return COOP_E_INVALID;
    if (g->deg0 || g->col_bu) (void)hipDeviceSynchronize();
    if (g->deg0) (void)hipFree(g->deg0);
    if (g->col_bu) (void)hipFree(g->col_bu);
    if (g->first2) (void)hipFree(g->first2);
    delete g;
    return COOP_OK;
}

// A BFS level's found vertices and their degree sum can ride on the barrier
// arrivals (24 and 28 bits of the arrival counter) when no level can exceed
// them: found <= n, mf <= arcs.
static uint32_t arrive_sums_ok(const coop_graph* g, const coop_launch_opts* opts) {
    if (opts && (opts->flags & COOP_F_SLOT_SUMS)) return 0u;
    return (g->n < (1u << 24) && g->arcs < (1ull << 28)) ? 1u : 0u;
}

int coop_bfs(coop_rt* rt, const coop_graph* g, const uint32_t* d_roots, uint32_t nroots, uint32_t* d_level,
             uint64_t out_stride, const coop_launch_opts* opts, coop_stream_t stream, coop_handle** out) {
    int rc = check_traversal_args(rt, g, d_roots, nroots, d_level, out_stride);
    if (rc) return rc;
    std::lock_guard<std::recursive_mutex> lk(rt->mu);
    reap(rt);
    Sizing sz{};
    if ((rc = size_launch(rt, opts, &sz))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    coop_handle* h = nullptr;
    if ((rc = begin_launch(rt, opts, sz, COOP_KERNEL_BFS, s, &h))) return rc;
    coop::BfsArgs& a = h->bfs;
    if ((rc = fill_traversal(h, g, d_roots, nroots, out_stride, opts, &a.t, true, false))) {
        handle_free(h);
        return rc;
    }
    coop_graph* gm = const_cast<coop_graph*>(g);
    if ((rc = ensure_deg0(rt, gm, s))) {
        handle_free(h);
        return rc;
    }
    a.words = g->words;
    a.vis = static_cast<uint32_t*>(scratch_buf(h, (size_t)a.words * 4));
    for (int i = 0; i < 3; ++i) a.fb[i] = static_cast<uint32_t*>(scratch_buf(h, (size_t)a.words * 4));
    a.deg0 = gm->deg0;
    a.level_out = d_level;
    a.direction_opt = (opts && (opts->flags & COOP_F_TOP_DOWN_ONLY)) ? 0u : 1u;
    a.alpha = (opts && opts->bu_alpha) ? opts->bu_alpha : kDefaultAlpha;
    a.beta = (opts && opts->bu_beta) ? opts->bu_beta : 24u;
    a.total_arcs = g->arcs;
    a.bu_prefetch = (opts && (opts->flags & (1u << 31))) ? 1u : 0u;
    a.col_bu = g->col_bu;
    a.first2 = g->first2;
    a.inline_on = (opts && (opts->flags & COOP_F_LEVEL_BARRIERS)) ? 0u : 1u;
    a.arrive_sums = arrive_sums_ok(g, opts);
    if (a.arrive_sums) a.t.cfg.mode |= coop::kModeArriveSums;
    a.flist = a.inline_on ? static_cast<uint32_t*>(scratch_buf(h, (size_t)sz.grid * (coop::kFlWgHost + 1) * 4))
                          : nullptr;
    if (!a.vis || !a.fb[0] || !a.fb[1] || !a.fb[2] || (a.inline_on && !a.flist)) {
        handle_free(h);
        return COOP_E_OOM;
    }
    (void)hipEventRecord(h->ev_init, s);
    (void)hipEventRecord(h->ev_start, s);
    return finish_launch(rt, h, relaunch(h, false, h->grid, s), out);
}

int coop_bfs_noalloc(coop_rt* rt, const coop_graph* g, const uint32_t* d_roots, uint32_t nroots,
                     uint32_t* d_level, uint64_t out_stride, const coop_launch_opts* opts, int32_t* d_status,
                     coop_stream_t stream) {
    int rc = check_traversal_args(rt, g, d_roots, nroots, d_level, out_stride);
    if (rc) return rc;
    if (!d_status || !rt->noalloc) return COOP_E_INVALID;
    // a host-driven target lives in pinned memory the library would allocate
    if (opts && (opts->flags & COOP_F_HOST_SCHEDULE)) return COOP_E_INVALID;
    Sizing sz{};
    if ((rc = size_launch(rt, opts, &sz))) return rc;
    const uint32_t th = (opts && opts->heavy_threshold) ? opts->heavy_threshold : kDefaultHeavy;
    const uint32_t strip = (opts && opts->strip) ? opts->strip : kDefaultStrip;
    uint64_t hs;
    {
        std::lock_guard<std::recursive_mutex> lk(rt->mu);
        hs = g->heavy_strips_lookup(th, strip);
    }
    if (hs > 0xFFFFFFFFull) return COOP_E_TOO_BIG;
    // the array's layout for this call: context | transmit block | slots |
    // found lists | heavy strips | visited, frontier x 3
    const size_t slot_words = (size_t)sz.grid * coop::kSlotWords;
    const bool inline_on = !(opts && (opts->flags & COOP_F_LEVEL_BARRIERS));
    const size_t o_work = align_up(sizeof(Ctx));
    const size_t o_slots = o_work + align_up(sizeof(Work));
    const size_t o_flist = o_slots + align_up(slot_words * 4);
    const size_t o_heavy = o_flist + (inline_on ? align_up((size_t)sz.grid * (coop::kFlWgHost + 1) * 4) : 0);
    const size_t o_bits = o_heavy + align_up(hs * sizeof(uint4));
    const size_t bm = align_up((size_t)g->words * 4);
    const size_t total = o_bits + 4 * bm;
    if (total > COOP_NOALLOC_SCRATCH_BYTES) return COOP_E_TOO_BIG;
    char* base = static_cast<char*>(rt->noalloc);
    coop::BfsArgs a{};
    fill_cfg(rt, opts, sz, nullptr, a.t.cfg);
    a.t.ctx = reinterpret_cast<Ctx*>(base);
    a.t.work = reinterpret_cast<Work*>(base + o_work);
    a.t.slots = reinterpret_cast<uint32_t*>(base + o_slots);
    a.t.row_ptr = g->row_ptr;
    a.t.col = g->col;
    a.t.w = g->w;
    a.t.n = g->n;
    a.t.N = sz.grid;
    a.t.heavy_th = th;
    a.t.strip = strip;
    a.t.heavy_cap = (uint32_t)hs;
    a.t.heavy = hs ? reinterpret_cast<uint4*>(base + o_heavy) : nullptr;
    a.t.roots = d_roots;
    a.t.nroots = nroots;
    a.t.out_stride = (uint32_t)out_stride;
    a.words = g->words;
    a.vis = reinterpret_cast<uint32_t*>(base + o_bits);
    for (int i = 0; i < 3; ++i) a.fb[i] = reinterpret_cast<uint32_t*>(base + o_bits + (size_t)(i + 1) * bm);
    a.deg0 = g->deg0;
    a.level_out = d_level;
    a.direction_opt = (opts && (opts->flags & COOP_F_TOP_DOWN_ONLY)) ? 0u : 1u;
    a.alpha = (opts && opts->bu_alpha) ? opts->bu_alpha : kDefaultAlpha;
    a.beta = (opts && opts->bu_beta) ? opts->bu_beta : 24u;
    a.total_arcs = g->arcs;
    a.bu_prefetch = (opts && (opts->flags & (1u << 31))) ? 1u : 0u;
    a.col_bu = g->col_bu;
    a.first2 = g->first2;
    a.inline_on = inline_on ? 1u : 0u;
    a.arrive_sums = arrive_sums_ok(g, opts);
    if (a.arrive_sums) a.t.cfg.mode |= coop::kModeArriveSums;
    a.flist = inline_on ? reinterpret_cast<uint32_t*>(base + o_flist) : nullptr;
    // the array keeps the previous call's contents: the context and the
    // slots are cleared here, the bitmaps by the kernel's per-source init
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = coop::launch_init_ctx(static_cast<Ctx*>(a.t.ctx), a.t.work, s);
    if (e == hipSuccess) e = coop::launch_fill_u32(a.t.slots, slot_words, 0u, s);
    if (e == hipSuccess) e = coop::launch_bfs(a, sz.coop, false, sz.grid, sz.block, sz.lds, s);
    if (e == hipSuccess) e = coop::launch_copy_status(a.t.ctx, d_status, s);
    return e == hipSuccess ? COOP_OK : hip_fail(rt, e);
}

int coop_sssp(coop_rt* rt, const coop_graph* g, const uint32_t* d_roots, uint32_t nroots, int32_t* d_dist,
              uint64_t out_stride, const coop_launch_opts* opts, coop_stream_t stream, coop_handle** out) {
    int rc = check_traversal_args(rt, g, d_roots, nroots, d_dist, out_stride);
    if (rc) return rc;
    if (!g->w && g->arcs) return COOP_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(rt->mu);
    reap(rt);
    Sizing sz{};
    if ((rc = size_launch(rt, opts, &sz))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    coop_handle* h = nullptr;
    if ((rc = begin_launch(rt, opts, sz, COOP_KERNEL_SSSP, s, &h))) return rc;
    coop::SsspArgs& a = h->sssp;
    if ((rc = fill_traversal(h, g, d_roots, nroots, out_stride, opts, &a.t, true, false))) {
        handle_free(h);
        return rc;
    }
    a.words = g->words;
    for (int i = 0; i < 3; ++i) a.fb[i] = static_cast<uint32_t*>(scratch_buf(h, (size_t)a.words * 4));
    a.lowered = static_cast<uint32_t*>(scratch_buf(h, (size_t)coop::kMaxXcds * 256));
    a.dist_out = d_dist;
    // whether a round lowered anything rides on the barrier arrivals (a count
    // of workgroups: it cannot overflow)
    a.arrive_sums = (opts && (opts->flags & COOP_F_SLOT_SUMS)) ? 0u : 1u;
    if (a.arrive_sums) a.t.cfg.mode |= coop::kModeArriveSums;
    if (!a.fb[0] || !a.fb[1] || !a.fb[2] || !a.lowered) { handle_free(h); return COOP_E_OOM; }
    (void)hipEventRecord(h->ev_init, s);
    (void)hipEventRecord(h->ev_start, s);
    return finish_launch(rt, h, relaunch(h, false, h->grid, s), out);
}

static int color_or_mis(coop_rt* rt, const coop_graph* g, uint64_t seed, uint32_t* colour, uint8_t* in_set,
                        const coop_launch_opts* opts, coop_stream_t stream, coop_handle** out) {
    if (!rt || !g || g->rt != rt || (!colour && !in_set)) return COOP_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(rt->mu);
    reap(rt);
    Sizing sz{};
    int rc = size_launch(rt, opts, &sz);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    coop_handle* h = nullptr;
    if ((rc = begin_launch(rt, opts, sz, in_set ? COOP_KERNEL_MIS : COOP_KERNEL_COLOR, s, &h))) return rc;
    coop::ColorArgs& a = h->color;
    static const uint32_t dummy_root = 0;
    (void)dummy_root;
    if ((rc = fill_traversal(h, g, nullptr, 1, 0, opts, &a.t, false, true))) { handle_free(h); return rc; }
    a.prio_seed = seed;
    a.pending = static_cast<uint32_t*>(scratch_buf(h, (size_t)g->n * 4));
    a.colour_out = colour;
    a.in_set_out = in_set;
    a.mis = in_set ? 1u : 0u;
    a.lanes = coop::color_lanes(g->arcs, g->n);
    if (!a.pending) { handle_free(h); return COOP_E_OOM; }
    (void)hipEventRecord(h->ev_init, s);
    (void)hipEventRecord(h->ev_start, s);
    return finish_launch(rt, h, relaunch(h, false, h->grid, s), out);
}

int coop_color(coop_rt* rt, const coop_graph* g, uint64_t prio_seed, uint32_t* d_colour,
               const coop_launch_opts* opts, coop_stream_t stream, coop_handle** out) {
    if (!d_colour) return COOP_E_INVALID;
    return color_or_mis(rt, g, prio_seed, d_colour, nullptr, opts, stream, out);
}

int coop_mis(coop_rt* rt, const coop_graph* g, uint64_t prio_seed, uint8_t* d_in_set,
             const coop_launch_opts* opts, coop_stream_t stream, coop_handle** out) {
    if (!d_in_set) return COOP_E_INVALID;
    return color_or_mis(rt, g, prio_seed, nullptr, d_in_set, opts, stream, out);
}

int coop_cc(coop_rt* rt, const coop_graph* g, uint32_t* d_label, const coop_launch_opts* opts,
            coop_stream_t stream, coop_handle** out) {
    if (!rt || !g || g->rt != rt || !d_label) return COOP_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(rt->mu);
    reap(rt);
    Sizing sz{};
    int rc = size_launch(rt, opts, &sz);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    coop_handle* h = nullptr;
    if ((rc = begin_launch(rt, opts, sz, COOP_KERNEL_CC, s, &h))) return rc;
    coop::CcArgs& a = h->cc;
    a.cfg = h->cfg;
    a.ctx = h->ctx;
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.n = g->n;
    a.label = d_label;
    a.changed = static_cast<uint32_t*>(scratch_buf(h, 512));
    if (!a.changed) { handle_free(h); return COOP_E_OOM; }
    hipError_t e = coop::launch_fill_u32(a.changed, 128, 0u, s);
    if (e != hipSuccess) { handle_free(h); return hip_fail(rt, e); }
    (void)hipEventRecord(h->ev_init, s);
    (void)hipEventRecord(h->ev_start, s);
    return finish_launch(rt, h, relaunch(h, false, h->grid, s), out);
}

int coop_launch(coop_rt* rt, int kernel_id, const coop_params* p, const coop_launch_opts* opts,
                coop_stream_t stream, coop_handle** out) {
    if (!rt || !p) return COOP_E_INVALID;
    switch (kernel_id) {
        case COOP_KERNEL_BFS:
            return coop_bfs(rt, p->graph, p->d_roots, p->nroots, static_cast<uint32_t*>(p->d_out),
                            p->out_stride, opts, stream, out);
        case COOP_KERNEL_SSSP:
            return coop_sssp(rt, p->graph, p->d_roots, p->nroots, static_cast<int32_t*>(p->d_out),
                             p->out_stride, opts, stream, out);
        case COOP_KERNEL_COLOR:
            return coop_color(rt, p->graph, p->prio_seed, static_cast<uint32_t*>(p->d_out), opts, stream, out);
        case COOP_KERNEL_MIS:
            return coop_mis(rt, p->graph, p->prio_seed, static_cast<uint8_t*>(p->d_out), opts, stream, out);
        case COOP_KERNEL_CC:
            return coop_cc(rt, p->graph, static_cast<uint32_t*>(p->d_out), opts, stream, out);
        case COOP_KERNEL_BARRIER: {
            if (p->barrier_iters == 0) return COOP_E_INVALID;
            std::lock_guard<std::recursive_mutex> lk(rt->mu);
            reap(rt);
            Sizing sz{};
            int rc = size_launch(rt, opts, &sz);
            if (rc) return rc;
            hipStream_t s = reinterpret_cast<hipStream_t>(stream);
            coop_handle* h = nullptr;
            if ((rc = begin_launch(rt, opts, sz, COOP_KERNEL_BARRIER, s, &h))) return rc;
            h->bb.cfg = h->cfg;
            h->bb.ctx = h->ctx;
            h->bb.work = h->work;
            h->bb.iters = p->barrier_iters;
            (void)hipEventRecord(h->ev_init, s);
            (void)hipEventRecord(h->ev_start, s);
            return finish_launch(rt, h, relaunch(h, false, h->grid, s), out);
        }
    }
    return COOP_E_INVALID;
}

// Statistics of a finished batched launch, summed over its instances.
static int batch_stats(coop_handle* h, coop_stats* stats) {
    coop_rt* rt = h->rt;
    const uint32_t count = h->batch.count;
    coop::BatchCtl ctl;
    coop::TaskState task;
    std::vector<coop::TeamState> ts(count);
    std::vector<uint64_t> slots(h->bslot_words / 2);
    hipError_t e = hipMemcpy(&ctl, h->bctl, sizeof(ctl), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&task, &h->ctx->task, sizeof(task), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(ts.data(), h->teams, (size_t)count * sizeof(coop::TeamState),
                                       hipMemcpyDeviceToHost);
    if (e == hipSuccess && !slots.empty())
        e = hipMemcpy(slots.data(), h->bslots, slots.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(rt, e);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, h->ev_start, h->ev_end);
    int rc = ctl.error;
    for (uint32_t i = 0; i < count && rc == COOP_OK; ++i) {
        if (ts[i].bfs_ctx.error) rc = ts[i].bfs_ctx.error;
        else if (ts[i].col_ctx.error) rc = ts[i].col_ctx.error;
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->error = rc;
        uint64_t arcs = 0, rows = 0, words = 0, found = 0;
        for (size_t i = 0; i + 8 <= slots.size(); i += 8) {
            arcs += slots[i + coop::kSlotArcs];
            rows += slots[i + coop::kSlotRows];
            words += slots[i + coop::kSlotBitmap];
            found += slots[i + coop::kSlotFoundAll];
        }
        uint32_t barriers = 0, levels = 0, td = 0, bu = 0, hp = 0;
        for (uint32_t i = 0; i < count; ++i) {
            barriers += ts[i].bfs_ctx.barriers + ts[i].col_ctx.barriers;
            levels += ts[i].bfs_work.x.levels_total;
            td += ts[i].bfs_work.x.td_levels;
            bu += ts[i].bfs_work.x.bu_levels;
            hp += ts[i].bfs_work.x.heavy_phases;
        }
        stats->barriers = barriers;
        stats->kills = task.kills;
        stats->forks = task.forks;
        stats->resizes = task.kills + task.forks;
        stats->min_groups = task.min_active == 0xFFFFFFFFu ? task.max_active : task.min_active;
        stats->max_groups = task.max_active;
        stats->final_groups = ctl.left;
        stats->grid = h->grid;
        stats->levels = levels;
        stats->kernel_ms = ms;
        stats->device_ms = 0.0;
        stats->arcs = arcs;
        stats->rows = rows;
        stats->found = found;
        stats->bitmap_words = words;
        stats->td_levels = td;
        stats->bu_levels = bu;
        stats->heavy_phases = hp;
    }
    return rc;
}

int coop_wait(coop_handle* h, coop_stats* stats) {
    if (!h || h->kind == COOP_KERNEL_SERVE) return COOP_E_INVALID;   // a server owns its launch
    coop_rt* rt = h->rt;
    // poll (a blocking event wait could hold runtime locks the injector
    // thread needs for its own launches while the kernel runs)
    hipError_t e;
    while ((e = hipEventQuery(h->ev_end)) == hipErrorNotReady)
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    // the kernel is finished: detach it from the injector (which may still
    // be forking joiners for it), then wait for those joiner grids
    if (rt->inj_handle.load() == h) {
        rt->inj_handle.store(nullptr);
        while (rt->inj_busy.load()) std::this_thread::yield();
    }
    {
        // and from the GPU sharer (which holds share_mu while it uses handles)
        std::lock_guard<std::mutex> sl(rt->share_mu);
        for (auto& e2 : rt->shared)
            if (e2.h == h) {
                if (!e2.ended) e2.t_end = now_ms();
                e2.ended = true;
                e2.h = nullptr;
            }
    }
    if (e == hipSuccess && h->joined) e = hipEventSynchronize(h->ev_join);
    if (h->kind == COOP_KERNEL_BATCH) {
        int rc = e == hipSuccess ? batch_stats(h, stats) : hip_fail(rt, e);
        std::lock_guard<std::recursive_mutex> lk(rt->mu);
        handle_free(h);
        return rc;
    }
    if (h->kind == COOP_KERNEL_OCTREE) {
        coop::OctCtl ctl{};
        coop::TaskState task{};
        if (e == hipSuccess) e = hipMemcpy(&ctl, h->octree.ctl, sizeof(ctl), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(&task, &h->ctx->task, sizeof(task), hipMemcpyDeviceToHost);
        float ms = 0.f;
        if (e == hipSuccess) (void)hipEventElapsedTime(&ms, h->ev_start, h->ev_end);
        int rc = e == hipSuccess ? ctl.error : hip_fail(rt, e);
        if (rc == COOP_OK && ctl.leaf_count > h->octree.leaf_cap) rc = COOP_E_INVALID;
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->error = rc;
            stats->grid = h->grid;
            stats->kills = task.kills;
            stats->forks = task.forks;
            stats->min_groups = task.min_active == 0xFFFFFFFFu ? task.max_active : task.min_active;
            stats->max_groups = task.max_active;
            stats->levels = ctl.tasks;
            stats->rows = ctl.leaf_count;
            stats->arcs = ctl.steals;
            stats->found = h->octree.n;
            stats->kernel_ms = ms;
        }
        std::lock_guard<std::recursive_mutex> lk(rt->mu);
        handle_free(h);
        return rc;
    }
    CtxCore c;
    Work w;
    std::vector<uint64_t> slots(h->slots ? (size_t)h->grid * coop::kSlotWords / 2 : 0);
    if (e == hipSuccess) e = hipMemcpy(&c, h->ctx, sizeof(CtxCore), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&w, h->work, sizeof(Work), hipMemcpyDeviceToHost);
    if (e == hipSuccess && h->slots)
        e = hipMemcpy(slots.data(), h->slots, slots.size() * 8, hipMemcpyDeviceToHost);
    uint64_t arcs = 0, rows = 0, words = 0, found = 0;
    for (size_t i = 0; i + 8 <= slots.size(); i += 8) {
        arcs += slots[i + coop::kSlotArcs];
        rows += slots[i + coop::kSlotRows];
        words += slots[i + coop::kSlotBitmap];
        found += slots[i + coop::kSlotFoundAll];
    }
    float ms = 0.f;
    if (e == hipSuccess) (void)hipEventElapsedTime(&ms, h->ev_start, h->ev_end);
    int rc = COOP_OK;
    if (e != hipSuccess) {
        rc = hip_fail(rt, e);
    } else {
        rc = c.error;
        if (stats) {
            stats->error = c.error;
            stats->barriers = c.barriers;
            stats->kills = c.kills;
            stats->forks = c.forks;
            stats->resizes = c.resizes;
            stats->min_groups = c.min_M == 0xFFFFFFFFu ? (h->coop ? 1u : h->grid) : c.min_M;
            if (c.min_M == 0xFFFFFFFFu && h->coop && c.max_M == 0) stats->min_groups = 1;
            stats->max_groups = c.max_M ? c.max_M : (h->coop ? 1u : h->grid);
            stats->final_groups = c.final_M;
            stats->grid = h->grid;
            stats->levels = w.x.levels_total;
            stats->kernel_ms = ms;
            stats->device_ms = (c.t_end > c.t_start && c.t_start)
                                   ? (double)(c.t_end - c.t_start) / (double)rt->wall_khz
                                   : 0.0;
            stats->arcs = arcs;
            stats->rows = rows;
            stats->found = found;
            stats->bitmap_words = words;
            stats->td_levels = w.x.td_levels;
            stats->bu_levels = w.x.bu_levels;
            stats->heavy_phases = w.x.heavy_phases;
            stats->join_full = c.join_full;
        }
    }
    std::lock_guard<std::recursive_mutex> lk(rt->mu);
    handle_free(h);
    return rc;
}

uint32_t coop_handle_groups(const coop_handle* h) { return h ? h->grid : 0; }

int coop_set_target(coop_handle* h, uint32_t target) {
    if (!h || !h->host) return COOP_E_INVALID;
    if (target < 1) target = 1;
    if (target > h->grid) target = h->grid;
    __atomic_store_n(&h->host->target, target, __ATOMIC_RELEASE);
    return COOP_OK;
}

int coop_fork_groups(coop_handle* h, uint32_t count) {
    if (!h || !h->coop) return COOP_E_INVALID;
    if (count == 0) return COOP_OK;
    coop_rt* rt = h->rt;
    std::lock_guard<std::recursive_mutex> lk(rt->mu);
    HIP_TRY(rt, hipStreamWaitEvent(rt->joiner_stream, h->ev_init, 0));
    HIP_TRY(rt, relaunch(h, true, count, rt->joiner_stream));
    HIP_TRY(rt, hipEventRecord(h->ev_join, rt->joiner_stream));
    h->joined = true;
    h->forked += count;
    return COOP_OK;
}

// ----------------------------------------------------------------- batched

void coop_tune_default(coop_tune* t) {
    if (!t) return;
    std::memset(t, 0, sizeof(*t));
    t->group_size = 1024;
    t->team_arcs = 1ull << 20;
    t->direction_opt = 1;
}

namespace {

int check_batch_item(coop_rt* rt, const coop_batch_item& it) {
    const coop_graph* g = it.graph;
    if (!g || g->rt != rt || g->n == 0) return COOP_E_INVALID;
    const uint32_t known = COOP_BATCH_BFS | COOP_BATCH_COLOR | COOP_BATCH_MIS;
    if (it.ops == 0 || (it.ops & ~known)) return COOP_E_INVALID;
    if ((it.ops & COOP_BATCH_COLOR) && (it.ops & COOP_BATCH_MIS)) return COOP_E_INVALID;
    if ((it.ops & COOP_BATCH_BFS) && (!it.d_level || it.bfs_root >= g->n)) return COOP_E_INVALID;
    if ((it.ops & COOP_BATCH_COLOR) && !it.d_colour) return COOP_E_INVALID;
    if ((it.ops & COOP_BATCH_MIS) && !it.d_in_set) return COOP_E_INVALID;
    return COOP_OK;
}

}  // namespace

int coop_batch_run(coop_rt* rt, const coop_batch_item* items, uint32_t count, const coop_tune* tune,
                   const coop_launch_opts* opts, coop_stream_t stream, coop_handle** out) {
    if (!rt || !items || count == 0) return COOP_E_INVALID;
    for (uint32_t i = 0; i < count; ++i) {
        int rc = check_batch_item(rt, items[i]);
        if (rc) return rc;
    }
    coop_tune tn;
    coop_tune_default(&tn);
    if (tune) {
        if (tune->group_size) tn.group_size = tune->group_size;
        tn.num_groups = tune->num_groups;
        if (tune->team_arcs) tn.team_arcs = tune->team_arcs;
        tn.team_max = tune->team_max;
        tn.direction_opt = tune->direction_opt;
        tn.heavy_threshold = tune->heavy_threshold;
        tn.strip = tune->strip;
    }
    if (tn.group_size % 64 || tn.group_size > coop::kMaxThreads) return COOP_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(rt->mu);
    reap(rt);
    coop_launch_opts o;
    coop_launch_opts_default(&o);
    if (opts) o = *opts;
    o.group_size = tn.group_size;
    o.num_groups = tn.num_groups;
    if (tn.heavy_threshold) o.heavy_threshold = tn.heavy_threshold;
    if (tn.strip) o.strip = tn.strip;
    Sizing sz{};
    int rc = size_launch(rt, &o, &sz, coop::kernel_lds_bytes_for(tn.group_size), coop::occupancy_batch);
    if (rc) return rc;
    const uint32_t team_max = tn.team_max ? tn.team_max : std::max<uint32_t>(1, sz.grid / 8);
    if (team_max > sz.grid) return COOP_E_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    coop_handle* h = nullptr;
    if ((rc = begin_launch(rt, &o, sz, COOP_KERNEL_BATCH, s, &h))) return rc;

    // ticket order: most work first (longest-processing-time order)
    std::vector<uint32_t> order(count);
    for (uint32_t i = 0; i < count; ++i) order[i] = i;
    auto work = [&](uint32_t i) { return items[i].graph->arcs + items[i].graph->n; };
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return work(a) > work(b); });

    const uint32_t heavy_th = o.heavy_threshold ? o.heavy_threshold : kDefaultHeavy;
    const uint32_t strip = o.strip ? o.strip : kDefaultStrip;
    // sizes of the per-instance regions
    std::vector<uint32_t> team(count);
    std::vector<uint64_t> hcap(count);
    h->batch_first.assign((size_t)count + 1, 0);
    size_t slot_words = 0, bytes = 0;
    for (uint32_t j = 0; j < count; ++j) {
        const coop_batch_item& it = items[order[j]];
        coop_graph* g = const_cast<coop_graph*>(it.graph);
        const uint64_t t = (work(order[j]) + tn.team_arcs - 1) / tn.team_arcs;
        team[j] = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(t, team_max));
        h->batch_first[j + 1] = h->batch_first[j] + team[j];
        slot_words += 2 * (size_t)team[j] * coop::kSlotWords;
        hcap[j] = (it.ops & COOP_BATCH_BFS) ? g->heavy_strips(heavy_th, strip) : 0;
        if (hcap[j] > 0xFFFFFFFFull) { handle_free(h); return COOP_E_INVALID; }
        if (it.ops & COOP_BATCH_BFS) bytes += 4 * align_up((size_t)g->words * 4) + align_up(hcap[j] * 16);
        if (it.ops & (COOP_BATCH_COLOR | COOP_BATCH_MIS)) bytes += 3 * align_up((size_t)g->n * 4 + 4);
        if ((it.ops & COOP_BATCH_BFS) && (rc = ensure_deg0(rt, g, s))) { handle_free(h); return rc; }
    }
    const size_t head = align_up((size_t)count * sizeof(coop::TeamState)) + align_up(sizeof(coop::BatchCtl)) +
                        align_up((size_t)count * sizeof(coop::BatchInst)) + align_up(((size_t)count + 1) * 4) +
                        align_up((size_t)count * 4) + align_up(slot_words * 4);
    char* base = static_cast<char*>(scratch_buf(h, head + bytes));
    if (!base) { handle_free(h); return COOP_E_OOM; }
    char* p = base;
    auto take = [&](size_t b) { char* r = p; p += align_up(b); return r; };
    h->teams = reinterpret_cast<coop::TeamState*>(take((size_t)count * sizeof(coop::TeamState)));
    h->bctl = reinterpret_cast<coop::BatchCtl*>(take(sizeof(coop::BatchCtl)));
    coop::BatchInst* d_inst = reinterpret_cast<coop::BatchInst*>(take((size_t)count * sizeof(coop::BatchInst)));
    uint32_t* d_first = reinterpret_cast<uint32_t*>(take(((size_t)count + 1) * 4));
    uint32_t* d_roots = reinterpret_cast<uint32_t*>(take((size_t)count * 4));
    h->bslots = reinterpret_cast<uint32_t*>(take(slot_words * 4));
    h->bslot_words = slot_words;

    h->batch_inst.assign(count, coop::BatchInst{});
    h->batch_roots.assign(count, 0);
    coop::Cfg icfg = h->cfg;           // per-team barrier constants: no scheduler, no traces
    icfg.mode = 0;
    icfg.host = nullptr;
    icfg.trace = nullptr;
    icfg.trace_cap = 0;
    icfg.wgtrace = nullptr;
    icfg.wgtrace_cap = 0;
    uint32_t* slot = h->bslots;
    for (uint32_t j = 0; j < count; ++j) {
        const coop_batch_item& it = items[order[j]];
        const coop_graph* g = it.graph;
        coop::BatchInst& I = h->batch_inst[j];
        I.team = team[j];
        I.ops = ((it.ops & COOP_BATCH_BFS) ? coop::kBatchBfs : 0u) |
                ((it.ops & (COOP_BATCH_COLOR | COOP_BATCH_MIS)) ? coop::kBatchColor : 0u);
        h->batch_roots[j] = it.bfs_root;
        coop::TraversalArgs t{};
        t.cfg = icfg;
        t.cfg.N = team[j];
        t.row_ptr = g->row_ptr;
        t.col = g->col;
        t.w = g->w;
        t.n = g->n;
        t.heavy_th = heavy_th;
        t.strip = strip;
        t.roots = d_roots + j;
        t.nroots = 1;
        t.out_stride = 0;
        t.N = team[j];
        // BFS
        I.bfs.t = t;
        I.bfs.t.ctx = &h->teams[j].bfs_ctx;
        I.bfs.t.work = &h->teams[j].bfs_work;
        I.bfs.t.slots = slot;
        slot += (size_t)team[j] * coop::kSlotWords;
        if (it.ops & COOP_BATCH_BFS) {
            I.bfs.words = g->words;
            I.bfs.vis = reinterpret_cast<uint32_t*>(take((size_t)g->words * 4));
            for (int k = 0; k < 3; ++k) I.bfs.fb[k] = reinterpret_cast<uint32_t*>(take((size_t)g->words * 4));
            I.bfs.t.heavy_cap = (uint32_t)hcap[j];
            I.bfs.t.heavy = hcap[j] ? reinterpret_cast<uint4*>(take(hcap[j] * 16)) : nullptr;
            I.bfs.deg0 = g->deg0;
            I.bfs.level_out = it.d_level;
            I.bfs.direction_opt = tn.direction_opt ? 1u : 0u;
            I.bfs.alpha = kDefaultAlpha;
            I.bfs.beta = 24;
            I.bfs.total_arcs = g->arcs;
            I.bfs.col_bu = g->col_bu;
            I.bfs.first2 = g->first2;
        }
        // colouring / MIS
        I.col.t = t;
        I.col.t.ctx = &h->teams[j].col_ctx;
        I.col.t.work = &h->teams[j].col_work;
        I.col.t.slots = slot;
        slot += (size_t)team[j] * coop::kSlotWords;
        if (it.ops & (COOP_BATCH_COLOR | COOP_BATCH_MIS)) {
            I.col.t.frontier[0] = reinterpret_cast<uint32_t*>(take((size_t)g->n * 4 + 4));
            I.col.t.frontier[1] = reinterpret_cast<uint32_t*>(take((size_t)g->n * 4 + 4));
            I.col.pending = reinterpret_cast<uint32_t*>(take((size_t)g->n * 4 + 4));
            I.col.prio_seed = it.prio_seed;
            I.col.colour_out = it.d_colour;
            I.col.in_set_out = it.d_in_set;
            I.col.mis = (it.ops & COOP_BATCH_MIS) ? 1u : 0u;
            I.col.lanes = coop::color_lanes(g->arcs, g->n);
        }
    }
    if ((size_t)(p - base) > head + bytes) { handle_free(h); return COOP_E_INTERNAL; }
    hipError_t e = hipMemcpyAsync(d_inst, h->batch_inst.data(), (size_t)count * sizeof(coop::BatchInst),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_first, h->batch_first.data(), ((size_t)count + 1) * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_roots, h->batch_roots.data(), (size_t)count * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && slot_words) e = coop::launch_fill_u32(h->bslots, slot_words, 0u, s);
    if (e == hipSuccess) e = coop::launch_batch_init(h->teams, d_inst, count, h->bctl, s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        handle_free(h);
        return hip_fail(rt, e);
    }
    coop::BatchArgs& a = h->batch;
    a.cfg = h->cfg;
    a.cfg.keep = team_max;                  // the scheduler never takes a launch below its largest team
    a.ctx = h->ctx;
    a.inst = d_inst;
    a.first = d_first;
    a.teams = h->teams;
    a.ctl = h->bctl;
    a.count = count;
    a.team_max = team_max;
    (void)hipEventRecord(h->ev_init, s);
    (void)hipEventRecord(h->ev_start, s);
    return finish_launch(rt, h, relaunch(h, false, h->grid, s), out);
}

namespace {

// The autotuner's cache: one schedule per device and batch shape (instance
// count, vertex and arc sums, largest instance, operations, launch mode),
// kept for the process and, through coop_tune_cache_save / _load, in a
// text file across processes.
struct TuneKey {
    std::string arch;
    uint32_t count;
    uint64_t sum_n, sum_arcs, max_work;
    uint32_t ops, mode;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, count, sum_n, sum_arcs, max_work, ops, mode) <
               std::tie(o.arch, o.count, o.sum_n, o.sum_arcs, o.max_work, o.ops, o.mode);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<coop_tune, double>> g_tune_cache;
constexpr const char* kTuneHeader = "coop-tune-cache v1";

}  // namespace

int coop_batch_autotune(coop_rt* rt, const coop_batch_item* items, uint32_t count, uint32_t stride,
                        uint32_t reps, const coop_launch_opts* opts, coop_stream_t stream, coop_tune* best,
                        double* best_ms, double* default_ms) {
    if (!rt || !items || count == 0 || !best) return COOP_E_INVALID;
    for (uint32_t i = 0; i < count; ++i) {
        int rc = check_batch_item(rt, items[i]);
        if (rc) return rc;
    }
    TuneKey key{rt->props.gcnArchName, count, 0, 0, 0, 0, opts ? opts->mode : (uint32_t)COOP_MODE_PLAIN};
    for (uint32_t i = 0; i < count; ++i) {
        key.sum_n += items[i].graph->n;
        key.sum_arcs += items[i].graph->arcs;
        key.max_work = std::max<uint64_t>(key.max_work, items[i].graph->n + items[i].graph->arcs);
        key.ops |= items[i].ops;
    }
    // names the device model only (the part before the feature list)
    key.arch = key.arch.substr(0, key.arch.find(':'));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *best = it->second.first;
            if (best_ms) *best_ms = it->second.second;
            if (default_ms) *default_ms = -1.0;
            return COOP_OK;
        }
    }
    if (stride == 0) stride = 1;
    if (reps == 0) reps = 3;
    std::vector<coop_batch_item> sub;
    for (uint32_t i = 0; i < count; i += stride) sub.push_back(items[i]);
    int err = COOP_OK;
    auto time_on = [&](const coop_batch_item* its, uint32_t n_its, const coop_tune& t) -> double {
        std::vector<double> ms;
        for (uint32_t r = 0; r < reps; ++r) {
            coop_handle* h = nullptr;
            int rc = coop_batch_run(rt, its, n_its, &t, opts, stream, &h);
            coop_stats st{};
            if (rc == COOP_OK) rc = coop_wait(h, &st);
            if (rc != COOP_OK) {
                if (rc != COOP_E_INVALID) err = rc;
                return 1e30;
            }
            ms.push_back(st.kernel_ms);
        }
        return percentile(ms, 0.5);
    };
    auto time_it = [&](const coop_tune& t) { return time_on(sub.data(), (uint32_t)sub.size(), t); };
    coop_tune cur;
    coop_tune_default(&cur);
    double cur_ms = time_it(cur);
    if (err) return err;
    double def_ms = cur_ms;
    // coordinate search, two passes: group size, workgroup count (as a share
    // of the resident workgroups), team work, team cap, BFS direction rule,
    // heavy-vertex threshold and strip; a candidate must beat the current
    // schedule by 2% (timing noise)
    const uint32_t cus = (uint32_t)std::max(1, rt->props.multiProcessorCount);
    auto try_it = [&](const coop_tune& c) {
        const double ms = time_it(c);
        if (ms < cur_ms * 0.98) {
            cur = c;
            cur_ms = ms;
        }
    };
    for (int pass = 0; pass < 2 && !err; ++pass) {
        for (uint32_t gs : {256u, 512u, 1024u}) {
            if (gs == cur.group_size) continue;
            coop_tune c = cur;
            c.group_size = gs;
            try_it(c);
        }
        for (uint32_t per_cu_x4 : {2u, 3u, 4u, 8u}) {          // 0.5, 0.75, 1 and 2 workgroups per CU
            coop_tune c = cur;
            c.num_groups = std::min<uint32_t>(coop::kMaxGroups, cus * per_cu_x4 / 4);
            if (c.num_groups == cur.num_groups) continue;
            try_it(c);
        }
        for (uint64_t ta : {1ull << 16, 1ull << 18, 1ull << 19, 1ull << 20, 1ull << 21, 1ull << 22, 1ull << 24}) {
            if (ta == cur.team_arcs) continue;
            coop_tune c = cur;
            c.team_arcs = ta;
            try_it(c);
        }
        for (uint32_t div : {16u, 8u, 4u, 2u}) {                 // team cap as a share of N (0 = N / 8)
            coop_tune c = cur;
            const uint32_t N = c.num_groups ? c.num_groups : std::min<uint32_t>(coop::kMaxGroups, cus);
            c.team_max = std::max<uint32_t>(1, N / div);
            if (c.team_max == cur.team_max) continue;
            try_it(c);
        }
        {
            coop_tune c = cur;
            c.direction_opt = cur.direction_opt ? 0u : 1u;
            try_it(c);
        }
        for (uint32_t th : {128u, 512u, 2048u}) {
            if (th == (cur.heavy_threshold ? cur.heavy_threshold : kDefaultHeavy)) continue;
            coop_tune c = cur;
            c.heavy_threshold = th;
            try_it(c);
        }
        for (uint32_t st : {256u, 512u, 1024u}) {
            if (st == (cur.strip ? cur.strip : kDefaultStrip)) continue;
            coop_tune c = cur;
            c.strip = st;
            try_it(c);
        }
    }
    if (err) return err;
    if (stride > 1) {
        // the subset has a fraction of the batch's work, so settings sized
        // to the work (workgroup count, team cap) can win there and lose on
        // the batch: the winner must also beat the default on the batch
        coop_tune dflt;
        coop_tune_default(&dflt);
        def_ms = time_on(items, count, dflt);
        const double won = err ? 1e30 : time_on(items, count, cur);
        if (err) return err;
        if (won < def_ms * 0.98) {
            cur_ms = won;
        } else {
            cur = dflt;
            cur_ms = def_ms;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = std::make_pair(cur, cur_ms);
    }
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    if (default_ms) *default_ms = def_ms;
    return COOP_OK;
}

int coop_tune_cache_save(const char* path, uint32_t* entries) {
    if (!path) return COOP_E_INVALID;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return COOP_E_INVALID;
    std::fprintf(f, "%s\n", kTuneHeader);
    for (const auto& kv : g_tune_cache) {
        const TuneKey& k = kv.first;
        const coop_tune& t = kv.second.first;
        std::fprintf(f, "%s %u %llu %llu %llu %u %u  %u %u %llu %u %u %u %u  %.6f\n", k.arch.c_str(), k.count,
                     (unsigned long long)k.sum_n, (unsigned long long)k.sum_arcs, (unsigned long long)k.max_work,
                     k.ops, k.mode, t.group_size, t.num_groups, (unsigned long long)t.team_arcs, t.team_max,
                     t.direction_opt, t.heavy_threshold, t.strip, kv.second.second);
    }
    const bool ok = std::fclose(f) == 0;
    if (entries) *entries = (uint32_t)g_tune_cache.size();
    return ok ? COOP_OK : COOP_E_INVALID;
}

int coop_tune_cache_load(const char* path, uint32_t* entries) {
    if (!path) return COOP_E_INVALID;
    FILE* f = std::fopen(path, "r");
    if (!f) return COOP_E_INVALID;
    char line[512];
    std::vector<std::pair<TuneKey, std::pair<coop_tune, double>>> got;
    bool ok = std::fgets(line, sizeof(line), f) && std::strncmp(line, kTuneHeader, std::strlen(kTuneHeader)) == 0;
    while (ok && std::fgets(line, sizeof(line), f)) {
        char arch[128];
        unsigned count, ops, mode, gs, ng, tm, dir, th, st;
        unsigned long long sn, sa, mw, ta;
        double ms;
        const int k = std::sscanf(line, "%127s %u %llu %llu %llu %u %u %u %u %llu %u %u %u %u %lf", arch, &count, &sn,
                                  &sa, &mw, &ops, &mode, &gs, &ng, &ta, &tm, &dir, &th, &st, &ms);
        if (k != 15 || gs == 0 || gs % 64 || gs > coop::kMaxThreads || ng > coop::kMaxGroups || dir > 1) {
            ok = false;
            break;
        }
        coop_tune t;
        coop_tune_default(&t);
        t.group_size = gs;
        t.num_groups = ng;
        t.team_arcs = ta;
        t.team_max = tm;
        t.direction_opt = dir;
        t.heavy_threshold = th;
        t.strip = st;
        got.push_back({TuneKey{arch, count, sn, sa, mw, ops, mode}, {t, ms}});
    }
    std::fclose(f);
    if (!ok) return COOP_E_INVALID;          // nothing of a malformed file is taken
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& e : got) g_tune_cache[e.first] = e.second;
    if (entries) *entries = (uint32_t)g_tune_cache.size();
    return COOP_OK;
}

void coop_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
}

// ----------------------------------------------------------------- serving

struct coop_server {
    coop_rt* rt = nullptr;
    coop_handle* h = nullptr;                  // the persistent launch
    hipStream_t stream = nullptr;
    std::vector<const coop_graph*> graphs;
    std::vector<uint32_t> team[2];             // per graph: team of a BFS / SSSP query
    uint32_t slots = 0, team_max = 1, owner_cap = 0;
    uint64_t slot_bytes = 0;
    // pinned host memory shared with the kernel
    coop::ServeHost* host = nullptr;
    coop::ServeReq* req = nullptr;
    uint32_t* owner = nullptr;
    coop::ServeDone* done = nullptr;
    // device memory (descriptors, slot lines, counters, slot state)
    void* dev = nullptr;
    coop::ServeCtl* ctl = nullptr;
    // host scheduling
    struct Query {
        uint32_t gi = 0, kind = 0, src = 0, slot = 0;
        void* out = nullptr;
        double t_submit = 0, t_admit = 0, t_done = 0;
        int state = 0;                          // 0 queued, 1 in a slot, 2 done
        int err = 0;
    };
    std::mutex mu;
    std::condition_variable cv;
    std::map<uint64_t, Query> queries;
    std::deque<uint64_t> pending;
    std::vector<uint64_t> slot_seq;            // query in each slot (0 = free)
    std::vector<uint32_t> free_slots;
    uint32_t next_ticket = 0;
    uint64_t next_seq = 1, submitted = 0, completed = 0;
    std::vector<double> lat[2], waits;
    int error = 0;
    std::thread poller;
    std::atomic<bool> stop_poller{false};
};

void coop_server_cfg_default(coop_server_cfg* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->mode = COOP_MODE_COOP;
    c->group_size = 1024;
    c->team_arcs_bfs = 1ull << 22;
    c->team_arcs_sssp = 1ull << 22;
    c->direction_opt = 1;
}

namespace {

// Publish a queued query into a free slot (server lock held).
void server_publish(coop_server* sv, uint64_t seq) {
    coop_server::Query& q = sv->queries[seq];
    const uint32_t slot = sv->free_slots.back();
    sv->free_slots.pop_back();
    const uint32_t t = sv->team[q.kind == COOP_QUERY_SSSP ? 1 : 0][q.gi];
    coop::ServeReq& r = sv->req[slot];
    r.desc = slot * (uint32_t)sv->graphs.size() + q.gi;
    r.kind = q.kind == COOP_QUERY_SSSP ? coop::kQuerySssp : coop::kQueryBfs;
    r.src = q.src;
    r.team = t;
    r.first = sv->next_ticket;
    r.out = reinterpret_cast<uint64_t>(q.out);
    r.seq = seq;
    for (uint32_t k = 0; k < t; ++k) sv->owner[(sv->next_ticket + k) % sv->owner_cap] = slot;
    sv->next_ticket += t;
    q.slot = slot;
    q.state = 1;
    q.t_admit = now_ms();
    sv->waits.push_back(q.t_admit - q.t_submit);
    sv->slot_seq[slot] = seq;
    __atomic_thread_fence(__ATOMIC_SEQ_CST);
    __atomic_store_n(&sv->host->ticket_end, sv->next_ticket, __ATOMIC_RELEASE);
}

// Completion records -> finished queries; queued queries -> freed slots.
void server_poll_once(coop_server* sv) {
    std::lock_guard<std::mutex> lk(sv->mu);
    bool any = false;
    for (uint32_t s = 0; s < sv->slots; ++s) {
        const uint64_t seq = sv->slot_seq[s];
        if (!seq) continue;
        if (__atomic_load_n(&sv->done[s].seq, __ATOMIC_ACQUIRE) != seq) continue;
        coop_server::Query& q = sv->queries[seq];
        q.state = 2;
        q.t_done = now_ms();
        q.err = __atomic_load_n(&sv->done[s].error, __ATOMIC_ACQUIRE);
        if (q.err && !sv->error) sv->error = q.err;
        sv->lat[q.kind == COOP_QUERY_SSSP ? 1 : 0].push_back(q.t_done - q.t_submit);
        sv->slot_seq[s] = 0;
        sv->free_slots.push_back(s);
        ++sv->completed;
        any = true;
    }
    while (!sv->pending.empty() && !sv->free_slots.empty()) {
        const uint64_t seq = sv->pending.front();
        sv->pending.pop_front();
        server_publish(sv, seq);
    }
    if (any) sv->cv.notify_all();
}

void server_free(coop_server* sv) {
    if (sv->host) (void)hipHostFree(sv->host);
    if (sv->req) (void)hipHostFree(sv->req);
    if (sv->owner) (void)hipHostFree(sv->owner);
    if (sv->done) (void)hipHostFree(sv->done);
    if (sv->dev) (void)hipFree(sv->dev);
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    delete sv;
}

}  // namespace

int coop_server_create(coop_rt* rt, const coop_graph* const* graphs, uint32_t ngraphs, uint64_t hbm_budget,
                       const coop_server_cfg* cfg, coop_server** out) {
    if (!rt || !graphs || ngraphs == 0 || !out) return COOP_E_INVALID;
    *out = nullptr;
    if (!kServerEnabled) return COOP_E_INVALID;
    coop_server_cfg c;
    coop_server_cfg_default(&c);
    if (cfg) c = *cfg;
    if (!c.group_size) c.group_size = 1024;
    if (!c.team_arcs_bfs) c.team_arcs_bfs = 1ull << 22;
    if (!c.team_arcs_sssp) c.team_arcs_sssp = 1ull << 22;
    uint32_t n_max = 0, words_max = 0;
    uint64_t heavy_max = 0;
    const uint32_t heavy_th = c.heavy_threshold ? c.heavy_threshold : kDefaultHeavy;
    const uint32_t strip = c.strip ? c.strip : kDefaultStrip;
    for (uint32_t i = 0; i < ngraphs; ++i) {
        const coop_graph* g = graphs[i];
        if (!g || g->rt != rt || g->n == 0) return COOP_E_INVALID;
        n_max = std::max(n_max, g->n);
        words_max = std::max(words_max, g->words);
        heavy_max = std::max(heavy_max, const_cast<coop_graph*>(g)->heavy_strips(heavy_th, strip));
    }
    // slot state: the BFS visited and frontier bitmaps (SSSP uses the three
    // frontier bitmaps; its distances live in the query's output), the SSSP
    // per-XCD round flags, the heavy-strip list and statistics slots
    const size_t bfs_b = 4 * align_up((size_t)words_max * 4) + (size_t)coop::kMaxXcds * 256;
    const size_t state_b = bfs_b + align_up(heavy_max * 16);

    coop_launch_opts o;
    coop_launch_opts_default(&o);
    o.mode = c.mode;
    o.flags = c.flags & COOP_F_HOST_SCHEDULE;
    o.num_groups = c.num_groups;
    o.group_size = c.group_size;
    o.watchdog_ns = c.watchdog_ns;
    std::lock_guard<std::recursive_mutex> lk(rt->mu);
    reap(rt);
    Sizing sz{};
    int rc = size_launch(rt, &o, &sz, coop::kernel_lds_bytes_for(c.group_size), coop::occupancy_serve);
    if (rc) return rc;
    if (!c.num_groups && sz.resident > 2 * rt->xcds * rt->ses) {
        // The server stays resident between queries, so by default it leaves
        // one workgroup slot per shader engine free: copies the host issues
        // meanwhile run as small kernels (so do other processes' kernels),
        // and the hardware gives a workgroup only a slot on the shader
        // engine it deals it to.
        o.num_groups = sz.resident - rt->xcds * rt->ses;
        if ((rc = size_launch(rt, &o, &sz, coop::kernel_lds_bytes_for(c.group_size), coop::occupancy_serve)))
            return rc;
    }
    const uint32_t team_max = c.team_max ? c.team_max : std::max<uint32_t>(1, sz.grid / 4);
    if (team_max > sz.grid) return COOP_E_INVALID;
    const size_t stats_b = align_up((size_t)team_max * coop::kSlotWords * 4);
    const uint64_t slot_bytes = state_b + stats_b + sizeof(coop::TeamState);
    uint64_t slots = hbm_budget / slot_bytes;
    const uint32_t cap = c.max_queries ? std::min<uint32_t>(c.max_queries, 1024u) : 1024u;
    slots = std::min<uint64_t>(slots, cap);
    if (slots == 0) return COOP_E_BUSY;

    coop_server* sv = new (std::nothrow) coop_server();
    if (!sv) return COOP_E_OOM;
    sv->rt = rt;
    sv->graphs.assign(graphs, graphs + ngraphs);
    sv->slots = (uint32_t)slots;
    sv->team_max = team_max;
    sv->slot_bytes = slot_bytes;
    for (int k = 0; k < 2; ++k) {
        const uint64_t ta = k ? c.team_arcs_sssp : c.team_arcs_bfs;
        for (const coop_graph* g : sv->graphs) {
            const uint64_t t = (g->arcs + g->n + ta - 1) / ta;
            sv->team[k].push_back((uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(t, team_max)));
        }
    }
    uint32_t oc = 1u << 16;
    while (oc < 2 * sv->slots * team_max) oc <<= 1;
    sv->owner_cap = oc;
    hipError_t e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    const unsigned pin = hipHostMallocCoherent | hipHostMallocMapped;
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sv->host), sizeof(coop::ServeHost), pin);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sv->req), slots * sizeof(coop::ServeReq), pin);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sv->owner), (size_t)oc * 4, pin);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sv->done), slots * sizeof(coop::ServeDone), pin);
    if (e != hipSuccess) { server_free(sv); return hip_fail(rt, e); }
    std::memset(sv->host, 0, sizeof(coop::ServeHost));
    std::memset(sv->req, 0, slots * sizeof(coop::ServeReq));
    std::memset(sv->owner, 0, (size_t)oc * 4);
    std::memset(sv->done, 0, slots * sizeof(coop::ServeDone));
    for (const coop_graph* g : sv->graphs) {
        if ((rc = ensure_deg0(rt, const_cast<coop_graph*>(g), sv->stream))) { server_free(sv); return rc; }
    }
    // device layout: descriptors | slot lines | counters | per slot: stats, state
    const size_t desc_b = align_up(slots * ngraphs * sizeof(coop::ServeDesc));
    const size_t team_b = align_up(slots * sizeof(coop::TeamState));
    const size_t ctl_b = align_up(sizeof(coop::ServeCtl));
    const size_t total = desc_b + team_b + ctl_b + slots * (stats_b + state_b);
    e = hipMalloc(&sv->dev, total);
    if (e != hipSuccess) { server_free(sv); return e == hipErrorOutOfMemory ? COOP_E_OOM : hip_fail(rt, e); }
    char* base = static_cast<char*>(sv->dev);
    coop::ServeDesc* d_desc = reinterpret_cast<coop::ServeDesc*>(base);
    coop::TeamState* teams = reinterpret_cast<coop::TeamState*>(base + desc_b);
    sv->ctl = reinterpret_cast<coop::ServeCtl*>(base + desc_b + team_b);
    char* slot_base = base + desc_b + team_b + ctl_b;

    // launch handle (events, pinned target word, sizing)
    coop_handle* h = nullptr;
    if ((rc = begin_launch(rt, &o, sz, COOP_KERNEL_SERVE, sv->stream, &h))) { server_free(sv); return rc; }
    sv->h = h;
    coop::Cfg tcfg = h->cfg;          // per-team barrier constants
    tcfg.mode = 0;
    tcfg.host = nullptr;
    tcfg.trace = nullptr;
    tcfg.trace_cap = 0;
    tcfg.wgtrace = nullptr;
    tcfg.wgtrace_cap = 0;
    tcfg.N = team_max;
    std::vector<coop::ServeDesc> desc(slots * ngraphs);
    for (uint32_t s = 0; s < slots; ++s) {
        char* sb = slot_base + (size_t)s * (stats_b + state_b);
        uint32_t* stats = reinterpret_cast<uint32_t*>(sb);
        char* st = sb + stats_b;
        uint4* heavy = heavy_max ? reinterpret_cast<uint4*>(st + bfs_b) : nullptr;
        for (uint32_t gi = 0; gi < ngraphs; ++gi) {
            const coop_graph* g = sv->graphs[gi];
            coop::ServeDesc& D = desc[(size_t)s * ngraphs + gi];
            coop::TraversalArgs t{};
            t.cfg = tcfg;
            t.ctx = &teams[s].bfs_ctx;
            t.work = &teams[s].bfs_work;
            t.slots = stats;
            t.row_ptr = g->row_ptr;
            t.col = g->col;
            t.w = g->w;
            t.n = g->n;
            t.heavy_th = heavy_th;
            t.strip = strip;
            t.heavy_cap = (uint32_t)const_cast<coop_graph*>(g)->heavy_strips(heavy_th, strip);
            t.heavy = heavy;
            t.roots = nullptr;
            t.nroots = 1;
            t.out_stride = 0;
            t.N = team_max;
            D.bfs.t = t;
            const size_t wb = align_up((size_t)words_max * 4);
            D.bfs.vis = reinterpret_cast<uint32_t*>(st);
            for (int k = 0; k < 3; ++k) D.bfs.fb[k] = reinterpret_cast<uint32_t*>(st + (k + 1) * wb);
            D.bfs.words = g->words;
            D.bfs.deg0 = g->deg0;
            D.bfs.level_out = nullptr;
            D.bfs.direction_opt = c.direction_opt ? 1u : 0u;
            D.bfs.alpha = kDefaultAlpha;
            D.bfs.beta = 24;
            D.bfs.total_arcs = g->arcs;
            D.bfs.col_bu = g->col_bu;
            D.bfs.first2 = g->first2;
            D.sssp.t = t;
            for (int k = 0; k < 3; ++k) D.sssp.fb[k] = D.bfs.fb[k];
            D.sssp.lowered = reinterpret_cast<uint32_t*>(st + 4 * wb);
            D.sssp.words = g->words;
            D.sssp.dist_out = nullptr;
        }
    }
    e = hipMemcpyAsync(d_desc, desc.data(), desc.size() * sizeof(coop::ServeDesc), hipMemcpyHostToDevice,
                       sv->stream);
    for (uint32_t s = 0; s < slots && e == hipSuccess; ++s)
        e = coop::launch_fill_u32(reinterpret_cast<uint32_t*>(slot_base + (size_t)s * (stats_b + state_b)),
                                  stats_b / 4, 0u, sv->stream);
    if (e == hipSuccess) e = coop::launch_serve_init(teams, (uint32_t)slots, sv->ctl, sv->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sv->stream);     // descriptors copied before `desc` goes
    if (e != hipSuccess) {
        handle_free(h);
        server_free(sv);
        return hip_fail(rt, e);
    }
    coop::ServeArgs& a = h->serve;
    a.cfg = h->cfg;
    a.cfg.keep = team_max;                           // never below the largest team
    if (a.cfg.host) a.cfg.mode |= coop::kModeRelayTarget;   // the relay copies the host target
    a.ctx = h->ctx;
    a.slots = (uint32_t)slots;
    a.ndesc = (uint32_t)(slots * ngraphs);
    a.desc = d_desc;
    a.teams = teams;
    a.ctl = sv->ctl;
    a.host = sv->host;
    a.req = sv->req;
    a.owner = sv->owner;
    a.done = sv->done;
    a.owner_cap = oc;
    a.team_max = team_max;
    sv->slot_seq.assign(slots, 0);
    for (uint32_t s = (uint32_t)slots; s-- > 0;) sv->free_slots.push_back(s);
    (void)hipEventRecord(h->ev_init, sv->stream);
    (void)hipEventRecord(h->ev_start, sv->stream);
    e = relaunch(h, false, h->grid, sv->stream);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(sv->stream);
        handle_free(h);
        server_free(sv);
        return hip_fail(rt, e);
    }
    (void)hipEventRecord(h->ev_end, sv->stream);
    sv->poller = std::thread([sv]() {
        (void)hipSetDevice(sv->rt->device);
        double beat = now_ms();
        while (!sv->stop_poller.load()) {
            server_poll_once(sv);
            const double t = now_ms();
            if (t - beat >= 1.0) {
                // tell the server's idle workgroups this process is alive
                __atomic_fetch_add(&sv->host->heartbeat, 1u, __ATOMIC_RELEASE);
                beat = t;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(10));
        }
    });
    *out = sv;
    return COOP_OK;
}

int coop_server_submit(coop_server* sv, const coop_graph* g, int kind, uint32_t src, void* d_out,
                       uint64_t* ticket) {
    if (!sv || !g || !d_out || (kind != COOP_QUERY_BFS && kind != COOP_QUERY_SSSP)) return COOP_E_INVALID;
    uint32_t gi = 0;
    while (gi < sv->graphs.size() && sv->graphs[gi] != g) ++gi;
    if (gi == sv->graphs.size() || src >= g->n) return COOP_E_INVALID;
    if (kind == COOP_QUERY_SSSP && !g->w && g->arcs) return COOP_E_INVALID;
    if (sv->slots == 0) return COOP_E_BUSY;
    std::lock_guard<std::mutex> lk(sv->mu);
    const uint64_t seq = sv->next_seq++;
    coop_server::Query& q = sv->queries[seq];
    q.gi = gi;
    q.kind = (uint32_t)kind;
    q.src = src;
    q.out = d_out;
    q.t_submit = now_ms();
    ++sv->submitted;
    if (!sv->free_slots.empty() && sv->pending.empty()) server_publish(sv, seq);
    else sv->pending.push_back(seq);
    if (ticket) *ticket = seq;
    return COOP_OK;
}

int coop_server_poll(coop_server* sv, uint64_t ticket, int* done, double* latency_ms) {
    if (!sv) return COOP_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->queries.find(ticket);
    if (it == sv->queries.end()) return COOP_E_INVALID;
    const bool fin = it->second.state == 2;
    if (done) *done = fin ? 1 : 0;
    if (fin && latency_ms) *latency_ms = it->second.t_done - it->second.t_submit;
    return fin ? it->second.err : COOP_OK;
}

int coop_server_wait(coop_server* sv, uint64_t ticket, double timeout_ms, double* latency_ms) {
    if (!sv) return COOP_E_INVALID;
    const double deadline = now_ms() + (timeout_ms > 0 ? timeout_ms : 1e12);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        auto it = sv->queries.find(ticket);
        if (it == sv->queries.end()) return COOP_E_INVALID;
        if (it->second.state == 2) {
            if (latency_ms) *latency_ms = it->second.t_done - it->second.t_submit;
            return it->second.err;
        }
        if (sv->error) return sv->error;
        if (now_ms() > deadline) return COOP_E_TIMEOUT;
        sv->cv.wait_for(lk, std::chrono::milliseconds(2));
    }
}

int coop_server_stats(coop_server* sv, coop_serve_stats* out) {
    if (!sv || !out) return COOP_E_INVALID;
    coop::ServeCtl ctl{};
    (void)hipMemcpyAsync(&ctl, sv->ctl, sizeof(ctl), hipMemcpyDeviceToHost, sv->rt->cotask_stream);
    (void)hipStreamSynchronize(sv->rt->cotask_stream);
    std::lock_guard<std::mutex> lk(sv->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->count_bfs = sv->lat[0].size();
    out->count_sssp = sv->lat[1].size();
    for (int k = 0; k < 2; ++k) {
        out->latency_p50_ms[k] = percentile(sv->lat[k], 0.50);
        out->latency_p99_ms[k] = percentile(sv->lat[k], 0.99);
    }
    out->wait_p50_ms = percentile(sv->waits, 0.50);
    out->wait_p99_ms = percentile(sv->waits, 0.99);
    out->slot_bytes = sv->slot_bytes;
    out->slots = sv->slots;
    out->in_flight = sv->slots - (uint32_t)sv->free_slots.size();
    out->queued = (uint32_t)sv->pending.size();
    coop::TaskState task{};
    (void)hipMemcpyAsync(&task, &sv->h->ctx->task, sizeof(task), hipMemcpyDeviceToHost, sv->rt->cotask_stream);
    (void)hipStreamSynchronize(sv->rt->cotask_stream);
    out->kills = task.kills;
    out->forks = task.forks;
    out->min_groups = task.min_active == 0xFFFFFFFFu ? task.max_active : task.min_active;
    out->max_groups = task.max_active;
    out->error = sv->error ? sv->error : ctl.error;
    return COOP_OK;
}

coop_handle* coop_server_handle(coop_server* sv) { return sv ? sv->h : nullptr; }

int coop_server_destroy(coop_server* sv) {
    if (!sv) return COOP_E_INVALID;
    coop_rt* rt = sv->rt;
    int rc = COOP_OK;
    // let queued and running queries finish (bounded), then stop the launch
    const double deadline = now_ms() + 120000.0;
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (sv->completed == sv->submitted || sv->error) break;
        }
        if (hipEventQuery(sv->h->ev_end) == hipSuccess) break;     // the launch ended early
        if (now_ms() > deadline) { rc = COOP_E_TIMEOUT; break; }
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    __atomic_store_n(&sv->host->stop, 1u, __ATOMIC_RELEASE);
    if (rt->inj_handle.load() == sv->h) {
        rt->inj_handle.store(nullptr);
        while (rt->inj_busy.load()) std::this_thread::yield();
    }
    hipError_t e;
    const double d2 = now_ms() + 60000.0;
    while ((e = hipEventQuery(sv->h->ev_end)) == hipErrorNotReady && now_ms() < d2)
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    if (e == hipErrorNotReady) return COOP_E_TIMEOUT;     // leave everything in place: the launch still runs
    if (sv->h->joined) (void)hipEventSynchronize(sv->h->ev_join);
    sv->stop_poller = true;
    if (sv->poller.joinable()) sv->poller.join();
    if (rc == COOP_OK) {
        coop::ServeCtl ctl{};
        if (hipMemcpy(&ctl, sv->ctl, sizeof(ctl), hipMemcpyDeviceToHost) == hipSuccess && ctl.error) rc = ctl.error;
        if (sv->error) rc = sv->error;
    }
    {
        std::lock_guard<std::recursive_mutex> lk(rt->mu);
        handle_free(sv->h);
    }
    server_free(sv);
    return rc;
}

// ----------------------------------------------------------------- co-task

static int cotask_once(coop_rt* rt, const coop_cotask_cfg* cfg, hipStream_t s, coop_handle* h,
                       double* lat, double* gat, double* busy_ms, double* t_req_out = nullptr,
                       double* t_end_out = nullptr) {
    const uint32_t lds = cfg->lds_bytes ? cfg->lds_bytes : kDefaultLds;
    coop::CotaskArgs a{};
    a.busy_ticks = cfg->busy_ns * (uint64_t)rt->wall_khz / 1000000ull;
    a.started = rt->d_cot;
    a.finished = rt->d_cot + 1;
    a.host_stamp = rt->h_stamp;
    a.nwg = cfg->groups;
    if (h && h->kind >= COOP_KERNEL_BFS && h->kind <= COOP_KERNEL_BARRIER) {
        a.release = &h->ctx->release;
        a.joined = &h->ctx->joined_grid;
    }
    __atomic_store_n(&rt->h_stamp[0], 0ull, __ATOMIC_RELEASE);
    __atomic_store_n(&rt->h_stamp[1], 0ull, __ATOMIC_RELEASE);
    __atomic_store_n(&rt->h_stamp[2], ~0ull, __ATOMIC_RELEASE);
    // the counters are cumulative, so no clearing kernel has to find a
    // compute unit before the co-task can start
    a.base = rt->cot_launched;
    const double t_req = now_ms();
    if (h) coop_set_target(h, h->grid > cfg->groups ? h->grid - cfg->groups : 1);
    HIP_TRY(rt, coop::launch_cotask(a, 256, lds, s));
    rt->cot_launched += cfg->groups;        // every launched workgroup counts once, even if we stop waiting
    double t_gather = -1, t_end = -1;
    const double deadline = t_req + 60000.0;
    while (now_ms() < deadline) {
        if (t_gather < 0 && __atomic_load_n(&rt->h_stamp[0], __ATOMIC_ACQUIRE)) t_gather = now_ms();
        if (__atomic_load_n(&rt->h_stamp[1], __ATOMIC_ACQUIRE)) { t_end = now_ms(); break; }
    }
    if (t_end < 0) return COOP_E_TIMEOUT;
    if (t_gather < 0) t_gather = t_end;
    if (h) coop_set_target(h, h->grid);
    if (lat) *lat = t_end - t_req;
    if (gat) *gat = t_gather - t_req;
    if (t_req_out) *t_req_out = t_req;
    if (t_end_out) *t_end_out = t_end;
    if (busy_ms) {
        const uint64_t a0 = __atomic_load_n(&rt->h_stamp[0], __ATOMIC_ACQUIRE);
        const uint64_t a1 = __atomic_load_n(&rt->h_stamp[1], __ATOMIC_ACQUIRE);
        *busy_ms = a1 > a0 ? (double)(a1 - a0) / (double)rt->wall_khz : 0.0;
    }
    HIP_TRY(rt, hipStreamSynchronize(s));
    return COOP_OK;
}

int coop_cotask_run(coop_rt* rt, const coop_cotask_cfg* cfg, coop_stream_t stream, double* latency_ms,
                    double* gather_ms) {
    if (!rt || !cfg || cfg->groups == 0 || cfg->groups > 0xFFFF) return COOP_E_INVALID;
    if (rt->injector.joinable()) return COOP_E_BUSY;
    return cotask_once(rt, cfg, reinterpret_cast<hipStream_t>(stream), nullptr, latency_ms, gather_ms, nullptr);
}

int coop_injector_start(coop_rt* rt, coop_handle* h, const coop_cotask_cfg* cfg) {
    if (!rt || !cfg || cfg->groups == 0 || cfg->period_ns == 0) return COOP_E_INVALID;
    if (h && (!h->coop || h->rt != rt)) return COOP_E_INVALID;
    if (rt->injector.joinable() || rt->sharer.joinable()) return COOP_E_BUSY;
    rt->inj_cfg = *cfg;
    rt->inj_stop = false;
    rt->inj_handle = h;
    rt->inj_lat.clear();
    rt->inj_gather.clear();
    rt->inj_busy_ms.clear();
    rt->inj_setup_max = rt->inj_restore_max = 0;
    rt->inj_late = 0;
    rt->inj_error = 0;
    rt->injector = std::thread([rt]() {
        (void)hipSetDevice(rt->device);
        const coop_cotask_cfg cfg = rt->inj_cfg;
        double next = now_ms();
        uint32_t done = 0;
        while (!rt->inj_stop.load() && (cfg.max_tasks == 0 || done < cfg.max_tasks)) {
            const double t = now_ms();
            if (t < next) {
                std::this_thread::sleep_for(std::chrono::microseconds(
                    (int64_t)std::min(1000.0, (next - t) * 1000.0)));
                continue;
            }
            const double period_ms = (double)cfg.period_ns / 1e6;
            if (t - next > period_ms) ++rt->inj_late;
            next += period_ms;
            rt->inj_busy = 1;
            coop_handle* h = rt->inj_handle.load();
            if (h && handle_done(h)) h = nullptr;
            double lat = 0, gat = 0, busy = 0, t_req = t, t_end = t;
            int rc = cotask_once(rt, &cfg, rt->cotask_stream, h, &lat, &gat, &busy, &t_req, &t_end);
            if (rc == COOP_OK && h && !handle_done(h)) {
                // fork joiners for the compute units the launch gave up:
                // N - M as the co-task saw it when done, less joiner
                // workgroups of earlier forks that have not started yet
                // (they take those units first). Launches that do not
                // report M: the co-task's groups plus what the engine-
                // balanced kill may have taken beyond them; joiners beyond
                // the room the target leaves give their unit back at once.
                const uint64_t seen = __atomic_load_n(&rt->h_stamp[2], __ATOMIC_ACQUIRE);
                uint32_t n;
                if (seen != ~0ull) {
                    const uint32_t M = (uint32_t)seen, started = (uint32_t)(seen >> 32);
                    const uint32_t pending = h->forked > started ? h->forked - started : 0u;
                    n = h->grid > M + pending ? h->grid - M - pending : 0u;
                } else {
                    n = cfg.groups + (h->cfg.engines > 1 ? h->cfg.engines - 1 : 0u);
                }
                rc = coop_fork_groups(h, std::min<uint32_t>(n, h->grid));
            }
            rt->inj_setup_max = std::max(rt->inj_setup_max, t_req - t);
            rt->inj_restore_max = std::max(rt->inj_restore_max, now_ms() - t_end);
            rt->inj_busy = 0;
            if (rc != COOP_OK) { rt->inj_error = rc; break; }
            rt->inj_lat.push_back(lat);
            rt->inj_gather.push_back(gat);
            rt->inj_busy_ms.push_back(busy);
            ++done;
        }
    });
    return COOP_OK;
}

int coop_injector_stop(coop_rt* rt, coop_cotask_stats* out) {
    if (!rt || !rt->injector.joinable()) return COOP_E_INVALID;
    rt->inj_stop = true;
    rt->injector.join();
    rt->inj_handle = nullptr;
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->count = (uint32_t)rt->inj_lat.size();
        out->latency_p50_ms = percentile(rt->inj_lat, 0.50);
        out->latency_p99_ms = percentile(rt->inj_lat, 0.99);
        out->latency_max_ms = percentile(rt->inj_lat, 1.0);
        out->gather_p50_ms = percentile(rt->inj_gather, 0.50);
        out->gather_p99_ms = percentile(rt->inj_gather, 0.99);
        out->gather_max_ms = percentile(rt->inj_gather, 1.0);
        double s = 0;
        for (double b : rt->inj_busy_ms) s += b;
        out->busy_mean_ms = rt->inj_busy_ms.empty() ? 0 : s / (double)rt->inj_busy_ms.size();
        out->setup_max_ms = rt->inj_setup_max;
        out->restore_max_ms = rt->inj_restore_max;
        out->late_periods = rt->inj_late;
    }
    return rt->inj_error;
}

// ---------------------------------------------------- work-stealing octree

int coop_octree(coop_rt* rt, const uint32_t* d_x, const uint32_t* d_y, const uint32_t* d_z, uint32_t n,
                uint32_t cap, uint32_t* d_out, uint32_t* d_leaves, uint32_t leaf_cap, const coop_launch_opts* opts,
                coop_stream_t stream, coop_handle** out) {
    if (!rt || (n && (!d_x || !d_y || !d_z || !d_out || !d_leaves)) || cap == 0 || leaf_cap == 0) return COOP_E_INVALID;
    if ((reinterpret_cast<uintptr_t>(d_out) & 15) != 0) return COOP_E_INVALID;
    std::lock_guard<std::recursive_mutex> lk(rt->mu);
    reap(rt);
    Sizing sz{};
    int rc = size_launch(rt, opts, &sz);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    coop_handle* h = nullptr;
    if ((rc = begin_launch(rt, opts, sz, COOP_KERNEL_OCTREE, s, &h))) return rc;
    coop::OctreeArgs& a = h->octree;
    a.cfg = h->cfg;
    a.n = n;
    a.cap = cap;
    // a cube that is split holds more than cap points and the cubes of one
    // depth are disjoint: at most n / (cap + 1) splits per depth
    const uint64_t nodes = (uint64_t)(coop::kOctMaxDepth + 1) * ((uint64_t)n / ((uint64_t)cap + 1) + 1);
    a.node_cap = (uint32_t)std::min<uint64_t>(nodes, 0xFFFFFFF0ull);
    a.leaf_cap = leaf_cap;
    a.buf[0] = reinterpret_cast<uint4*>(d_out);
    a.buf[1] = static_cast<uint4*>(scratch_buf(h, (size_t)std::max<uint32_t>(n, 1) * 16));
    a.nodes = static_cast<uint32_t*>(scratch_buf(h, (size_t)a.node_cap * 32));
    a.leaves = d_leaves;
    a.ctl = static_cast<coop::OctCtl*>(scratch_buf(h, sizeof(coop::OctCtl)));
    a.q = static_cast<coop::OctQueue*>(scratch_buf(h, (size_t)h->grid * sizeof(coop::OctQueue)));
    a.ctx = h->ctx;
    if (!a.buf[1] || !a.nodes || !a.ctl || !a.q) { handle_free(h); return COOP_E_OOM; }
    hipError_t e = coop::launch_octree_init(a, d_x, d_y, d_z, s);
    if (e != hipSuccess) { handle_free(h); return hip_fail(rt, e); }
    (void)hipEventRecord(h->ev_init, s);
    (void)hipEventRecord(h->ev_start, s);
    return finish_launch(rt, h, relaunch(h, false, h->grid, s), out);
}

// ------------------------------------------------- several cooperative launches

namespace {

// One pass of the sharer (share_mu held): drop finished launches, give every
// live one its weighted share of the resident workgroups as its target, and
// fork joiners for a launch whose share grew (the engine-balanced kill of
// another launch may also have freed up to engines - 1 more).
void share_pass(coop_rt* rt) {
    uint64_t wsum = 0;
    uint32_t live = 0, N = 0;
    for (auto& e : rt->shared) {
        if (e.ended || !e.h) continue;
        if (handle_done(e.h)) {
            e.ended = true;
            e.t_end = now_ms();
            continue;
        }
        wsum += e.weight;
        ++live;
        N = std::max(N, e.h->grid);
    }
    if (!live) return;
    uint32_t given = 0, first = ~0u;
    std::vector<uint32_t> want(rt->shared.size(), 0);
    for (size_t i = 0; i < rt->shared.size(); ++i) {
        auto& e = rt->shared[i];
        if (e.ended || !e.h) continue;
        if (first == ~0u) first = (uint32_t)i;
        want[i] = std::max<uint32_t>(1, (uint32_t)((uint64_t)N * e.weight / wsum));
        given += want[i];
    }
    if (given < N) want[first] += N - given;        // the remainder goes to the oldest launch
    for (size_t i = 0; i < rt->shared.size(); ++i) {
        auto& e = rt->shared[i];
        if (e.ended || !e.h || want[i] == e.share) continue;
        (void)coop_set_target(e.h, want[i]);
        if (e.share && want[i] > e.share) {
            const uint32_t extra = e.h->cfg.engines > 1 ? e.h->cfg.engines - 1 : 0u;
            const int rc = coop_fork_groups(e.h, std::min(want[i] - e.share + extra, e.h->grid));
            if (rc && !rt->share_error) rt->share_error = rc;
            ++rt->share_forks;
        }
        e.share = want[i];
        ++rt->share_updates;
    }
}

}  // namespace

int coop_share_start(coop_rt* rt, uint32_t period_us) {
    if (!rt) return COOP_E_INVALID;
    if (rt->sharer.joinable() || rt->injector.joinable()) return COOP_E_BUSY;
    {
        std::lock_guard<std::mutex> sl(rt->share_mu);
        rt->shared.clear();
        rt->share_updates = rt->share_forks = 0;
        rt->share_error = 0;
        rt->share_period_us = period_us ? period_us : 200u;
    }
    rt->share_stop = false;
    rt->sharer = std::thread([rt]() {
        (void)hipSetDevice(rt->device);
        while (!rt->share_stop.load()) {
            {
                std::lock_guard<std::mutex> sl(rt->share_mu);
                share_pass(rt);
            }
            std::this_thread::sleep_for(std::chrono::microseconds(rt->share_period_us));
        }
    });
    return COOP_OK;
}

int coop_share_add(coop_rt* rt, coop_handle* h, uint32_t weight) {
    if (!rt || !h || h->rt != rt || !h->coop || !h->cfg.host || weight == 0) return COOP_E_INVALID;
    if (!rt->sharer.joinable()) return COOP_E_INVALID;
    std::lock_guard<std::mutex> sl(rt->share_mu);
    for (const auto& e : rt->shared)
        if (e.h == h) return COOP_E_INVALID;
    coop_rt::Shared e;
    e.h = h;
    e.weight = weight;
    e.t_add = now_ms();
    rt->shared.push_back(e);
    share_pass(rt);                                  // targets change now, not a period later
    return COOP_OK;
}

int coop_share_stop(coop_rt* rt, coop_share_stats* out) {
    if (!rt || !rt->sharer.joinable()) return COOP_E_INVALID;
    rt->share_stop = true;
    rt->sharer.join();
    std::lock_guard<std::mutex> sl(rt->share_mu);
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->launches = (uint32_t)rt->shared.size();
        out->target_updates = rt->share_updates;
        out->fork_calls = rt->share_forks;
    }
    rt->shared.clear();
    return rt->share_error;
}

int coop_barrier_bench(coop_rt* rt, const coop_launch_opts* opts, uint32_t iters, coop_stream_t stream,
                       double* ns_per_barrier, coop_stats* stats) {
    if (!rt || iters == 0) return COOP_E_INVALID;
    coop_params p{};
    p.barrier_iters = iters;
    coop_handle* h = nullptr;
    int rc = coop_launch(rt, COOP_KERNEL_BARRIER, &p, opts, stream, &h);
    if (rc) return rc;
    coop_stats st{};
    rc = coop_wait(h, &st);
    if (stats) *stats = st;
    if (ns_per_barrier) *ns_per_barrier = st.device_ms * 1e6 / (double)iters;
    return rc;
}

}  // extern "C"
