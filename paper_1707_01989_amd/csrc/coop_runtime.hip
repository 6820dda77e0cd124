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
#include <thread>
#include <vector>

#include "coop.h"
#include "coop_device.hpp"
#include "coop_internal.h"

using coop::Ctx;
using coop::HostCtl;
using coop::Work;

namespace {

constexpr uint32_t kDefaultLds = 96 * 1024;       // > half a CU's 160 KiB: one workgroup per CU
constexpr uint32_t kDefaultHeavy = 128;
constexpr uint32_t kDefaultStrip = 4096;
constexpr uint64_t kDefaultWatchdogNs = 10ull * 1000 * 1000 * 1000;
constexpr uint32_t kDefaultStartupNs = 20 * 1000;

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
    coop::BfsArgs bfs{};
    coop::SsspArgs sssp{};
    coop::ColorArgs color{};
    coop::BarrierBenchArgs bb{};
};

struct coop_rt {
    int device = 0;
    hipDeviceProp_t props{};
    uint32_t wall_khz = 100000;
    hipStream_t joiner_stream = nullptr;
    hipStream_t cotask_stream = nullptr;
    std::recursive_mutex mu;
    int last_hip = 0;
    std::multimap<size_t, void*> pool;         // free device buffers by size
    std::vector<HostCtl*> host_pool;           // free pinned control blocks
    std::vector<coop_handle*> detached;        // handles the caller did not keep
    // co-task state (counters on the device, stamps in pinned host memory)
    uint32_t* d_cot = nullptr;                 // [0] started, [1] finished
    uint64_t* h_stamp = nullptr;               // [0] all started, [1] all finished
    // injector
    std::thread injector;
    std::atomic<bool> inj_stop{false};
    std::atomic<coop_handle*> inj_handle{nullptr};
    std::atomic<uint32_t> inj_busy{0};         // 1 while the injector touches inj_handle
    coop_cotask_cfg inj_cfg{};
    std::vector<double> inj_lat, inj_gather, inj_busy_ms;
    int inj_error = 0;
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

void* scratch(coop_handle* h, size_t bytes) {
    void* p = pool_get(h->rt, bytes);
    if (p) h->scratch.emplace_back(p, bytes);
    return p;
}

struct Sizing {
    uint32_t grid, block, lds, mode;
    uint64_t watchdog_ticks;
    uint32_t startup_ticks, sched_p16;
    bool coop;
};

int size_launch(coop_rt* rt, const coop_launch_opts* o, Sizing* s) {
    coop_launch_opts d;
    coop_launch_opts_default(&d);
    if (!o) o = &d;
    if (o->mode != COOP_MODE_PLAIN && o->mode != COOP_MODE_COOP) return COOP_E_INVALID;
    s->coop = o->mode == COOP_MODE_COOP;
    s->block = o->group_size ? o->group_size : 1024;
    if (s->block % 64 || s->block > coop::kMaxThreads || s->block == 0) return COOP_E_INVALID;
    s->lds = std::max<uint32_t>(o->lds_bytes ? o->lds_bytes : kDefaultLds, coop::kernel_lds_bytes());
    if (s->lds > (uint32_t)rt->props.maxSharedMemoryPerMultiProcessor) return COOP_E_INVALID;
    const uint32_t cus = (uint32_t)rt->props.multiProcessorCount;
    // residency per CU from the LDS request (the binding resource here) and
    // the wave slots (32 per CU on CDNA)
    uint32_t by_lds = (uint32_t)rt->props.maxSharedMemoryPerMultiProcessor / s->lds;
    uint32_t by_waves = 32 / (s->block / 64);
    uint32_t per_cu = std::max<uint32_t>(1, std::min(by_lds, by_waves));
    const uint32_t resident = cus * per_cu;
    s->grid = o->num_groups ? o->num_groups : resident;
    if (s->grid == 0 || s->grid > 0xFFFF) return COOP_E_INVALID;
    if (!s->coop && s->grid > resident) return COOP_E_INVALID;   // a plain barrier needs residency
    if (s->coop && (o->flags & COOP_F_RANDOM_SCHEDULE) && (o->sched_p < 0 || o->sched_p > 1))
        return COOP_E_INVALID;
    s->mode = 0;
    if (s->coop) {
        s->mode |= coop::kModeCoop;
        if (o->flags & COOP_F_PARK_KILLED) s->mode |= coop::kModePark;
        if (o->flags & COOP_F_RANDOM_SCHEDULE) s->mode |= coop::kModeRandomSched;
    }
    s->sched_p16 = (uint32_t)std::lround(std::min(1.0, std::max(0.0, o->sched_p)) * 65536.0);
    const uint64_t wd = o->watchdog_ns ? o->watchdog_ns : kDefaultWatchdogNs;
    s->watchdog_ticks = wd * (uint64_t)rt->wall_khz / 1000000ull;
    if (s->watchdog_ticks == 0) s->watchdog_ticks = 1;
    const uint64_t su = o->startup_wait_ns ? o->startup_wait_ns : kDefaultStartupNs;
    s->startup_ticks = (uint32_t)std::min<uint64_t>(0xFFFFFFFFu, su * (uint64_t)rt->wall_khz / 1000000ull);
    return COOP_OK;
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
    char* cw = static_cast<char*>(scratch(h, cbytes));
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
    coop::Cfg& cfg = h->cfg;
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
        t->heavy = static_cast<uint4*>(scratch(h, hs * sizeof(uint4)));
        if (!t->heavy) return COOP_E_OOM;
    }
    t->frontier[0] = t->frontier[1] = nullptr;
    if (queues) {
        for (int i = 0; i < 2; ++i) {
            t->frontier[i] = static_cast<uint32_t*>(scratch(h, (size_t)g->n * 4 + 4));
            if (!t->frontier[i]) return COOP_E_OOM;
        }
    }
    const size_t slot_words = (size_t)h->grid * coop::kSlotWords;
    t->slots = static_cast<uint32_t*>(scratch(h, slot_words * 4));
    if (!t->slots) return COOP_E_OOM;
    h->slots = t->slots;
    hipError_t e = coop::launch_fill_u32(t->slots, slot_words, 0u, h->stream);
    if (e != hipSuccess) return hip_fail(h->rt, e);
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
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&rt->h_stamp), 64,
                                           hipHostMallocCoherent | hipHostMallocMapped);
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
    (void)hipDeviceSynchronize();
    for (coop_handle* h : rt->detached) handle_free(h);
    rt->detached.clear();
    for (auto& kv : rt->pool) (void)hipFree(kv.second);
    rt->pool.clear();
    for (HostCtl* h : rt->host_pool) (void)hipHostFree(h);
    rt->host_pool.clear();
    if (rt->d_cot) (void)hipFree(rt->d_cot);
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
        if (rp[v + 1] < rp[v]) { delete g; return COOP_E_INVALID; }
        g->deg[v] = rp[v + 1] - rp[v];
        g->max_deg = std::max(g->max_deg, g->deg[v]);
    }
    *out = g;
    return COOP_OK;
}

int coop_graph_release(coop_graph* g) {
    if (!g) return COOP_E_INVALID;
    if (g->deg0) {
        (void)hipDeviceSynchronize();
        (void)hipFree(g->deg0);
    }
    delete g;
    return COOP_OK;
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
    if (!gm->deg0) {
        hipError_t e = hipMalloc(&gm->deg0, (size_t)gm->words * 4);
        if (e == hipSuccess) e = coop::launch_deg0_bitmap(g->row_ptr, g->n, gm->deg0, gm->words, s);
        if (e != hipSuccess) {
            if (gm->deg0) (void)hipFree(gm->deg0);
            gm->deg0 = nullptr;
            handle_free(h);
            return hip_fail(rt, e);
        }
    }
    a.words = g->words;
    a.vis = static_cast<uint32_t*>(scratch(h, (size_t)a.words * 4));
    for (int i = 0; i < 3; ++i) a.fb[i] = static_cast<uint32_t*>(scratch(h, (size_t)a.words * 4));
    a.deg0 = gm->deg0;
    a.level_out = d_level;
    a.direction_opt = (opts && (opts->flags & COOP_F_TOP_DOWN_ONLY)) ? 0u : 1u;
    a.alpha = 14;
    a.beta = 24;
    a.total_arcs = g->arcs;
    if (!a.vis || !a.fb[0] || !a.fb[1] || !a.fb[2]) { handle_free(h); return COOP_E_OOM; }
    (void)hipEventRecord(h->ev_init, s);
    (void)hipEventRecord(h->ev_start, s);
    return finish_launch(rt, h, relaunch(h, false, h->grid, s), out);
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
    if ((rc = fill_traversal(h, g, d_roots, nroots, out_stride, opts, &a.t, true, true))) {
        handle_free(h);
        return rc;
    }
    a.state = static_cast<uint64_t*>(scratch(h, (size_t)g->n * 8));
    a.dist_out = d_dist;
    if (!a.state) { handle_free(h); return COOP_E_OOM; }
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
    a.pending = static_cast<uint32_t*>(scratch(h, (size_t)g->n * 4));
    a.colour_out = colour;
    a.in_set_out = in_set;
    a.mis = in_set ? 1u : 0u;
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

int coop_wait(coop_handle* h, coop_stats* stats) {
    if (!h) return COOP_E_INVALID;
    coop_rt* rt = h->rt;
    hipError_t e = hipEventSynchronize(h->ev_end);
    // the kernel is finished: detach it from the injector (which may still
    // be forking joiners for it), then wait for those joiner grids
    if (rt->inj_handle.load() == h) {
        rt->inj_handle.store(nullptr);
        while (rt->inj_busy.load()) std::this_thread::yield();
    }
    if (e == hipSuccess && h->joined) e = hipEventSynchronize(h->ev_join);
    Ctx c;
    Work w;
    std::vector<uint64_t> slots(h->slots ? (size_t)h->grid * coop::kSlotWords / 2 : 0);
    if (e == hipSuccess) e = hipMemcpy(&c, h->ctx, offsetof(Ctx, join_entry), hipMemcpyDeviceToHost);
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
            stats->reserved = 0;
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
    return COOP_OK;
}

// ----------------------------------------------------------------- co-task

static int cotask_once(coop_rt* rt, const coop_cotask_cfg* cfg, hipStream_t s, coop_handle* h,
                       double* lat, double* gat, double* busy_ms) {
    const uint32_t lds = cfg->lds_bytes ? cfg->lds_bytes : kDefaultLds;
    coop::CotaskArgs a{};
    a.busy_ticks = cfg->busy_ns * (uint64_t)rt->wall_khz / 1000000ull;
    a.started = rt->d_cot;
    a.finished = rt->d_cot + 1;
    a.host_stamp = rt->h_stamp;
    a.nwg = cfg->groups;
    __atomic_store_n(&rt->h_stamp[0], 0ull, __ATOMIC_RELEASE);
    __atomic_store_n(&rt->h_stamp[1], 0ull, __ATOMIC_RELEASE);
    HIP_TRY(rt, hipMemsetAsync(rt->d_cot, 0, 8, s));
    const double t_req = now_ms();
    if (h) coop_set_target(h, h->grid > cfg->groups ? h->grid - cfg->groups : 1);
    HIP_TRY(rt, coop::launch_cotask(a, 256, lds, s));
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
    if (rt->injector.joinable()) return COOP_E_BUSY;
    rt->inj_cfg = *cfg;
    rt->inj_stop = false;
    rt->inj_handle = h;
    rt->inj_lat.clear();
    rt->inj_gather.clear();
    rt->inj_busy_ms.clear();
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
            next += (double)cfg.period_ns / 1e6;
            rt->inj_busy = 1;
            coop_handle* h = rt->inj_handle.load();
            if (h && handle_done(h)) h = nullptr;
            double lat = 0, gat = 0, busy = 0;
            int rc = cotask_once(rt, &cfg, rt->cotask_stream, h, &lat, &gat, &busy);
            if (rc == COOP_OK && h && !handle_done(h)) rc = coop_fork_groups(h, cfg.groups);
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
    }
    return rt->inj_error;
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
