// Cooperative graph-traversal kernels for gfx950.
//
// Every algorithm is one persistent kernel whose workgroups run the
// level-synchronous loop of the paper's cooperative graph-traversal figure:
// take the work of the current level, process it, meet at one resizing
// global barrier, repeat until the frontier is empty. Between barriers the
// active workgroup count M is fixed; at each barrier the scheduler may fork
// waiting workgroups in or claim the top ids back.
//
// Design rules measured on MI355X: a device-scope atomic on one address
// costs ~11 ns and serialises across the chip, random atomics execute at
// the memory side (~27 G/s), random L2-hit loads reach ~270 G/s. So:
//  * work of a level is distributed statically over the M x (waves per
//    workgroup) wave slots of the interval (units u, u + W, u + 2W, ...);
//    no claim counter;
//  * per-workgroup statistics go to a private slot (one cache line per
//    logical id) summed by the master step; no shared counter;
//  * queue outputs are compacted (wave ballot + mbcnt) into per-wave LDS
//    buffers and flushed with one atomic per workgroup per phase;
//  * BFS keeps its frontiers as bitmaps (three rotating ones) and switches
//    between top-down levels (walk the frontier's neighbour lists, claim
//    targets with one atomic OR) and bottom-up levels (every unvisited
//    vertex looks for a parent in the frontier bitmap; no atomics at all)
//    by the frontier/unvisited edge-count rule of Beamer, Asanovic and
//    Patterson (SC 2012);
//  * a wave walks the concatenated neighbour lists of up to 64 vertices,
//    64 x UNROLL arcs per step, each lane finding its source vertex by a
//    binary search over the wave's degree prefix in LDS; vertices above a
//    degree threshold are cut into fixed-size arc strips processed by all
//    waves in a HEAVY phase of the same level.
#include "traverse.h"

namespace {

template <bool Coop>
__device__ void bfs_body(const BfsArgs& p, bool joiner_grid) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    const TraversalArgs& t = p.t;
    Ctx* c = static_cast<Ctx*>(t.ctx);
    Work* wk = t.work;

    if (threadIdx.x == 0) {
        Member m = register_member(c, t.cfg, !Coop, joiner_grid);
        if (Coop && m.alive && m.epoch == 0) startup_wait(c, t.cfg);
        sh.level = m.alive && m.epoch != 0 ? wk->x.level : 0u;
        sh.root = m.alive && m.epoch != 0 ? wk->x.root : 0u;
        for (int i = 0; i < 8; ++i) sh.acc[i] = 0;
        sh.bar.member = m;
        sh.bar.killed = 0;
    }
    __syncthreads();
    Member m = sh.bar.member;
    uint32_t level = sh.level, root = sh.root;
    bool fresh = m.epoch == 0;      // initial members begin at the registration barrier

    for (;;) {
        if (!m.alive) {
            if (Coop && sh.bar.killed && (t.cfg.mode & kModePark)) {
                __syncthreads();
                if (threadIdx.x == 0) {
                    sh.bar.member = join_queue(c, t.cfg);
                    sh.bar.killed = 0;
                    sh.level = wk->x.level;
                    sh.root = wk->x.root;
                }
                __syncthreads();
                m = sh.bar.member;
                level = sh.level;
                root = sh.root;
                if (m.alive) continue;
            }
            return;
        }
        const uint32_t ph = fresh ? kPhStart : (m.flags & kPhMask);
        fresh = false;
        wg_trace(t.cfg, m.epoch, m.id, kTrStart);
        bfs_phase(p, sh, ph, m.flags, level, root, m.id, m.M);
        wg_trace(t.cfg, m.epoch, m.id, kTrWorkDone);
        const uint32_t cur_flags = m.flags;
        barrier<Coop>(c, t.cfg, m, sh.bar,
                      [&](uint32_t, uint32_t) -> uint32_t { return bfs_master(p, sh, c, ph, cur_flags); });
        bfs_follow(ph, m.flags, level, root);
    }
}

// ----------------------------------------------------------------- SSSP

struct SsspVisit {
    uint64_t* state;        // {distance (hi) | tag (lo)}
    const uint32_t* w;
    uint32_t tag;           // tag meaning "queued for the next round"
    CtxCore* ctx;
    uint32_t* out_tail;
    uint32_t* out;

    __device__ __forceinline__ uint32_t payload(uint32_t v) const {
        return (uint32_t)(ld_relaxed64(&state[v]) >> 32);
    }
    __device__ __forceinline__ uint32_t strip_payload(uint32_t, uint32_t v) const { return payload(v); }
    __device__ __forceinline__ void maybe_flush(WaveLds& wl) {
        if (wl.out_n > kFlushAt) wave_flush(wl, out_tail, out);
    }

    // Frontier Bellman-Ford relaxation. One 64-bit atomicMin on {distance,
    // tag} lowers the distance and, through the old tag it returns, tells
    // whether the vertex is already queued for the next round (tags only
    // grow, so an equal distance never changes the word).
    __device__ __forceinline__ void step(const bool* ok, const uint32_t* arc, const uint32_t* u,
                                         const uint32_t* pay, WaveLds& wl, Stats& st) {
        uint32_t wt[kUnroll];
        uint32_t du[kUnroll];
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) wt[j] = ok[j] ? __builtin_nontemporal_load(&w[arc[j]]) : 0u;
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) du[j] = ok[j] ? (uint32_t)(state[u[j]] >> 32) : 0u;
        bool win[kUnroll];
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) {
            win[j] = false;
            if (!ok[j]) continue;
            const uint64_t nd64 = (uint64_t)pay[j] + (uint64_t)wt[j];
            if (nd64 >= 0x7FFFFFFFull) {
                if (pay[j] != 0x7FFFFFFFu) raise_error(ctx, kErrOverflow);
                continue;
            }
            const uint32_t nd = (uint32_t)nd64;
            if (nd < du[j]) {
                const uint64_t old = __hip_atomic_fetch_min(&state[u[j]], ((uint64_t)nd << 32) | tag,
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                win[j] = nd < (uint32_t)(old >> 32) && (uint32_t)old != tag;
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) {
            st.found += win[j] ? 1u : 0u;
            wave_push(wl, win[j], u[j]);
        }
    }
};

// Queue engine (SSSP): phases INIT (clear), TD (expand the input queue,
// 64-entry units distributed statically), HEAVY; one barrier per phase.
template <bool Coop>
__device__ void sssp_body(const SsspArgs& p, bool joiner_grid) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    const TraversalArgs& t = p.t;
    Ctx* c = static_cast<Ctx*>(t.ctx);
    Work* wk = t.work;
    const uint32_t nw = num_waves();

    if (threadIdx.x == 0) {
        Member m = register_member(c, t.cfg, !Coop, joiner_grid);
        if (Coop && m.alive && m.epoch == 0) startup_wait(c, t.cfg);
        const bool joined = m.alive && m.epoch != 0;
        sh.root = joined ? wk->x.root : 0u;
        sh.aux = joined ? wk->x.round : 0u;
        for (uint32_t i = 0; i < num_waves(); ++i) sh.wave[i].out_n = 0;
        for (int i = 0; i < 8; ++i) sh.acc[i] = 0;
        sh.bar.member = m;
        sh.bar.killed = 0;
    }
    __syncthreads();
    Member m = sh.bar.member;
    uint32_t root = sh.root, round = sh.aux;
    bool fresh = m.epoch == 0;

    for (;;) {
        if (!m.alive) {
            if (Coop && sh.bar.killed && (t.cfg.mode & kModePark)) {
                __syncthreads();
                if (threadIdx.x == 0) {
                    sh.bar.member = join_queue(c, t.cfg);
                    sh.bar.killed = 0;
                    sh.root = wk->x.root;
                    sh.aux = wk->x.round;
                }
                __syncthreads();
                m = sh.bar.member;
                root = sh.root;
                round = sh.aux;
                if (m.alive) continue;
            }
            return;
        }
        const uint32_t ph = fresh ? kPhStart : (m.flags & kPhMask);
        fresh = false;
        const bool sel = (m.flags & kFlagSel) != 0;
        uint32_t* in = t.frontier[sel ? 1 : 0];
        uint32_t* out = t.frontier[sel ? 0 : 1];
        int32_t* dist = p.dist_out + (size_t)root * t.out_stride;
        const uint32_t gw = m.id * nw + wave_id();
        const uint32_t W = m.M * nw;
        Stats st;

        if (ph == kPhInit) {
            // distances to "unreached"; tags to 0 (no round uses tag 0)
            const uint32_t tid = m.id * blockDim.x + threadIdx.x, stride = m.M * blockDim.x;
            for (uint32_t i = tid; i < t.n; i += stride) p.state[i] = 0x7FFFFFFFull << 32;
        } else if (ph == kPhOut) {
            const uint32_t tid = m.id * blockDim.x + threadIdx.x, stride = m.M * blockDim.x;
            for (uint32_t i = tid; i < t.n; i += stride) dist[i] = (int32_t)(p.state[i] >> 32);
        } else if (ph == kPhTD || ph == kPhHeavy) {
            wg_trace(t.cfg, m.epoch, m.id, kTrStart);
            if (threadIdx.x == 0) sh.in_size = wk->x.in_size;
            __syncthreads();
            const uint32_t size = sh.in_size;
            SsspVisit vis{p.state, t.w, round + 2, c, &wk->out_tail, out};
            WaveLds& w = sh.wave[wave_id()];
            if (ph == kPhTD) {
                const uint32_t units = (size + kWave - 1) / kWave;
                for (uint32_t u = gw; u < units; u += W) {
                    const uint32_t i = u * kWave + lane_id();
                    const bool act = i < size;
                    expand_batch(t, wk, w, act, act ? in[i] : 0u, vis, st);
                }
            } else {
                heavy_phase(t, size, gw, W, w, vis, st);
            }
            wg_flush(sh, &wk->out_tail, out);
            stats_to_lds(sh, st);
            __syncthreads();
            acc_to_slot(sh, t.slots, m.id);
            wg_trace(t.cfg, m.epoch, m.id, kTrWorkDone);
        }

        const uint32_t cur_flags = m.flags;
        barrier<Coop>(c, t.cfg, m, sh.bar, [&](uint32_t, uint32_t) -> uint32_t {
            uint64_t tot[2];
            master_sum_slots(sh, t.slots, t.N, tot);
            if (threadIdx.x == 0) {
                XferR x = wk->load_x();                 // one batch of loads
                const uint32_t hs = ld_relaxed(&wk->heavy_tail);
                const uint32_t ot = ld_relaxed(&wk->out_tail);
                uint32_t res;
                const uint32_t flags = cur_flags & kFlagSel;
                if (ph == kPhStart) {
                    x.root() = 0;
                    res = kPhInit;
                } else if (ph == kPhOut) {
                    x.root() += 1;
                    res = x.root() >= t.nroots ? kFlagDone : kPhInit;
                } else if (ph == kPhInit) {
                    const uint32_t r = t.roots[x.root()];
                    p.state[r] = (uint64_t)(x.round() + 1);      // distance 0, queued for this round
                    t.frontier[0][0] = r;
                    x.in_size() = 1;
                    wk->out_tail = 0;
                    wk->heavy_tail = 0;
                    res = kPhTD;               // input = buffer 0
                } else if (ph == kPhTD && hs > 0) {
                    if (hs > t.heavy_cap) raise_error(c, kErrInternal);
                    x.in_size() = hs;
                    wk->heavy_tail = 0;
                    x.heavy_phases() += 1;
                    res = flags | kPhHeavy;
                } else {
                    // round done: the output queue becomes the input
                    wk->out_tail = 0;
                    if (hs) wk->heavy_tail = 0;
                    x.in_size() = ot;
                    x.level() += 1;
                    x.round() += 1;
                    x.levels_total() += 1;
                    res = ot == 0 ? (kPhOut | kFlagAdv) : ((flags ^ kFlagSel) | kPhTD | kFlagAdv);
                }
                wk->store_x(x);
                sh.bar.flags = res;
            }
            __syncthreads();
            return sh.bar.flags;
        });
        const uint32_t nph = m.flags & kPhMask;
        if (m.flags & kFlagAdv) round += 1;
        if (nph == kPhInit && ph == kPhOut) root += 1;
    }
}

template <bool Coop>
__device__ void color_body(const ColorArgs& p, bool joiner_grid) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    const TraversalArgs& t = p.t;
    Ctx* c = static_cast<Ctx*>(t.ctx);

    if (threadIdx.x == 0) {
        Member m = register_member(c, t.cfg, !Coop, joiner_grid);
        if (Coop && m.alive && m.epoch == 0) startup_wait(c, t.cfg);
        for (uint32_t i = 0; i < num_waves(); ++i) sh.wave[i].out_n = 0;
        for (int i = 0; i < 8; ++i) sh.acc[i] = 0;
        sh.bar.member = m;
        sh.bar.killed = 0;
    }
    __syncthreads();
    Member m = sh.bar.member;
    bool fresh = m.epoch == 0;

    for (;;) {
        if (!m.alive) {
            if (Coop && sh.bar.killed && (t.cfg.mode & kModePark)) {
                __syncthreads();
                if (threadIdx.x == 0) {
                    sh.bar.member = join_queue(c, t.cfg);
                    sh.bar.killed = 0;
                }
                __syncthreads();
                m = sh.bar.member;
                if (m.alive) continue;
            }
            return;
        }
        const uint32_t ph = fresh ? kPhStart : (m.flags & kPhMask);
        fresh = false;
        color_phase(p, sh, ph, m.flags, m.id, m.M);
        const uint32_t cur_flags = m.flags;
        barrier<Coop>(c, t.cfg, m, sh.bar,
                      [&](uint32_t, uint32_t) -> uint32_t { return color_master(p, sh, ph, cur_flags); });
    }
}

// ----------------------------------------------------- barrier benchmark

template <bool Coop>
__device__ void barrier_bench_body(const BarrierBenchArgs& p, bool joiner_grid) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    Ctx* c = p.ctx;
    if (threadIdx.x == 0) {
        Member m = register_member(c, p.cfg, !Coop, joiner_grid);
        if (Coop && m.alive && m.epoch == 0) startup_wait(c, p.cfg);
        sh.bar.member = m;
        sh.bar.killed = 0;
    }
    __syncthreads();
    Member m = sh.bar.member;
    for (;;) {
        if (!m.alive) return;
        barrier<Coop>(c, p.cfg, m, sh.bar, [&](uint32_t, uint32_t ne) -> uint32_t {
            if (ne == 1 && threadIdx.x == 0) c->t_start = now_ticks();
            return ne > p.iters ? kFlagDone : 0u;
        });
    }
}

}  // namespace

// ------------------------------------------------------------ entry points

#define COOP_KERNEL_BOUNDS __launch_bounds__(1024)

template <bool Coop>
__global__ void COOP_KERNEL_BOUNDS bfs_kernel(BfsArgs a, int joiner) { bfs_body<Coop>(a, joiner != 0); }
template <bool Coop>
__global__ void COOP_KERNEL_BOUNDS sssp_kernel(SsspArgs a, int joiner) { sssp_body<Coop>(a, joiner != 0); }
template <bool Coop>
__global__ void COOP_KERNEL_BOUNDS color_kernel(ColorArgs a, int joiner) { color_body<Coop>(a, joiner != 0); }
template <bool Coop>
__global__ void COOP_KERNEL_BOUNDS barrier_bench_kernel(BarrierBenchArgs a, int joiner) {
    barrier_bench_body<Coop>(a, joiner != 0);
}

__global__ void init_ctx_kernel(Ctx* c, Work* w) {
    const uint32_t tid = threadIdx.x;
    uint32_t* cw = reinterpret_cast<uint32_t*>(c);
    const uint32_t head_words = sizeof(CtxCore) / 4;
    for (uint32_t i = tid; i < head_words; i += blockDim.x) cw[i] = 0;
    for (uint32_t i = tid; i < kJoinCap; i += blockDim.x) c->join_entry[i] = ~0ull;
    uint32_t* ww = reinterpret_cast<uint32_t*>(w);
    for (uint32_t i = tid; i < sizeof(Work) / 4; i += blockDim.x) ww[i] = 0;
    __syncthreads();
    if (tid == 0) {
        c->min_M = 0xFFFFFFFFu;
        c->release = make_release(0, 1, 0);
    }
}

__global__ void fill_u32_kernel(uint32_t* p, uint64_t count, uint32_t value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// Bit v of `bits` is set when vertex v has no arcs; bits past n are set too.
__global__ void deg0_bitmap_kernel(const uint32_t* row_ptr, uint32_t n, uint32_t* bits, uint32_t words) {
    for (uint32_t wi = blockIdx.x * blockDim.x + threadIdx.x; wi < words; wi += gridDim.x * blockDim.x) {
        uint32_t b = 0;
        for (uint32_t k = 0; k < 32; ++k) {
            const uint32_t v = wi * 32 + k;
            const bool none = v >= n || row_ptr[v + 1] == row_ptr[v];
            b |= (none ? 1u : 0u) << k;
        }
        bits[wi] = b;
    }
}

// A non-cooperative co-task: every workgroup holds its compute unit for a
// fixed wall-clock time (the stand-in for the paper's graphics workload).
// Its LDS request makes it exclusive with a traversal workgroup per CU.
__global__ void __launch_bounds__(256) cotask_kernel(CotaskArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    if (threadIdx.x == 0) {
        const uint64_t t0 = now_ticks();
        lds_raw[0] = 1;
        const uint32_t s = add_relaxed(a.started, 1u);
        if (s + 1 == a.nwg && a.host_stamp)
            __hip_atomic_store(&a.host_stamp[0], t0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        while (now_ticks() - t0 < a.busy_ticks) __builtin_amdgcn_s_sleep(8);
        const uint32_t f = add_relaxed(a.finished, 1u);
        if (f + 1 == a.nwg && a.host_stamp)
            __hip_atomic_store(&a.host_stamp[1], now_ticks(), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();
}

namespace coop {

uint32_t kernel_lds_bytes() { return (uint32_t)sizeof(BlockLds); }

uint32_t kernel_lds_bytes_for(uint32_t block) {
    return (uint32_t)(offsetof(BlockLds, wave) + (size_t)(block / 64) * sizeof(WaveLds));
}

template <class K, class A>
static hipError_t launch_persistent(K kern_coop, K kern_plain, const A& a, bool coop, bool joiner_grid,
                                    uint32_t grid, uint32_t block, uint32_t lds_bytes, hipStream_t s) {
    K k = coop ? kern_coop : kern_plain;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_bytes);
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds_bytes, s, a, joiner_grid ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_bfs(const BfsArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                      uint32_t lds_bytes, hipStream_t s) {
    return launch_persistent(bfs_kernel<true>, bfs_kernel<false>, a, coop, joiner_grid, grid, block,
                             lds_bytes, s);
}
hipError_t launch_sssp(const SsspArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                       uint32_t lds_bytes, hipStream_t s) {
    return launch_persistent(sssp_kernel<true>, sssp_kernel<false>, a, coop, joiner_grid, grid, block,
                             lds_bytes, s);
}
hipError_t launch_color(const ColorArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                        uint32_t lds_bytes, hipStream_t s) {
    return launch_persistent(color_kernel<true>, color_kernel<false>, a, coop, joiner_grid, grid, block,
                             lds_bytes, s);
}
hipError_t launch_barrier_bench(const BarrierBenchArgs& a, bool coop, bool joiner_grid, uint32_t grid,
                                uint32_t block, uint32_t lds_bytes, hipStream_t s) {
    return launch_persistent(barrier_bench_kernel<true>, barrier_bench_kernel<false>, a, coop, joiner_grid,
                             grid, block, lds_bytes, s);
}

hipError_t launch_init_ctx(Ctx* c, Work* w, hipStream_t s) {
    hipLaunchKernelGGL(init_ctx_kernel, dim3(1), dim3(256), 0, s, c, w);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s) {
    if (count == 0) return hipSuccess;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t launch_deg0_bitmap(const uint32_t* row_ptr, uint32_t n, uint32_t* bits, uint32_t words,
                              hipStream_t s) {
    uint32_t blocks = (words + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(deg0_bitmap_kernel, dim3(blocks), dim3(256), 0, s, row_ptr, n, bits, words);
    return hipGetLastError();
}

hipError_t launch_cotask(const CotaskArgs& a, uint32_t block, uint32_t lds_bytes, hipStream_t s) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(cotask_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    hipLaunchKernelGGL(cotask_kernel, dim3(a.nwg), dim3(block), lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace coop
