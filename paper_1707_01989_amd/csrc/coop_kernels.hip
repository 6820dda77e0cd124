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

// Every body below is written against the programming-model calls of
// coop_device.hpp (coop_start, coop_resizing_global_barrier,
// coop_get_group_id / coop_get_num_groups, coop_rejoin); the level state a
// joiner takes over is the Work block's transmit words, written by the
// barrier's single step.

template <bool Coop, bool Small>
__device__ __forceinline__ void bfs_body(const BfsArgs& p, bool joiner_grid) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    const TraversalArgs& t = p.t;
    Ctx* c = static_cast<Ctx*>(t.ctx);
    Group g(c, t.cfg, sh.bar);
    Work* wk = t.work;

    coop_start<Coop>(g, joiner_grid);
    if (threadIdx.x == 0) {
        const bool joined = g.bar.member.alive && coop_joined(g);
        sh.level = joined ? wk->x.level : 0u;
        sh.root = joined ? wk->x.root : 0u;
        for (int i = 0; i < 8; ++i) sh.acc[i] = 0;
        sh.fl_n = 0;
    }
    __syncthreads();
    uint32_t level = sh.level, root = sh.root;
    bool fresh = !coop_joined(g);   // initial members begin at the registration barrier

    for (;;) {
        if (!g.bar.member.alive) {
            if (!coop_rejoin<Coop>(g)) return;
            if (threadIdx.x == 0) {
                sh.level = wk->x.level;
                sh.root = wk->x.root;
            }
            __syncthreads();
            level = sh.level;
            root = sh.root;
            continue;
        }
        const uint32_t cur_flags = coop_flags(g);
        const uint32_t ph = fresh ? kPhStart : (cur_flags & kPhMask);
        const uint32_t id = coop_get_group_id(g), M = coop_get_num_groups(g);
        fresh = false;
        wg_trace(t.cfg, g.bar.member.epoch, id, kTrStart);
        const uint64_t pay = bfs_phase<Small>(p, sh, ph, cur_flags, level, root, id, M, p.level_out);
        wg_trace(t.cfg, g.bar.member.epoch, id, kTrWorkDone);
        coop_resizing_global_barrier<Coop>(g, [&](uint32_t M_now, uint32_t) -> uint32_t {
            return bfs_master<Small>(p, sh, c, ph, cur_flags, t.roots, p.level_out, M_now);
        }, pay);
        bfs_follow(ph, coop_flags(g), level, root, wk);
    }
}

// ----------------------------------------------------------------- SSSP

template <bool Coop>
__device__ __forceinline__ void sssp_body(const SsspArgs& p, bool joiner_grid) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    const TraversalArgs& t = p.t;
    Ctx* c = static_cast<Ctx*>(t.ctx);
    Group g(c, t.cfg, sh.bar);
    Work* wk = t.work;

    coop_start<Coop>(g, joiner_grid);
    if (threadIdx.x == 0) {
        const bool joined = g.bar.member.alive && coop_joined(g);
        sh.root = joined ? wk->x.root : 0u;
        for (uint32_t i = 0; i < num_waves(); ++i) sh.wave[i].out_n = 0;
        for (int i = 0; i < 8; ++i) sh.acc[i] = 0;
    }
    __syncthreads();
    uint32_t root = sh.root;
    bool fresh = !coop_joined(g);

    for (;;) {
        if (!g.bar.member.alive) {
            if (!coop_rejoin<Coop>(g)) return;
            if (threadIdx.x == 0) sh.root = wk->x.root;
            __syncthreads();
            root = sh.root;
            continue;
        }
        const uint32_t cur_flags = coop_flags(g);
        const uint32_t ph = fresh ? kPhStart : (cur_flags & kPhMask);
        const uint32_t id = coop_get_group_id(g), M = coop_get_num_groups(g);
        fresh = false;
        wg_trace(t.cfg, g.bar.member.epoch, id, kTrStart);
        const uint64_t pay = sssp_phase(p, sh, ph, cur_flags, p.dist_out + (size_t)root * t.out_stride, id, M);
        wg_trace(t.cfg, g.bar.member.epoch, id, kTrWorkDone);
        coop_resizing_global_barrier<Coop>(g, [&](uint32_t, uint32_t) -> uint32_t {
            return sssp_master(p, sh, c, ph, cur_flags, t.roots, p.dist_out);
        }, pay);
        sssp_follow(ph, coop_flags(g), root);
    }
}

template <bool Coop>
__device__ __forceinline__ void color_body(const ColorArgs& p, bool joiner_grid) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    const TraversalArgs& t = p.t;
    Ctx* c = static_cast<Ctx*>(t.ctx);
    Group g(c, t.cfg, sh.bar);

    coop_start<Coop>(g, joiner_grid);
    if (threadIdx.x == 0) {
        for (uint32_t i = 0; i < num_waves(); ++i) sh.wave[i].out_n = 0;
        for (int i = 0; i < 8; ++i) sh.acc[i] = 0;
    }
    __syncthreads();
    bool fresh = !coop_joined(g);

    for (;;) {
        if (!g.bar.member.alive) {
            if (!coop_rejoin<Coop>(g)) return;
            continue;
        }
        const uint32_t cur_flags = coop_flags(g);
        const uint32_t ph = fresh ? kPhStart : (cur_flags & kPhMask);
        fresh = false;
        color_phase(p, sh, ph, cur_flags, coop_get_group_id(g), coop_get_num_groups(g));
        coop_resizing_global_barrier<Coop>(g, [&](uint32_t, uint32_t) -> uint32_t {
            return color_master(p, sh, ph, cur_flags);
        });
    }
}

// ----------------------------------------------------- barrier benchmark

template <bool Coop>
__device__ void barrier_bench_body(const BarrierBenchArgs& p, bool joiner_grid) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    Ctx* c = p.ctx;
    Group g(c, p.cfg, sh.bar);
    if (!coop_start<Coop>(g, joiner_grid)) return;
    bool first = true;
    while (coop_resizing_global_barrier<Coop>(g, [&](uint32_t, uint32_t ne) -> uint32_t {
        if (ne == 1 && threadIdx.x == 0) c->t_start = now_ticks();
        return ne > p.iters ? kFlagDone : 0u;
    })) {
        // test of the bounded wait: the last member goes missing (no kill,
        // no leave): the others' next waits run out on the watchdog
        if ((p.cfg.mode & kModeLoseOne) && first && coop_get_group_id(g) + 1 == coop_get_num_groups(g)) return;
        first = false;
    }
}

}  // namespace

// ------------------------------------------------------------ entry points

#define COOP_KERNEL_BOUNDS __launch_bounds__(1024)

template <bool Coop>
__global__ void COOP_KERNEL_BOUNDS bfs_kernel(BfsArgs a, int joiner) { bfs_body<Coop, true>(a, joiner != 0); }
// ... built without the master step's small levels, for launches that give
// every level its own phase and barrier (BfsArgs::inline_on = 0)
template <bool Coop>
__global__ void COOP_KERNEL_BOUNDS bfs_levels_kernel(BfsArgs a, int joiner) { bfs_body<Coop, false>(a, joiner != 0); }
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
    for (uint32_t i = tid; i < kMaxXcds; i += blockDim.x) {
        c->xcd_arrive[i].count = 0;
        c->xcd.members[i] = 0;
    }
    if (tid == 0) c->xcd.groups = 0;
    uint32_t* tw = reinterpret_cast<uint32_t*>(&c->task);
    for (uint32_t i = tid; i < sizeof(TaskState) / 4; i += blockDim.x) tw[i] = 0;
    for (uint32_t i = tid; i < 64; i += blockDim.x) c->transmit[i] = 0;
    uint32_t* ww = reinterpret_cast<uint32_t*>(w);
    for (uint32_t i = tid; i < sizeof(Work) / 4; i += blockDim.x) ww[i] = 0;
    __syncthreads();
    if (tid == 0) {
        c->min_M = 0xFFFFFFFFu;
        c->task.min_active = 0xFFFFFFFFu;
        c->release = make_release(0, 1, 0);
    }
}

// Every workgroup records its XCD and shader engine (the runtime counts
// them). The launch asks for more than half a CU's LDS, so a CU holds one
// probe workgroup, and each holds its CU for `hold` wall-clock ticks: the
// first grid-full lands on every CU, hence on every shader engine, instead
// of a few fast CUs taking all of them.
__global__ void place_probe_kernel(uint32_t* out, uint64_t hold) {
    extern __shared__ uint32_t probe_lds[];
    if (threadIdx.x == 0) {
        const uint64_t t0 = now_ticks();
        probe_lds[0] = blockIdx.x;
        out[2 * blockIdx.x] = __builtin_amdgcn_s_getreg((3u << 11) | (0u << 6) | 20u) & 0xFu;
        out[2 * blockIdx.x + 1] = (__builtin_amdgcn_s_getreg((31u << 11) | (0u << 6) | 4u) >> 13) & 7u;
        while (now_ticks() - t0 < hold) __builtin_amdgcn_s_sleep(8);
    }
}

__global__ void fill_u32_kernel(uint32_t* p, uint64_t count, uint32_t value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void copy_status_kernel(const CtxCore* c, int32_t* out) {
    if (threadIdx.x == 0) *out = ld_relaxed_i(&c->error);
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

// Column indices outside [0, n), counted into *bad (graph check).
__global__ void check_cols_kernel(const uint32_t* col, uint64_t arcs, uint32_t n, uint32_t* bad) {
    uint32_t b = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < arcs; i += (uint64_t)gridDim.x * blockDim.x)
        b += col[i] >= n ? 1u : 0u;
    if (b) atomicAdd(bad, b);
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
        if (s + 1 == a.base + a.nwg && a.host_stamp)
            __hip_atomic_store(&a.host_stamp[0], t0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        while (now_ticks() - t0 < a.busy_ticks) __builtin_amdgcn_s_sleep(8);
        const uint32_t f = add_relaxed(a.finished, 1u);
        if (f + 1 == a.base + a.nwg && a.host_stamp) {
            if (a.release) {
                // what the resizable launch looks like while the co-task
                // still holds its compute units: the host forks joiners
                // for exactly the units it gives back
                const uint64_t r = ld_relaxed64(a.release);
                const uint32_t j = ld_relaxed(a.joined);
                __hip_atomic_store(&a.host_stamp[2], (uint64_t)rel_M(r) | ((uint64_t)j << 32), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            }
            __hip_atomic_store(&a.host_stamp[1], now_ticks(), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    __syncthreads();
}

namespace coop {

uint32_t kernel_lds_bytes() { return (uint32_t)sizeof(BlockLds); }

hipError_t launch_place_probe(uint32_t* out, uint32_t groups, uint32_t lds_bytes, uint64_t hold_ticks,
                              hipStream_t s) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(place_probe_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    hipLaunchKernelGGL(place_probe_kernel, dim3(groups), dim3(64), lds_bytes, s, out, hold_ticks);
    return hipGetLastError();
}

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
    if (!a.inline_on)
        return launch_persistent(bfs_levels_kernel<true>, bfs_levels_kernel<false>, a, coop, joiner_grid, grid,
                                 block, lds_bytes, s);
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

hipError_t launch_copy_status(const CtxCore* c, int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(copy_status_kernel, dim3(1), dim3(64), 0, s, c, out);
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

hipError_t launch_check_cols(const uint32_t* col, uint64_t arcs, uint32_t n, uint32_t* bad, hipStream_t s) {
    hipError_t e = launch_fill_u32(bad, 1, 0u, s);
    if (e != hipSuccess) return e;
    uint64_t blocks = (arcs + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(check_cols_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, col, arcs, n, bad);
    return hipGetLastError();
}

hipError_t launch_cotask(const CotaskArgs& a, uint32_t block, uint32_t lds_bytes, hipStream_t s) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(cotask_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    hipLaunchKernelGGL(cotask_kernel, dim3(a.nwg), dim3(block), lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace coop
