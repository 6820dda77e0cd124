// Cooperative graph-traversal kernels for gfx950.
//
// Every algorithm is one persistent kernel whose workgroups run the
// level-synchronous loop of the paper's cooperative graph-traversal figure:
// take work from the input frontier, process it, meet at one resizing
// global barrier per level, repeat until the frontier is empty. Between
// barriers the active workgroup count M is fixed; at each barrier the
// scheduler may fork waiting workgroups in or claim the top ids back.
//
// Frontier expansion is built for CDNA waves (64 lanes):
//  * work is claimed by a workgroup 1024 frontier entries at a time from a
//    64-bit {size | next} word, then handed to waves 64 entries at a time
//    through an LDS counter;
//  * a wave loads its 64 vertices' CSR ranges, scans the degrees across the
//    wave, and walks the concatenated neighbour lists 64 x UNROLL arcs per
//    step (coalesced col/w loads; each lane finds its owner vertex by a
//    binary search over the wave's degree prefix in LDS);
//  * vertices whose degree exceeds a threshold are not walked by one wave:
//    they are cut into fixed-size arc strips pushed to a strip queue and
//    processed by all waves in a second phase of the same level;
//  * new frontier entries are compacted with a wave ballot + mbcnt into a
//    per-wave LDS buffer and flushed with one atomic per flush.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "coop_device.hpp"
#include "coop_internal.h"

using namespace coop;

namespace {

constexpr uint32_t kWave = 64;
constexpr uint32_t kUnroll = 8;                   // arcs per lane per step
constexpr uint32_t kOutCap = 1024;                // per-wave output buffer (entries)
constexpr uint32_t kFlushAt = kOutCap - kWave * kUnroll;
constexpr uint32_t kInf = 0xFFFFFFFFu;

// BFS / SSSP / colouring phases carried in the release flags
constexpr uint32_t kPhShift = 4;
constexpr uint32_t kPhMask = 7u << kPhShift;
constexpr uint32_t kPhStart = 0u << kPhShift;     // registration barrier
constexpr uint32_t kPhInit = 1u << kPhShift;      // clear per-root state
constexpr uint32_t kPhLight = 2u << kPhShift;     // walk the input frontier
constexpr uint32_t kPhHeavy = 3u << kPhShift;     // walk the heavy strips
constexpr uint32_t kPhSetup = 4u << kPhShift;     // colouring: count higher neighbours
constexpr uint32_t kFlagSel = 1u << 8;            // which frontier buffer is input
constexpr uint32_t kFlagAdv = 1u << 9;            // this barrier advanced the level

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t wave_id() { return threadIdx.x / kWave; }
__device__ __forceinline__ uint32_t num_waves() { return blockDim.x / kWave; }

__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const uint32_t l = lane_id();
#pragma unroll
    for (uint32_t d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if (l >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t bcast(uint32_t x, uint32_t src) { return __shfl(x, src, kWave); }

// ----------------------------------------------------------- LDS layout

struct WaveLds {
    uint32_t excl[kWave + 1];   // degree prefix of the wave's vertices
    uint32_t start[kWave];      // first arc of each vertex
    uint32_t pay[kWave];        // algorithm payload (vertex id or distance)
    uint32_t out_n;             // entries in the output buffer
    uint32_t out[kOutCap];
};

struct BlockLds {
    Member member;
    uint32_t killed;
    uint32_t chunk_lo, chunk_hi, sub;
    uint32_t level, root, aux;
    WaveLds wave[kMaxWaves];
};

// ------------------------------------------------------ output frontier

// Append this wave's ballot winners (lanes with `win`) to its LDS buffer.
__device__ __forceinline__ void wave_push(WaveLds& w, bool win, uint32_t v) {
    const uint64_t mask = __ballot(win);
    if (!mask) return;
    const uint32_t base = w.out_n;
    if (win) w.out[base + mbcnt(mask)] = v;
    __builtin_amdgcn_wave_barrier();
    if (lane_id() == 0) w.out_n = base + (uint32_t)__popcll(mask);
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void wave_flush(WaveLds& w, uint32_t* out_tail, uint32_t* out) {
    const uint32_t cnt = w.out_n;
    if (cnt == 0) return;
    uint32_t base = 0;
    if (lane_id() == 0) base = add_relaxed(out_tail, cnt);
    base = bcast(base, 0);
    for (uint32_t i = lane_id(); i < cnt; i += kWave) out[base + i] = w.out[i];
    __builtin_amdgcn_wave_barrier();
    if (lane_id() == 0) w.out_n = 0;
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------- expansion

// Owner of flattened arc index e inside the wave: largest i with excl[i] <= e.
__device__ __forceinline__ uint32_t owner_of(const WaveLds& w, uint32_t e) {
    uint32_t lo = 0, hi = kWave;        // excl[lo] <= e < excl[hi]
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const uint32_t mid = (lo + hi) >> 1;
        if (w.excl[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// Walk the concatenated neighbour lists described by excl/start/pay (total
// arcs `total`), UNROLL arcs per lane per step. `visit(lane_valid, arc, u,
// payload)` returns (win, value) through references; winners are pushed.
template <class Visit>
__device__ __forceinline__ void walk_arcs(WaveLds& w, uint32_t total, const uint32_t* __restrict__ col,
                                          uint32_t* out_tail, uint32_t* out, Visit& visit) {
    for (uint32_t base = 0; base < total; base += kWave * kUnroll) {
        uint32_t arc[kUnroll], u[kUnroll], pay[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) {
            const uint32_t e = base + j * kWave + lane_id();
            ok[j] = e < total;
            const uint32_t o = owner_of(w, ok[j] ? e : 0u);
            arc[j] = w.start[o] + (e - w.excl[o]);
            pay[j] = w.pay[o];
        }
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) u[j] = ok[j] ? __builtin_nontemporal_load(&col[arc[j]]) : 0u;
        visit.step(ok, arc, u, pay, w);
        if (w.out_n > kFlushAt) wave_flush(w, out_tail, out);
    }
}

// Per-wave processing of one heavy strip {vertex payload, first arc, length}.
template <class Visit>
__device__ __forceinline__ void walk_strip(WaveLds& w, uint32_t pay0, uint32_t a0, uint32_t len,
                                           const uint32_t* __restrict__ col, uint32_t* out_tail,
                                           uint32_t* out, Visit& visit) {
    for (uint32_t base = 0; base < len; base += kWave * kUnroll) {
        uint32_t arc[kUnroll], u[kUnroll], pay[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) {
            const uint32_t e = base + j * kWave + lane_id();
            ok[j] = e < len;
            arc[j] = a0 + (ok[j] ? e : 0u);
            pay[j] = pay0;
        }
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) u[j] = ok[j] ? __builtin_nontemporal_load(&col[arc[j]]) : 0u;
        visit.step(ok, arc, u, pay, w);
        if (w.out_n > kFlushAt) wave_flush(w, out_tail, out);
    }
}

// One LIGHT phase: claim frontier chunks, expand light vertices, queue the
// heavy ones as strips.
template <class Visit>
__device__ void light_phase(const TraversalArgs& a, Work* wk, BlockLds& sh, const uint32_t* in,
                            uint32_t* out, Visit& visit) {
    // `visit.payload(v)` gives a vertex's payload (e.g. its distance).
    WaveLds& w = sh.wave[wave_id()];
    const uint32_t nw = num_waves();
    const uint32_t chunk = nw * kWave;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint64_t c = add_relaxed64(&wk->claim, chunk);
            const uint32_t next = (uint32_t)c, size = (uint32_t)(c >> 32);
            sh.chunk_lo = next;
            sh.chunk_hi = next < size ? (next + chunk < size ? next + chunk : size) : next;
            sh.sub = 0;
        }
        __syncthreads();
        const uint32_t lo = sh.chunk_lo, hi = sh.chunk_hi;
        if (lo >= hi) break;
        for (;;) {
            uint32_t s = 0;
            if (lane_id() == 0) s = atomicAdd(&sh.sub, 1u);
            s = bcast(s, 0);
            const uint32_t i0 = lo + s * kWave;
            if (i0 >= hi) break;
            const uint32_t i = i0 + lane_id();
            uint32_t v = 0, st = 0, deg = 0, pay = 0;
            if (i < hi) {
                v = in[i];
                st = a.row_ptr[v];
                deg = a.row_ptr[v + 1] - st;
                pay = visit.payload(v);
            }
            // heavy vertices become strips for the HEAVY phase
            const bool heavy = deg > a.heavy_th;
            const uint64_t hmask = __ballot(heavy);
            if (hmask) {
                const uint32_t ns = heavy ? (deg + a.strip - 1) / a.strip : 0u;
                const uint32_t incl = wave_incl_scan(ns);
                const uint32_t tot = bcast(incl, kWave - 1);
                uint32_t b = 0;
                if (lane_id() == kWave - 1) b = add_relaxed(&wk->heavy_tail, tot);
                b = bcast(b, kWave - 1);
                if (heavy) {
                    uint32_t k = b + incl - ns;
                    for (uint32_t j = 0; j < ns; ++j, ++k) {
                        const uint32_t off = j * a.strip;
                        const uint32_t len = deg - off < a.strip ? deg - off : a.strip;
                        if (k < a.heavy_cap) a.heavy[k] = make_uint4(pay, st + off, len, v);
                    }
                }
                if (heavy) deg = 0;
            }
            const uint32_t incl = wave_incl_scan(deg);
            w.excl[lane_id()] = incl - deg;
            w.start[lane_id()] = st;
            w.pay[lane_id()] = pay;
            if (lane_id() == kWave - 1) w.excl[kWave] = incl;
            __builtin_amdgcn_wave_barrier();
            const uint32_t total = bcast(incl, kWave - 1);
            walk_arcs(w, total, a.col, &wk->out_tail, out, visit);
            __builtin_amdgcn_wave_barrier();
        }
    }
}

template <class Visit>
__device__ void heavy_phase(const TraversalArgs& a, Work* wk, BlockLds& sh, uint32_t* out, Visit& visit) {
    WaveLds& w = sh.wave[wave_id()];
    for (;;) {
        uint64_t c = 0;
        if (lane_id() == 0) c = add_relaxed64(&wk->hclaim, 1);
        const uint32_t s = bcast((uint32_t)c, 0);
        const uint32_t n = bcast((uint32_t)(c >> 32), 0);
        if (s >= n) break;
        const uint4 rec = a.heavy[s];
        const uint32_t pay = visit.strip_payload(rec.x, rec.w);
        walk_strip(w, pay, rec.y, rec.z, a.col, &wk->out_tail, out, visit);
    }
}

__device__ __forceinline__ void flush_all(BlockLds& sh, Work* wk, uint32_t* out) {
    wave_flush(sh.wave[wave_id()], &wk->out_tail, out);
}

// ------------------------------------------------------------------ BFS

struct BfsAlgo {
    using Args = BfsArgs;
    struct Visit {
        uint32_t* bitmap;
        uint32_t* level;        // output slice of the current root
        uint32_t next_level;

        __device__ __forceinline__ uint32_t payload(uint32_t) const { return 0; }
        __device__ __forceinline__ uint32_t strip_payload(uint32_t p, uint32_t) const { return p; }

        // Claim unvisited targets: a plain load filters most arcs, the
        // atomic OR decides the single winner, which writes the level.
        __device__ __forceinline__ void step(const bool* ok, const uint32_t*, const uint32_t* u,
                                             const uint32_t*, WaveLds& w) {
            uint32_t word[kUnroll];
#pragma unroll
            for (uint32_t j = 0; j < kUnroll; ++j) word[j] = ok[j] ? bitmap[u[j] >> 5] : ~0u;
            bool win[kUnroll];
#pragma unroll
            for (uint32_t j = 0; j < kUnroll; ++j) {
                const uint32_t bit = 1u << (u[j] & 31);
                win[j] = false;
                if (ok[j] && !(word[j] & bit)) {
                    const uint32_t old = __hip_atomic_fetch_or(&bitmap[u[j] >> 5], bit, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                    win[j] = !(old & bit);
                }
            }
#pragma unroll
            for (uint32_t j = 0; j < kUnroll; ++j) {
                if (win[j]) level[u[j]] = next_level;
                wave_push(w, win[j], u[j]);
            }
        }
    };

    __device__ static uint32_t* out_slice(const Args& p, uint32_t root) {
        return p.level_out + (size_t)root * p.t.out_stride;
    }
    __device__ static Visit visit(const Args& p, uint32_t level, uint32_t, uint32_t root) {
        return Visit{p.bitmap, out_slice(p, root), level + 1};
    }
    // INIT phase: clear the visited set and the root's level slice.
    __device__ static void init_range(const Args& p, uint32_t root, uint32_t tid, uint32_t stride) {
        uint32_t* lvl = out_slice(p, root);
        const uint32_t n = p.t.n, words = (n + 31) / 32;
        for (uint32_t i = tid; i < n; i += stride) lvl[i] = kInf;
        for (uint32_t i = tid; i < words; i += stride) p.bitmap[i] = 0;
    }
    // Master step: the root is at level 0 and visited.
    __device__ static void place_root(const Args& p, uint32_t root, uint32_t r, uint32_t) {
        out_slice(p, root)[r] = 0;
        p.bitmap[r >> 5] |= 1u << (r & 31);
    }
};

// ----------------------------------------------------------------- SSSP

struct SsspAlgo {
    using Args = SsspArgs;
    struct Visit {
        int32_t* dist;
        uint32_t* stamp;
        const uint32_t* w;
        uint32_t tag;           // stamp value meaning "queued for the next round"
        Ctx* ctx;

        __device__ __forceinline__ uint32_t payload(uint32_t v) const {
            return (uint32_t)__hip_atomic_load(&dist[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __device__ __forceinline__ uint32_t strip_payload(uint32_t, uint32_t v) const { return payload(v); }

        // Frontier Bellman-Ford relaxation: atomicMin the candidate; a vertex
        // whose distance dropped is queued once per round (stamp exchange).
        __device__ __forceinline__ void step(const bool* ok, const uint32_t* arc, const uint32_t* u,
                                             const uint32_t* pay, WaveLds& wl) {
            uint32_t wt[kUnroll];
            int32_t du[kUnroll];
#pragma unroll
            for (uint32_t j = 0; j < kUnroll; ++j) wt[j] = ok[j] ? __builtin_nontemporal_load(&w[arc[j]]) : 0u;
#pragma unroll
            for (uint32_t j = 0; j < kUnroll; ++j) du[j] = ok[j] ? dist[u[j]] : 0;
            bool win[kUnroll];
#pragma unroll
            for (uint32_t j = 0; j < kUnroll; ++j) {
                win[j] = false;
                if (!ok[j]) continue;
                const int64_t nd64 = (int64_t)(int32_t)pay[j] + (int64_t)wt[j];
                if (nd64 >= 0x7FFFFFFF) {
                    raise_error(ctx, kErrOverflow);
                    continue;
                }
                const int32_t nd = (int32_t)nd64;
                if (nd < du[j]) {
                    const int32_t old = __hip_atomic_fetch_min(&dist[u[j]], nd, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                    if (nd < old) {
                        const uint32_t prev = __hip_atomic_exchange(&stamp[u[j]], tag, __ATOMIC_RELAXED,
                                                                    __HIP_MEMORY_SCOPE_AGENT);
                        win[j] = prev != tag;
                    }
                }
            }
#pragma unroll
            for (uint32_t j = 0; j < kUnroll; ++j) wave_push(wl, win[j], u[j]);
        }
    };

    __device__ static int32_t* out_slice(const Args& p, uint32_t root) {
        return p.dist_out + (size_t)root * p.t.out_stride;
    }
    __device__ static Visit visit(const Args& p, uint32_t, uint32_t round, uint32_t root) {
        return Visit{out_slice(p, root), p.stamp, p.t.w, round + 2, p.t.ctx};
    }
    __device__ static void init_range(const Args& p, uint32_t root, uint32_t tid, uint32_t stride) {
        int32_t* d = out_slice(p, root);
        for (uint32_t i = tid; i < p.t.n; i += stride) d[i] = 0x7FFFFFFF;
    }
    __device__ static void place_root(const Args& p, uint32_t root, uint32_t r, uint32_t round) {
        out_slice(p, root)[r] = 0;
        p.stamp[r] = round + 1;
    }
};

// -------------------------------------------------- generic traversal body

// The level loop of the cooperative graph-traversal figure, one resizing
// barrier per level. Phases per source: INIT (clear), then per level LIGHT
// (+ HEAVY when heavy strips were queued). The master step swaps the
// frontiers, resets the output counter and increments the level; the
// transmitted state (level, source index, round) lives in Work::xfer_*.
template <bool Coop, class Algo>
__device__ void traverse(const typename Algo::Args& p, bool joiner_grid) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    const TraversalArgs& t = p.t;
    Ctx* c = t.ctx;
    Work* wk = t.work;

    if (threadIdx.x == 0) {
        Member m = register_member(c, !Coop, joiner_grid);
        if (Coop && m.alive && m.epoch == 0) startup_wait(c);
        if (m.alive && m.epoch != 0) {
            // admitted joiner: take over the transmitted state of workgroup 0
            sh.level = wk->xfer_level;
            sh.root = wk->xfer_root;
            sh.aux = wk->xfer_round;
        } else {
            sh.level = 0;
            sh.root = 0;
            sh.aux = 0;
        }
        for (uint32_t i = 0; i < kMaxWaves; ++i) sh.wave[i].out_n = 0;
        sh.member = m;
        sh.killed = 0;
    }
    __syncthreads();
    Member m = sh.member;
    uint32_t level = sh.level, root = sh.root, round = sh.aux;
    bool fresh = m.epoch == 0;    // initial members begin at the registration barrier

    for (;;) {
        if (!m.alive) {
            if (Coop && sh.killed && (c->mode & kModePark)) {
                // park mode: a claimed workgroup queues again as a joiner
                __syncthreads();
                if (threadIdx.x == 0) {
                    Member j = join_queue(c);
                    sh.member = j;
                    sh.killed = 0;
                    sh.level = wk->xfer_level;
                    sh.root = wk->xfer_root;
                    sh.aux = wk->xfer_round;
                }
                __syncthreads();
                m = sh.member;
                level = sh.level;
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

        if (ph == kPhInit) {
            Algo::init_range(p, root, m.id * blockDim.x + threadIdx.x, m.M * blockDim.x);
        } else if (ph == kPhLight) {
            auto vis = Algo::visit(p, level, round, root);
            light_phase(t, wk, sh, in, out, vis);
            flush_all(sh, wk, out);
        } else if (ph == kPhHeavy) {
            auto vis = Algo::visit(p, level, round, root);
            heavy_phase(t, wk, sh, out, vis);
            flush_all(sh, wk, out);
        }

        const uint32_t cur_flags = m.flags;
        barrier<Coop>(c, m, &sh.member, &sh.killed, [&](uint32_t, uint32_t) -> uint32_t {
            uint32_t flags = cur_flags & kFlagSel;
            if (ph == kPhStart) {
                wk->xfer_root = 0;
                wk->xfer_level = 0;
                return kPhInit;
            }
            if (ph == kPhInit) {
                const uint32_t r = t.roots[wk->xfer_root];
                Algo::place_root(p, wk->xfer_root, r, wk->xfer_round);
                t.frontier[0][0] = r;
                wk->xfer_level = 0;
                __hip_atomic_store(&wk->claim, (uint64_t)1 << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&wk->out_tail, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&wk->heavy_tail, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return kPhLight;   // input = buffer 0
            }
            const uint32_t hs = ld_relaxed(&wk->heavy_tail);
            if (ph == kPhLight && hs > 0) {
                if (hs > t.heavy_cap) {
                    raise_error(c, kErrInternal);
                    return kFlagAbort;
                }
                __hip_atomic_store(&wk->hclaim, (uint64_t)hs << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return flags | kPhHeavy;
            }
            // level done: swap frontiers, reset the output counter, level++
            const uint32_t size = ld_relaxed(&wk->out_tail);
            __hip_atomic_store(&wk->out_tail, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&wk->heavy_tail, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&wk->claim, (uint64_t)size << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            wk->xfer_level += 1;
            wk->xfer_round += 1;
            wk->levels_total += 1;
            if (size == 0) {
                wk->xfer_root += 1;
                if (wk->xfer_root >= t.nroots) return kFlagDone;
                return kPhInit | kFlagAdv;
            }
            return (flags ^ kFlagSel) | kPhLight | kFlagAdv;
        });
        // follow the transmitted state locally
        const uint32_t nph = m.flags & kPhMask;
        if (m.flags & kFlagAdv) round += 1;
        if (nph == kPhInit) {
            if (ph != kPhStart) root += 1;
            level = 0;
        } else if (nph == kPhLight) {
            if (ph == kPhInit) level = 0;
            else if (m.flags & kFlagAdv) level += 1;
        }
    }
}

// ----------------------------------------------- colouring and MIS (JP DAG)

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

// Priority key (h(v), v), higher first; h(v) = output v of SplitMix64 from
// state prio_seed.
__device__ __forceinline__ bool key_higher(uint64_t hu, uint32_t u, uint64_t hv, uint32_t v) {
    return hu > hv || (hu == hv && u > v);
}
__device__ __forceinline__ uint64_t key_hash(uint64_t seed, uint32_t v) {
    return splitmix64(seed + (uint64_t)v * kGamma);
}

// Process one decided vertex v (all higher-key neighbours are final):
// colour = mex of their colours (or MIS membership), then release the
// lower-key neighbours; a neighbour whose count reaches 0 is queued.
__device__ __forceinline__ bool color_vertex(const ColorArgs& p, uint32_t v, WaveLds& w, bool valid,
                                             uint32_t* out_tail, uint32_t* out) {
    uint32_t pushed_any = 0;
    if (valid) {
        const uint64_t hv = key_hash(p.prio_seed, v);
        const uint32_t a0 = p.t.row_ptr[v], a1 = p.t.row_ptr[v + 1];
        if (p.mis) {
            bool blocked = false;
            for (uint32_t e = a0; e < a1 && !blocked; ++e) {
                const uint32_t u = p.t.col[e];
                if (key_higher(key_hash(p.prio_seed, u), u, hv, v)) blocked = p.in_set_out[u] != 0;
            }
            p.in_set_out[v] = blocked ? 0 : 1;
        } else {
            uint32_t base = 0, c = 0;
            for (;;) {
                uint64_t used = 0;
                for (uint32_t e = a0; e < a1; ++e) {
                    const uint32_t u = p.t.col[e];
                    if (key_higher(key_hash(p.prio_seed, u), u, hv, v)) {
                        const uint32_t cu = p.colour_out[u] - base;
                        if (cu < 64) used |= 1ull << cu;
                    }
                }
                if (~used) { c = base + (uint32_t)__ffsll((long long)~used) - 1; break; }
                base += 64;
            }
            p.colour_out[v] = c;
        }
    }
    (void)pushed_any;
    return valid;
}

__device__ __forceinline__ void release_lower(const ColorArgs& p, uint32_t v, bool valid, WaveLds& w,
                                              uint32_t* out_tail, uint32_t* out) {
    const uint64_t hv = valid ? key_hash(p.prio_seed, v) : 0;
    uint32_t e = valid ? p.t.row_ptr[v] : 0;
    const uint32_t a1 = valid ? p.t.row_ptr[v + 1] : 0;
    // lanes walk their own lists; the wave keeps pushing until all are done
    for (;;) {
        const bool more = e < a1;
        if (!__ballot(more)) break;
        bool win = false;
        uint32_t u = 0;
        if (more) {
            u = p.t.col[e];
            if (!key_higher(key_hash(p.prio_seed, u), u, hv, v)) {
                const uint32_t old = __hip_atomic_fetch_sub(&p.pending[u], 1u, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                win = old == 1;
            }
            ++e;
        }
        wave_push(w, win, u);
        if (w.out_n > kFlushAt) wave_flush(w, out_tail, out);
    }
}

// Colouring / MIS body: SETUP counts every vertex's higher-key neighbours
// and queues the sources of the priority DAG; each round then decides its
// frontier and releases the next one.
template <bool Coop>
__device__ void color_body(const ColorArgs& p, bool joiner_grid) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    const TraversalArgs& t = p.t;
    Ctx* c = t.ctx;
    Work* wk = t.work;

    if (threadIdx.x == 0) {
        Member m = register_member(c, !Coop, joiner_grid);
        if (Coop && m.alive && m.epoch == 0) startup_wait(c);
        for (uint32_t i = 0; i < kMaxWaves; ++i) sh.wave[i].out_n = 0;
        sh.member = m;
        sh.killed = 0;
    }
    __syncthreads();
    Member m = sh.member;
    bool fresh = m.epoch == 0;
    WaveLds& w = sh.wave[wave_id()];

    for (;;) {
        if (!m.alive) {
            if (Coop && sh.killed && (c->mode & kModePark)) {
                __syncthreads();
                if (threadIdx.x == 0) {
                    sh.member = join_queue(c);
                    sh.killed = 0;
                }
                __syncthreads();
                m = sh.member;
                if (m.alive) continue;
            }
            return;
        }
        const uint32_t ph = fresh ? kPhStart : (m.flags & kPhMask);
        fresh = false;
        const bool sel = (m.flags & kFlagSel) != 0;
        uint32_t* in = t.frontier[sel ? 1 : 0];
        uint32_t* out = t.frontier[sel ? 0 : 1];

        if (ph == kPhSetup) {
            // count higher-key neighbours; vertices with none are ready
            const uint32_t tid = m.id * blockDim.x + threadIdx.x, stride = m.M * blockDim.x;
            const uint32_t n = t.n;
            for (uint32_t base = m.id * blockDim.x; base < n; base += stride) {
                const uint32_t v = base + threadIdx.x;
                const bool valid = v < n;
                uint32_t cnt = 0;
                if (valid) {
                    const uint64_t hv = key_hash(p.prio_seed, v);
                    for (uint32_t e = t.row_ptr[v]; e < t.row_ptr[v + 1]; ++e) {
                        const uint32_t u = t.col[e];
                        cnt += key_higher(key_hash(p.prio_seed, u), u, hv, v) ? 1u : 0u;
                    }
                    p.pending[v] = cnt;
                }
                wave_push(w, valid && cnt == 0, v);
                if (w.out_n > kFlushAt) wave_flush(w, &wk->out_tail, out);
            }
            (void)tid;
            flush_all(sh, wk, out);
        } else if (ph == kPhLight) {
            // decide the frontier: claims of blockDim.x vertices, one per lane
            for (;;) {
                __syncthreads();
                if (threadIdx.x == 0) {
                    const uint64_t cl = add_relaxed64(&wk->claim, blockDim.x);
                    sh.chunk_lo = (uint32_t)cl;
                    sh.chunk_hi = (uint32_t)(cl >> 32);
                }
                __syncthreads();
                const uint32_t lo = sh.chunk_lo, size = sh.chunk_hi;
                if (lo >= size) break;
                const uint32_t i = lo + threadIdx.x;
                const bool valid = i < size;
                const uint32_t v = valid ? in[i] : 0u;
                color_vertex(p, v, w, valid, &wk->out_tail, out);
                release_lower(p, v, valid, w, &wk->out_tail, out);
            }
            flush_all(sh, wk, out);
        }

        barrier<Coop>(c, m, &sh.member, &sh.killed, [&](uint32_t, uint32_t) -> uint32_t {
            if (ph == kPhStart) {
                __hip_atomic_store(&wk->out_tail, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return kPhSetup;          // SETUP writes buffer 1 (sel = 0)
            }
            const uint32_t flags = m.flags & kFlagSel;
            const uint32_t size = ld_relaxed(&wk->out_tail);
            __hip_atomic_store(&wk->out_tail, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&wk->claim, (uint64_t)size << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            wk->xfer_level += 1;
            wk->levels_total += 1;
            if (size == 0) return kFlagDone;
            return (flags ^ kFlagSel) | kPhLight | kFlagAdv;
        });
    }
}

// ----------------------------------------------------- barrier benchmark

template <bool Coop>
__device__ void barrier_bench_body(const BarrierBenchArgs& p, bool joiner_grid) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    Ctx* c = p.ctx;
    if (threadIdx.x == 0) {
        Member m = register_member(c, !Coop, joiner_grid);
        if (Coop && m.alive && m.epoch == 0) startup_wait(c);
        sh.member = m;
        sh.killed = 0;
    }
    __syncthreads();
    Member m = sh.member;
    for (;;) {
        if (!m.alive) return;
        barrier<Coop>(c, m, &sh.member, &sh.killed, [&](uint32_t, uint32_t ne) -> uint32_t {
            if (ne == 1) c->t_start = now_ticks();
            return ne > p.iters ? kFlagDone : 0u;
        });
    }
}

}  // namespace

// ------------------------------------------------------------ entry points

#define COOP_KERNEL_BOUNDS __launch_bounds__(1024)

template <bool Coop>
__global__ void COOP_KERNEL_BOUNDS bfs_kernel(BfsArgs a, int joiner) { traverse<Coop, BfsAlgo>(a, joiner != 0); }
template <bool Coop>
__global__ void COOP_KERNEL_BOUNDS sssp_kernel(SsspArgs a, int joiner) { traverse<Coop, SsspAlgo>(a, joiner != 0); }
template <bool Coop>
__global__ void COOP_KERNEL_BOUNDS color_kernel(ColorArgs a, int joiner) { color_body<Coop>(a, joiner != 0); }
template <bool Coop>
__global__ void COOP_KERNEL_BOUNDS barrier_bench_kernel(BarrierBenchArgs a, int joiner) {
    barrier_bench_body<Coop>(a, joiner != 0);
}

__global__ void init_ctx_kernel(Ctx* c, Work* w, uint32_t N, uint32_t mode, uint32_t wg_size,
                                uint64_t sched_seed, uint32_t sched_p16, uint64_t watchdog_ticks,
                                uint32_t epoch0_wait, HostCtl* host) {
    const uint32_t tid = threadIdx.x;
    uint32_t* cw = reinterpret_cast<uint32_t*>(c);
    const uint32_t head_words = offsetof(Ctx, join_entry) / 4;
    for (uint32_t i = tid; i < head_words; i += blockDim.x) cw[i] = 0;
    for (uint32_t i = tid; i < kJoinCap; i += blockDim.x) c->join_entry[i] = ~0ull;
    uint32_t* ww = reinterpret_cast<uint32_t*>(w);
    for (uint32_t i = tid; i < sizeof(Work) / 4; i += blockDim.x) ww[i] = 0;
    __syncthreads();
    if (tid == 0) {
        c->N = N;
        c->mode = mode;
        c->wg_size = wg_size;
        c->sched_seed = sched_seed;
        c->sched_p16 = sched_p16;
        c->watchdog_ticks = watchdog_ticks;
        c->epoch0_wait = epoch0_wait;
        c->host = host;
        c->T_dev = N;
        c->min_M = 0xFFFFFFFFu;
        c->max_M = 0;
        c->t_start = 0;
        c->release = make_release(0, 1, 0);
    }
}

__global__ void fill_u32_kernel(uint32_t* p, uint64_t count, uint32_t value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
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

template <class K, class A>
static hipError_t launch_persistent(K kern_coop, K kern_plain, const A& a, bool coop, bool joiner_grid,
                                    uint32_t grid, uint32_t block, uint32_t lds_bytes, hipStream_t s) {
    K k = coop ? kern_coop : kern_plain;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    (void)e;
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

hipError_t launch_init_ctx(Ctx* c, Work* w, uint32_t N, uint32_t mode, uint32_t wg_size,
                           uint64_t sched_seed, uint32_t sched_p16, uint64_t watchdog_ticks,
                           uint32_t epoch0_wait, HostCtl* host, hipStream_t s) {
    hipLaunchKernelGGL(init_ctx_kernel, dim3(1), dim3(256), 0, s, c, w, N, mode, wg_size, sched_seed,
                       sched_p16, watchdog_ticks, epoch0_wait, host);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s) {
    if (count == 0) return hipSuccess;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t launch_cotask(const CotaskArgs& a, uint32_t block, uint32_t lds_bytes, hipStream_t s) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(cotask_kernel),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    hipLaunchKernelGGL(cotask_kernel, dim3(a.nwg), dim3(block), lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace coop
