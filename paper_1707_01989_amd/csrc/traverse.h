// Device building blocks of the level-synchronous traversals, shared by the
// resizable persistent kernels (one traversal over all workgroups) and the
// batched kernel (one team of workgroups per graph instance).
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
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
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

// phases and flags carried in the release word
constexpr uint32_t kPhShift = 4;
constexpr uint32_t kPhMask = 7u << kPhShift;
constexpr uint32_t kPhStart = 0u << kPhShift;     // registration barrier
constexpr uint32_t kPhInit = 1u << kPhShift;      // clear per-source state
constexpr uint32_t kPhTD = 2u << kPhShift;        // top-down: walk the frontier
constexpr uint32_t kPhHeavy = 3u << kPhShift;     // walk the heavy strips
constexpr uint32_t kPhBU = 4u << kPhShift;        // bottom-up: unvisited vertices look for a parent
constexpr uint32_t kPhSetup = 5u << kPhShift;     // colouring: count higher-priority neighbours
constexpr uint32_t kPhOut = 6u << kPhShift;       // SSSP: copy a source's distances out
constexpr uint32_t kFlagSel = 1u << 8;            // queue engine: which buffer is input
constexpr uint32_t kFlagAdv = 1u << 9;            // this barrier advanced the level
constexpr uint32_t kRotShift = 10;                // BFS: frontier bitmap rotation (0..2)
constexpr uint32_t kRotMask = 3u << kRotShift;
constexpr uint32_t kFlagEnd = 1u << 12;           // a served query finished (the team goes on)
constexpr uint32_t kFlagPreSplit = 1u << 13;      // BFS top-down: the frontier's heavy vertices are strips already
constexpr uint32_t kFlagJump = 1u << 14;          // BFS: the master step ran levels itself; the level is x.level
constexpr uint32_t kFlagRecord = 1u << 15;        // BFS: the phase lists what it finds (a small level may follow)
constexpr uint64_t kRecordArcs = 1u << 16;        // ... when the frontier has at most this many arcs
constexpr uint32_t kFlWg = coop::kFlWgHost;       // BFS: found vertices a workgroup lists per level

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
        const uint32_t y = __shfl_up(x, d, kWave);
        if (l >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t bcast(uint32_t x, uint32_t src) { return __shfl(x, src, kWave); }

__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
#pragma unroll
    for (uint32_t d = kWave / 2; d >= 1; d >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)x, d, kWave);
        const uint32_t hi = __shfl_xor((uint32_t)(x >> 32), d, kWave);
        x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

// Wave slot of this wave in the interval: units are dealt one per
// workgroup before any workgroup gets a second, from the highest logical id
// down. A small frontier (a few heavy strips, a thin SSSP wavefront) is then
// spread over as many compute units (and XCDs) as it has units instead of
// queueing on one compute unit's memory pipeline, and it avoids workgroup 0,
// which also relays the scheduler target every barrier.
__device__ __forceinline__ uint32_t wave_slot(uint32_t id, uint32_t M, uint32_t nw) {
    (void)nw;
    return wave_id() * M + (M - 1 - id);
}

// ----------------------------------------------------------- LDS layout

struct WaveLds {
    uint32_t excl[kWave + 1];   // degree prefix of the wave's vertices
    uint32_t start[kWave];      // first arc of each vertex
    uint32_t pay[kWave];        // algorithm payload (distance, degree ...)
    uint32_t out_n;             // entries in the output buffer
    uint32_t out[kOutCap];
    uint32_t lng[2 * kWave];    // bottom-up: candidates with long lists, scanned by the whole wave
    uint32_t lngk[2 * kWave];   // ... and the arc where the lane's probes stopped
};

struct BlockLds {
    BarrierLds bar;
    uint32_t level, root, aux, in_size;
    uint32_t wave_base[kMaxWaves];
    uint64_t acc[8];            // per-workgroup statistics of the phase
    uint64_t red[8][kMaxWaves]; // master reductions
    uint32_t mb[4];             // master step: values thread 0 shares with the workgroup
    uint32_t fl_n;              // BFS: vertices this workgroup found in the phase
    uint32_t fl[kFlWg];         // ... the first kFlWg of them
    uint32_t il_c[2], il_go;    // BFS master step: small-level list lengths, whether to run them
    uint32_t il_v[6];           // ... values thread 0 shares with the workgroup
    XferR il_x;                 // BFS master step: thread 0's copy of the transmit block
    WaveLds wave[kMaxWaves];
};

// Per-wave statistics, flushed to the workgroup accumulators at phase end.
struct Stats {
    uint64_t found = 0, mf = 0, arcs = 0, rows = 0, words = 0;
};

__device__ void stats_to_lds(BlockLds& sh, const Stats& s) {
    const uint64_t v[5] = {wave_sum64(s.found), wave_sum64(s.mf), wave_sum64(s.arcs),
                           wave_sum64(s.rows), wave_sum64(s.words)};
    if (lane_id() == 0)
        for (int i = 0; i < 5; ++i)
            if (v[i]) atomicAdd(reinterpret_cast<unsigned long long*>(&sh.acc[i]),
                                (unsigned long long)v[i]);
}

// Add the workgroup's phase statistics to its slot (after a __syncthreads);
// fire-and-forget atomics, so nobody waits for the round trip. Every field
// only grows: fields 0 and 1 (found, mf) are kept only when the master step
// reads them (BFS whose level counts do not come with the barrier
// arrivals), which takes a level's values as the difference from the sums
// it saw at the previous level.
__device__ void acc_to_slot(BlockLds& sh, uint32_t* slots, uint32_t id, bool per_level = true) {
    if (threadIdx.x < 5) {
        uint64_t* s = reinterpret_cast<uint64_t*>(slots + (size_t)id * kSlotWords);
        const uint64_t v = sh.acc[threadIdx.x];
        if (v) {
            if (per_level || threadIdx.x >= 2) add_nr64(&s[threadIdx.x], v);
            if (threadIdx.x == 0) add_nr64(&s[kSlotFoundAll], v);
        }
        sh.acc[threadIdx.x] = 0;
    }
}

// Master step helper: sum fields 0 and 1 (found, mf) of every slot (all N
// logical ids). They are never cleared (a clear would leave dirty lines for
// the release to write back); the caller subtracts the previous sums.
// Called by all threads of the master workgroup; tot[0..1] valid in all.
__device__ void master_sum_slots(BlockLds& sh, const uint32_t* slots, uint32_t N, uint64_t* tot) {
    uint64_t part[2] = {0, 0};
    for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) {
        const uint64_t* s = reinterpret_cast<const uint64_t*>(slots + (size_t)i * kSlotWords);
        part[0] += s[0];
        part[1] += s[1];
    }
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const uint64_t w = wave_sum64(part[f]);
        if (lane_id() == 0) sh.red[f][wave_id()] = w;
    }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        uint64_t t = 0;
        for (uint32_t w = 0; w < num_waves(); ++w) t += sh.red[f][w];
        tot[f] = t;
    }
    __syncthreads();
}

// ------------------------------------------------------ output queue

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

// End of a phase: one reservation for the whole workgroup.
__device__ void wg_flush(BlockLds& sh, uint32_t* out_tail, uint32_t* out) {
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (uint32_t w = 0; w < num_waves(); ++w) {
            sh.wave_base[w] = tot;
            tot += sh.wave[w].out_n;
        }
        const uint32_t base = tot ? add_relaxed(out_tail, tot) : 0u;
        for (uint32_t w = 0; w < num_waves(); ++w) sh.wave_base[w] += base;
    }
    __syncthreads();
    WaveLds& w = sh.wave[wave_id()];
    const uint32_t cnt = w.out_n, base = sh.wave_base[wave_id()];
    for (uint32_t i = lane_id(); i < cnt; i += kWave) out[base + i] = w.out[i];
    __builtin_amdgcn_wave_barrier();
    if (lane_id() == 0) w.out_n = 0;
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
// arcs `total`), UNROLL arcs per lane per step, coalesced column loads.
template <class Visit>
__device__ __forceinline__ void walk_arcs(WaveLds& w, uint32_t total, const uint32_t* __restrict__ col,
                                          Visit& visit, Stats& st) {
    st.arcs += lane_id() == 0 ? total : 0u;
    for (uint32_t base = 0; base < total; base += kWave * kUnroll) {
        uint32_t arc[kUnroll], u[kUnroll], pay[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) {
            const uint32_t e = base + j * kWave + lane_id();
            ok[j] = e < total;
            const uint32_t o = owner_of(w, ok[j] ? e : 0u);
            arc[j] = w.start[o] + (ok[j] ? e - w.excl[o] : 0u);
            pay[j] = w.pay[o];
        }
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) u[j] = ok[j] ? __builtin_nontemporal_load(&col[arc[j]]) : 0u;
        visit.step(ok, arc, u, pay, w, st);
        visit.maybe_flush(w);
    }
}

// One heavy strip {payload, first arc, length} walked by one wave.
template <class Visit>
__device__ __forceinline__ void walk_strip(WaveLds& w, uint32_t pay0, uint32_t a0, uint32_t len,
                                           const uint32_t* __restrict__ col, Visit& visit, Stats& st) {
    st.arcs += lane_id() == 0 ? len : 0u;
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
        visit.step(ok, arc, u, pay, w, st);
        visit.maybe_flush(w);
    }
}

// Expand one batch of up to 64 vertices (lane l holds vertex v if `act`):
// heavy vertices are queued as strips, the rest are walked by this wave.
// With `queue_heavy` false the heavy vertices are skipped: their strips
// were queued already (and are walked in the same phase).
template <class Visit>
__device__ __forceinline__ void expand_batch(const TraversalArgs& a, Work* wk, WaveLds& w, bool act,
                                             uint32_t v, Visit& visit, Stats& st, bool queue_heavy = true) {
    uint32_t s0 = 0, deg = 0, pay = 0;
    if (act) {
        s0 = a.row_ptr[v];
        deg = a.row_ptr[v + 1] - s0;
        pay = visit.payload(v);
        st.rows += 1;
    }
    const bool heavy = deg > a.heavy_th;
    if (!queue_heavy && heavy) deg = 0;
    const uint64_t hmask = queue_heavy ? __ballot(heavy) : 0ull;
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
                if (k < a.heavy_cap) a.heavy[k] = make_uint4(pay, s0 + off, len, v);
            }
            deg = 0;
        }
    }
    const uint32_t incl = wave_incl_scan(deg);
    w.excl[lane_id()] = incl - deg;
    w.start[lane_id()] = s0;
    w.pay[lane_id()] = pay;
    if (lane_id() == kWave - 1) w.excl[kWave] = incl;
    __builtin_amdgcn_wave_barrier();
    const uint32_t total = bcast(incl, kWave - 1);
    if (total) walk_arcs(w, total, a.col, visit, st);
    __builtin_amdgcn_wave_barrier();
}

// HEAVY phase: strips distributed statically over the interval's waves.
template <class Visit>
__device__ void heavy_phase(const TraversalArgs& a, uint32_t nstrips, uint32_t gw, uint32_t W, WaveLds& w,
                            Visit& visit, Stats& st) {
    if (nstrips > a.heavy_cap) nstrips = a.heavy_cap;
    for (uint32_t s = gw; s < nstrips; s += W) {
        const uint4 rec = a.heavy[s];
        const uint32_t pay = visit.strip_payload(rec.x, rec.w);
        walk_strip(w, pay, rec.y, rec.z, a.col, visit, st);
    }
}

// ------------------------------------------------------------------ BFS

// Count the wave's found vertices (`c` per lane) into the workgroup's LDS
// list; `emit(pos)` writes a lane's vertices from list position pos on
// (positions at or past kFlWg are dropped). `on` (wave-uniform) turns off once
// the count passes kFlWg: it then only tells the master step that the list
// overflowed (the master also checks the counts against the level's total).
template <class Emit>
__device__ __forceinline__ void fl_record(uint32_t* fl_n, bool& on, uint32_t c, Emit&& emit) {
    const uint32_t incl = wave_incl_scan(c);
    const uint32_t tot = bcast(incl, kWave - 1);
    if (tot == 0) return;
    uint32_t base = 0;
    if (lane_id() == kWave - 1) base = atomicAdd(fl_n, tot);
    base = bcast(base, kWave - 1);
    if (base + tot > kFlWg) on = false;
    if (c && base + incl - c < kFlWg) emit(base + incl - c);
}

struct BfsTopDown {
    uint32_t* vis;
    uint32_t* nxt;
    uint32_t* level;
    const uint32_t* row_ptr;
    uint32_t next_level;
    uint32_t count_mf;
    uint32_t* fl_n = nullptr;   // LDS found list of the workgroup (null: none kept)
    uint32_t* fl = nullptr;
    bool fl_on = false;

    __device__ __forceinline__ uint32_t payload(uint32_t) const { return 0; }
    __device__ __forceinline__ uint32_t strip_payload(uint32_t p, uint32_t) const { return p; }
    __device__ __forceinline__ void maybe_flush(WaveLds&) {}

    // Claim unvisited targets: a plain load filters most arcs, the atomic OR
    // on the visited set decides the single winner, which writes the level
    // and marks the next frontier. All claims of a step are issued before
    // any result is examined, so a step costs one atomic round trip however
    // many of its arcs reach unvisited vertices.
    __device__ __forceinline__ void step(const bool* ok, const uint32_t*, const uint32_t* u, const uint32_t*,
                                         WaveLds&, Stats& st) {
        uint32_t word[kUnroll], old[kUnroll];
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) word[j] = ok[j] ? vis[u[j] >> 5] : ~0u;
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) {
            const uint32_t bit = 1u << (u[j] & 31);
            old[j] = ~0u;
            if (!(word[j] & bit))
                old[j] = __hip_atomic_fetch_or(&vis[u[j] >> 5], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        bool won[kUnroll];
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) {
            const uint32_t bit = 1u << (u[j] & 31);
            won[j] = !(old[j] & bit);
            if (won[j]) {
                __builtin_nontemporal_store(next_level, &level[u[j]]);
                __hip_atomic_fetch_or(&nxt[u[j] >> 5], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                st.found += 1;
            }
        }
        if (fl_on) {
            uint32_t c = 0;
#pragma unroll
            for (uint32_t j = 0; j < kUnroll; ++j) c += won[j] ? 1u : 0u;
            fl_record(fl_n, fl_on, c, [&](uint32_t pos) {
#pragma unroll
                for (uint32_t j = 0; j < kUnroll; ++j)
                    if (won[j]) {
                        if (pos < kFlWg) fl[pos] = u[j];
                        ++pos;
                    }
            });
        }
        if (count_mf) {
            uint32_t r0[kUnroll], r1[kUnroll];
#pragma unroll
            for (uint32_t j = 0; j < kUnroll; ++j) {
                r0[j] = r1[j] = 0;
                if (won[j]) {
                    r0[j] = row_ptr[u[j]];
                    r1[j] = row_ptr[u[j] + 1];
                }
            }
#pragma unroll
            for (uint32_t j = 0; j < kUnroll; ++j) {
                st.mf += r1[j] - r0[j];
                st.rows += won[j] ? 1u : 0u;
            }
        }
    }
};

// Bottom-up level: every unvisited vertex with arcs scans its neighbours for
// one in the current frontier; the first hit makes it a member of the next
// level. A wave owns blocks of 32 bitmap words (1024 vertices): lanes 0..31
// load one visited word each, the unvisited vertices with arcs are compacted
// into an LDS list, and each lane probes two candidates at a time, taking the
// next candidate from the list as soon as one resolves, so two independent
// load chains stay in flight per lane until the list runs dry. A lane gives
// a candidate up after kLaneRounds steps of 4 arcs; such candidates (long
// lists without an early hit) are scanned by the whole wave, 256 arcs per
// step, so one long list does not hold the wave (and the level) for hundreds
// of dependent steps. Found bits are gathered in LDS
// and each block's visited and next-frontier words are written once, with
// plain stores (no other wave owns them).
constexpr uint32_t kLaneRounds = 8;

// One bottom-up probe: the aligned 16 bytes of the probe-order columns that
// hold arc k, i.e. arcs (k & ~3) .. (k & ~3) + 3 (the copy is 16-byte
// aligned and padded, so the load never leaves it); a lane tests the ones
// in [k, e). One load instruction per probe, one cache line per lane.
__device__ __forceinline__ uint4 probe_chunk(const uint32_t* __restrict__ col_bu, uint32_t k) {
    return *reinterpret_cast<const uint4*>(col_bu + (k & ~3u));
}

// Whether arcs max(k, k & ~3) .. min(e, (k & ~3) + 4) - 1 of chunk q reach
// the frontier `cur`; `got` = how many arcs that was.
__device__ __forceinline__ bool probe_hits(const uint32_t* __restrict__ cur, uint4 q, uint32_t k, uint32_t e,
                                          uint32_t& got) {
    const uint32_t b0 = k & ~3u;
    const uint32_t end = e < b0 + 4 ? e : b0 + 4;
    got = end - k;
    const uint32_t u[4] = {q.x, q.y, q.z, q.w};
    bool hit = false;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t a = b0 + j;
        if (a >= k && a < end) hit |= ((cur[u[j] >> 5] >> (u[j] & 31)) & 1u) != 0;
    }
    return hit;
}

// (`word0`: the block's first bitmap word; fw holds the block's found bits)
__device__ __forceinline__ void bu_mark(const BfsArgs& p, uint32_t* fw, uint32_t* level, uint32_t v,
                                        uint32_t next_level, uint32_t word0, uint32_t deg, Stats& st) {
    __builtin_nontemporal_store(next_level, &level[v]);
    atomicOr(&fw[(v >> 5) - word0], 1u << (v & 31));
    st.found += 1;
    st.mf += deg;
}

// Scan the deferred long lists with the whole wave, one candidate at a time,
// 256 arcs per step, from where the lane left off (lngk).
__device__ void bu_scan_long(const BfsArgs& p, WaveLds& wl, const uint32_t* cur, uint32_t* fw, uint32_t* level,
                             uint32_t next_level, uint32_t word0, uint32_t nlong, Stats& st) {
    const uint32_t l = lane_id();
    for (uint32_t i = 0; i < nlong; ++i) {
        const uint32_t vv = wl.lng[i];
        const uint32_t a0 = p.t.row_ptr[vv], a1 = p.t.row_ptr[vv + 1];
        bool found = false;
        for (uint32_t kk = wl.lngk[i]; kk < a1 && !found; kk += 4 * kWave) {
            uint32_t u[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t a = kk + j * kWave + l;
                u[j] = a < a1 ? p.col_bu[a] : 0xFFFFFFFFu;
            }
            bool h = false;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (u[j] != 0xFFFFFFFFu) h |= ((cur[u[j] >> 5] >> (u[j] & 31)) & 1u) != 0;
            found = __ballot(h) != 0;
            st.arcs += l == 0 ? (a1 - kk < 4 * kWave ? a1 - kk : 4 * kWave) : 0u;
        }
        if (found && l == 0) bu_mark(p, fw, level, vv, next_level, word0, a1 - a0, st);
    }
    __builtin_amdgcn_wave_barrier();
}

__device__ void bfs_bottom_up(const BfsArgs& p, WaveLds& wl, const uint32_t* cur, uint32_t* nxt,
                              uint32_t* level, uint32_t next_level, uint32_t gw, uint32_t W, Stats& st,
                              uint32_t* fl_n, uint32_t* fl) {
    bool fl_on = fl_n != nullptr;
    constexpr uint32_t kBlockWords = 32;
    const uint32_t blocks = p.words / kBlockWords;
    const uint32_t l = lane_id();
    uint32_t* list = wl.out;            // up to 1024 candidates
    uint32_t* fw = wl.excl;             // found bits of the block's 32 words
    for (uint32_t b = gw; b < blocks; b += W) {
        const uint32_t wi = b * kBlockWords + (l & 31);
        uint32_t vw = 0, cand = 0;
        if (l < 32) {
            vw = p.vis[wi];
            cand = ~(vw | p.deg0[wi]);
            fw[l] = 0;
        }
        st.words += (l == 0) ? 2u * kBlockWords : 0u;
        const uint32_t cnt = __popc(cand);
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t total = bcast(incl, kWave - 1);
        if (total == 0) continue;
        uint32_t pos = incl - cnt;
        while (cand) {
            list[pos++] = wi * 32u + (uint32_t)(__ffs(cand) - 1);
            cand &= cand - 1;
        }
        __builtin_amdgcn_wave_barrier();
        const bool dense = p.first2 != nullptr;     // skewed graphs only (see graph_prep)
        uint32_t pend = total;                      // candidates left for the probe slots
        if (dense) {
            // first pass on a skewed graph: every candidate's first two
            // neighbours from the dense array, 4 x 64 candidates at a time
            // (consecutive candidates read adjacent entries, and the loads
            // of the four are in flight together); most candidates end
            // here, the others go back to the list for the probe slots,
            // which start at their third arc
            uint32_t nrem = 0;
            for (uint32_t base = 0; base < total; base += 4 * kWave) {
                uint32_t vv[4], a0[4], a1[4];
                uint2 f[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t i = base + j * kWave + l;
                    vv[j] = i < total ? list[i] : 0xFFFFFFFFu;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    a0[j] = a1[j] = 0;
                    f[j] = make_uint2(0, 0);
                    if (vv[j] != 0xFFFFFFFFu) {
                        f[j] = p.first2[vv[j]];
                        a0[j] = p.t.row_ptr[vv[j]];
                        a1[j] = p.t.row_ptr[vv[j] + 1];
                    }
                }
                bool hit[4], more[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t d = a1[j] - a0[j];        // >= 1 for a candidate
                    hit[j] = false;
                    more[j] = false;
                    if (vv[j] != 0xFFFFFFFFu) {
                        hit[j] = ((cur[f[j].x >> 5] >> (f[j].x & 31)) & 1u) != 0;
                        if (d > 1) hit[j] |= ((cur[f[j].y >> 5] >> (f[j].y & 31)) & 1u) != 0;
                        more[j] = !hit[j] && d > 2;
                        st.arcs += d < 2 ? d : 2u;
                        st.rows += 1;
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (hit[j]) bu_mark(p, fw, level, vv[j], next_level, b * kBlockWords, a1[j] - a0[j], st);
                    // the misses with more arcs, in list order; the entries
                    // written lie below the ones this round has read
                    const uint64_t mask = __ballot(more[j]);
                    if (more[j]) list[nrem + mbcnt(mask)] = vv[j];
                    nrem += (uint32_t)__popcll(mask);
                }
            }
            pend = nrem;
            __builtin_amdgcn_wave_barrier();
        }
        // Two probe slots per lane; a slot that resolves its candidate takes
        // the next one from the list, so the wave keeps 128 chains busy
        // instead of waiting for the slowest lane of a batch.
        uint32_t next = 0, nlong = 0;
        uint32_t v[2] = {0, 0}, k[2] = {0, 0}, e[2] = {0, 0}, s0[2] = {0, 0}, rounds[2] = {0, 0};
        bool act[2] = {false, false};
        for (;;) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const bool need = !act[c];
                const uint64_t mask = __ballot(need);
                if (next < pend && mask) {
                    const uint32_t idx = next + mbcnt(mask);
                    if (need && idx < pend) {
                        v[c] = list[idx];
                        act[c] = true;
                        s0[c] = k[c] = p.t.row_ptr[v[c]];
                        e[c] = p.t.row_ptr[v[c] + 1];
                        if (dense) k[c] += 2;            // the first pass probed two arcs
                        rounds[c] = 0;
                        st.rows += 1;
                    }
                    next += (uint32_t)__popcll(mask);
                }
            }
            if (!__ballot(act[0] || act[1])) break;
            // every round probes an aligned 4-arc chunk of col_bu
            uint4 q[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) q[c] = act[c] ? probe_chunk(p.col_bu, k[c]) : make_uint4(0, 0, 0, 0);
            bool defer[2] = {false, false};
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (!act[c]) continue;
                uint32_t got;
                const bool hit = probe_hits(cur, q[c], k[c], e[c], got);
                st.arcs += got;
                k[c] += got;
                rounds[c] += 1;
                if (hit) {
                    bu_mark(p, fw, level, v[c], next_level, b * kBlockWords, e[c] - s0[c], st);
                    act[c] = false;
                } else if (k[c] >= e[c]) {
                    act[c] = false;                  // no parent in this frontier
                } else if (rounds[c] == kLaneRounds) {
                    defer[c] = true;                 // long list: the whole wave scans it
                    act[c] = false;
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const uint64_t mask = __ballot(defer[c]);
                if (defer[c]) {
                    wl.lng[nlong + mbcnt(mask)] = v[c];
                    wl.lngk[nlong + mbcnt(mask)] = k[c];
                }
                nlong += (uint32_t)__popcll(mask);
            }
            if (nlong) {                             // at most 2 x 64 deferrals: the list's capacity
                __builtin_amdgcn_wave_barrier();
                bu_scan_long(p, wl, cur, fw, level, next_level, b * kBlockWords, nlong, st);
                nlong = 0;
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (l < 32) {
            const uint32_t f = fw[l];
            if (f) {
                p.vis[wi] = vw | f;
                nxt[wi] = f;
            }
        }
        if (fl_on) {
            const uint32_t f = l < 32 ? fw[l] : 0u;
            fl_record(fl_n, fl_on, __popc(f), [&](uint32_t pos) {
                for (uint32_t m = f; m && pos < kFlWg; m &= m - 1) fl[pos++] = wi * 32u + (uint32_t)(__ffs(m) - 1);
            });
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Bottom-up level with the block's row ranges staged in LDS. A wave owns
// blocks of 16 bitmap words (512 vertices): lanes 0..15 load one visited
// word each, the whole wave reads the block's 513 row_ptr entries with one
// coalesced pass into LDS, and the unvisited vertices with arcs are
// compacted into a list of block offsets. Each lane then probes two
// candidates at a time as in bfs_bottom_up, but a candidate's arc range
// comes from LDS, so its dependent chain is column -> frontier bit (two
// global round trips instead of three).
__device__ void bfs_bottom_up_rp(const BfsArgs& p, WaveLds& wl, const uint32_t* cur, uint32_t* nxt,
                                 uint32_t* level, uint32_t next_level, uint32_t gw, uint32_t W, Stats& st,
                                 uint32_t* fl_n, uint32_t* fl) {
    bool fl_on = fl_n != nullptr;
    constexpr uint32_t kBlockWords = 16, kBlockV = kBlockWords * 32;
    const uint32_t blocks = p.words / kBlockWords;
    const uint32_t l = lane_id();
    const uint32_t n = p.t.n;
    uint32_t* list = wl.out;                 // candidates as block offsets (< 512)
    uint32_t* rp = wl.out + kBlockV;         // row_ptr of the block's vertices 0..511
    uint32_t* fw = wl.excl;                  // found bits of the block's 16 words
    for (uint32_t b = gw; b < blocks; b += W) {
        const uint32_t wi = b * kBlockWords + (l & 15);
        const uint32_t v0 = b * kBlockV;
        uint32_t vw = 0, cand = 0;
        if (l < 16) {
            vw = p.vis[wi];
            cand = ~(vw | p.deg0[wi]);
            fw[l] = 0;
        }
        st.words += (l == 0) ? 2u * kBlockWords : 0u;
        const uint32_t cnt = __popc(cand);
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t total = bcast(incl, kWave - 1);
        if (total == 0) continue;
        // row ranges of the whole block (vertices past n read row_ptr[n])
#pragma unroll
        for (uint32_t j = 0; j < kBlockV / kWave; ++j) {
            const uint32_t v = v0 + j * kWave + l;
            rp[j * kWave + l] = p.t.row_ptr[v < n ? v : n];
        }
        const uint32_t vend = v0 + kBlockV;
        const uint32_t rp_end = p.t.row_ptr[vend < n ? vend : n];
        st.rows += (l == 0) ? kBlockV : 0u;
        uint32_t pos = incl - cnt;
        const uint32_t wbase = (l & 15) * 32u;
        while (cand) {
            list[pos++] = wbase + (uint32_t)(__ffs(cand) - 1);
            cand &= cand - 1;
        }
        __builtin_amdgcn_wave_barrier();
        uint32_t next = 0, nlong = 0;
        uint32_t o[2] = {0, 0}, k[2] = {0, 0}, e[2] = {0, 0}, s0[2] = {0, 0}, rounds[2] = {0, 0};
        bool act[2] = {false, false};
        for (;;) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const bool need = !act[c];
                const uint64_t mask = __ballot(need);
                if (next < total && mask) {
                    const uint32_t idx = next + mbcnt(mask);
                    if (need && idx < total) {
                        o[c] = list[idx];
                        act[c] = true;
                        rounds[c] = 0;
                        s0[c] = k[c] = rp[o[c]];
                        e[c] = o[c] + 1 < kBlockV ? rp[o[c] + 1] : rp_end;
                    }
                    next += (uint32_t)__popcll(mask);
                }
            }
            if (!__ballot(act[0] || act[1])) break;
            uint4 q[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) q[c] = act[c] ? probe_chunk(p.col_bu, k[c]) : make_uint4(0, 0, 0, 0);
            bool defer[2] = {false, false};
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (!act[c]) continue;
                uint32_t got;
                const bool hit = probe_hits(cur, q[c], k[c], e[c], got);
                st.arcs += got;
                k[c] += got;
                rounds[c] += 1;
                if (hit) {
                    bu_mark(p, fw, level, v0 + o[c], next_level, b * kBlockWords, e[c] - s0[c], st);
                    act[c] = false;
                } else if (k[c] >= e[c]) {
                    act[c] = false;                  // no parent in this frontier
                } else if (rounds[c] == kLaneRounds) {
                    defer[c] = true;                 // long list: the whole wave scans it
                    act[c] = false;
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const uint64_t mask = __ballot(defer[c]);
                if (defer[c]) {
                    wl.lng[nlong + mbcnt(mask)] = v0 + o[c];
                    wl.lngk[nlong + mbcnt(mask)] = k[c];
                }
                nlong += (uint32_t)__popcll(mask);
            }
            if (nlong) {
                __builtin_amdgcn_wave_barrier();
                bu_scan_long(p, wl, cur, fw, level, next_level, b * kBlockWords, nlong, st);
                nlong = 0;
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (l < 16) {
            const uint32_t f = fw[l];
            if (f) {
                p.vis[wi] = vw | f;
                nxt[wi] = f;
            }
        }
        if (fl_on) {
            const uint32_t f = l < 16 ? fw[l] : 0u;
            fl_record(fl_n, fl_on, __popc(f), [&](uint32_t pos) {
                for (uint32_t m = f; m && pos < kFlWg; m &= m - 1) fl[pos++] = wi * 32u + (uint32_t)(__ffs(m) - 1);
            });
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Top-down step over a frontier bitmap. A unit is one bitmap word (32
// vertices) and unit u belongs to wave slot u mod W, so a frontier that
// fills a few hundred adjacent words still spreads over as many waves (and
// workgroups). A wave gathers up to 32 of its words at a time (lane j loads
// word gw + (k + j) W), compacts their set bits into its LDS list and
// expands them 64 vertices per batch.
template <class Visit>
__device__ void expand_bitmap(const TraversalArgs& a, Work* wk, WaveLds& w, const uint32_t* cur, uint32_t words,
                              uint32_t gw, uint32_t W, Visit& vis, Stats& st, bool queue_heavy = true) {
    const uint32_t l = lane_id();
    uint32_t* list = w.out;             // up to 32 x 32 = 1024 vertices
    for (uint32_t k = 0; gw + k * W < words; k += 32) {
        const uint32_t wi = gw + (k + (l & 31)) * W;
        uint32_t word = (l < 32 && wi < words) ? cur[wi] : 0u;
        st.words += (l < 32 && wi < words) ? 1u : 0u;
        const uint32_t cnt = __popc(word);
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t total = bcast(incl, kWave - 1);
        if (total == 0) continue;
        uint32_t pos = incl - cnt;
        while (word) {
            list[pos++] = wi * 32u + (uint32_t)(__ffs(word) - 1);
            word &= word - 1;
        }
        __builtin_amdgcn_wave_barrier();
        for (uint32_t base = 0; base < total; base += kWave) {
            const uint32_t i = base + l;
            const bool act = i < total;
            expand_batch(a, wk, w, act, act ? list[i] : 0u, vis, st, queue_heavy);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

__device__ void bfs_top_down(const BfsArgs& p, Work* wk, WaveLds& w, const uint32_t* cur, BfsTopDown& vis,
                             uint32_t gw, uint32_t W, Stats& st, bool queue_heavy = true) {
    expand_bitmap(p.t, wk, w, cur, p.words, gw, W, vis, st, queue_heavy);
}

// Clear a bitmap share: words gw*64 + lane, then + W*64 ...
__device__ __forceinline__ void clear_share(uint32_t* bm, uint32_t words, uint32_t gw, uint32_t W) {
    for (uint32_t i = gw * kWave + lane_id(); i < words; i += W * kWave) bm[i] = 0;
}

// Level partials that survive the TD -> HEAVY barrier live in Work::pad5.
// One BFS phase for member `id` of `M` (the interval's membership):
// INIT clears the per-source state, TD/HEAVY expand the frontier, BU probes
// the unvisited vertices. Statistics go to the member's slot.
// Returns (thread 0) the workgroup's share of the level's found and mf for
// the barrier arrival when the launch takes them that way, else 0.
template <bool Small = false>
__device__ __forceinline__ uint64_t bfs_phase(const BfsArgs& p, BlockLds& sh, uint32_t ph, uint32_t flags,
                                              uint32_t level, uint32_t root, uint32_t id, uint32_t M,
                                              uint32_t* lvl_base) {
    const TraversalArgs& t = p.t;
    Work* wk = t.work;
    const uint32_t nw = num_waves();
    const uint32_t rot = (flags & kRotMask) >> kRotShift;
    uint32_t* cur = p.fb[rot];
    uint32_t* nxt = p.fb[(rot + 1) % 3];
    uint32_t* spare = p.fb[(rot + 2) % 3];
    uint32_t* lvl = lvl_base + (size_t)root * t.out_stride;
    const uint32_t gw = wave_slot(id, M, nw);
    const uint32_t W = M * nw;
    Stats st;
    if (ph == kPhInit) {
        const uint32_t tid = id * blockDim.x + threadIdx.x, stride = M * blockDim.x;
        // the level array is output only: streamed, so it does not sit dirty
        // in L2 for the next barrier's release to write back
        for (uint32_t i = tid; i < t.n; i += stride) __builtin_nontemporal_store(kInf, &lvl[i]);
        for (uint32_t i = tid; i < p.words; i += stride) {
            p.vis[i] = 0;
            p.fb[0][i] = 0;
            p.fb[1][i] = 0;
            p.fb[2][i] = 0;
        }
    } else if (ph == kPhTD || ph == kPhHeavy) {
        BfsTopDown vis{p.vis, nxt, lvl, t.row_ptr, level + 1, p.direction_opt};
        if (Small && p.flist && (flags & kFlagRecord)) {
            vis.fl_n = &sh.fl_n;
            vis.fl = sh.fl;
            vis.fl_on = true;
        }
        WaveLds& w = sh.wave[wave_id()];
        if (ph == kPhTD) {
            clear_share(spare, p.words, gw, W);
            const bool pre = (flags & kFlagPreSplit) != 0;
            if (pre) heavy_phase(t, wk->x.in_size, gw, W, w, vis, st);   // the master step's strips
            bfs_top_down(p, wk, w, cur, vis, gw, W, st, !pre);
        } else {
            heavy_phase(t, wk->x.in_size, gw, W, w, vis, st);
        }
    } else if (ph == kPhBU) {
        clear_share(spare, p.words, gw, W);
        uint32_t* fn = (Small && p.flist && (flags & kFlagRecord)) ? &sh.fl_n : nullptr;
        if (p.bu_prefetch) bfs_bottom_up_rp(p, sh.wave[wave_id()], cur, nxt, lvl, level + 1, gw, W, st, fn, sh.fl);
        else bfs_bottom_up(p, sh.wave[wave_id()], cur, nxt, lvl, level + 1, gw, W, st, fn, sh.fl);
    }
    uint64_t pay = 0;
    if (ph != kPhStart && ph != kPhInit) {
        stats_to_lds(sh, st);
        __syncthreads();
        // read before acc_to_slot clears the accumulators (the same wave)
        if (p.arrive_sums && threadIdx.x == 0) pay = arrive_payload(sh.acc[0], sh.acc[1]);
        acc_to_slot(sh, t.slots, id, !p.arrive_sums);
        if (Small && p.flist && (flags & kFlagRecord) && threadIdx.x < kWave) {
            // the phase's found list, for a master step that may run the
            // next levels itself: count, then up to kFlWg vertices (wave 0
            // reads the count before lane 0 clears it for the next phase)
            const uint32_t nf = sh.fl_n;
            uint32_t* dst = p.flist + (size_t)id * (kFlWg + 1);
            if (threadIdx.x < nf && threadIdx.x < kFlWg) dst[1 + threadIdx.x] = sh.fl[threadIdx.x];
            if (threadIdx.x == 0) {
                dst[0] = nf;
                sh.fl_n = 0;
            }
        }
    }
    return pay;
}

// ------------------------------------------- small levels in the master step
//
// A level whose frontier is small costs far more in its phase's start and
// end (every workgroup scans its share of the frontier bitmap, then meets at
// the barrier) than in its arcs. The master workgroup runs such levels
// itself, one after another, inside the master step: on R-MAT the first
// level after a low-degree source and the last one or two levels of every
// traversal touch a few thousand arcs at most. A level qualifies when its
// frontier fits the master's LDS lists (il_cap) and its arcs are at most
// kInlineLevelArcs per thread (walked in rounds of kInlineArcs per thread:
// the smaller round costs the kernel's phases fewer registers); it is
// walked top-down whatever the direction rule would pick for a phase. The
// results are those of the phases: the same claims on the visited bitmap,
// the same levels, the same next frontier in the bitmap the next phase
// reads.
//
// The lists live in the master's wave output buffers (idle in a master
// step): two frontier lists, the first arc of each vertex and its degree
// (then degree prefix), each il_cap entries, indexed through il_at.
constexpr uint32_t kInlineArcs = 3;      // arcs per thread of the master workgroup per round
constexpr uint32_t kInlineLevelArcs = 4; // arcs per thread of a level the master step takes (more rounds)
constexpr uint32_t kInlineLevels = 16;   // levels per master step at most (a barrier, and its
                                         // offer_kill, still comes after that many)

__device__ __forceinline__ uint32_t il_cap(uint32_t nw) {
    const uint32_t c = (nw * kOutCap - 1) / 6;
    return c < 2048u ? c : 2048u;
}
__device__ __forceinline__ uint32_t& il_at(BlockLds& sh, uint32_t i) { return sh.wave[i / kOutCap].out[i % kOutCap]; }

// Exclusive prefix sum of entries [base, base + n) in place; returns the
// total (all threads).
__device__ __forceinline__ uint32_t il_scan(BlockLds& sh, uint32_t base, uint32_t n) {
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t i0 = threadIdx.x * per;
    uint32_t loc = 0;
    for (uint32_t j = 0; j < per; ++j)
        if (i0 + j < n) loc += il_at(sh, base + i0 + j);
    const uint32_t incl = wave_incl_scan(loc);
    if (lane_id() == kWave - 1) sh.wave_base[wave_id()] = incl;
    __syncthreads();
    uint32_t run = incl - loc, tot = 0;
    for (uint32_t w = 0; w < num_waves(); ++w) {
        const uint32_t b = sh.wave_base[w];
        run += w < wave_id() ? b : 0u;
        tot += b;
    }
    for (uint32_t j = 0; j < per; ++j)
        if (i0 + j < n) {
            uint32_t& e = il_at(sh, base + i0 + j);
            const uint32_t d = e;
            e = run;
            run += d;
        }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(tot);
}

// The last index i < n whose prefix entry [base + i] is <= k.
__device__ __forceinline__ uint32_t il_owner(BlockLds& sh, uint32_t base, uint32_t n, uint32_t k) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (il_at(sh, base + mid) <= k) lo = mid; else hi = mid;
    }
    return lo;
}

// The found lists of the phase just ended (members 0 .. M-1, nf vertices
// in all) into frontier list 0, with each vertex's first arc and degree.
// False (all threads) if a workgroup found more than it could list.
__device__ __forceinline__ bool il_gather(BlockLds& sh, const uint32_t* flist, const uint32_t* row_ptr, uint32_t M,
                                          uint32_t nf) {
    const uint32_t F = il_cap(num_waves());
    if (M > 5 * F || nf > F) return false;
    const uint32_t T0 = F;                     // the M counts, then their offsets
    if (threadIdx.x == 0) sh.il_go = 1u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) {
        const uint32_t c = flist[(size_t)i * (kFlWg + 1)];
        il_at(sh, T0 + i) = c;
        if (c > kFlWg) sh.il_go = 0u;
    }
    __syncthreads();
    const uint32_t tot = il_scan(sh, T0, M);
    if (!__builtin_amdgcn_readfirstlane(sh.il_go) || tot != nf) return false;
    for (uint32_t k = threadIdx.x; k < nf; k += blockDim.x) {
        const uint32_t i = il_owner(sh, T0, M, k);
        il_at(sh, k) = flist[(size_t)i * (kFlWg + 1) + 1 + (k - il_at(sh, T0 + i))];
    }
    __syncthreads();
    uint32_t arcs = 0;
    for (uint32_t k = threadIdx.x; k < nf; k += blockDim.x) {
        const uint32_t v = il_at(sh, k);
        const uint32_t a0 = row_ptr[v];
        const uint32_t d = row_ptr[v + 1] - a0;
        il_at(sh, 2 * F + k) = a0;
        il_at(sh, 4 * F + k) = d;
        arcs += d;
    }
    // the level's arcs (the phases only sum them when they choose directions)
    const uint64_t wa = wave_sum64(arcs);
    if (lane_id() == 0) sh.red[0][wave_id()] = wa;
    __syncthreads();
    uint64_t all = 0;
    for (uint32_t w = 0; w < num_waves(); ++w) all += sh.red[0][w];
    __syncthreads();
    return all <= (uint64_t)kInlineLevelArcs * blockDim.x;
}

// One round of a master-step level: arcs e0 .. e0 + kInlineArcs * blockDim.x
// - 1 of the frontier in list region LA/SA/PA (PA: degree prefix). Claimed
// neighbours get level lvl + 1 and their bit in bm, and go to list region
// LB/SB/PB (counted in *len); returns the lane's sum of their degrees.
__device__ __forceinline__ uint64_t il_round(BlockLds& sh, uint32_t* vis, uint32_t* bm, uint32_t* lv,
                                             const uint32_t* col, const uint32_t* row_ptr, uint32_t lvl, uint32_t e0,
                                             uint32_t total, uint32_t nf, uint32_t SA, uint32_t PA, uint32_t LB,
                                             uint32_t SB, uint32_t PB, uint32_t F, uint32_t* len) {
    uint32_t u[kInlineArcs], s[kInlineArcs], d[kInlineArcs];
    bool won[kInlineArcs];
    // all loads of a step are issued before their results are used
#pragma unroll
    for (uint32_t j = 0; j < kInlineArcs; ++j) {
        const uint32_t e = e0 + threadIdx.x + j * blockDim.x;
        u[j] = 0xFFFFFFFFu;
        if (e < total) {
            const uint32_t i = il_owner(sh, PA, nf, e);
            u[j] = col[il_at(sh, SA + i) + (e - il_at(sh, PA + i))];
        }
    }
    // claims without a filtering load first (at most a few thousand arcs:
    // one round trip less per level)
#pragma unroll
    for (uint32_t j = 0; j < kInlineArcs; ++j) {
        const uint32_t bit = 1u << (u[j] & 31);
        uint32_t old = ~0u;
        if (u[j] != 0xFFFFFFFFu)
            old = __hip_atomic_fetch_or(&vis[u[j] >> 5], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        won[j] = !(old & bit);
    }
    uint32_t cnt = 0;
#pragma unroll
    for (uint32_t j = 0; j < kInlineArcs; ++j) {
        s[j] = d[j] = 0;
        if (won[j]) {
            __builtin_nontemporal_store(lvl + 1, &lv[u[j]]);
            __hip_atomic_fetch_or(&bm[u[j] >> 5], 1u << (u[j] & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s[j] = row_ptr[u[j]];
            d[j] = row_ptr[u[j] + 1];
            ++cnt;
        }
    }
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t wtot = bcast(incl, kWave - 1);
    uint32_t base = 0;
    if (lane_id() == kWave - 1 && wtot) base = atomicAdd(len, wtot);
    base = bcast(base, kWave - 1);
    uint32_t pos = base + incl - cnt;
    uint64_t mf = 0;
#pragma unroll
    for (uint32_t j = 0; j < kInlineArcs; ++j)
        if (won[j]) {
            d[j] -= s[j];
            mf += d[j];
            if (pos < F) {
                il_at(sh, LB + pos) = u[j];
                il_at(sh, SB + pos) = s[j];
                il_at(sh, PB + pos) = d[j];
            }
            ++pos;
        }
    return mf;
}

struct IlArgs {                  // what the master-step levels read, by value (no kernel-argument address)
    uint32_t* vis;
    uint32_t* bm;                // the frontier bitmap the levels keep current
    const uint32_t* col;
    const uint32_t* row_ptr;
    uint32_t* slots;
    uint32_t* lv;                // the source's level array
    uint64_t total_arcs;
    uint32_t alpha, direction_opt, nroots, record;
};

// Run levels in the master step (all threads). On entry frontier list 0
// holds the nf vertices of level `lvl` with their first arcs and degrees;
// their bits are all of fb[(r + 1) % 3], and fb[(r + 2) % 3] is clear (the
// state after a phase at rotation r). Each level claims the frontier's
// unvisited neighbours on the visited bitmap, gives them level lvl + 1 and
// sets their bits in the same bitmap while clearing the frontier's, so the
// bitmap always holds exactly the current frontier. It stops when the
// source is finished, when the next level is too large, or after
// kInlineLevels levels; the next phase then runs at rotation (r + 1) % 3
// (current = that bitmap, next = the clear one), in the direction the rule
// picks. `x` and the returned release flags are thread 0's.
__device__ __forceinline__ uint32_t bfs_inline_levels(const IlArgs& q, BlockLds& sh, XferR& x, uint32_t nf,
                                                      uint32_t lvl, uint32_t r) {
    const uint32_t F = il_cap(num_waves());
    const uint32_t round = kInlineArcs * blockDim.x;
    uint32_t* bm = q.bm;
    uint32_t* lv = q.lv;
    uint64_t arcs_all = 0, rows_all = 0, found_all = 0;
    uint32_t a = 0, res = 0;
    for (uint32_t done = 1;; ++done) {
        const uint32_t LA = a * F, SA = (2 + a) * F, PA = (4 + a) * F;
        const uint32_t LB = (1 - a) * F, SB = (3 - a) * F, PB = (5 - a) * F;
        // the next list's length (last read two levels ago; the scan's
        // workgroup barriers order the reset before any append)
        if (threadIdx.x == 0) sh.il_c[1 - a] = 0;
        const uint32_t total = il_scan(sh, PA, nf);      // degrees -> first arc of each vertex in the level's arcs
        // one round per level under the entry conditions; a longer level
        // (a frontier whose arcs the phases did not count) takes more
        uint64_t mf = 0;
        for (uint32_t e0 = 0; e0 < total; e0 += round)
            mf += il_round(sh, q.vis, bm, lv, q.col, q.row_ptr, lvl, e0, total, nf, SA, PA, LB, SB, PB, F,
                           &sh.il_c[1 - a]);
        // the level's own bits leave the bitmap (the winners are other vertices)
        for (uint32_t i = threadIdx.x; i < nf; i += blockDim.x) {
            const uint32_t v = il_at(sh, LA + i);
            __hip_atomic_fetch_and(&bm[v >> 5], ~(1u << (v & 31)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const uint64_t wmf = wave_sum64(mf);
        if (lane_id() == 0) sh.red[0][wave_id()] = wmf;
        __syncthreads();                           // every claim, mark and clear has completed
        const uint32_t nb = __builtin_amdgcn_readfirstlane(sh.il_c[1 - a]);
        if (threadIdx.x == 0) {
            uint64_t mfb = 0;
            for (uint32_t w = 0; w < num_waves(); ++w) mfb += sh.red[0][w];
            arcs_all += total;
            rows_all += nf + nb;
            found_all += nb;
            x.levels_total() += 1;
            x.td_levels() += 1;
            uint32_t go = 0;
            if (nb == 0) {
                x.root() += 1;
                res = x.root() >= q.nroots ? kFlagDone : (kPhInit | kFlagAdv);
            } else {
                const uint64_t mv = join64(x.m_visited_lo(), x.m_visited_hi()) + mfb;
                x.m_visited_lo() = (uint32_t)mv;
                x.m_visited_hi() = (uint32_t)(mv >> 32);
                const uint64_t m_u = q.total_arcs > mv ? q.total_arcs - mv : 0;
                const uint32_t nph = (q.direction_opt && mfb * q.alpha > m_u) ? kPhBU : kPhTD;
                x.level() = lvl + 1;
                x.nf_prev() = nb;
                // a level this small goes here whatever the direction rule
                // says (the rule picks the cheaper walk for a phase of all
                // workgroups; either gives the same levels)
                go = (nb <= F && mfb <= (uint64_t)kInlineLevelArcs * blockDim.x && done < kInlineLevels) ? 1u : 0u;
                if (!go)
                    res = nph | kFlagAdv | kFlagJump | (((r + 1) % 3) << kRotShift) |
                          (q.record && mfb <= kRecordArcs ? kFlagRecord : 0u);
            }
            sh.il_go = go;
        }
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(sh.il_go)) break;
        nf = nb;
        lvl += 1;
        a = 1 - a;
    }
    if (threadIdx.x == 0) {
        uint64_t* s0 = reinterpret_cast<uint64_t*>(q.slots);
        add_nr64(&s0[kSlotArcs], arcs_all);
        add_nr64(&s0[kSlotRows], rows_all);
        if (found_all) add_nr64(&s0[kSlotFoundAll], found_all);
    }
    return res;
}

// Start source x.root() in the master step (all threads of the master
// workgroup; `x` is thread 0's): the source gets level 0, and when its list
// has at most one arc per thread the workgroup expands it at once -- every
// neighbour claimed on the visited bitmap gets level 1 and a bit in the
// next frontier -- so the source needs no top-down phase (and barrier) for
// level 0. The marks are atomics, as every later claim of the same words is.
// Returns the release flags (thread 0).
template <bool Small>
__device__ uint32_t bfs_master_source(const BfsArgs& p, BlockLds& sh, CtxCore* c, XferR& x, const uint32_t* roots,
                                      uint32_t* lvl_base) {
    const TraversalArgs& t = p.t;
    if (threadIdx.x == 0) {
        const uint32_t src = roots[x.root()];
        uint32_t a0 = 0, deg = 0;
        if (src < t.n) {
            a0 = t.row_ptr[src];
            deg = t.row_ptr[src + 1] - a0;
            uint32_t* lv = lvl_base + (size_t)x.root() * t.out_stride;
            __builtin_nontemporal_store(0u, &lv[src]);
            atomicOr(&p.vis[src >> 5], 1u << (src & 31));
            atomicOr(&p.fb[0][src >> 5], 1u << (src & 31));
        }
        sh.mb[0] = src;
        sh.mb[1] = a0;
        sh.mb[2] = deg;
        sh.mb[3] = x.root();
        sh.il_c[0] = 0;
    }
    __syncthreads();
    const uint32_t src = sh.mb[0], a0 = sh.mb[1], deg = sh.mb[2];
    if (src >= t.n) {
        // a source outside the graph ends the launch before anything is
        // written for it (earlier sources are complete)
        if (threadIdx.x == 0) {
            raise_error(c, kErrInvalid);
            sh.il_go = 0;
        }
        return kFlagAbort;
    }
    const bool inline_l0 = deg <= blockDim.x;
    uint64_t found = 0, mf = 0, strips = 0;
    uint32_t* lv = lvl_base + (size_t)sh.mb[3] * t.out_stride;
    uint32_t u = 0, u0 = 0, du = 0;
    bool won = false;
    if (inline_l0) {
        if (threadIdx.x < deg) {
            u = t.col[a0 + threadIdx.x];
            const uint32_t bit = 1u << (u & 31);
            if (!(atomicOr(&p.vis[u >> 5], bit) & bit)) {
                __builtin_nontemporal_store(1u, &lv[u]);
                atomicOr(&p.fb[1][u >> 5], bit);
                won = true;
                found = 1;
                u0 = t.row_ptr[u];
                du = t.row_ptr[u + 1] - u0;
                mf = du;
                // a heavy vertex of level 1: unless the master step runs
                // level 1 itself, its strips are queued below, so level 1's
                // own phase walks them (no HEAVY phase)
                if (du > t.heavy_th) strips = (du + t.strip - 1) / t.strip;
            }
        }
        if (Small && p.inline_on) {
            // level 1 as frontier list 0 of the master-step levels (at most
            // one vertex per thread, within il_cap)
            const uint32_t F = il_cap(num_waves());
            const uint32_t cw = won ? 1u : 0u;
            const uint32_t incl = wave_incl_scan(cw);
            const uint32_t wtot = bcast(incl, kWave - 1);
            uint32_t base = 0;
            if (lane_id() == kWave - 1 && wtot) base = atomicAdd(&sh.il_c[0], wtot);
            base = bcast(base, kWave - 1);
            if (won) {
                const uint32_t pos = base + incl - 1;
                il_at(sh, pos) = u;
                il_at(sh, 2 * F + pos) = u0;
                il_at(sh, 4 * F + pos) = du;
            }
        }
        const uint64_t wf = wave_sum64(found), wm = wave_sum64(mf), ws = wave_sum64(strips);
        if (lane_id() == 0) {
            sh.red[0][wave_id()] = wf;
            sh.red[1][wave_id()] = wm;
            sh.red[2][wave_id()] = ws;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            found = mf = strips = 0;
            for (uint32_t w = 0; w < num_waves(); ++w) {
                found += sh.red[0][w];
                mf += sh.red[1][w];
                strips += sh.red[2][w];
            }
        }
    }
    uint32_t res = 0;
    bool il = false;
    if (threadIdx.x == 0) {
        x.level() = 0;
        x.nf_prev() = 1;
        x.m_visited_lo() = deg;
        x.m_visited_hi() = 0;
        x.lvl_found() = 0;
        x.lvl_mf_lo() = x.lvl_mf_hi() = 0;
        t.work->heavy_tail = 0;
        if (!inline_l0) {
            res = kPhTD;                        // rotation 0: current = fb[0]
        } else {
            x.levels_total() += 1;
            x.td_levels() += 1;
            // the level's work in the cumulative statistics (slot of id 0)
            uint64_t* s0 = reinterpret_cast<uint64_t*>(t.slots);
            add_nr64(&s0[kSlotArcs], deg);
            add_nr64(&s0[kSlotRows], 1 + found);
            if (found) add_nr64(&s0[kSlotFoundAll], found);
            if (found == 0) {
                x.root() += 1;
                res = x.root() >= t.nroots ? kFlagDone : (kPhInit | kFlagAdv);
            } else {
                const uint64_t mv = (uint64_t)deg + mf;
                x.m_visited_lo() = (uint32_t)mv;
                x.m_visited_hi() = (uint32_t)(mv >> 32);
                const uint64_t m_u = p.total_arcs > mv ? p.total_arcs - mv : 0;
                const uint32_t nph = (p.direction_opt && mf * p.alpha > m_u) ? kPhBU : kPhTD;
                x.nf_prev() = (uint32_t)found;
                x.level() = 1;
                res = nph | kFlagAdv | (1u << kRotShift) |   // level 1: current = fb[1]
                      (Small && p.flist && (mf <= kRecordArcs || !p.direction_opt) ? kFlagRecord : 0u);
                il = Small && p.inline_on && mf <= (uint64_t)kInlineLevelArcs * blockDim.x;
                if (strips && !il) {
                    // the strips stay queued for a top-down level 1 (a
                    // bottom-up one does not walk the frontier's lists)
                    x.in_size() = (uint32_t)strips;
                    if (nph == kPhTD) res |= kFlagPreSplit;
                    if (strips > t.heavy_cap) {
                        raise_error(c, kErrInternal);
                        res |= kFlagAbort;
                    }
                }
            }
        }
        // level 1 is small: the master step runs it (and what follows),
        // from frontier list 0 (the caller runs the levels)
        sh.il_go = il ? 1u : 0u;
        sh.il_v[0] = 0;             // strips placed so far (positions from 0: the list is empty)
        sh.il_v[1] = 1;             // the list's level
        sh.il_v[2] = 0;             // rotation: level 1 is all of fb[1], fb[2] is clear
        sh.il_v[3] = sh.mb[3];      // source index
        sh.il_v[4] = 0;             // no found lists to gather
    }
    __syncthreads();
    if (!sh.il_go && won && du > t.heavy_th) {
        const uint32_t ns = (du + t.strip - 1) / t.strip;
        const uint32_t b = atomicAdd(&sh.il_v[0], ns);
        for (uint32_t j = 0; j < ns; ++j) {
            const uint32_t off = j * t.strip;
            if (b + j < t.heavy_cap) t.heavy[b + j] = make_uint4(0u, u0 + off, du - off < t.strip ? du - off : t.strip, u);
        }
    }
    return res;
}

// The small levels a master step runs (all threads of the master
// workgroup; the way in is in sh.il_*: the frontier in list 0 or in the
// phase's found lists, its level, rotation and source). Thread 0 publishes
// the release flags and the transmit block; a gather that cannot take the
// lists changes nothing. Only the BFS kernel built with small levels runs
// it: its code in a kernel costs the phases' loops some registers (a few
// percent on R-MAT), so launches that give every level a barrier use a
// build without it.
__device__ __forceinline__ void bfs_small_levels(BlockLds& sh, uint32_t M, uint32_t* vis, uint32_t* fb0, uint32_t* fb1,
                                              uint32_t* fb2, const uint32_t* col, const uint32_t* row_ptr,
                                              uint32_t* slots, const uint32_t* flist, uint32_t* lvl_base,
                                              uint32_t out_stride, uint64_t total_arcs, uint32_t alpha,
                                              uint32_t direction_opt, uint32_t nroots, Work* work) {
    const uint32_t nf = __builtin_amdgcn_readfirstlane(sh.il_c[0]);
    const uint32_t lvl = __builtin_amdgcn_readfirstlane(sh.il_v[1]);
    const uint32_t r = __builtin_amdgcn_readfirstlane(sh.il_v[2]);
    const uint32_t root = __builtin_amdgcn_readfirstlane(sh.il_v[3]);
    const bool gather = __builtin_amdgcn_readfirstlane(sh.il_v[4]) != 0;
    if (gather && !il_gather(sh, flist, row_ptr, M, nf)) return;
    const IlArgs q{vis, r == 0 ? fb1 : (r == 1 ? fb2 : fb0), col, row_ptr, slots,
                   lvl_base + (size_t)root * out_stride, total_arcs, alpha, direction_opt, nroots,
                   flist != nullptr ? 1u : 0u};
    const uint32_t res = bfs_inline_levels(q, sh, sh.il_x, nf, lvl, r);
    if (threadIdx.x == 0) {
        sh.bar.flags = res;
        work->store_x(sh.il_x);
    }
}

// BFS master step (all threads of the master workgroup): per-level
// bookkeeping, HEAVY follow-up, direction of the next level (Beamer's
// alpha/beta rule), next source or done. `roots` / `lvl_base`: the sources
// and the output (the launch's, or a served query's). Returns the release
// flags.
template <bool Small = false>
__device__ __forceinline__ uint32_t bfs_master(const BfsArgs& p, BlockLds& sh, CtxCore* c, uint32_t ph,
                                               uint32_t cur_flags, const uint32_t* roots, uint32_t* lvl_base,
                                               uint32_t M) {
    const TraversalArgs& t = p.t;
    Work* wk = t.work;
    // thread 0 loads the transmit block before the slot sums, so both round
    // trips overlap (the values stay undefined in the other threads)
    XferR x;
    uint32_t hs;
    if (threadIdx.x == 0) {
        x = wk->load_x();
        hs = ld_relaxed(&wk->heavy_tail);
    }
    // the phase's found and mf: from the barrier arrivals, or as the growth
    // of the slot sums
    uint64_t tot[2] = {0, 0};
    if (!p.arrive_sums) master_sum_slots(sh, t.slots, t.N, tot);
    if (ph == kPhInit) {
        const uint32_t res = bfs_master_source<Small>(p, sh, c, x, roots, lvl_base);
        if (threadIdx.x == 0) {
            sh.bar.flags = res;
            wk->store_x(x);
            if (sh.il_go) sh.il_x = x;
        }
    }
    bool il = false;
    if (ph != kPhInit && threadIdx.x == 0) {
        uint32_t res = 0;
        const uint32_t r = (cur_flags & kRotMask) >> kRotShift;
        if (ph == kPhStart) {
            x.root() = 0;
            res = kPhInit;
        } else {
            // this phase's finds: the growth of the slot sums (modulo 2^32:
            // a level finds fewer vertices and arcs than that); level
            // partials (a TD level may be followed by a HEAVY phase)
            uint32_t d_found, d_mf;
            if (p.arrive_sums) {
                d_found = sums_a(sh.bar.sums);
                d_mf = sums_b(sh.bar.sums);
            } else {
                d_found = (uint32_t)tot[0] - x.sum_found();
                d_mf = (uint32_t)tot[1] - x.sum_mf();
                x.sum_found() = (uint32_t)tot[0];
                x.sum_mf() = (uint32_t)tot[1];
            }
            const uint64_t mf_lvl = join64(x.lvl_mf_lo(), x.lvl_mf_hi()) + d_mf;
            const uint32_t nf_lvl = x.lvl_found() + d_found;
            if (ph == kPhTD && hs > 0) {
                x.in_size() = hs;
                wk->heavy_tail = 0;
                x.lvl_found() = nf_lvl;
                x.lvl_mf_lo() = (uint32_t)mf_lvl;
                x.lvl_mf_hi() = (uint32_t)(mf_lvl >> 32);
                x.heavy_phases() += 1;
                res = (cur_flags & kRotMask) | kPhHeavy;
                if (hs > t.heavy_cap) {                 // the strip list overflowed
                    raise_error(c, kErrInternal);
                    res |= kFlagAbort;
                }
            } else {
                x.lvl_found() = 0;
                x.lvl_mf_lo() = x.lvl_mf_hi() = 0;
                if (hs) wk->heavy_tail = 0;
                x.levels_total() += 1;
                if (ph == kPhBU) x.bu_levels() += 1; else x.td_levels() += 1;
                if (nf_lvl == 0) {
                    x.root() += 1;
                    res = x.root() >= t.nroots ? kFlagDone : (kPhInit | kFlagAdv);
                } else {
                    // direction of the next level
                    const uint64_t mv = join64(x.m_visited_lo(), x.m_visited_hi()) + mf_lvl;
                    x.m_visited_lo() = (uint32_t)mv;
                    x.m_visited_hi() = (uint32_t)(mv >> 32);
                    const uint64_t m_u = p.total_arcs > mv ? p.total_arcs - mv : 0;
                    uint32_t nph = kPhTD;
                    if (p.direction_opt) {
                        if (ph == kPhBU)
                            nph = ((uint64_t)nf_lvl * p.beta < t.n && nf_lvl < x.nf_prev()) ? kPhTD : kPhBU;
                        else
                            nph = (mf_lvl * p.alpha > m_u) ? kPhBU : kPhTD;
                    }
                    x.nf_prev() = nf_lvl;
                    x.level() += 1;
                    res = nph | kFlagAdv | (((r + 1) % 3) << kRotShift);
                    // a frontier with few arcs finds few vertices: its phase
                    // lists them (top-down-only launches do not sum mf and
                    // always list)
                    if (Small && p.flist && (mf_lvl <= kRecordArcs || !p.direction_opt)) res |= kFlagRecord;
                    // a small level next: the master step may run it (the
                    // phase's found lists hold the frontier; a HEAVY phase
                    // rewrote them with its own finds only). The gather
                    // checks the arcs that top-down-only launches do not sum.
                    il = Small && p.inline_on && p.flist && (cur_flags & kFlagRecord) && ph != kPhHeavy &&
                         nf_lvl <= il_cap(num_waves()) && mf_lvl <= (uint64_t)kInlineLevelArcs * blockDim.x;
                    sh.il_c[0] = nf_lvl;
                    sh.il_v[1] = x.level();
                    sh.il_v[2] = r;
                    sh.il_v[3] = x.root();
                    sh.il_v[4] = 1;     // the frontier is in the phase's found lists
                }
            }
        }
        sh.bar.flags = res;
        sh.il_go = il ? 1u : 0u;
        // the transmit block as it stands; the levels below work on an
        // LDS copy (no registers held through them) and store it again
        wk->store_x(x);
        if (il) sh.il_x = x;
    }
    __syncthreads();
    if constexpr (Small) {
        // small levels in the master step (one call site for both ways in)
        if (sh.il_go)
            bfs_small_levels(sh, M, p.vis, p.fb[0], p.fb[1], p.fb[2], t.col, t.row_ptr, t.slots, p.flist,
                             lvl_base, t.out_stride, p.total_arcs, p.alpha, p.direction_opt, t.nroots, wk);
        __syncthreads();
    }
    return sh.bar.flags;
}

// Follow the transmitted BFS state locally after a barrier (JUMP: the
// master step ran levels itself, the level is the transmit block's).
__device__ __forceinline__ void bfs_follow(uint32_t ph, uint32_t nflags, uint32_t& level, uint32_t& root,
                                           const Work* wk) {
    const uint32_t nph = nflags & kPhMask;
    if (nph == kPhInit) {
        if (ph != kPhStart) root += 1;
        level = 0;
    } else if (nflags & kFlagJump) {
        level = __hip_atomic_load(&wk->x.level, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (ph == kPhInit) {
        level = (nflags & kFlagAdv) ? 1u : 0u;   // ADV: the master step expanded level 0 itself
    } else if (nflags & kFlagAdv) {
        level += 1;
    }
}

// ----------------------------------------------------------------- SSSP

constexpr uint32_t kRelaxBatch = 8;        // SSSP relaxations in flight per lane

// Frontier Bellman-Ford on the BFS engine's frontier bitmaps. The distances
// live in the output array itself (INT32_MAX = unreached); a round expands
// the vertices of the current bitmap and a relaxation that lowers dist[u]
// sets u in the next bitmap, so no queue, no reservation and no per-vertex
// round stamp are needed (setting a bit twice is harmless).
struct SsspVisit {
    uint32_t* dist;         // distances of the current source
    const uint32_t* w;
    uint32_t* nxt;          // frontier bitmap of the next round
    CtxCore* ctx;

    // a value read while other workgroups lower it can only be too large:
    // the relaxation is then weaker, and the vertex is in the next round's
    // bitmap anyway (whoever lowered it set its bit)
    __device__ __forceinline__ uint32_t payload(uint32_t v) const { return dist[v]; }
    __device__ __forceinline__ uint32_t strip_payload(uint32_t, uint32_t v) const { return payload(v); }
    __device__ __forceinline__ void maybe_flush(WaveLds&) {}

    // The arcs that would lower their target (by a plain probe) are decided
    // for the whole step first; each issues its atomic minimum and marks its
    // target in the next bitmap without waiting for either. Marking on the
    // probe is exact: the probe read this round's value or a later (lower)
    // one, so a candidate below it means the target's distance dropped in
    // this round, by this relaxation or by one that marked it as well; a
    // candidate not below it cannot lower the target.
    __device__ __forceinline__ void step(const bool* ok, const uint32_t* arc, const uint32_t* u,
                                         const uint32_t* pay, WaveLds&, Stats& st) {
        uint32_t wt[kUnroll];
        uint32_t du[kUnroll];
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) wt[j] = ok[j] ? __builtin_nontemporal_load(&w[arc[j]]) : 0u;
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) du[j] = ok[j] ? dist[u[j]] : 0u;
        uint32_t nd[kUnroll];
        bool tr[kUnroll], ovf = false;
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) {
            const uint64_t nd64 = (uint64_t)pay[j] + (uint64_t)wt[j];
            const bool big = nd64 >= 0x7FFFFFFFull;
            ovf |= ok[j] && big && pay[j] != 0x7FFFFFFFu;
            nd[j] = (uint32_t)nd64;
            tr[j] = ok[j] && !big && nd[j] < du[j];
        }
        if (ovf) raise_error(ctx, kErrOverflow);
#pragma unroll
        for (uint32_t j = 0; j < kUnroll; ++j) {
            if (tr[j]) {
                (void)__hip_atomic_fetch_min(&dist[u[j]], nd[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                (void)__hip_atomic_fetch_or(&nxt[u[j] >> 5], 1u << (u[j] & 31), __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
                st.found += 1;
            }
        }
    }
};

// One SSSP phase for member `id` of `M`: INIT sets the source's distances
// to unreached and clears the bitmaps, TD relaxes the arcs of the vertices
// in the current bitmap (one-word units) and clears the bitmap two rounds
// ahead, HEAVY walks strips of heavy vertices. A workgroup that lowered any
// distance raises the round's "next bitmap not empty" word.
// Returns (thread 0) the workgroup's arrival payload when the launch takes
// the round's outcome that way: 1 in the first sum if it lowered a distance.
__device__ __forceinline__ uint64_t sssp_phase(const SsspArgs& p, BlockLds& sh, uint32_t ph, uint32_t flags,
                                               int32_t* dist_i, uint32_t id, uint32_t M) {
    const TraversalArgs& t = p.t;
    Work* wk = t.work;
    const uint32_t nw = num_waves();
    uint32_t* dist = reinterpret_cast<uint32_t*>(dist_i);
    const uint32_t rot = (flags & kRotMask) >> kRotShift;
    uint32_t* cur = p.fb[rot];
    uint32_t* nxt = p.fb[(rot + 1) % 3];
    uint32_t* spare = p.fb[(rot + 2) % 3];
    const uint32_t gw = wave_slot(id, M, nw);
    const uint32_t W = M * nw;
    Stats st;
    uint64_t pay = 0;
    if (ph == kPhInit) {
        const uint32_t tid = id * blockDim.x + threadIdx.x, stride = M * blockDim.x;
        for (uint32_t i = tid; i < t.n; i += stride) dist[i] = 0x7FFFFFFFu;
        for (uint32_t i = tid; i < p.words; i += stride) {
            p.fb[0][i] = 0;
            p.fb[1][i] = 0;
            p.fb[2][i] = 0;
        }
    } else if (ph == kPhTD || ph == kPhHeavy) {
        SsspVisit vis{dist, t.w, nxt, t.ctx};
        WaveLds& w = sh.wave[wave_id()];
        if (ph == kPhTD) {
            clear_share(spare, p.words, gw, W);
            expand_bitmap(t, wk, w, cur, p.words, gw, W, vis, st);
        } else {
            heavy_phase(t, wk->x.in_size, gw, W, w, vis, st);
        }
        stats_to_lds(sh, st);
        __syncthreads();
        // one flag per XCD: a single shared word took every workgroup's
        // store in turn at the end of the round (or a count on the arrivals)
        if (threadIdx.x == 0 && sh.acc[0]) {
            if (p.arrive_sums) pay = arrive_payload(1u, 0u);
            else __hip_atomic_store(&p.lowered[xcc_id() * 64u], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        acc_to_slot(sh, t.slots, id, false);
    }
    return pay;
}

// SSSP master step: place the next source, switch a round to its HEAVY
// phase, or end the round: the next bitmap becomes the current one, or, if
// no distance was lowered, the source is finished and the next one starts.
// `roots` / `dist_base`: the sources and the distances (the launch's, or a
// served query's). Returns the release flags.
__device__ __forceinline__ uint32_t sssp_master(const SsspArgs& p, BlockLds& sh, CtxCore* c, uint32_t ph,
                                                uint32_t cur_flags, const uint32_t* roots, int32_t* dist_base) {
    const TraversalArgs& t = p.t;
    Work* wk = t.work;
    if (threadIdx.x == 0) {
        XferR x = wk->load_x();                 // one batch of loads
        const uint32_t hs = ld_relaxed(&wk->heavy_tail);
        uint32_t lw[kMaxXcds];
        uint32_t lowered = 0;
        if (p.arrive_sums) {
            // workgroups that lowered a distance in this phase, counted by
            // the arrivals (a TD phase's count waits in lvl_found while its
            // HEAVY phase runs)
#pragma unroll
            for (uint32_t i = 0; i < kMaxXcds; ++i) lw[i] = 0;
            lowered = sums_a(sh.bar.sums);
        } else {
#pragma unroll
            for (uint32_t i = 0; i < kMaxXcds; ++i) lw[i] = ld_relaxed(&p.lowered[i * 64u]);
#pragma unroll
            for (uint32_t i = 0; i < kMaxXcds; ++i) lowered |= lw[i];
        }
        const uint32_t r = (cur_flags & kRotMask) >> kRotShift;
        uint32_t res;
        if (ph == kPhStart) {
            x.root() = 0;
            res = kPhInit;
        } else if (ph == kPhInit) {
            const uint32_t src = roots[x.root()];
            if (src >= t.n) {                   // as in BFS: fail before any write
                raise_error(c, kErrInvalid);
                res = kFlagAbort;
            } else {
                int32_t* d = dist_base + (size_t)x.root() * t.out_stride;
                d[src] = 0;
                p.fb[0][src >> 5] = 1u << (src & 31);
                x.level() = 0;
#pragma unroll
                for (uint32_t i = 0; i < kMaxXcds; ++i) p.lowered[i * 64u] = 0;
                wk->heavy_tail = 0;
                res = kPhTD;                    // rotation 0: current = fb[0]
            }
        } else if (ph == kPhTD && hs > 0) {
            x.in_size() = hs;
            wk->heavy_tail = 0;
            x.heavy_phases() += 1;
            if (p.arrive_sums) x.lvl_found() = lowered;   // the HEAVY phase's master adds it
            res = (cur_flags & kRotMask) | kPhHeavy;
            if (hs > t.heavy_cap) {                     // the strip list overflowed
                raise_error(c, kErrInternal);
                res |= kFlagAbort;
            }
        } else {
            if (hs) wk->heavy_tail = 0;
            if (p.arrive_sums) {
                lowered += x.lvl_found();
                x.lvl_found() = 0;
            }
#pragma unroll
            for (uint32_t i = 0; i < kMaxXcds; ++i)
                if (lw[i]) p.lowered[i * 64u] = 0;
            x.level() += 1;
            x.levels_total() += 1;
            if (!lowered) {
                x.root() += 1;
                res = x.root() >= t.nroots ? kFlagDone : (kPhInit | kFlagAdv);
            } else {
                res = kPhTD | kFlagAdv | (((r + 1) % 3) << kRotShift);
            }
        }
        wk->store_x(x);
        sh.bar.flags = res;
    }
    __syncthreads();
    return sh.bar.flags;
}

// Follow the transmitted SSSP state locally after a barrier: the source
// index advances when a new source starts.
__device__ __forceinline__ void sssp_follow(uint32_t ph, uint32_t nflags, uint32_t& root) {
    if ((nflags & kPhMask) == kPhInit && ph != kPhStart) root += 1;
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

// Arcs a lane takes at a time in the colouring walks: their loads are all
// issued before any is used (a lane's walk of a 32-arc list is then four
// round trips per step instead of thirty-two).
constexpr uint32_t kColorBatch = 8;

// OR of x over a lane group: G consecutive lanes, G a power of two that
// divides the wave.
__device__ __forceinline__ uint32_t group_or32(uint32_t x, uint32_t G) {
    for (uint32_t o = 1; o < G; o <<= 1) x |= __shfl_xor(x, o, kWave);
    return x;
}
__device__ __forceinline__ uint64_t group_or64(uint64_t x, uint32_t G) {
    for (uint32_t o = 1; o < G; o <<= 1) x |= __shfl_xor(x, o, kWave);
    return x;
}

// Decide frontier vertex v (its higher-priority neighbours are all decided):
// the smallest colour none of them has, or (MIS) whether none of them is in
// the set. The vertex's G lanes (consecutive lanes, G a power of two) take
// its arcs sub, sub + G, ... kColorBatch at a time (their loads in flight
// together) and OR their findings across the group; the group's first lane
// writes the result. Every lane of the wave makes the call (`valid` false:
// no vertex), so the group reductions see all of their lanes.
__device__ __forceinline__ void color_vertex(const ColorArgs& p, uint32_t v, bool valid, uint32_t sub, uint32_t G,
                                             Stats& st) {
    const uint64_t hv = valid ? key_hash(p.prio_seed, v) : 0;
    const uint32_t a0 = valid ? p.t.row_ptr[v] : 0, a1 = valid ? p.t.row_ptr[v + 1] : 0;
    if (valid && sub == 0) {
        st.rows += 1;
        st.arcs += a1 - a0;
    }
    const uint32_t step = G * kColorBatch;
    if (p.mis) {
        uint32_t blocked = 0;
        for (uint32_t e0 = a0 + sub; e0 < a1 && !blocked; e0 += step) {
            uint32_t u[kColorBatch];
            uint8_t in[kColorBatch];
#pragma unroll
            for (uint32_t j = 0; j < kColorBatch; ++j) u[j] = e0 + j * G < a1 ? p.t.col[e0 + j * G] : 0xFFFFFFFFu;
#pragma unroll
            for (uint32_t j = 0; j < kColorBatch; ++j) {
                in[j] = 0;
                if (u[j] != 0xFFFFFFFFu && key_higher(key_hash(p.prio_seed, u[j]), u[j], hv, v))
                    in[j] = p.in_set_out[u[j]];
            }
#pragma unroll
            for (uint32_t j = 0; j < kColorBatch; ++j) blocked |= in[j] != 0 ? 1u : 0u;
        }
        blocked = group_or32(blocked, G);
        if (valid && sub == 0) p.in_set_out[v] = blocked ? 0 : 1;
    } else {
        uint32_t base = 0, c = 0;
        for (;;) {
            uint64_t used = 0;
            for (uint32_t e0 = a0 + sub; e0 < a1; e0 += step) {
                uint32_t u[kColorBatch], cu[kColorBatch];
#pragma unroll
                for (uint32_t j = 0; j < kColorBatch; ++j) u[j] = e0 + j * G < a1 ? p.t.col[e0 + j * G] : 0xFFFFFFFFu;
#pragma unroll
                for (uint32_t j = 0; j < kColorBatch; ++j) {
                    cu[j] = 0xFFFFFFFFu;           // no colour is that large
                    if (u[j] != 0xFFFFFFFFu && key_higher(key_hash(p.prio_seed, u[j]), u[j], hv, v))
                        cu[j] = p.colour_out[u[j]];
                }
#pragma unroll
                for (uint32_t j = 0; j < kColorBatch; ++j) {
                    const uint32_t d = cu[j] - base;
                    if (cu[j] != 0xFFFFFFFFu && d < 64) used |= 1ull << d;
                }
            }
            // the whole wave takes the same number of windows: a group that
            // still needs one more keeps every lane of the wave in the loop
            used = group_or64(used, G);
            const bool need = ~used == 0;
            if (!need) c = base + (uint32_t)__ffsll((long long)~used) - 1;
            if (!__ballot(valid && need)) break;
            if (need) base += 64;
        }
        if (valid && sub == 0) p.colour_out[v] = c;
    }
}

// Release the lower-priority neighbours of v; one whose count of undecided
// higher neighbours reaches 0 is queued for the next round. The vertex's G
// lanes take its arcs as in color_vertex, kColorBatch at a time: their
// loads, then their decrements, issued back to back.
__device__ __forceinline__ void release_lower(const ColorArgs& p, uint32_t v, bool valid, uint32_t sub, uint32_t G,
                                              WaveLds& w, uint32_t* out_tail, uint32_t* out, Stats& st) {
    const uint64_t hv = valid ? key_hash(p.prio_seed, v) : 0;
    uint32_t e = valid ? p.t.row_ptr[v] + sub : 0;
    const uint32_t a1 = valid ? p.t.row_ptr[v + 1] : 0;
    for (;;) {
        const bool more = e < a1;
        if (!__ballot(more)) break;
        uint32_t u[kColorBatch], old[kColorBatch];
        bool lower[kColorBatch];
#pragma unroll
        for (uint32_t j = 0; j < kColorBatch; ++j) u[j] = e + j * G < a1 ? p.t.col[e + j * G] : 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t j = 0; j < kColorBatch; ++j) {
            lower[j] = u[j] != 0xFFFFFFFFu && !key_higher(key_hash(p.prio_seed, u[j]), u[j], hv, v);
            old[j] = 0;
            if (lower[j])
                old[j] = __hip_atomic_fetch_sub(&p.pending[u[j]], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (uint32_t j = 0; j < kColorBatch; ++j) {
            const bool win = lower[j] && old[j] == 1;
            st.found += win ? 1u : 0u;
            wave_push(w, win, u[j]);
            if (w.out_n > kFlushAt) wave_flush(w, out_tail, out);
        }
        e += G * kColorBatch;
    }
}

// Colouring / MIS: SETUP counts every vertex's higher-priority neighbours
// and queues the sources of the priority DAG; each round decides its
// frontier and releases the next one.
// One colouring/MIS phase for member `id` of `M`: SETUP counts every
// vertex's higher-priority neighbours and queues the sources of the
// priority DAG; TD decides the round's frontier and releases the next one.
__device__ __forceinline__ void color_phase(const ColorArgs& p, BlockLds& sh, uint32_t ph, uint32_t flags,
                                            uint32_t id, uint32_t M) {
    const TraversalArgs& t = p.t;
    Work* wk = t.work;
    const uint32_t nw = num_waves();
    const bool sel = (flags & kFlagSel) != 0;
    uint32_t* in = t.frontier[sel ? 1 : 0];
    uint32_t* out = t.frontier[sel ? 0 : 1];
    const uint32_t gw = wave_slot(id, M, nw);
    const uint32_t W = M * nw;
    WaveLds& w = sh.wave[wave_id()];
    Stats st;
    if (ph == kPhSetup) {
        const uint32_t units = (t.n + kWave - 1) / kWave;
        for (uint32_t u = gw; u < units; u += W) {
            const uint32_t v = u * kWave + lane_id();
            const bool valid = v < t.n;
            uint32_t cnt = 0;
            if (valid) {
                const uint64_t hv = key_hash(p.prio_seed, v);
                const uint32_t a1 = t.row_ptr[v + 1];
                for (uint32_t e0 = t.row_ptr[v]; e0 < a1; e0 += kColorBatch) {
                    uint32_t x[kColorBatch];
#pragma unroll
                    for (uint32_t j = 0; j < kColorBatch; ++j) x[j] = e0 + j < a1 ? t.col[e0 + j] : 0xFFFFFFFFu;
#pragma unroll
                    for (uint32_t j = 0; j < kColorBatch; ++j)
                        cnt += (x[j] != 0xFFFFFFFFu && key_higher(key_hash(p.prio_seed, x[j]), x[j], hv, v)) ? 1u : 0u;
                }
                p.pending[v] = cnt;
            }
            wave_push(w, valid && cnt == 0, v);
            if (w.out_n > kFlushAt) wave_flush(w, &wk->out_tail, out);
        }
        wg_flush(sh, &wk->out_tail, out);
    } else if (ph == kPhTD) {
        if (threadIdx.x == 0) sh.in_size = wk->x.in_size;
        __syncthreads();
        const uint32_t size = sh.in_size;
        // G consecutive lanes per frontier vertex (G divides the wave)
        const uint32_t G = p.lanes == 2 || p.lanes == 4 || p.lanes == 8 ? p.lanes : 1u;
        const uint32_t lg = __builtin_ctz(G);
        const uint32_t per = kWave >> lg;
        const uint32_t units = (size + per - 1) >> (6 - lg);
        for (uint32_t u = gw; u < units; u += W) {
            const uint32_t i = u * per + (lane_id() >> lg);
            const uint32_t sub = lane_id() & (G - 1);
            const bool valid = i < size;
            const uint32_t v = valid ? in[i] : 0u;
            color_vertex(p, v, valid, sub, G, st);
            release_lower(p, v, valid, sub, G, w, &wk->out_tail, out, st);
        }
        wg_flush(sh, &wk->out_tail, out);
        stats_to_lds(sh, st);
        __syncthreads();
        acc_to_slot(sh, t.slots, id, false);
    }
}

// Colouring master step: the output queue of the round becomes the input
// of the next; an empty queue ends the run.
__device__ __forceinline__ uint32_t color_master(const ColorArgs& p, BlockLds& sh, uint32_t ph, uint32_t cur_flags) {
    const TraversalArgs& t = p.t;
    Work* wk = t.work;
    if (threadIdx.x == 0) {
        XferR x = wk->load_x();
        const uint32_t ot = ld_relaxed(&wk->out_tail);
        uint32_t res;
        if (ph == kPhStart) {
            if (ot) wk->out_tail = 0;
            res = kPhSetup;           // SETUP writes buffer 1 (sel = 0)
        } else {
            wk->out_tail = 0;
            x.in_size() = ot;
            x.level() += 1;
            x.levels_total() += 1;
            res = ot == 0 ? kFlagDone : (((cur_flags & kFlagSel) ^ kFlagSel) | kPhTD | kFlagAdv);
        }
        wk->store_x(x);
        sh.bar.flags = res;
    }
    __syncthreads();
    return sh.bar.flags;
}

}  // namespace
