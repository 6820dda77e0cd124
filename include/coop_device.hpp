// Device-side cooperative-kernel primitives for gfx950 (HIP).
//
// This header is what a cooperative kernel includes. It implements the
// primitives of the cooperative-kernels programming model (paper section
// "Semantics of Cooperative Kernels"): a workgroup-count M that can shrink
// and grow between 1 and the launch limit N, offer_kill (a workgroup offers
// to leave), request_fork (waiting workgroups join), get_num_groups (current
// M), global_barrier and resizing_global_barrier, plus the scheduler query
// of the paper's efficient resizing barrier (section "Scheduler Design").
//
// Design on MI355X (not the paper's OpenCL megakernel):
//  * One long-lived persistent kernel. Every launched workgroup registers by
//    ticket; ticket 0 becomes logical workgroup 0 (M starts at 1) and every
//    other workgroup -- including those dispatched late and those of a
//    separately launched "joiner" grid -- waits in a joiner queue and is
//    admitted at a barrier. The barrier therefore only ever waits for
//    workgroups that are running, whatever the hardware made resident.
//  * The barrier is a counter in HBM: each workgroup's thread 0 adds 1 with
//    agent-scope release; the last arrival (count == M) runs the critical
//    section ("master step") with all of its threads while everybody else is
//    parked, then publishes one 64-bit release word {epoch, M', flags}.
//  * In the master step: per-level bookkeeping (a callback), fork = admit up
//    to k in [0, N-M] waiting joiners as ids [M, M+k-1] (the master
//    workgroup's threads admit them in parallel), query = read the scheduler
//    target T (host-written word in pinned memory, or a seeded device-side
//    schedule), and kill = the top W = min(max(0, M+k-T), M+k-1) ids leave.
//    Workgroup 0 is never killed.
//  * Waiters read (epoch, M') as one word. An alive member is needed by the
//    next barrier, so it can never miss an epoch; a waiter that sees the
//    epoch advance by more than one was therefore killed at the epoch it
//    missed. (Reading the count separately would let a slow killed
//    workgroup pick up a later epoch's count and continue with a stale id.)
//  * Launch constants travel as kernel arguments (Cfg), so the master step
//    touches only a few lines of HBM state, loaded in one batch.
//  * Every spin is bounded by a wall-clock watchdog; expiry sets an error
//    and an abort flag that every waiter honours, so the grid always drains.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace coop {

constexpr uint32_t kMaxThreads = 1024;
constexpr uint32_t kMaxWaves = kMaxThreads / 64;
constexpr uint32_t kJoinCap = 8192;          // joiner admission ring
constexpr uint32_t kMaxGroups = 2048;        // launch limit N

// release-word flags
constexpr uint32_t kFlagDone = 1u;          // kernel finished: everybody leaves
constexpr uint32_t kFlagAbort = 2u;         // watchdog fired or error: leave
constexpr uint32_t kFlagRenum = 4u;         // kills chose their victims: read the new id
constexpr uint32_t kFlagFlat = 8u;          // next arrival per workgroup (joiners' XCDs not yet known)
constexpr uint32_t kFlagUser0 = 16u;        // algorithm-specific bits start here

// Cfg::mode bits
constexpr uint32_t kModeCoop = 1u;          // cooperative (resizable) launch
constexpr uint32_t kModePark = 2u;          // killed workgroups re-queue as joiners
constexpr uint32_t kModeRandomSched = 4u;   // device-side seeded kill/fork schedule
constexpr uint32_t kModeRegular = 8u;       // regular resizing barrier: at most one kill per barrier
constexpr uint32_t kModeRelayTarget = 16u;  // the host target is relayed into Ctx::T_seen by the kernel itself
constexpr uint32_t kModeLoseOne = 32u;      // test: the barrier benchmark's last workgroup goes missing
constexpr uint32_t kModeArriveSums = 64u;   // the arrivals carry sums (64-bit counters; else 32-bit adds)

// error codes written to ctx->error (match COOP_E_* of coop.h)
constexpr int32_t kErrInvalid = -1;
constexpr int32_t kErrTimeout = -4;
constexpr int32_t kErrOverflow = -6;
constexpr int32_t kErrInternal = -7;

// Host-written control words (pinned, fine-grained host memory).
struct alignas(64) HostCtl {
    uint32_t target;          // scheduler target T (query), 1..N
    uint32_t pad0[15];
};

// Launch constants (kernel argument; immutable like the paper's kernel
// parameters).
struct Cfg {
    uint32_t N;               // launch limit (max active workgroups)
    uint32_t mode;            // kMode* bits
    uint32_t sched_p16;       // random schedule: P(target changes) * 65536
    uint32_t trace_cap;       // barriers the trace buffer holds
    uint64_t sched_seed;
    uint64_t watchdog_ticks;  // wall-clock ticks before a spin gives up
    HostCtl* host;            // host-written target, or null
    uint64_t* trace;          // optional: 2 words per barrier (master start, publish|flags)
    uint32_t epoch0_wait;     // ticks ticket 0 waits for the grid to register
    uint32_t wgtrace_cap;     // barriers the per-workgroup trace holds
    uint64_t* wgtrace;        // optional: per barrier and logical id, 4 timestamps
    uint32_t engines;         // shader engines workgroups are dealt over (XCDs x engines per XCD)
    uint32_t ses;             // shader engines per XCD
    uint32_t slots_per_engine;  // workgroups of this kernel one shader engine holds at once
    uint32_t join_window;     // joiners that may wait in the admission ring at once (<= kJoinCap - N)
    uint32_t keep;            // task pattern: fewest active workgroups the scheduler leaves (0 = 1)
};

// The shader engine this workgroup runs on, numbered XCD-major: the XCD
// from hardware register XCC_ID (bits 3:0) and the engine inside it from
// HW_ID (bits 15:13). The hardware deals a kernel's workgroups round-robin
// over the XCDs and, inside each XCD, over its shader engines. `ses` is the
// engine count per XCD the runtime observed; an engine index beyond it is
// folded onto the last one, so that id / ses is always the XCD (the arrival
// by XCD counts members with it).
__device__ __forceinline__ uint32_t engine_id(uint32_t ses) {
    const uint32_t xcc = __builtin_amdgcn_s_getreg((3u << 11) | (0u << 6) | 20u) & 0xFu;
    const uint32_t se = (__builtin_amdgcn_s_getreg((31u << 11) | (0u << 6) | 4u) >> 13) & 7u;
    const uint32_t n = ses ? ses : 1u;
    return xcc * n + (se < n ? se : n - 1u);
}
constexpr uint32_t kMaxEngines = 64;
constexpr uint32_t kRelayThread = 64;        // first lane of the second wave
constexpr uint32_t kMaxXcds = 16;

__device__ __forceinline__ uint32_t xcc_id() { return __builtin_amdgcn_s_getreg((3u << 11) | (0u << 6) | 20u) & 0xFu; }

// Per-workgroup phase trace points (debugging and tuning only).
enum WgTracePoint : uint32_t { kTrStart = 0, kTrWorkDone = 1, kTrArrive = 2, kTrReleased = 3 };
__device__ __forceinline__ void wg_trace(const Cfg cfg, uint32_t epoch, uint32_t id, uint32_t point) {
    if (cfg.wgtrace && epoch < cfg.wgtrace_cap && threadIdx.x == 0)
        cfg.wgtrace[((size_t)epoch * cfg.N + id) * 4 + point] = wall_clock64();
}

// Barrier state: the lines every barrier touches. A team of workgroups
// inside a batched launch uses one of these on its own (no joiners).
struct alignas(256) CtxCore {
    // ---- line: barrier arrival counter (per workgroup, or per group of
    //      workgroups in a resizable launch), with the arrivals' sums
    //      (arrive_sums)
    uint64_t arrive;
    uint32_t _pa[62];
    // ---- line: release word {epoch:32 (lo) | M:16 | flags:16 (hi)}
    uint64_t release;
    uint64_t _pr[31];
    // ---- line: registration
    uint32_t ticket;          // start-up tickets
    uint32_t join_tail;       // next joiner slot
    uint32_t join_full;       // joiners that found the admission ring full and left
    uint32_t joined_grid;     // workgroups of joiner grids that started
    uint32_t cohort;          // tickets the first barrier admitted as ids 0 .. cohort-1
    uint32_t _pj[59];
    // ---- line: error and the host target as read by workgroup 0
    int32_t error;
    uint32_t T_seen;
    uint32_t _pe[62];
    // ---- line: master-only scheduler state and statistics
    uint32_t join_head;       // first slot not yet admitted
    uint32_t T_dev;           // device-side target (random schedule)
    uint32_t barriers;
    uint32_t kills;
    uint32_t forks;
    uint32_t resizes;
    uint32_t min_M;
    uint32_t max_M;
    uint32_t final_M;
    uint32_t tail_prev;       // join_tail as the previous barrier's master read it
    uint64_t t_start;
    uint64_t t_end;
    uint32_t _pm[50];
};

// Context of a resizable launch: barrier lines, the joiner admission ring
// (entries {slot:32 (lo) | epoch_lo:16 | id:16 (hi)}), the shader engine of
// every logical id, and the new ids of a barrier that chose its kill victims
// ({epoch_lo:16 (hi) | new id:16 (lo)}, new id 0xFFFF = killed).
// Arrival by XCD. An agent-scope release on gfx950 writes back the XCD's
// whole L2 and an acquire invalidates it; with every workgroup doing both
// on one counter the arrival took about 6 us for 256 workgroups. Instead a
// workgroup waits for its own memory operations (they then sit in its XCD's
// L2), adds to its XCD's counter without a fence, and only the last of each
// XCD releases (one L2 write-back per XCD) on the top counter; the last of
// those is the master. The master keeps the per-XCD member counts of the
// next interval (from engine_of) and sets kFlagFlat for an interval whose
// joiners have not recorded their XCD yet; that interval arrives per
// workgroup with release-acquire as before.
struct alignas(256) ArriveLine {
    uint64_t count;           // arrivals, with their sums (arrive_sums)
    uint32_t _p[62];
};

// A barrier arrival adds one to its counter and, in the same atomic, two
// counts the workgroup brings (an algorithm's per-phase totals, e.g. the
// vertices a BFS level found and their degree sum): the count of arrivals
// in the low 12 bits, a 24-bit and a 28-bit sum above it. The last arrival
// of an XCD gets its XCD's sums from the value its add returns and passes
// them on with its arrival on the top counter, so the master step receives
// the totals of all members without reading anything. The launch must keep
// the sums in range (the host only enables them when they cannot overflow).
constexpr uint32_t kArriveCountBits = 12;                      // up to kMaxGroups arrivals
constexpr uint64_t kArriveCount = (1ull << kArriveCountBits) - 1;
__device__ __forceinline__ uint64_t arrive_payload(uint64_t a24, uint64_t b28) {
    return (a24 << kArriveCountBits) | (b28 << (kArriveCountBits + 24));
}
__device__ __forceinline__ uint32_t sums_a(uint64_t sums) { return (uint32_t)(sums & 0xFFFFFFu); }
__device__ __forceinline__ uint32_t* arrive_lo(uint64_t* counter) { return reinterpret_cast<uint32_t*>(counter); }
__device__ __forceinline__ uint32_t sums_b(uint64_t sums) { return (uint32_t)(sums >> 24); }
struct alignas(256) XcdCounts {
    uint32_t members[kMaxXcds];   // members of this interval per XCD
    uint32_t groups;              // XCDs with members
    uint32_t _p[64 - kMaxXcds - 1];
};

// State of a launch whose kernel calls offer_kill and request_fork directly
// between tasks instead of meeting at resizing barriers (the work-stealing
// pattern of the paper's programming section). Ids are slots in [0, N)
// that a workgroup claims when it becomes active and frees when it leaves,
// so a workgroup can leave whatever its id (kill in any order, Appendix B).
constexpr uint32_t kTransmitWords = 16;
struct alignas(256) TaskState {
    uint32_t active;          // M: active workgroups
    uint32_t kills;           // offers the scheduler accepted
    uint32_t forks;           // joiners that became active
    uint32_t min_active;      // fewest active after a kill
    uint32_t max_active;      // most active
    uint32_t decisions;       // seeded schedule: offers decided so far
    uint32_t join_tickets;    // joiners that asked to come in
    uint32_t join_granted;    // joiners request_fork has let in (tickets below this may enter)
    uint32_t _p[56];
    uint32_t active_x[kMaxEngines];          // active workgroups per shader engine
    uint32_t transmit[kTransmitWords];       // state the last request_fork transmitted
    uint32_t _q[64 - kTransmitWords];
    uint32_t slot_owner[kMaxGroups];         // 1 while a workgroup holds the id
};

struct alignas(256) Ctx : CtxCore {
    uint64_t join_entry[kJoinCap];
    uint32_t engine_of[kMaxGroups];
    uint32_t renum[kMaxGroups];
    ArriveLine xcd_arrive[kMaxXcds];
    XcdCounts xcd;
    uint32_t transmit[64];    // interval pattern: state joiners take over (kTransmitWords used)
    TaskState task;
};

// Launch contexts (not the small per-team ones) arrive by XCD.
template <class C>
constexpr bool kGroupedArrival = std::is_same<C, Ctx>::value;

// ------------------------------------------------------------- atomics

__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_relaxed_i(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_relaxed64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_relaxed(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Fire-and-forget add (the result is unused, so no round trip is waited for).
__device__ __forceinline__ void add_nr64(uint64_t* p, uint64_t v) {
    (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_system(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

__device__ __forceinline__ uint64_t now_ticks() { return wall_clock64(); }

__device__ __forceinline__ uint32_t rel_epoch(uint64_t r) { return (uint32_t)r; }
__device__ __forceinline__ uint32_t rel_M(uint64_t r) { return (uint32_t)(r >> 32) & 0xFFFFu; }
__device__ __forceinline__ uint32_t rel_flags(uint64_t r) { return (uint32_t)(r >> 48); }
__device__ __forceinline__ uint64_t make_release(uint32_t epoch, uint32_t M, uint32_t flags) {
    return (uint64_t)epoch | ((uint64_t)(M & 0xFFFFu) << 32) | ((uint64_t)(flags & 0xFFFFu) << 48);
}

// SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// --------------------------------------------------------------- state

// Workgroup-uniform view of the scheduler state, kept in registers/LDS.
struct Member {
    uint32_t id;        // logical workgroup id in [0, M)
    uint32_t M;         // active workgroups in this resizing-barrier interval
    uint32_t epoch;     // last release epoch observed
    uint32_t flags;     // flags of that release
    uint32_t alive;     // 1 while this workgroup is an active member
    uint32_t xm, xg;    // arrival by XCD: this XCD's members and the XCDs with members,
                        // as last loaded (xg = 0: not loaded since the master recounted)
};

// Whether the master that published `n` (after the interval described by
// `m`) recounted the members per XCD: exactly when the next interval arrives
// by XCD and the membership may have changed.
__device__ __forceinline__ bool counts_changed(const Member& m, const Member& n) {
    if (n.flags & (kFlagDone | kFlagAbort | kFlagFlat)) return false;
    return m.epoch == 0 || (m.flags & kFlagFlat) || n.M != m.M || (n.flags & kFlagRenum);
}

// The scheduler words a master step reads (loaded while the algorithm's
// master step runs).
struct MasterPre {
    int32_t err;
    uint32_t tail, T_seen, join_head, T_dev, nb, kills, forks, resizes, min_M, max_M, tail_prev;
    // the scheduler's decision for a barrier after which the kernel goes on
    // (master_decide); master_schedule sets it aside when the algorithm's
    // flags end the kernel
    uint32_t T, T_dev_new, M0, kmax, drain, quiet;
};

// Workgroup-shared state of the barrier.
struct BarrierLds {
    Member member;
    uint64_t sums;          // master: the arrivals' sums (sums_a / sums_b)
    uint32_t killed;        // this workgroup left because the scheduler claimed it
    uint32_t is_master;     // this workgroup runs the master step
    uint32_t flags;         // master step result (broadcast inside the master)
    uint32_t head, kmax, T;
    uint32_t my_new;                   // placed kill: the master's new id
    uint32_t top_kill;                 // placed kill: no engine owes, the top W ids leave
    uint32_t drain_span, drained;      // ring slots checked for given-up joiners, and how many lead
    uint32_t offers;                   // task pattern: offer_kill calls so far (thread 0)
    uint32_t cut, tail_prev;           // admission: slots taken before the first new unannounced one
    uint32_t m0;                       // members before this barrier's forks (the start-up admission's count)
    uint32_t quiet;                    // the master step changes nothing but the epoch
    uint32_t valid[kMaxGroups / 32];   // admission: ring slots whose joiner was still waiting
    uint32_t xcnt[kMaxEngines];        // placed kill: members per engine, then victims per engine
    uint32_t wsum[kMaxWaves + 1];      // placed kill: survivors per wave of ids
    uint8_t xcd[kMaxGroups];           // placed kill: shader engine of every logical id
    uint8_t renum_alive[kMaxGroups];   // placed kill: 1 if the id survives
};

// Raise the abort flag so every spinning workgroup leaves.
__device__ inline void raise_error(CtxCore* c, int32_t err) {
    atomicCAS(&c->error, 0, err);
    __hip_atomic_fetch_or(&c->release, (uint64_t)kFlagAbort << 48, __ATOMIC_RELEASE,
                          __HIP_MEMORY_SCOPE_AGENT);
}

// Joiner admission ring. Slot s (taken in arrival order from join_tail)
// lives in entry s % kJoinCap as {slot:32 (lo) | tag:32 (hi)}; the tag is
// an admission {epoch_lo:16 | id:16 (hi)} or one of the states below. A
// joiner announces itself (waiting) with a compare-and-swap, and gives up by
// turning its own waiting entry into withdrawn; the master turns a waiting
// entry into an admission with a compare-and-swap and closes any other slot
// it passes (consumed), so a slot counts as a member only if its joiner was
// still waiting, and a joiner that announces too late sees that it was
// passed. Nothing else bounds how many joiners take slots between two
// admissions (under a co-task, surplus joiner workgroups the hardware starts
// late take slots and withdraw while the target leaves no room), so a joiner
// whose slot lies more than the ring's window ahead of the master's head
// leaves at once without touching the ring: its entry may still belong to
// an older slot. The window keeps one barrier's worth of slots (at most N)
// back, so the entries of joiners admitted at the last barrier, whose final
// ids they read after the release, are not reused under them; for the same
// reason the master passes given-up slots without admitting (a drain) only
// at barriers that admit nobody.
constexpr uint32_t kTagWithdrawn = 0xFFFFFFFFu;
constexpr uint32_t kTagWaiting = 0xFFFFFFFEu;
constexpr uint32_t kTagConsumed = 0xFFFFFFFDu;
constexpr uint32_t kDrainMin = 64;           // queued slots before the master drains given-up ones
__device__ __forceinline__ uint64_t ring_entry(uint32_t slot, uint32_t tag) {
    return (uint64_t)slot | ((uint64_t)tag << 32);
}
__device__ __forceinline__ uint64_t admit_entry(uint32_t slot, uint32_t epoch, uint32_t id) {
    return (uint64_t)slot | ((uint64_t)(epoch & 0xFFFFu) << 32) | ((uint64_t)id << 48);
}
__device__ __forceinline__ bool cas64(uint64_t* p, uint64_t& expected, uint64_t desired) {
    return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
}

// Master side of one slot: admit its joiner as `id` if it is waiting, else
// close the slot. Returns true if admitted. Terminates: every failed
// compare-and-swap means the joiner moved its entry on (announced, or
// withdrew), which it does at most twice.
__device__ inline bool ring_admit(uint64_t* ent, uint32_t slot, uint32_t epoch, uint32_t id) {
    uint64_t cur = __hip_atomic_load(ent, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (cur == ring_entry(slot, kTagWithdrawn) || cur == ring_entry(slot, kTagConsumed)) return false;
        if (cur == ring_entry(slot, kTagWaiting)) {
            if (cas64(ent, cur, admit_entry(slot, epoch, id))) return true;
        } else if (cas64(ent, cur, ring_entry(slot, kTagConsumed))) {
            return false;   // not announced (yet, or ever): passed
        }
    }
}

// Wait for the release word to move past `epoch` (or abort/done). Returns
// the word. Bounded by the watchdog.
__device__ inline uint64_t wait_release(CtxCore* c, const Cfg cfg, uint32_t epoch) {
    const uint64_t t0 = now_ticks();
    uint32_t spins = 0;
    for (;;) {
        const uint64_t r = ld_relaxed64(&c->release);
        if (rel_epoch(r) != epoch || (rel_flags(r) & (kFlagAbort | kFlagDone))) return r;
        if (++spins > 32) {
            __builtin_amdgcn_s_sleep(1);
            if ((spins & 255) == 0) {
                if (ld_relaxed_i(&c->error)) return r | ((uint64_t)kFlagAbort << 48);
                if (now_ticks() - t0 > cfg.watchdog_ticks) {
                    raise_error(c, kErrTimeout);
                    return ld_relaxed64(&c->release) | ((uint64_t)kFlagAbort << 48);
                }
            }
        }
    }
}

// Joiner queue (thread 0 only): wait until admitted at a barrier, until
// the kernel is done, or until giving the compute unit back because the
// scheduler target leaves no room (host-driven schedule only), the
// admission ring is full or the watchdog expires.
__device__ inline Member join_queue(Ctx* c, const Cfg cfg) {
    Member m{};
    m.alive = 0;
    const uint32_t slot = add_relaxed(&c->join_tail, 1u);
    uint64_t* ent = &c->join_entry[slot % kJoinCap];
    if (slot - __hip_atomic_load(&c->join_head, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= cfg.join_window) {
        add_relaxed(&c->join_full, 1u);
        return m;
    }
    {
        // announce over the entry of an older slot only: our own slot's
        // value means the master passed it, a newer slot's that the ring
        // went a whole lap round while this joiner stood still (slots are
        // compared modulo 2^32, so a launch sees at most 2^31 joiners)
        uint64_t cur = __hip_atomic_load(ent, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (;;) {
            if (cur != ~0ull && (int32_t)((uint32_t)cur - slot) >= 0) return m;
            if (cas64(ent, cur, ring_entry(slot, kTagWaiting))) break;
        }
    }
    const uint64_t t0 = now_ticks();
    for (uint32_t it = 0;; ++it) {
        const uint64_t e = __hip_atomic_load(ent, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint64_t r = ld_relaxed64(&c->release);
        if (e != ring_entry(slot, kTagWaiting)) {
            if ((e >> 32) >= kTagConsumed) return m;     // not ours to take (cannot happen after announcing)
            // admitted at epoch (e >> 32) & 0xFFFF: wait until that epoch's
            // release is visible, then read the final id (the master may
            // renumber before it publishes) and start after the fork point
            const uint32_t aep = (uint32_t)(e >> 32) & 0xFFFFu;
            // wait until the release of that epoch is published (the entry is
            // written before it); an epoch already past it means this joiner
            // was not a member of that interval (see below)
            while (((rel_epoch(r) - aep) & 0xFFFFu) >= 0x8000u && !(rel_flags(r) & (kFlagAbort | kFlagDone))) {
                __builtin_amdgcn_s_sleep(1);
                r = ld_relaxed64(&c->release);
            }
            fence_acquire();
            const uint64_t f = __hip_atomic_load(ent, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            m.id = (uint32_t)(f >> 48);
            m.M = rel_M(r);
            m.epoch = rel_epoch(r);
            m.flags = rel_flags(r);
            m.alive = (m.flags & (kFlagAbort | kFlagDone)) ? 0u : 1u;
            // admitted and killed at once (the master admits at most T - M
            // joiners and kills only M + admitted - T, so it does not
            // happen; an id at or above M would count as an extra arrival)
            if (m.id >= m.M || (rel_epoch(r) & 0xFFFFu) != aep) m.alive = 0u;
            if (m.alive) st_relaxed(&c->engine_of[m.id], engine_id(cfg.ses));
            return m;
        }
        bool leave = (rel_flags(r) & (kFlagAbort | kFlagDone)) != 0;
        if (!leave && cfg.host && !(cfg.mode & kModePark) && (it & 15) == 15) {
            // no room under the current target: give the compute unit back
            leave = ld_system(&cfg.host->target) <= rel_M(r);
        }
        if (!leave && now_ticks() - t0 > cfg.watchdog_ticks) leave = true;
        if (leave) {
            uint64_t expected = e;
            if (cas64(ent, expected, ring_entry(slot, kTagWithdrawn)))
                return m;            // withdrawn: the master will skip this slot
            continue;                // the master admitted us meanwhile: re-read
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

// Registration (thread 0 only). In a plain launch the workgroup id is the
// block id and M is the grid size. In a cooperative launch the launch's own
// workgroups draw tickets: ticket 0 becomes logical 0 (M starts at 1), and
// every later ticket waits for the first release, whose master step admits
// the tickets drawn before it as ids 0 .. cohort-1 (the start-up admission:
// the Fork rule with the ids given in ticket order, no joiner ring and no
// host reads). A later ticket, a workgroup of a joiner grid and a killed
// workgroup re-queued in park mode wait in the joiner queue.
__device__ inline Member register_member(Ctx* c, const Cfg cfg, bool plain, bool joiner_grid) {
    Member m{};
    if (plain) {
        m.id = blockIdx.x;
        m.M = gridDim.x;
        m.alive = 1;
        st_relaxed(&c->engine_of[m.id], engine_id(cfg.ses));
        return m;
    }
    if (!joiner_grid) {
        const uint32_t t = add_relaxed(&c->ticket, 1u);
        if (t == 0) {
            m.id = 0;
            m.M = 1;
            m.alive = 1;
            st_relaxed(&c->engine_of[0], engine_id(cfg.ses));
            return m;
        }
        const uint64_t r = wait_release(c, cfg, 0u);
        fence_acquire();
        if (rel_flags(r) & (kFlagAbort | kFlagDone)) {
            m.alive = 0;
            return m;
        }
        if (t < ld_relaxed(&c->cohort)) {
            // admitted at the first barrier, which cannot release the next
            // one without this member: r is that first release
            m.id = t;
            m.M = rel_M(r);
            m.epoch = rel_epoch(r);
            m.flags = rel_flags(r);
            m.alive = 1;
            st_relaxed(&c->engine_of[t], engine_id(cfg.ses));
            return m;
        }
    } else {
        add_relaxed(&c->joined_grid, 1u);
    }
    return join_queue(c, cfg);
}

// Start-up: in a cooperative launch ticket 0 waits briefly for the rest of
// the grid to draw tickets, so the first barrier can admit them together.
__device__ inline void startup_wait(Ctx* c, const Cfg cfg) {
    const uint64_t t0 = now_ticks();
    while (ld_relaxed(&c->ticket) < gridDim.x && now_ticks() - t0 < cfg.epoch0_wait)
        __builtin_amdgcn_s_sleep(2);
}

// The thread that loads the scheduler words and runs the scheduler's
// decisions. In a cooperative launch: the last wave's first lane, a wave the
// algorithms' master steps leave idle (a wave waits for its loads in issue
// order, so from thread 0 the dozen scheduler loads held up the master
// step's own: 0.4 us of each SSSP round). A plain launch loads two words and
// keeps thread 0 (one wave fewer between the master step and the release).
template <bool Coop>
__device__ __forceinline__ uint32_t sched_thread() {
    return Coop ? blockDim.x - 64u : 0u;
}

// Inputs of the scheduler part of the master step, loaded by the
// scheduling thread as soon as its workgroup knows it is the master, so
// that their round trip
// overlaps the algorithm's own master step. An error raised by another
// workgroup after this load is caught at the next barrier (the error word
// stays set); the algorithm's master step reports its own errors in the
// flags it returns.
template <bool Coop, class C>
__device__ __forceinline__ MasterPre master_prefetch(C* c, const Cfg cfg, bool relay_self) {
    MasterPre p;
    p.err = ld_relaxed_i(&c->error);
    p.tail = Coop ? ld_relaxed(&c->join_tail) : 0u;
    // the target workgroup 0 relayed while it waited; when it has nobody
    // to wait for (M = 1) it reads the host word here, the PCIe round trip
    // overlapping the algorithm's master step (with M > 1 a barrier that
    // workgroup 0 masters uses the value of the one before)
    p.T_seen = (Coop && cfg.host) ? (relay_self ? ld_system(&cfg.host->target) : ld_relaxed(&c->T_seen)) : 0u;
    // and leaves it for the masters after it (nobody relayed while M was 1)
    if (Coop && cfg.host && relay_self) st_relaxed(&c->T_seen, p.T_seen);
    p.join_head = ld_relaxed(&c->join_head);
    p.T_dev = c->T_dev;
    p.nb = c->barriers;
    p.kills = c->kills;
    p.forks = c->forks;
    p.resizes = c->resizes;
    p.min_M = c->min_M;
    p.max_M = c->max_M;
    p.tail_prev = c->tail_prev;
    return p;
}

// The scheduler's decision (scheduling thread, from the words master_prefetch
// loaded) for a barrier after which the kernel goes on: the target, the
// start-up cohort, how many waiting joiners to admit or pass, and whether
// the barrier is quiet. In a cooperative launch the scheduling thread, in
// a wave the algorithms' master steps leave idle, takes it while their
// master step runs (its loads are the first thing it waits for); a plain
// launch decides little and keeps it after the master step, in thread 0.
template <bool Coop, class C>
__device__ __forceinline__ void master_decide(C* c, const Cfg cfg, const Member& m, MasterPre& p, bool resize) {
    const uint32_t ne = m.epoch + 1;
    // a barrier that may not resize is one whose fork admits nobody and
    // whose kill claims nobody (k = 0 and the Kill-No-Op rule)
    const bool live = Coop && resize && !p.err;
    uint32_t T_dev = p.T_dev;
    uint32_t T = cfg.N;
    if (live) {
        if (cfg.mode & kModeRandomSched) {
            const uint64_t h = splitmix64(cfg.sched_seed + (uint64_t)ne * 0x9E3779B97F4A7C15ull);
            if ((uint32_t)(h & 0xFFFFu) < cfg.sched_p16) T_dev = 1u + (uint32_t)((h >> 16) % cfg.N);
            T = T_dev ? T_dev : cfg.N;      // no draw yet: nothing competes
        } else if (cfg.host) {
            T = p.T_seen;
        }
        if (T < 1u) T = 1u;
        if (T > cfg.N) T = cfg.N;
    }
    // start-up admission (the first barrier of a cooperative launch): the
    // launch's tickets drawn so far (every arrival drew one before it
    // arrived), at most the target, become ids 0 .. M0-1 (the members
    // before this barrier's forks); each reads M0 after the release
    uint32_t M0 = m.M;
    if (live && m.epoch == 0) {
        const uint32_t drawn = ld_relaxed(&c->ticket);
        M0 = drawn < T ? drawn : T;
        if (M0 < 1u) M0 = 1u;
    }
    const uint32_t ready = p.tail - p.join_head;
    const uint32_t room = cfg.N - M0;
    const uint32_t want = T > M0 ? T - M0 : 0u;
    uint32_t kmax = live ? ready : 0u;
    kmax = kmax < room ? kmax : room;
    kmax = kmax < want ? kmax : want;
    // with no room, pass the slots at the head whose joiners have given up
    // already, so that they do not fill the ring's window (never at a
    // barrier that admits: see the ring's comment)
    const uint32_t span = ready < blockDim.x ? ready : blockDim.x;
    const uint32_t drain = (live && kmax == 0 && span >= kDrainMin) ? span : 0u;
    p.T = T;
    p.T_dev_new = T_dev;
    p.M0 = M0;
    p.kmax = kmax;
    p.drain = drain;
    // the common barrier: nothing to admit, drain or kill, no recount of
    // the members per XCD (the algorithm's flags may still rule it out),
    // the kernel goes on (the Kill-No-Op rule and a fork of k = 0); only
    // the bookkeeping in master_schedule runs
    p.quiet = (m.epoch != 0 && p.nb != 0 && !(m.flags & kFlagFlat) && kmax == 0 && drain == 0 && T >= m.M &&
               T_dev == p.T_dev) ? 1u : 0u;
}

// Scheduler part of the master step, run by every thread of the master
// workgroup: fork (admit waiting joiners, in parallel), query (the target)
// and kill (the top ids). Thread 0 then publishes the release word.
template <bool Coop, class C>
__device__ inline void master_schedule(C* c, const Cfg cfg, Member& m, BarrierLds& b, uint32_t flags,
                                       uint64_t t_in, MasterPre& pre, bool resize) {
    uint32_t T_dev = 0, nb = 0, kills = 0, forks = 0, resizes = 0, min_M = 0, max_M = 0;
    uint32_t kmax0 = 0, head0 = 0, drain0 = 0;     // the scheduling thread's copies of what it shares in LDS
    // one thread decides and publishes: the thread that loaded the
    // scheduler words (MasterPre) while the algorithm's master step ran
    const uint32_t sched = sched_thread<Coop>();
    if (threadIdx.x == sched) {
        if constexpr (!Coop) master_decide<Coop>(c, cfg, m, pre, resize);
        nb = pre.nb;
        kills = pre.kills;
        forks = pre.forks;
        resizes = pre.resizes;
        min_M = pre.min_M;
        max_M = pre.max_M;
        if (pre.err) flags |= kFlagAbort;
        // the decision stands unless the algorithm ended the kernel: then
        // nothing is admitted, drained or killed
        const bool live = Coop && resize && !(flags & (kFlagDone | kFlagAbort));
        T_dev = live ? pre.T_dev_new : pre.T_dev;
        const uint32_t M0 = live ? pre.M0 : m.M;
        if (live && m.epoch == 0) st_relaxed(&c->cohort, M0);
        b.m0 = M0;
        const uint32_t kmax = live ? pre.kmax : 0u;
        kmax0 = kmax;
        head0 = pre.join_head;
        b.head = pre.join_head;
        b.kmax = kmax;
        b.T = live ? pre.T : cfg.N;
        b.flags = flags;
        b.tail_prev = pre.tail_prev;
        drain0 = live ? pre.drain : 0u;
        b.drain_span = drain0;
        b.quiet = (pre.quiet && !(flags & (kFlagDone | kFlagAbort | kFlagRenum | kFlagFlat))) ? 1u : 0u;
    }
    const uint32_t ne = m.epoch + 1;
    // every thread reads what the scheduling thread just shared (b.flags decides below
    // whether the whole workgroup recounts the members per XCD, a block with
    // workgroup barriers inside): in every launch mode, since an
    // algorithm's single step need not have left the flags in b.flags, and
    // the LDS may still hold an earlier launch's value (a plain launch that
    // read it unsynchronised split its barriers between the threads that saw
    // DONE there and thread 0, and miscounted the arrivals)
    __syncthreads();
    if (b.quiet) {
        if (threadIdx.x == sched) {
            c->barriers = nb + 1;
            if (Coop) c->tail_prev = pre.tail;
            if (cfg.trace && nb < cfg.trace_cap) {
                cfg.trace[2 * nb] = t_in;
                cfg.trace[2 * nb + 1] = (now_ticks() & 0xFFFFFFFFFFFFull) | ((uint64_t)(flags & 0xFFFFu) << 48);
            }
            st_release64(&c->release, make_release(ne, m.M, flags));
            Member n = m;
            n.epoch = ne;
            n.flags = flags;
            n.alive = 1u;
            b.member = n;
            b.killed = 0u;
        }
        return;
    }
    const uint32_t M0 = b.m0;
    uint32_t admitted = 0;
    if constexpr (Coop) {
        const uint32_t kmax = b.kmax, head = b.head;
        if (b.drain_span) {
            if (threadIdx.x == 0) b.drained = b.drain_span;
            __syncthreads();
            if (threadIdx.x < b.drain_span) {
                const uint32_t slot = head + threadIdx.x;
                const uint64_t e = __hip_atomic_load(&c->join_entry[slot % kJoinCap], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                if (e != ring_entry(slot, kTagWithdrawn)) atomicMin(&b.drained, threadIdx.x);
            }
            __syncthreads();
        }
        if (kmax) {
            // a slot taken since the previous barrier whose joiner has not
            // announced itself yet ends this barrier's admissions (it will
            // announce within moments); an older unannounced slot belongs to
            // a joiner that left beyond the window and is closed
            if (threadIdx.x == 0) b.cut = kmax;
            const uint32_t nwords0 = (kmax + 31) / 32;
            for (uint32_t w = threadIdx.x; w < nwords0; w += blockDim.x) b.valid[w] = 0;
            __syncthreads();
            for (uint32_t j = threadIdx.x; j < kmax; j += blockDim.x) {
                const uint32_t slot = head + j;
                const uint64_t e = __hip_atomic_load(&c->join_entry[slot % kJoinCap], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                const bool known = e == ring_entry(slot, kTagWaiting) || e == ring_entry(slot, kTagWithdrawn) ||
                                   e == ring_entry(slot, kTagConsumed);
                if (!known && (int32_t)(slot - b.tail_prev) >= 0) atomicMin(&b.cut, j);
            }
            __syncthreads();
            const uint32_t kcut = b.cut;
            const uint32_t nwords = (kcut + 31) / 32;
            // fork: admit ring slots head .. head+kcut-1 as ids M .. M+kcut-1
            for (uint32_t j = threadIdx.x; j < kcut; j += blockDim.x) {
                const uint32_t slot = head + j;
                if (ring_admit(&c->join_entry[slot % kJoinCap], slot, ne, M0 + j))
                    atomicOr(&b.valid[j / 32], 1u << (j % 32));
            }
            __syncthreads();
            // passed slots leave holes: renumber the admitted ones densely
            // (a joiner reads its final id after the release is published)
            for (uint32_t j = threadIdx.x; j < kcut; j += blockDim.x) {
                const uint32_t wj = j / 32, bj = j % 32;
                if (!((b.valid[wj] >> bj) & 1u)) continue;
                uint32_t rank = __popc(b.valid[wj] & ((1u << bj) - 1u));
                for (uint32_t q = 0; q < wj; ++q) rank += __popc(b.valid[q]);
                if (rank != j) {
                    const uint32_t slot = head + j;
                    __hip_atomic_store(&c->join_entry[slot % kJoinCap], admit_entry(slot, ne, M0 + rank),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            for (uint32_t q = 0; q < nwords; ++q) admitted += __popc(b.valid[q]);
            __syncthreads();
        }
    }
    // kill decision: W = the surplus over the target, never workgroup 0
    // (every thread computes it from the shared values of this step)
    uint32_t W = 0;
    if constexpr (Coop) {
        if (!(b.flags & (kFlagDone | kFlagAbort))) {
            const uint32_t M2 = M0 + admitted;
            W = M2 > b.T ? M2 - b.T : 0u;
            if (W > M2 - 1) W = M2 - 1;
            // the regular barrier (section 4.2): one offer_kill per arrival,
            // which in the worst arrival order claims only the top id
            if ((cfg.mode & kModeRegular) && W > 1) W = 1;
        }
    }
    // A host-driven target asks for compute units for another kernel, whose
    // workgroups the hardware deals round-robin over the XCDs and their
    // shader engines: choose the victims so that every engine frees its
    // share (then renumber the rest densely). The share is that of all
    // N - T units the other kernel needs, not of this barrier's surplus:
    // units already idle have usually been taken by the other kernel's
    // first workgroups, so an engine keeps at most slots - ceil((N - T) /
    // engines) of ours. The regular barrier takes one victim, on the engine
    // that owes most. If no engine owes (a launch smaller than the device),
    // the top ids leave as in the plain kill.
    bool renum = false;
    uint32_t Mn_sel = 0, my_new = m.id;
    if constexpr (Coop) {
        if (W && cfg.host && !(cfg.mode & kModeRandomSched) && cfg.engines > 1 && cfg.engines <= kMaxEngines) {
            renum = true;
            const uint32_t M2 = M0 + admitted;
            for (uint32_t t = threadIdx.x; t < M2; t += blockDim.x) b.xcd[t] = (uint8_t)ld_relaxed(&c->engine_of[t]);
            if (threadIdx.x < kMaxEngines) b.xcnt[threadIdx.x] = 0;
            __syncthreads();
            for (uint32_t t = threadIdx.x; t < M2; t += blockDim.x) atomicAdd(&b.xcnt[b.xcd[t] % kMaxEngines], 1u);
            __syncthreads();
            if (threadIdx.x == 0) {
                const uint32_t want_free = cfg.N > b.T ? cfg.N - b.T : 0u;
                const uint32_t need = (want_free + cfg.engines - 1) / cfg.engines;
                uint32_t best = kMaxEngines, best_k = 0;
                for (uint32_t x = 0; x < kMaxEngines; ++x) {
                    const uint32_t cnt = b.xcnt[x];
                    const uint32_t idle = x < cfg.engines && cfg.slots_per_engine > cnt ? cfg.slots_per_engine - cnt : 0u;
                    uint32_t k = need > idle ? need - idle : 0u;
                    const uint32_t cap = cnt - (x == b.xcd[0] ? 1u : 0u);     // workgroup 0 stays
                    b.xcnt[x] = k < cap ? k : cap;
                    if (b.xcnt[x] > best_k) {
                        best_k = b.xcnt[x];
                        best = x;
                    }
                }
                if (cfg.mode & kModeRegular)           // one victim: on the engine that owes most
                    for (uint32_t x = 0; x < kMaxEngines; ++x) b.xcnt[x] = x == best ? 1u : 0u;
                b.top_kill = best_k == 0 ? 1u : 0u;
            }
            __syncthreads();
            // id t is a victim if fewer than xcnt[its XCD] higher ids share its XCD
            uint32_t carry = 0;
            for (uint32_t base = 0; base < M2; base += blockDim.x) {
                const uint32_t t = base + threadIdx.x;
                bool alive = false;
                if (t < M2) {
                    const uint32_t x = b.xcd[t];
                    uint32_t above = 0;
                    for (uint32_t u = t + 1; u < M2; ++u) above += b.xcd[u] == x ? 1u : 0u;
                    alive = b.top_kill ? t < M2 - W : (t == 0 || above >= b.xcnt[x % kMaxEngines]);
                }
                const uint64_t bal = __ballot(alive);
                if ((threadIdx.x & 63) == 0) b.wsum[threadIdx.x / 64] = (uint32_t)__popcll(bal);
                __syncthreads();
                uint32_t before = carry;
                for (uint32_t w = 0; w < threadIdx.x / 64; ++w) before += b.wsum[w];
                const uint32_t nid = before + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                if (t < M2) {
                    __hip_atomic_store(&c->renum[t], ((ne & 0xFFFFu) << 16) | (alive ? nid : 0xFFFFu),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (alive) st_relaxed(&c->engine_of[nid], b.xcd[t]);
                    b.renum_alive[t] = alive ? 1u : 0u;
                }
                if (t == m.id) b.my_new = alive ? nid : 0xFFFFu;
                for (uint32_t w = 0; w < blockDim.x / 64; ++w) carry += b.wsum[w];
                __syncthreads();
            }
            Mn_sel = carry;
            my_new = b.my_new;
            __syncthreads();
        }
    }
    // members per XCD for the next interval's arrival (launch contexts):
    // recounted when the membership changed or the interval just ending
    // could not arrive by XCD; joiners admitted now have not recorded their
    // XCD yet, so the next interval arrives per workgroup (kFlagFlat)
    if constexpr (kGroupedArrival<C>) {
        const bool over = (b.flags & (kFlagDone | kFlagAbort)) != 0;
        const uint32_t M2 = M0 + admitted;
        const uint32_t Mn = renum ? Mn_sel : M2 - W;
        if (!over && admitted == 0 && M0 == m.M && (m.epoch == 0 || (m.flags & kFlagFlat) || Mn != m.M || renum)) {
            if (threadIdx.x < kMaxXcds) b.xcnt[threadIdx.x] = 0;
            __syncthreads();
            if (renum) {
                // survivors' XCDs are in LDS (the new table is being written)
                for (uint32_t t = threadIdx.x; t < M2; t += blockDim.x)
                    if (t == 0 || b.renum_alive[t]) atomicAdd(&b.xcnt[(b.xcd[t] / cfg.ses) % kMaxXcds], 1u);
            } else {
                for (uint32_t t = threadIdx.x; t < Mn; t += blockDim.x)
                    atomicAdd(&b.xcnt[(ld_relaxed(&c->engine_of[t]) / cfg.ses) % kMaxXcds], 1u);
            }
            __syncthreads();
            // the scheduling thread stores the counts: its release below
            // orders its own stores only
            if (threadIdx.x == sched) {
                Ctx* cx = reinterpret_cast<Ctx*>(c);
                uint32_t groups = 0;
                for (uint32_t x = 0; x < kMaxXcds; ++x) {
                    cx->xcd.members[x] = b.xcnt[x];
                    groups += b.xcnt[x] ? 1u : 0u;
                }
                cx->xcd.groups = groups;
            }
        }
    }
    if (threadIdx.x == sched) {
        // `flags` is still the value the scheduling thread shared as b.flags
        uint32_t Mn = m.M;
        // newcomers (admitted or started up here) have not recorded their
        // XCD yet: the next interval arrives per workgroup
        const uint32_t newcomers = admitted + (M0 - m.M);
        if (kGroupedArrival<C> && !(flags & (kFlagDone | kFlagAbort)) && newcomers) flags |= kFlagFlat;
        if (Coop && !(flags & (kFlagDone | kFlagAbort))) {
            const uint32_t M2 = M0 + admitted;
            const uint32_t Wk = renum ? M2 - Mn_sel : W;
            Mn = M2 - Wk;
            if (renum) flags |= kFlagRenum;
            if (kmax0) st_relaxed(&c->join_head, head0 + b.cut);
            else if (drain0 && b.drained) st_relaxed(&c->join_head, head0 + b.drained);
            if (cfg.mode & kModeRandomSched) c->T_dev = T_dev;
            if (newcomers) c->forks = forks + newcomers;
            if (Wk) c->kills = kills + Wk;
            if (Mn != m.M) c->resizes = resizes + 1;
            if (Mn < min_M) c->min_M = Mn;
            if (Mn > max_M) c->max_M = Mn;
        }
        c->barriers = nb + 1;
        if (Coop) c->tail_prev = pre.tail;
        if (nb == 0) c->t_start = t_in;
        if (flags & kFlagDone) {
            c->final_M = m.M;
            c->t_end = now_ticks();
        }
        if (cfg.trace && nb < cfg.trace_cap) {
            cfg.trace[2 * nb] = t_in;
            cfg.trace[2 * nb + 1] = (now_ticks() & 0xFFFFFFFFFFFFull) | ((uint64_t)(flags & 0xFFFFu) << 48);
        }
        st_release64(&c->release, make_release(ne, Mn, flags));
        Member n = m;
        n.epoch = m.epoch + 1;
        n.M = Mn;
        n.flags = flags;
        const bool over = (flags & (kFlagDone | kFlagAbort)) != 0;
        bool gone = false;
        if (Coop && !over) gone = renum ? my_new == 0xFFFFu : n.id >= Mn;
        if (renum && !gone) n.id = my_new;
        n.alive = (over || gone) ? 0u : 1u;
        if (counts_changed(m, n)) n.xm = n.xg = 0;
        b.member = n;
        b.killed = gone ? 1u : 0u;
    }
}

// The (resizing) global barrier. Called by every thread of every active
// workgroup. The last workgroup to arrive runs the master step with all of
// its threads: `master_fn(M, new_epoch)` does the per-level bookkeeping
// (it may use __syncthreads and must return the same flags in every
// thread); kFlagDone ends the kernel. In a cooperative launch the master
// then admits joiners and applies the scheduler target. Only workgroup 0
// reads the host-written target (one PCIe read per barrier), before it
// arrives.
template <bool Coop, class C, class MasterFn>
__device__ inline void barrier(C* c, const Cfg cfg, Member& m, BarrierLds& b, MasterFn&& master_fn,
                               bool resize = true, uint64_t payload = 0) {
    // by XCD: every wave's memory operations must have reached the L2 that
    // its XCD's last arriver writes back
    const bool by_xcd = kGroupedArrival<C> && m.epoch != 0 && !(m.flags & kFlagFlat);
    // the counters are 64-bit only in a launch whose arrivals carry sums
    // (a 64-bit add costs the contended counters more); otherwise every
    // add is 32-bit on the low word, whose high word stays 0
    const bool wide = (cfg.mode & kModeArriveSums) != 0;
    if (by_xcd) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    wg_trace(cfg, m.epoch, m.id, kTrArrive);
    if (threadIdx.x == 0) {
        // workgroup 0 passes the host target to the master: here in
        // one-wave workgroups (and at a first barrier it does not master
        // alone), otherwise while it waits for a release (below); alone
        // (M = 1, as at the first barrier) it reads it in its master step
        if (Coop && cfg.host && m.id == 0 && m.M > 1 && (m.epoch == 0 || blockDim.x <= kRelayThread))
            __hip_atomic_store(&c->T_seen, ld_system(&cfg.host->target), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        uint32_t last = 0;
        if (by_xcd) {
            Ctx* cx = reinterpret_cast<Ctx*>(c);
            const uint32_t x = xcc_id();
            if (m.xg == 0) {
                // the counts changed at the last release: load them once
                m.xm = ld_relaxed(&cx->xcd.members[x]);
                m.xg = ld_relaxed(&cx->xcd.groups);
            }
            const uint32_t members = m.xm, groups = m.xg;
            __builtin_amdgcn_s_waitcnt(0);       // our T_seen store is in the L2 too
            if (wide) {
                const uint64_t o = __hip_atomic_fetch_add(&cx->xcd_arrive[x].count, 1ull + payload,
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((uint32_t)(o & kArriveCount) + 1 == members) {
                    // last of this XCD: reset its counter, write back its L2
                    // and arrive for the XCD with the XCD's sums
                    __hip_atomic_store(&cx->xcd_arrive[x].count, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t xs = (o + 1ull + payload) & ~kArriveCount;
                    const uint64_t o2 = __hip_atomic_fetch_add(&c->arrive, 1ull + xs, __ATOMIC_ACQ_REL,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                    last = ((uint32_t)(o2 & kArriveCount) + 1 == groups) ? 1u : 0u;
                    b.sums = (o2 + 1ull + xs) >> kArriveCountBits;
                }
            } else {
                const uint32_t o = __hip_atomic_fetch_add(arrive_lo(&cx->xcd_arrive[x].count), 1u, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                if (o + 1 == members) {
                    // last of this XCD: reset its counter, write back its L2
                    // and arrive for the XCD
                    __hip_atomic_store(arrive_lo(&cx->xcd_arrive[x].count), 0u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t o2 = __hip_atomic_fetch_add(arrive_lo(&c->arrive), 1u, __ATOMIC_ACQ_REL,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                    last = (o2 + 1 == groups) ? 1u : 0u;
                }
            }
        } else if (wide) {
            const uint64_t old = __hip_atomic_fetch_add(&c->arrive, 1ull + payload, __ATOMIC_ACQ_REL,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            last = ((uint32_t)(old & kArriveCount) + 1 == m.M) ? 1u : 0u;
            b.sums = (old + 1ull + payload) >> kArriveCountBits;
        } else {
            const uint32_t old = __hip_atomic_fetch_add(arrive_lo(&c->arrive), 1u, __ATOMIC_ACQ_REL,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            last = (old + 1 == m.M) ? 1u : 0u;
        }
        b.is_master = last;
        if (b.is_master) {
            if (wide) __hip_atomic_store(&c->arrive, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else __hip_atomic_store(arrive_lo(&c->arrive), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    if (b.is_master) {
        // master step: everybody else is parked in the barrier
        const uint64_t t_in = now_ticks();
        MasterPre pre;
        if (threadIdx.x == sched_thread<Coop>()) {
            pre = master_prefetch<Coop>(c, cfg, m.M == 1);
            if constexpr (Coop) master_decide<Coop>(c, cfg, m, pre, resize);
        }
        const uint32_t flags = master_fn(m.M, m.epoch + 1);
        master_schedule<Coop, C>(c, cfg, m, b, flags, t_in, pre, resize);
    } else if (Coop && cfg.host && m.id == 0 && threadIdx.x == kRelayThread) {
        // workgroup 0 reads the host target over PCIe while it waits, in a
        // wave other than the waiting one: the read (about 2 us) then sits
        // neither in a phase's loads nor on the master's path; the master of
        // the next barrier finds the value (one barrier late if workgroup 0
        // is this barrier's master and skips the read)
        __hip_atomic_store(&c->T_seen, ld_system(&cfg.host->target), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (threadIdx.x == 0) {
        const uint64_t r = wait_release(c, cfg, m.epoch);
        fence_acquire();
        Member n = m;
        const uint32_t e = rel_epoch(r);
        n.flags = rel_flags(r);
        n.M = rel_M(r);
        n.epoch = e;
        // an alive member cannot miss an epoch: a gap means it was killed
        uint32_t k = (Coop && e != m.epoch + 1) ? 1u : 0u;
        if constexpr (Coop) {
            if (!k && (n.flags & kFlagRenum)) {
                // victims chosen by XCD: the entry of this epoch holds the
                // new id; an entry of a later epoch means it was killed here
                const uint32_t ent = ld_relaxed(&c->renum[m.id]);
                if ((ent >> 16) != (e & 0xFFFFu) || (ent & 0xFFFFu) == 0xFFFFu) k = 1;
                else n.id = ent & 0xFFFFu;
            }
        }
        if (Coop && !(n.flags & kFlagRenum) && n.id >= n.M) k = 1;
        if (n.flags & (kFlagDone | kFlagAbort)) k = 0;
        n.alive = (!k && !(n.flags & (kFlagDone | kFlagAbort))) ? 1u : 0u;
        if (counts_changed(m, n)) n.xm = n.xg = 0;
        b.member = n;
        b.killed = k;
    }
    __syncthreads();
    wg_trace(cfg, m.epoch, m.id, kTrReleased);
    m = b.member;
}

// Barrier of a team: a fixed set of `m.M` workgroups that work on one
// instance inside a batched launch, with its own barrier lines and no
// scheduler (kill and fork happen between instances). A one-workgroup team
// needs no global atomics: every wave waits for its own memory operations,
// the workgroup meets at s_barrier, one agent-scope acquire drops stale
// L1 lines (other waves' atomics were performed in L2), and the workgroup
// runs the master step itself.
template <class MasterFn>
__device__ inline void team_barrier(CtxCore* c, const Cfg cfg, Member& m, BarrierLds& b, MasterFn&& master_fn,
                                    uint64_t payload = 0) {
    if (m.M > 1) {
        barrier<false>(c, cfg, m, b, master_fn, true, payload);
        return;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        b.sums = payload >> kArriveCountBits;
    }
    __syncthreads();
    uint32_t flags = master_fn(1u, m.epoch + 1);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (ld_relaxed_i(&c->error)) flags |= kFlagAbort;
        c->barriers += 1;
        b.flags = flags;
    }
    __syncthreads();
    flags = b.flags;
    m.epoch += 1;
    m.flags = flags;
    m.alive = (flags & (kFlagDone | kFlagAbort)) ? 0u : 1u;
}

// ==================================================================
// The programming model as device calls (paper section 3.1, "Semantics of
// Cooperative Kernels", and the rules of Appendix A). Every call is a
// workgroup-level function: all threads of the workgroup make it, with the
// same arguments (the paper's uniformity requirement); `Coop` is false in a
// plain launch, where M is fixed and nothing is killed or forked.
//
// Two ways to write a cooperative kernel, as in the paper's programming
// section:
//  * interval pattern (graph traversal): the kernel meets at
//    coop_resizing_global_barrier / coop_global_barrier; M and the ids stay
//    fixed between two barriers, so work can be split statically by
//    coop_get_group_id / coop_get_num_groups. Forks and kills happen inside
//    the resizing barrier (fork first, then kill; the query barrier of the
//    paper's scheduler design). Joiners start after a barrier and read the
//    transmitted state with coop_transmit_block().
//  * task pattern (work stealing): the kernel calls coop_offer_kill and
//    coop_request_fork itself, typically before each task, and never meets
//    at a global barrier. Ids are slots that a workgroup keeps until it
//    leaves, so the scheduler may take any workgroup (Appendix B).
// A kernel uses one pattern; the launch context (Ctx) carries the state of
// both.

// A workgroup's handle on its launch: the launch context in HBM, the
// launch constants (the kernel argument) and the workgroup's membership and
// barrier scratch in LDS.
struct Group {
    Ctx* ctx;
    const Cfg& cfg;
    BarrierLds& bar;
    __device__ Group(Ctx* c, const Cfg& f, BarrierLds& b) : ctx(c), cfg(f), bar(b) {}
};

// get_group_id: this workgroup's id (section 3.1, "Active Workgroups"): in
// [0, M) in the interval pattern, a slot in [0, N) in the task pattern.
__device__ __forceinline__ uint32_t coop_get_group_id(const Group& g) { return g.bar.member.id; }

// get_num_groups: the active workgroup count M of the current resizing-
// barrier interval (interval pattern; section 3.2, "A Changing Workgroup
// Count"). In the task pattern M changes at any time: this returns the
// count as last read, a hint only.
__device__ __forceinline__ uint32_t coop_get_num_groups(const Group& g) { return g.bar.member.M; }

// The flags the last barrier's single step published (algorithm bits from
// kFlagUser0 up, and kFlagDone once the kernel has finished).
__device__ __forceinline__ uint32_t coop_flags(const Group& g) { return g.bar.member.flags; }

// The state a joiner takes over (the transmit qualifier of section 3.1).
// Interval pattern: the single step of a resizing barrier writes it, as the
// state of workgroup 0 that forked joiners receive ("Global Barriers"), and
// a joiner reads it once coop_start or coop_rejoin has let it in. Task
// pattern: coop_request_fork writes it, a joiner reads it once
// coop_task_start has let it in (the state of the most recent fork that let
// joiners in).
__device__ __forceinline__ uint32_t* coop_transmit_block(const Group& g) { return g.ctx->transmit; }
__device__ __forceinline__ const uint32_t* coop_task_transmitted(const Group& g) { return g.ctx->task.transmit; }

// The host-written target, read over PCIe, or (kModeRelayTarget) the copy
// one of the kernel's own workgroups keeps in device memory.
__device__ __forceinline__ uint32_t host_target(const Group& g) {
    return (g.cfg.mode & kModeRelayTarget) ? ld_relaxed(&g.ctx->T_seen) : ld_system(&g.cfg.host->target);
}

// query: the number of workgroups the scheduler wants the kernel to keep,
// the value the paper's efficient resizing barrier asks the scheduler for
// (section 4.2): the seeded device schedule's current target, the
// host-written target, or N when nothing else is competing.
__device__ __forceinline__ uint32_t coop_query(const Group& g) {
    uint32_t T = g.cfg.N;
    if (g.cfg.mode & kModeRandomSched) {
        // the seeded schedule's target (set at resizing barriers; a
        // task-pattern launch has none and is sized by its kill offers)
        const uint32_t d = ld_relaxed(&g.ctx->T_dev);
        if (d) T = d;
    } else if (g.cfg.host) {
        T = host_target(g);
    }
    if (T < 1u) T = 1u;
    return T < g.cfg.N ? T : g.cfg.N;
}

// --------------------------------------------------- interval pattern

// Kernel entry. Returns true if this workgroup is active. In a plain launch
// every workgroup is (id = block id, M = grid). In a cooperative launch
// workgroup ticket 0 starts as workgroup 0 with M = 1 (at least one
// workgroup is active, section 3.1), and every other workgroup -- late ones
// of the grid and those of joiner grids (coop_fork_groups on the host) --
// waits to be forked in at a resizing barrier; it returns false if it gave
// its compute unit back without being admitted. coop_joined() tells a
// workgroup that entered at a later barrier, which must read the
// transmitted state.
template <bool Coop>
__device__ inline bool coop_start(Group& g, bool joiner_grid) {
    if (threadIdx.x == 0) {
        Member m = register_member(g.ctx, g.cfg, !Coop, joiner_grid);
        if (Coop && m.alive && m.epoch == 0) startup_wait(g.ctx, g.cfg);
        g.bar.member = m;
        g.bar.killed = 0;
    }
    __syncthreads();
    return g.bar.member.alive != 0;
}
__device__ __forceinline__ bool coop_joined(const Group& g) { return g.bar.member.epoch != 0; }

// resizing_global_barrier (section 3.1, "Global Barriers"; Appendix A,
// Resizing-Barrier rule): every active workgroup arrives; the last one to
// arrive runs `single(M, epoch)` with all of its threads while the others
// wait (the work the paper puts between two barriers: swap the frontiers,
// reset, level++; it may write the transmit block and returns the flags to
// publish, kFlagDone to end the kernel); then the scheduler sets the new
// count M': joiners are forked in first (ids M .. M'-1, the transmit block
// as their state), then the surplus over the target is killed (Kill rule:
// the top ids, never workgroup 0; with a host-driven target the victims are
// chosen per shader engine and the others renumbered densely, Appendix B).
// Returns false if this workgroup was killed or the kernel is over: the
// caller leaves (or re-queues with coop_rejoin). All global memory accesses
// issued before the barrier are complete and visible after it.
// `payload` (thread 0's value counts; arrive_payload) is this workgroup's
// share of two sums the master step finds in g.bar.sums: what every member
// brought to this barrier, added up by the arrival atomics themselves.
template <bool Coop, class Single>
__device__ inline bool coop_resizing_global_barrier(Group& g, Single&& single, uint64_t payload = 0) {
    Member m = g.bar.member;
    barrier<Coop>(g.ctx, g.cfg, m, g.bar, single, true, payload);
    return m.alive != 0;
}
template <bool Coop>
__device__ inline bool coop_resizing_global_barrier(Group& g) {
    return coop_resizing_global_barrier<Coop>(g, [](uint32_t, uint32_t) -> uint32_t { return 0u; });
}

// global_barrier (section 3.1, "Global Barriers"; Appendix A, Barrier rule):
// the same meeting with the active count left unchanged (no fork, no kill).
// Returns false only when the kernel is over (kFlagDone or an error).
template <bool Coop, class Single>
__device__ inline bool coop_global_barrier(Group& g, Single&& single) {
    Member m = g.bar.member;
    barrier<Coop>(g.ctx, g.cfg, m, g.bar, single, false);
    return m.alive != 0;
}
template <bool Coop>
__device__ inline bool coop_global_barrier(Group& g) {
    return coop_global_barrier<Coop>(g, [](uint32_t, uint32_t) -> uint32_t { return 0u; });
}

// A workgroup the scheduler killed at a resizing barrier waits to be forked
// in again (a launch with COOP_F_PARK_KILLED: the compute unit stays with
// the kernel, which exercises kill and fork without a competing task).
// Returns true once admitted (it resumes after that barrier, as a joiner).
template <bool Coop>
__device__ inline bool coop_rejoin(Group& g) {
    if (!Coop || !g.bar.killed || !(g.cfg.mode & kModePark)) return false;
    __syncthreads();
    if (threadIdx.x == 0) {
        g.bar.member = join_queue(g.ctx, g.cfg);
        g.bar.killed = 0;
    }
    __syncthreads();
    return g.bar.member.alive != 0;
}

// ------------------------------------------------------- task pattern

// The scheduler's decision for one workgroup on shader engine `x` that
// offers to leave (thread 0): accept if the launch holds more than
// max(T, floor) workgroups and, when the other kernel's workgroups are
// dealt over `engines` shader engines, this engine holds more than its
// share ceil(T / engines). The engine's count is claimed first with
// compare-and-swap, so workgroups of one engine that decide together
// cannot all leave it; if the launch-wide count is already at its floor
// the engine's count is given back.
__device__ inline bool task_leave(TaskState* ts, uint32_t T, uint32_t floor, uint32_t engines, uint32_t x) {
    const uint32_t lo = T > floor ? T : floor;
    const bool placed = engines > 1 && engines <= kMaxEngines;
    const uint32_t share = placed ? (T + engines - 1) / engines : T;
    uint32_t* ax = &ts->active_x[x % kMaxEngines];
    if (placed) {
        uint32_t e = ld_relaxed(ax);
        for (;;) {
            if (e <= share) return false;
            if (__hip_atomic_compare_exchange_strong(ax, &e, e - 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT))
                break;
        }
    }
    uint32_t a = ld_relaxed(&ts->active);
    while (a > lo) {
        if (__hip_atomic_compare_exchange_strong(&ts->active, &a, a - 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
            if (!placed) add_relaxed(ax, 0xFFFFFFFFu);
            add_relaxed(&ts->kills, 1u);
            atomicMin(&ts->min_active, a - 1);
            return true;
        }
    }
    if (placed) add_relaxed(ax, 1u);          // the launch is at its floor: stay
    return false;
}

// Thread 0: become active in slot `s` or the next free one after it.
__device__ inline bool task_claim(Ctx* c, const Cfg& cfg, uint32_t s0, Member& m) {
    TaskState* ts = &c->task;
    for (uint32_t k = 0; k < cfg.N; ++k) {
        const uint32_t s = (s0 + k) % cfg.N;
        uint32_t expected = 0;
        if (__hip_atomic_compare_exchange_strong(&ts->slot_owner[s], &expected, 1u, __ATOMIC_ACQUIRE,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            const uint32_t x = engine_id(cfg.ses);
            st_relaxed(&c->engine_of[s], x);
            add_relaxed(&ts->active_x[x % kMaxEngines], 1u);
            m.id = s;
            m.alive = 1;
            return true;
        }
    }
    return false;
}

// Task-pattern entry. Workgroups of the launch's own grid are scheduled
// initially (section 3.1: the scheduler may start fewer than N; every one
// that starts is active) and take a slot. A workgroup of a joiner grid is a
// fork: it waits until an active workgroup's coop_request_fork lets it in
// (then it starts after that call, with the transmitted state), and gives
// its compute unit back if the kernel finishes, the target leaves no room,
// or the watchdog expires first. Returns true if this workgroup is active.
template <bool Coop>
__device__ inline bool coop_task_start(Group& g, bool joiner_grid) {
    if (threadIdx.x == 0) {
        Ctx* c = g.ctx;
        TaskState* ts = &c->task;
        Member m{};
        m.alive = 0;
        const uint32_t lim = g.cfg.N;
        if (!joiner_grid || !Coop) {
            // the initial schedule: at most N workgroups
            uint32_t a = ld_relaxed(&ts->active);
            bool room = false;
            while (a < lim) {
                if (__hip_atomic_compare_exchange_strong(&ts->active, &a, a + 1, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    room = true;
                    break;
                }
            }
            if (room) {
                if (task_claim(c, g.cfg, blockIdx.x % lim, m)) atomicMax(&ts->max_active, a + 1);
                else add_relaxed(&ts->active, 0xFFFFFFFFu);
            }
        } else {
            const uint32_t t = add_relaxed(&ts->join_tickets, 1u);
            const uint64_t t0 = now_ticks();
            for (uint32_t it = 0;; ++it) {
                const uint64_t r = ld_relaxed64(&c->release);
                if ((rel_flags(r) & (kFlagAbort | kFlagDone)) || ld_relaxed_i(&c->error)) break;
                if ((int32_t)(ld_relaxed(&ts->join_granted) - t) > 0) {
                    // let in: take a unit of room under the target, then a slot
                    fence_acquire();
                    uint32_t T = lim;
                    if (g.cfg.host) T = host_target(g);
                    if (T < 1u) T = 1u;
                    const uint32_t cap = T < lim ? T : lim;
                    uint32_t a = ld_relaxed(&ts->active);
                    bool room = false;
                    while (a < cap) {
                        if (__hip_atomic_compare_exchange_strong(&ts->active, &a, a + 1, __ATOMIC_RELAXED,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            room = true;
                            break;
                        }
                    }
                    if (room) {
                        if (task_claim(c, g.cfg, (blockIdx.x * 2654435761u) % lim, m)) {
                            atomicMax(&ts->max_active, a + 1);
                            add_relaxed(&ts->forks, 1u);
                        } else {
                            add_relaxed(&ts->active, 0xFFFFFFFFu);
                        }
                    }
                    break;
                }
                if (g.cfg.host && (it & 15) == 15 && host_target(g) <= ld_relaxed(&ts->active))
                    break;                          // no room under the target: give the unit back
                if (now_ticks() - t0 > g.cfg.watchdog_ticks) break;
                __builtin_amdgcn_s_sleep(4);
            }
        }
        m.M = ld_relaxed(&ts->active);
        g.bar.member = m;
        g.bar.killed = 0;
        g.bar.offers = 0;
    }
    __syncthreads();
    return g.bar.member.alive != 0;
}

// offer_kill (section 3.1, "Semantics for offer_kill"; Appendix A, Kill and
// Kill-No-Op rules, with the any-order kill of Appendix B): the scheduler
// may take this workgroup back; returns false if it did, and the workgroup
// must then leave the kernel (its slot is free for a joiner). The decision:
// a seeded device schedule accepts with the launch's probability; a
// host-driven target accepts while the launch holds more than the target,
// choosing workgroups on the shader engines the other kernel needs
// (task_leave); otherwise the offer is a no-op. The host target is read on
// every eighth offer (the others are no-ops, which the Kill-No-Op rule
// allows), and never fewer than Cfg::keep workgroups stay.
template <bool Coop>
__device__ inline bool coop_offer_kill(Group& g) {
    if (!Coop) return true;
    if (threadIdx.x == 0) {
        TaskState* ts = &g.ctx->task;
        const uint32_t floor = g.cfg.keep ? g.cfg.keep : 1u;
        const uint32_t x = ld_relaxed(&g.ctx->engine_of[g.bar.member.id]);
        bool killed = false;
        if (g.cfg.mode & kModeRandomSched) {
            const uint32_t d = add_relaxed(&ts->decisions, 1u);
            const uint64_t h = splitmix64(g.cfg.sched_seed + (uint64_t)d * 0x9E3779B97F4A7C15ull);
            if ((uint32_t)(h & 0xFFFFu) < g.cfg.sched_p16) killed = task_leave(ts, 0u, floor, 1u, x);
        } else if (g.cfg.host && (g.bar.offers++ & 7u) == 0) {
            killed = task_leave(ts, host_target(g), floor, g.cfg.engines, x);
        }
        if (killed) {
            __hip_atomic_store(&ts->slot_owner[g.bar.member.id], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            g.bar.member.alive = 0;
            g.bar.killed = 1;
        }
    }
    __syncthreads();
    return g.bar.member.alive != 0;
}

// request_fork (section 3.1, "Semantics for offer_fork"; Appendix A, Fork
// rule): the scheduler chooses k in [0, N - M] -- here the joiners waiting
// to come in, at most the room the target leaves -- and that many join after
// this call, each with the `words` words of `state` (the transmitted
// variables of thread 0, read by joiners with coop_task_transmitted). Returns k
// (joiners let in: each takes a unit of room when it starts, so a joiner
// that finds none gives its compute unit back). k = 0 is always legal.
template <bool Coop>
__device__ inline uint32_t coop_request_fork(Group& g, const uint32_t* state = nullptr, uint32_t words = 0) {
    if (!Coop) return 0;
    __shared__ uint32_t forked;
    if (threadIdx.x == 0) {
        TaskState* ts = &g.ctx->task;
        const uint32_t waiting = ld_relaxed(&ts->join_tickets) - ld_relaxed(&ts->join_granted);
        uint32_t k = 0;
        if ((int32_t)waiting > 0) {
            const uint32_t T = coop_query(g);
            const uint32_t a = ld_relaxed(&ts->active);
            const uint32_t room = T > a ? T - a : 0u;
            k = waiting < room ? waiting : room;
            if (k) {
                for (uint32_t i = 0; i < words && i < kTransmitWords; ++i) st_relaxed(&ts->transmit[i], state[i]);
                __hip_atomic_fetch_add(&ts->join_granted, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        forked = k;
    }
    __syncthreads();
    return forked;
}

// The kernel's work is over (task pattern): joiners still waiting leave.
__device__ inline void coop_task_finish(Group& g) {
    if (threadIdx.x == 0)
        __hip_atomic_fetch_or(&g.ctx->release, (uint64_t)kFlagDone << 48, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// A task-pattern workgroup leaving for a reason of its own (work finished,
// error): its slot and its unit of the active count are given back.
__device__ inline void coop_task_leave(Group& g) {
    if (threadIdx.x == 0 && g.bar.member.alive) {
        TaskState* ts = &g.ctx->task;
        const uint32_t id = g.bar.member.id;
        add_relaxed(&ts->active_x[ld_relaxed(&g.ctx->engine_of[id]) % kMaxEngines], 0xFFFFFFFFu);
        add_relaxed(&ts->active, 0xFFFFFFFFu);
        __hip_atomic_store(&ts->slot_owner[id], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        g.bar.member.alive = 0;
    }
    __syncthreads();
}

}  // namespace coop
