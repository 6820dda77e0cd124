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
//    section ("master step") while everybody else is parked, then publishes
//    one 64-bit release word {epoch, M', flags} with agent-scope release.
//  * In the master step: per-level bookkeeping (a callback), fork = admit up
//    to k in [0, N-M] waiting joiners as ids [M, M+k-1], query = read the
//    scheduler target T (host-written word in pinned memory, or a seeded
//    device-side schedule), and kill = the top W = min(max(0, M+k-T), M+k-1)
//    ids leave. Workgroup 0 is never killed.
//  * Waiters read (epoch, M') as one word. An alive member is needed by the
//    next barrier, so it can never miss an epoch; a waiter that sees the
//    epoch advance by more than one was therefore killed at the epoch it
//    missed. (Reading the count separately would let a slow killed
//    workgroup pick up a later epoch's count and continue with a stale id.)
//  * Every spin is bounded by a wall-clock watchdog; expiry sets an error
//    and an abort flag that every waiter honours, so the grid always drains.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace coop {

constexpr uint32_t kMaxThreads = 1024;
constexpr uint32_t kMaxWaves = kMaxThreads / 64;
constexpr uint32_t kJoinCap = 8192;          // joiner admission ring

// release-word flags
constexpr uint32_t kFlagDone = 1u;          // kernel finished: everybody leaves
constexpr uint32_t kFlagAbort = 2u;         // watchdog fired or error: leave
constexpr uint32_t kFlagUser0 = 16u;        // algorithm-specific bits start here

// ctx->mode bits
constexpr uint32_t kModeCoop = 1u;          // cooperative (resizable) launch
constexpr uint32_t kModePark = 2u;          // killed workgroups re-queue as joiners
constexpr uint32_t kModeRandomSched = 4u;   // device-side seeded kill/fork schedule
constexpr uint32_t kModeTrace = 8u;         // record per-barrier timestamps

// error codes written to ctx->error (match COOP_E_* of coop.h)
constexpr int32_t kErrTimeout = -4;
constexpr int32_t kErrOverflow = -6;
constexpr int32_t kErrInternal = -7;

// Host-written control words (pinned, fine-grained host memory).
struct alignas(64) HostCtl {
    uint32_t target;          // scheduler target T (query), 1..N
    uint32_t pad0[15];
    uint32_t exited;          // workgroups released to the scheduler (device writes)
    uint32_t pad1[15];
};

struct alignas(256) Ctx {
    // ---- line: barrier arrival counter (one atomic per workgroup per barrier)
    uint32_t arrive;
    uint32_t _pa[63];
    // ---- line: release word {epoch:32 (lo) | M:16 | flags:16 (hi)}
    uint64_t release;
    uint64_t _pr[31];
    // ---- line: registration / joiner queue
    uint32_t ticket;          // start-up tickets
    uint32_t join_tail;       // next joiner slot
    uint32_t join_head;       // first slot not yet admitted (master only)
    uint32_t _pj[61];
    // ---- line: configuration (written by the init kernel, read-only after)
    uint32_t N;               // launch limit (max active workgroups)
    uint32_t mode;
    uint32_t sched_p16;       // random schedule: P(change) * 65536
    uint32_t wg_size;
    uint64_t sched_seed;
    uint64_t watchdog_ticks;  // wall-clock ticks before a spin gives up
    HostCtl* host;            // nullable
    uint32_t T_dev;           // device-side target (random schedule)
    uint32_t epoch0_wait;     // ticks ticket 0 waits for the first joiners
    uint32_t _pc[52];
    // ---- line: results / statistics (master only, plus error by anyone)
    int32_t error;
    uint32_t barriers;
    uint32_t kills;
    uint32_t forks;
    uint32_t resizes;
    uint32_t min_M;
    uint32_t max_M;
    uint32_t final_M;
    uint64_t t_start;
    uint64_t t_end;
    uint32_t _ps[52];
    // ---- joiner admission ring: {slot:32 (lo) | epoch_lo:16 | id:16 (hi)}
    uint64_t join_entry[kJoinCap];
};

// ------------------------------------------------------------- atomics

__device__ __forceinline__ uint32_t ld_acquire(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
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
__device__ __forceinline__ uint64_t add_relaxed64(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_system(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

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
};

// Raise the abort flag so every spinning workgroup leaves.
__device__ inline void raise_error(Ctx* c, int32_t err) {
    atomicCAS(&c->error, 0, err);
    __hip_atomic_fetch_or(&c->release, (uint64_t)kFlagAbort << 48, __ATOMIC_RELEASE,
                          __HIP_MEMORY_SCOPE_AGENT);
}

// The scheduler target this barrier sees (the paper's `query`): either the
// host-written word or a seeded device-side random schedule.
__device__ inline uint32_t query_target(Ctx* c, uint32_t epoch, uint32_t host_T) {
    const uint32_t N = c->N;
    uint32_t T;
    if (c->mode & kModeRandomSched) {
        uint64_t h = splitmix64(c->sched_seed + (uint64_t)epoch * 0x9E3779B97F4A7C15ull);
        T = c->T_dev;
        if ((uint32_t)(h & 0xFFFFu) < c->sched_p16) {
            T = 1u + (uint32_t)((h >> 16) % N);
            c->T_dev = T;
        }
    } else if (c->host) {
        T = host_T;
    } else {
        T = N;
    }
    if (T < 1u) T = 1u;
    if (T > N) T = N;
    return T;
}

// Joiner admission entries: {slot:32 (lo) | epoch_lo:16 | id:16 (hi)}.
// A joiner that gives up writes a "withdrawn" entry for its slot with a
// compare-and-swap; the master admits with an exchange and skips a slot
// whose previous value was that joiner's withdrawal. Both sides therefore
// agree on whether the slot was admitted.
__device__ __forceinline__ uint64_t withdrawn_entry(uint32_t slot) {
    return (uint64_t)slot | (0xFFFFFFFFull << 32);
}

// Master step, part 2: fork (admit joiners) and kill (query). Returns M'.
// Runs while every other member is parked in the barrier.
__device__ inline uint32_t resize_at_barrier(Ctx* c, uint32_t M, uint32_t new_epoch,
                                             uint32_t host_T) {
    const uint32_t N = c->N;
    const uint32_t T = query_target(c, new_epoch, host_T);
    // fork: k in [0, N - M], limited by registered joiners and the target
    uint32_t head = c->join_head;
    const uint32_t tail = ld_relaxed(&c->join_tail);
    const uint32_t want = T > M ? T - M : 0u;
    const uint32_t room = N - M;
    uint32_t k = 0;
    while (head != tail && k < room && k < want) {
        const uint32_t slot = head++;
        const uint64_t e = (uint64_t)slot | ((uint64_t)(new_epoch & 0xFFFFu) << 32) |
                           ((uint64_t)(M + k) << 48);
        const uint64_t prev = __hip_atomic_exchange(&c->join_entry[slot % kJoinCap], e,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == withdrawn_entry(slot)) continue;   // that joiner already left
        ++k;
    }
    c->join_head = head;
    const uint32_t M2 = M + k;
    // query/kill: the top W ids leave; workgroup 0 always stays
    uint32_t W = M2 > T ? M2 - T : 0u;
    if (W > M2 - 1) W = M2 - 1;
    const uint32_t Mn = M2 - W;
    if (k) c->forks += k;
    if (W) c->kills += W;
    if (Mn != M) c->resizes += 1;
    if (Mn < c->min_M) c->min_M = Mn;
    if (Mn > c->max_M) c->max_M = Mn;
    return Mn;
}

// Wait for the release word to move past `epoch` (or abort/done). Returns
// the word. Bounded by the watchdog.
__device__ inline uint64_t wait_release(Ctx* c, uint32_t epoch) {
    const uint64_t t0 = now_ticks();
    uint32_t spins = 0;
    for (;;) {
        const uint64_t r = ld_relaxed64(&c->release);
        if (rel_epoch(r) != epoch || (rel_flags(r) & (kFlagAbort | kFlagDone))) return r;
        if (++spins > 32) {
            __builtin_amdgcn_s_sleep(1);
            if ((spins & 255) == 0) {
                if (__hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    return r | ((uint64_t)kFlagAbort << 48);
                if (now_ticks() - t0 > c->watchdog_ticks) {
                    raise_error(c, kErrTimeout);
                    return ld_relaxed64(&c->release) | ((uint64_t)kFlagAbort << 48);
                }
            }
        }
    }
}

// Registration (thread 0 only). In a plain launch the workgroup id is the
// block id and M is the grid size. In a cooperative launch ticket 0 becomes
// logical 0 (M starts at 1); everybody else -- late-dispatched workgroups,
// workgroups of a joiner grid, killed workgroups re-queued in park mode --
// waits in the joiner queue until admitted at a barrier, until the kernel is
// done, or until it gives its compute unit back because the scheduler target
// leaves no room (host-driven schedule only) or the watchdog expires.
__device__ inline Member join_queue(Ctx* c) {
    Member m{};
    m.alive = 0;
    const uint32_t slot = add_relaxed(&c->join_tail, 1u);
    uint64_t* ent = &c->join_entry[slot % kJoinCap];
    const uint64_t t0 = now_ticks();
    for (uint32_t it = 0;; ++it) {
        uint64_t e = __hip_atomic_load(ent, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint64_t r = ld_relaxed64(&c->release);
        if ((uint32_t)e == slot && (e >> 32) != 0xFFFFFFFFull) {
            // admitted at epoch (e >> 32) & 0xFFFF as id (e >> 48): wait until
            // that epoch's release is visible, then start after the fork point
            const uint32_t aep = (uint32_t)(e >> 32) & 0xFFFFu;
            while ((rel_epoch(r) & 0xFFFFu) != aep &&
                   !(rel_flags(r) & (kFlagAbort | kFlagDone))) {
                __builtin_amdgcn_s_sleep(1);
                r = ld_relaxed64(&c->release);
            }
            fence_acquire();
            m.id = (uint32_t)(e >> 48);
            m.M = rel_M(r);
            m.epoch = rel_epoch(r);
            m.flags = rel_flags(r);
            m.alive = (m.flags & (kFlagAbort | kFlagDone)) ? 0u : 1u;
            return m;
        }
        bool leave = (rel_flags(r) & (kFlagAbort | kFlagDone)) != 0;
        if (!leave && c->host && !(c->mode & kModePark) && (it & 15) == 15) {
            // no room under the current target: give the compute unit back
            leave = ld_system(&c->host->target) <= rel_M(r);
        }
        if (!leave && now_ticks() - t0 > c->watchdog_ticks) leave = true;
        if (leave) {
            uint64_t expected = e;
            if (__hip_atomic_compare_exchange_strong(ent, &expected, withdrawn_entry(slot),
                                                     __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT))
                return m;            // withdrawn: the master will skip this slot
            continue;                // the master admitted us meanwhile: re-read
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

__device__ inline Member register_member(Ctx* c, bool plain, bool joiner_grid) {
    Member m{};
    if (plain) {
        m.id = blockIdx.x;
        m.M = gridDim.x;
        m.epoch = 0;
        m.flags = 0;
        m.alive = 1;
        return m;
    }
    if (!joiner_grid) {
        const uint32_t t = add_relaxed(&c->ticket, 1u);
        if (t == 0) {
            m.id = 0;
            m.M = 1;
            m.epoch = 0;
            m.flags = 0;
            m.alive = 1;
            return m;
        }
    }
    return join_queue(c);
}

// The (resizing) global barrier. Called by every thread of every active
// workgroup. `master_fn(M, new_epoch)` runs in thread 0 of the last
// arrival while all other members wait; it does the per-level bookkeeping
// and returns the flags to publish (kFlagDone ends the kernel). In a
// cooperative launch the barrier then admits joiners and applies the
// scheduler's target. `sh` is a workgroup-shared slot used to broadcast the
// new membership; `killed` tells the caller whether this workgroup left
// because the scheduler claimed it (as opposed to the kernel ending).
template <bool Coop, class MasterFn>
__device__ inline void barrier(Ctx* c, Member& m, Member* sh, uint32_t* killed, MasterFn&& master_fn) {
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t host_T = 0;
        if (Coop && c->host) host_T = ld_system(&c->host->target);   // prefetch the query
        const uint32_t old = __hip_atomic_fetch_add(&c->arrive, 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        Member n = m;
        uint32_t k = 0;
        if (old + 1 == m.M) {
            // master step: everybody else is parked in the barrier
            __hip_atomic_store(&c->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t ne = m.epoch + 1;
            uint32_t flags = master_fn(m.M, ne);
            if (__hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                flags |= kFlagAbort;
            uint32_t Mn = m.M;
            if (Coop && !(flags & (kFlagDone | kFlagAbort))) Mn = resize_at_barrier(c, m.M, ne, host_T);
            c->barriers += 1;
            if (flags & kFlagDone) { c->final_M = m.M; c->t_end = now_ticks(); }
            st_release64(&c->release, make_release(ne, Mn, flags));
            n.epoch = ne;
            n.M = Mn;
            n.flags = flags;
        } else {
            const uint64_t r = wait_release(c, m.epoch);
            fence_acquire();
            const uint32_t e = rel_epoch(r);
            n.flags = rel_flags(r);
            n.M = rel_M(r);
            n.epoch = e;
            // an alive member cannot miss an epoch: a gap means we were killed
            if (Coop && e != m.epoch + 1) k = 1;
        }
        if (Coop && n.id >= n.M) k = 1;
        if (n.flags & (kFlagDone | kFlagAbort)) k = 0;
        n.alive = (!k && !(n.flags & (kFlagDone | kFlagAbort))) ? 1u : 0u;
        *sh = n;
        *killed = k;
    }
    __syncthreads();
    m = *sh;
}

// Start-up: in a cooperative launch ticket 0 waits briefly for the rest of
// the grid to register, so the first barrier can admit them together.
__device__ inline void startup_wait(Ctx* c) {
    const uint64_t t0 = now_ticks();
    while (ld_relaxed(&c->join_tail) + 1 < gridDim.x && now_ticks() - t0 < c->epoch0_wait)
        __builtin_amdgcn_s_sleep(2);
}

}  // namespace coop
