// Serving kernel for gfx950: one persistent cooperative launch that runs
// BFS and SSSP queries on resident graphs as they arrive (continuous
// batching), each query by a team of workgroups.
//
//  * The host publishes a query by writing its record into the query's slot
//    (pinned memory), the slot index into the ticket-owner map for each of
//    the team's tickets, and then the end of the published ticket range.
//    A workgroup with nothing to do polls that word; it draws the next
//    ticket (compare-and-swap below the published end) and becomes rank
//    (ticket - first) of the query's team. Tickets are drawn in order, so
//    at most one team is incomplete at any time.
//  * A slot's barrier lines live on across its queries: members take the
//    current epoch when they start and the last barrier of a query carries
//    an END flag instead of DONE. The last member to leave a query writes
//    the slot's completion record, so the host reuses a slot only when no
//    member can still be waiting on its barrier.
//  * Between queries a workgroup may leave for the scheduler (offer_kill
//    against the host target, never below team_max workgroups). Inside a
//    query a team's master may also give up its top members at a barrier
//    (the resizing barrier, per team), so a co-task does not have to wait
//    for long queries to end. Joiner grids launched later enter between
//    queries (request_fork). These are the task-pattern calls of
//    coop_device.hpp on the launch context.
//  * One idle workgroup at a time, the relay, reads the host's words (ticket
//    end, stop, heartbeat, scheduler target) over PCIe and republishes them
//    in device memory; every other idle workgroup polls those copies, so
//    PCIe sees one reader however many workgroups are idle.
//  * Every value read from host memory is checked before it is used as an
//    index or a pointer (slot, descriptor, kind, rank, team, output); a bad
//    one stops the server with COOP_E_INTERNAL instead of being followed.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "traverse.h"

namespace {

typedef __attribute__((address_space(4))) const ServeDesc ConstDesc;

__device__ __forceinline__ uint64_t ld_system64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void fence_acquire_system() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, ""); }

// Barrier of a query's team. One-workgroup teams synchronise locally; larger
// teams use the counter barrier on the slot's lines, and in a cooperative
// launch with a host target the master may release its top members (never
// member 0) while the target is below the active count.
template <bool Coop, class MasterFn>
__device__ void serve_barrier(const ServeArgs& a, CtxCore* c, const Cfg tcfg, Member& m, BarrierLds& b,
                              const uint32_t* slots, MasterFn&& master_fn) {
    if (m.M == 1) {
        team_barrier(c, tcfg, m, b, master_fn);
        return;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t old = __hip_atomic_fetch_add(&c->arrive, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        b.is_master = ((uint32_t)(old & kArriveCount) + 1 == m.M) ? 1u : 0u;
        if (b.is_master) __hip_atomic_store(&c->arrive, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (b.is_master) {
        uint32_t flags = master_fn(m.M, m.epoch + 1);
        if (threadIdx.x == 0) {
            if (ld_relaxed_i(&c->error)) flags |= kFlagAbort;
            uint32_t Mn = m.M;
            if (Coop && a.cfg.host && !(flags & (kFlagEnd | kFlagAbort | kFlagDone))) {
                // give up top members while the launch holds more than the
                // target and their shader engine more than its share
                // (member 0 stays)
                const uint32_t T = ld_relaxed(&a.ctx->T_seen);       // the relayed host target
                const uint32_t engines = a.cfg.engines;
                while (Mn > 1) {
                    const uint32_t x = ld_relaxed(&slots[(size_t)(Mn - 1) * kSlotWords + kSlotEngine]);
                    if (!task_leave(&a.ctx->task, T, a.team_max, engines, x)) break;
                    --Mn;
                }
            }
            c->barriers += 1;
            const uint32_t ne = m.epoch + 1;
            st_release64(&c->release, make_release(ne, Mn, flags));
            Member n = m;
            n.epoch = ne;
            n.M = Mn;
            n.flags = flags;
            n.alive = ((flags & kFlagAbort) || n.id >= Mn) ? 0u : 1u;
            b.member = n;
            b.killed = n.id >= Mn ? 1u : 0u;
        }
    } else if (threadIdx.x == 0) {
        const uint64_t r = wait_release(c, tcfg, m.epoch);
        fence_acquire();
        Member n = m;
        n.epoch = rel_epoch(r);
        n.M = rel_M(r);
        n.flags = rel_flags(r);
        // a member that sees the epoch move by more than one was let go at
        // the epoch it missed (the next release needs every member), and
        // the slot may already be serving a later query: that query's
        // release is not this member's
        const bool gap = n.epoch != m.epoch + 1;
        const bool out = gap || n.id >= n.M;
        n.alive = ((n.flags & kFlagAbort) || out) ? 0u : 1u;
        b.member = n;
        b.killed = out ? 1u : 0u;
    }
    __syncthreads();
    m = b.member;
}

// Query start (thread 0): the slot's current epoch, this member's shader
// engine (for the team's master), and (rank 0) the transmit block's source
// index reset for this query.
__device__ __forceinline__ void query_start(BlockLds& sh, CtxCore* c, Work* wk, uint32_t* slots, uint32_t rank,
                                            uint32_t ses) {
    if (threadIdx.x == 0) {
        st_relaxed(&slots[(size_t)rank * kSlotWords + kSlotEngine], engine_id(ses));
        const uint64_t r = ld_relaxed64(&c->release);
        fence_acquire();
        sh.level = rel_epoch(r);
        if (rank == 0) st_relaxed(&wk->x.root, 0u);
    }
    __syncthreads();
}

// A BFS query. Returns the team size at the query's end, or 0 if this
// workgroup was released to the scheduler (or the slot aborted) and must
// leave the kernel.
template <bool Coop>
__device__ __forceinline__ uint32_t serve_bfs(const ServeArgs& a, const BfsArgs& p, BlockLds& sh, uint32_t rank,
                                          uint32_t team, const uint32_t* roots, uint32_t* out) {
    CtxCore* c = p.t.ctx;
    query_start(sh, c, p.t.work, p.t.slots, rank, p.t.cfg.ses);
    Member m{rank, team, sh.level, 0u, 1u};
    uint32_t level = 0, root = 0, ph = kPhInit;
    for (;;) {
        bfs_phase(p, sh, ph, m.flags, level, root, m.id, m.M, out);
        const uint32_t cur_flags = m.flags, cur_ph = ph;
        serve_barrier<Coop>(a, c, p.t.cfg, m, sh.bar, p.t.slots, [&](uint32_t M, uint32_t) -> uint32_t {
            uint32_t f = bfs_master(p, sh, c, cur_ph, cur_flags, roots, out, M);
            return (f & kFlagDone) ? ((f & ~kFlagDone) | kFlagEnd) : f;
        });
        if (!m.alive) return 0;
        if (m.flags & kFlagEnd) return m.M;
        bfs_follow(ph, m.flags, level, root, p.t.work);
        ph = m.flags & kPhMask;
    }
}

// An SSSP query (frontier Bellman-Ford); distances go to `out`, which is
// also the query's working state.
template <bool Coop>
__device__ __forceinline__ uint32_t serve_sssp(const ServeArgs& a, const SsspArgs& p, BlockLds& sh, uint32_t rank,
                                           uint32_t team, const uint32_t* roots, int32_t* out) {
    CtxCore* c = p.t.ctx;
    query_start(sh, c, p.t.work, p.t.slots, rank, p.t.cfg.ses);
    Member m{rank, team, sh.level, 0u, 1u};
    uint32_t root = 0, ph = kPhInit;
    for (;;) {
        sssp_phase(p, sh, ph, m.flags, out, m.id, m.M);
        const uint32_t cur_flags = m.flags, cur_ph = ph;
        serve_barrier<Coop>(a, c, p.t.cfg, m, sh.bar, p.t.slots, [&](uint32_t, uint32_t) -> uint32_t {
            uint32_t f = sssp_master(p, sh, c, cur_ph, cur_flags, roots, out);
            return (f & kFlagDone) ? ((f & ~kFlagDone) | kFlagEnd) : f;
        });
        if (!m.alive) return 0;
        if (m.flags & kFlagEnd) return m.M;
        sssp_follow(ph, m.flags, root);
        ph = m.flags & kPhMask;
    }
}

// Leaving a finished query: the last member (all of them are past the final
// barrier) resets the leave count and writes the completion record with
// system-scope release, after which the host may reuse the slot.
__device__ void query_leave(const ServeArgs& a, CtxCore* c, uint32_t slot, uint32_t M, uint64_t seq) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t old = __hip_atomic_fetch_add(&c->ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == M) {
            __hip_atomic_store(&c->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ServeDone* d = &a.done[slot];
            __hip_atomic_store(&d->t_end, now_ticks(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&d->error, ld_relaxed_i(&c->error), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&d->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            add_relaxed(&a.ctl->queries, 1u);
        }
    }
}

// Thread 0 of an idle workgroup: the next ticket, or why to leave (1 error,
// 2 taken by the scheduler, 3 stop). The relay reads the host's words and
// republishes them; the others read the copies.
template <bool Coop>
__device__ uint32_t serve_next_ticket(const ServeArgs& a, Group& g, uint32_t& k, uint32_t& hb_seen,
                                      uint64_t& hb_t, uint32_t& beat_seen, uint64_t& beat_t) {
    ServeCtl* ctl = a.ctl;
    bool relay = false;
    uint32_t idle = 0;
    for (uint32_t it = 0;; ++it) {
        if (ld_relaxed_i(&ctl->error)) break;
        if (!relay && ld_relaxed(&ctl->relay) == 0) {
            uint32_t z = 0;
            relay = __hip_atomic_compare_exchange_strong(&ctl->relay, &z, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
        }
        const uint64_t now = now_ticks();
        if (relay) {
            st_relaxed(&ctl->end, ld_system(&a.host->ticket_end));
            st_relaxed(&ctl->stop, ld_system(&a.host->stop));
            if (Coop && a.cfg.host) st_relaxed(&a.ctx->T_seen, ld_system(&a.cfg.host->target));
            add_relaxed(&ctl->beat, 1u);
            if ((it & 63) == 63) {
                // the host's poller advances its heartbeat every millisecond:
                // a server whose process has gone stops itself
                const uint32_t hb = ld_system(&a.host->heartbeat);
                if (hb != hb_seen) {
                    hb_seen = hb;
                    hb_t = now;
                } else if (now - hb_t > a.cfg.watchdog_ticks) {
                    atomicCAS(&ctl->error, 0, kErrTimeout);
                    break;
                }
            }
        } else if ((it & 63) == 63) {
            // the relay itself must be alive: its beat moves at every poll
            const uint32_t b = ld_relaxed(&ctl->beat);
            if (b != beat_seen) {
                beat_seen = b;
                beat_t = now;
            } else if (ld_relaxed(&ctl->relay) != 0 && now - beat_t > a.cfg.watchdog_ticks) {
                atomicCAS(&ctl->error, 0, kErrTimeout);
                break;
            }
        }
        uint32_t t = ld_relaxed(&ctl->ticket);
        const uint32_t end = ld_relaxed(&ctl->end);
        if (t < end) {
            if (__hip_atomic_compare_exchange_strong(&ctl->ticket, &t, t + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
                k = t;
                if (relay) st_relaxed(&ctl->relay, 0u);      // hand the role to another idle workgroup
                return 0;
            }
            continue;
        }
        if (ld_relaxed(&ctl->stop)) {
            if (relay) st_relaxed(&ctl->relay, 0u);
            return 3;
        }
        // idle: back off to about 10 us between polls (the relay polls faster)
        idle = idle < 16 ? idle + 1 : 16;
        for (uint32_t z = 0; z < (relay ? 1u : idle); ++z) __builtin_amdgcn_s_sleep(16);
    }
    if (relay) st_relaxed(&ctl->relay, 0u);
    return 1;
}

template <bool Coop>
__device__ __forceinline__ void serve_body(const ServeArgs& a, bool joiner) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    ServeCtl* ctl = a.ctl;
    // the launch-wide membership (task pattern) keeps its own LDS: sh.bar
    // holds the team barrier of the query being served
    __shared__ BarrierLds gbar;
    Group g(a.ctx, a.cfg, gbar);
    __shared__ uint32_t q_desc, q_kind, q_rank, q_team, q_slot, q_leave;
    __shared__ uint64_t q_out, q_seq;
    if (threadIdx.x == 0) {
        for (uint32_t i = 0; i < num_waves(); ++i) sh.wave[i].out_n = 0;
        for (int i = 0; i < 8; ++i) sh.acc[i] = 0;
    }
    if (!coop_task_start<Coop>(g, joiner)) return;
    uint32_t hb_seen = 0, beat_seen = 0;
    uint64_t hb_t = now_ticks(), beat_t = hb_t;
    for (;;) {
        // between queries: offer this workgroup to the scheduler, let
        // waiting joiners in
        if (!coop_offer_kill<Coop>(g)) return;
        coop_request_fork<Coop>(g);
        if (threadIdx.x == 0) {
            uint32_t k = 0;
            uint32_t leave = serve_next_ticket<Coop>(a, g, k, hb_seen, hb_t, beat_seen, beat_t);
            if (!leave) {
                fence_acquire_system();
                // every value from host memory is checked before it is used
                const uint32_t slot = ld_system(&a.owner[k % a.owner_cap]);
                bool ok = slot < a.slots;
                if (ok) {
                    const ServeReq* q = &a.req[slot];
                    q_desc = ld_system(&q->desc);
                    q_kind = ld_system(&q->kind);
                    q_team = ld_system(&q->team);
                    const uint32_t first = ld_system(&q->first);
                    q_rank = k - first;
                    q_out = ld_system64(&q->out);
                    q_seq = ld_system64(&q->seq);
                    q_slot = slot;
                    ok = q_desc < a.ndesc && (q_kind == kQueryBfs || q_kind == kQuerySssp) && q_team >= 1 &&
                         q_team <= a.team_max && (int32_t)(k - first) >= 0 && q_rank < q_team && q_out != 0;
                }
                if (!ok) {
                    atomicCAS(&ctl->error, 0, kErrInternal);
                    leave = 1;
                }
            }
            if (leave) add_relaxed(&ctl->left, 1u);
            q_leave = leave;
        }
        __syncthreads();
        if (q_leave) {
            coop_task_leave(g);
            return;
        }
        const uint32_t di = __builtin_amdgcn_readfirstlane(q_desc);
        const uint32_t kind = __builtin_amdgcn_readfirstlane(q_kind);
        const uint32_t rank = __builtin_amdgcn_readfirstlane(q_rank);
        const uint32_t team = __builtin_amdgcn_readfirstlane(q_team);
        const uint32_t slot = __builtin_amdgcn_readfirstlane(q_slot);
        const uint64_t out = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(q_out >> 32)) << 32) |
                             __builtin_amdgcn_readfirstlane((uint32_t)q_out);
        const uint64_t seq = q_seq;
        const ServeDesc& D = *(const ServeDesc*)((ConstDesc*)(uintptr_t)a.desc + di);
        const uint32_t* roots = &a.req[slot].src;
        uint32_t stay;
        CtxCore* c;
        if (kind == kQueryBfs) {
            c = D.bfs.t.ctx;
            stay = serve_bfs<Coop>(a, D.bfs, sh, rank, team, roots, reinterpret_cast<uint32_t*>(out));
        } else {
            c = D.sssp.t.ctx;
            stay = serve_sssp<Coop>(a, D.sssp, sh, rank, team, roots, reinterpret_cast<int32_t*>(out));
        }
        if (stay == 0) {
            // let go by the team's master (already taken off the active
            // count, its slot with it) or the query failed
            if (threadIdx.x == 0) {
                if (!sh.bar.killed) {
                    atomicCAS(&ctl->error, 0, ld_relaxed_i(&c->error) ? ld_relaxed_i(&c->error) : kErrInternal);
                } else {
                    __hip_atomic_store(&a.ctx->task.slot_owner[coop_get_group_id(g)], 0u, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    g.bar.member.alive = 0;
                }
            }
            __syncthreads();
            coop_task_leave(g);
            return;
        }
        query_leave(a, c, slot, stay, seq);
        __syncthreads();
    }
}

}  // namespace

template <bool Coop>
__global__ void __launch_bounds__(1024) serve_kernel(ServeArgs a, int joiner) { serve_body<Coop>(a, joiner != 0); }

// Zero the slots' barrier lines (release word: epoch 0) and the counters.
__global__ void serve_init_kernel(TeamState* teams, uint32_t slots, ServeCtl* ctl) {
    constexpr uint32_t words = sizeof(TeamState) / 4;
    for (uint32_t t = blockIdx.x; t < slots; t += gridDim.x) {
        uint32_t* w = reinterpret_cast<uint32_t*>(&teams[t]);
        for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0;
    }
    if (blockIdx.x == 0) {
        uint32_t* w = reinterpret_cast<uint32_t*>(ctl);
        for (uint32_t i = threadIdx.x; i < sizeof(ServeCtl) / 4; i += blockDim.x) w[i] = 0;
        __syncthreads();
    }
}

namespace coop {

hipError_t launch_serve_init(TeamState* teams, uint32_t slots, ServeCtl* ctl, hipStream_t s) {
    const uint32_t grid = slots < 1024 ? (slots ? slots : 1) : 1024;
    hipLaunchKernelGGL(serve_init_kernel, dim3(grid), dim3(256), 0, s, teams, slots, ctl);
    return hipGetLastError();
}

hipError_t launch_serve(const ServeArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                        uint32_t lds_bytes, hipStream_t s) {
    auto k = coop ? serve_kernel<true> : serve_kernel<false>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_bytes);
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds_bytes, s, a, joiner_grid ? 1 : 0);
    return hipGetLastError();
}

uint32_t occupancy_serve(bool coop, uint32_t block, uint32_t lds_bytes) {
    auto k = coop ? serve_kernel<true> : serve_kernel<false>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_bytes);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, (int)block, lds_bytes) != hipSuccess) return 1;
    return n > 0 ? (uint32_t)n : 1u;
}

}  // namespace coop
