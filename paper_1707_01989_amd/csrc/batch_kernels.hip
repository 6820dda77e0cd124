// Batched persistent kernel for gfx950: hundreds of independent graph
// instances in one launch, each run by a team of workgroups with its own
// barrier.
//
// The paper's cooperative kernel runs one blocking algorithm over all
// workgroups. A batch of small, uneven graphs would spend most of its time
// in global barriers that way, so this kernel gives every instance a team
// sized to its work and lets the teams run side by side:
//  * instances are laid out in ticket order (largest first); instance i owns
//    tickets [first[i], first[i] + team_i). A workgroup draws the next
//    ticket with one atomic and becomes rank (ticket - first[i]) of team i.
//    Tickets are drawn in order, so at most one team is ever incomplete;
//    every other team's members are running, finish and draw again, so the
//    incomplete team fills as long as at least team_max workgroups remain;
//  * a team runs the same level-synchronous BFS (direction-optimising) and
//    Jones-Plassmann colouring/MIS phases as the single-traversal kernels,
//    with a barrier over its own members (a one-workgroup team needs no
//    global atomics at all);
//  * between instances a workgroup holds no team state, which is where the
//    cooperative scheduler may take it (offer_kill: the host target or a
//    seeded random schedule, never below team_max workgroups) or where
//    workgroups of a later joiner grid come in (request_fork).
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "traverse.h"

namespace {

typedef __attribute__((address_space(4))) const BatchInst ConstInst;
typedef __attribute__((address_space(4))) const uint32_t ConstU32;

// BFS of one instance by rank `rank` of a team of `team` workgroups; the
// first phase clears the instance's state, the first master step places
// the source.
__device__ __forceinline__ void bfs_team(const BfsArgs& p, BlockLds& sh, uint32_t rank, uint32_t team) {
    CtxCore* c = p.t.ctx;
    Member m{rank, team, 0u, 0u, 1u};
    uint32_t level = 0, root = 0, ph = kPhInit;
    for (;;) {
        bfs_phase(p, sh, ph, m.flags, level, root, m.id, m.M, p.level_out);
        const uint32_t cur_flags = m.flags, cur_ph = ph;
        team_barrier(c, p.t.cfg, m, sh.bar,
                     [&](uint32_t M, uint32_t) -> uint32_t {
                         return bfs_master(p, sh, c, cur_ph, cur_flags, p.t.roots, p.level_out, M);
                     });
        if (!m.alive) return;
        bfs_follow(ph, m.flags, level, root, p.t.work);
        ph = m.flags & kPhMask;
    }
}

// Colouring / MIS of one instance: SETUP, then one round per barrier.
__device__ __forceinline__ void color_team(const ColorArgs& p, BlockLds& sh, uint32_t rank, uint32_t team) {
    CtxCore* c = p.t.ctx;
    Member m{rank, team, 0u, 0u, 1u};
    uint32_t ph = kPhSetup;
    for (;;) {
        color_phase(p, sh, ph, m.flags, m.id, m.M);
        const uint32_t cur_flags = m.flags, cur_ph = ph;
        team_barrier(c, p.t.cfg, m, sh.bar,
                     [&](uint32_t, uint32_t) -> uint32_t { return color_master(p, sh, cur_ph, cur_flags); });
        if (!m.alive) return;
        ph = m.flags & kPhMask;
    }
}

template <bool Coop>
__device__ __forceinline__ void batch_body(const BatchArgs& a, bool joiner) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    BlockLds& sh = *reinterpret_cast<BlockLds*>(lds_raw);
    BatchCtl* ctl = a.ctl;
    Group g(a.ctx, a.cfg, sh.bar);
    ConstU32* first = (ConstU32*)(uintptr_t)a.first;
    const uint32_t total = first[a.count];
    if (threadIdx.x == 0) {
        // only the waves of this group size have LDS behind them
        for (uint32_t i = 0; i < num_waves(); ++i) sh.wave[i].out_n = 0;
        for (int i = 0; i < 8; ++i) sh.acc[i] = 0;
    }
    // the task pattern of the programming model: a workgroup holds no team
    // state between instances, which is where it offers itself to the
    // scheduler (offer_kill: host target or seeded schedule, never below
    // team_max workgroups) and lets waiting joiners in (request_fork)
    if (!coop_task_start<Coop>(g, joiner)) return;
    for (;;) {
        if (!coop_offer_kill<Coop>(g)) return;
        coop_request_fork<Coop>(g);
        if (threadIdx.x == 0) {
            uint32_t leave = ld_relaxed_i(&ctl->error) ? 1u : 0u;
            if (!leave) {
                const uint32_t k = add_relaxed(&ctl->ticket, 1u);
                if (k >= total) {
                    leave = 3;
                } else {
                    uint32_t lo = 0, hi = a.count;       // first[lo] <= k < first[hi]
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (first[mid] <= k) lo = mid; else hi = mid;
                    }
                    sh.root = lo;
                    sh.aux = k - first[lo];
                }
            }
            if (leave) add_relaxed(&ctl->left, 1u);
            sh.level = leave;
        }
        __syncthreads();
        if (sh.level) {
            // out of work (or an instance failed): joiners still waiting go too
            coop_task_leave(g);
            coop_task_finish(g);
            return;
        }
        const uint32_t i = __builtin_amdgcn_readfirstlane(sh.root);
        const uint32_t rank = __builtin_amdgcn_readfirstlane(sh.aux);
        const BatchInst& I = *(const BatchInst*)((ConstInst*)(uintptr_t)a.inst + i);
        const uint32_t ops = I.ops, team = I.team;
        // the team barriers keep their membership in the same LDS block as
        // the launch-wide (task-pattern) one, and leave it at the team's
        // rank and not alive when the instance ends: the launch-wide one is
        // put back before the next offer_kill
        const Member task_member = g.bar.member;
        if (ops & kBatchBfs) bfs_team(I.bfs, sh, rank, team);
        if (ops & kBatchColor) color_team(I.col, sh, rank, team);
        if (threadIdx.x == 0) {
            int32_t e = ld_relaxed_i(&I.bfs.t.ctx->error);
            if (!e) e = ld_relaxed_i(&I.col.t.ctx->error);
            if (e) atomicCAS(&ctl->error, 0, e);
            g.bar.member = task_member;
            g.bar.killed = 0;
        }
        __syncthreads();
    }
}

}  // namespace

template <bool Coop>
__global__ void __launch_bounds__(1024) batch_kernel(BatchArgs a, int joiner) { batch_body<Coop>(a, joiner != 0); }

// Zero every team block and set its release words (epoch 0, M = team).
__global__ void batch_init_kernel(TeamState* teams, const BatchInst* inst, uint32_t count, BatchCtl* ctl) {
    constexpr uint32_t words = sizeof(TeamState) / 4;
    for (uint32_t t = blockIdx.x; t < count; t += gridDim.x) {
        uint32_t* w = reinterpret_cast<uint32_t*>(&teams[t]);
        for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t team = inst[t].team;
            teams[t].bfs_ctx.release = make_release(0, team, 0);
            teams[t].col_ctx.release = make_release(0, team, 0);
            teams[t].bfs_ctx.min_M = team;
            teams[t].col_ctx.min_M = team;
        }
        __syncthreads();
    }
    if (blockIdx.x == 0) {
        uint32_t* w = reinterpret_cast<uint32_t*>(ctl);
        for (uint32_t i = threadIdx.x; i < sizeof(BatchCtl) / 4; i += blockDim.x) w[i] = 0;
        __syncthreads();
    }
}

namespace coop {

hipError_t launch_batch_init(TeamState* teams, const BatchInst* inst, uint32_t count, BatchCtl* ctl,
                             hipStream_t s) {
    const uint32_t grid = count < 1024 ? (count ? count : 1) : 1024;
    hipLaunchKernelGGL(batch_init_kernel, dim3(grid), dim3(256), 0, s, teams, inst, count, ctl);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                        uint32_t lds_bytes, hipStream_t s) {
    auto k = coop ? batch_kernel<true> : batch_kernel<false>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_bytes);
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds_bytes, s, a, joiner_grid ? 1 : 0);
    return hipGetLastError();
}

uint32_t occupancy_batch(bool coop, uint32_t block, uint32_t lds_bytes) {
    auto k = coop ? batch_kernel<true> : batch_kernel<false>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_bytes);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, (int)block, lds_bytes) != hipSuccess) return 1;
    return n > 0 ? (uint32_t)n : 1u;
}

}  // namespace coop
