// Connected components by minimum-label propagation, written only against
// the programming-model calls of coop_device.hpp (coop_start,
// coop_get_group_id, coop_get_num_groups, coop_resizing_global_barrier,
// coop_transmit_block, coop_rejoin): the level-by-level pattern of the
// paper's cooperative graph traversal, where every round is one resizing-
// barrier interval whose work is split statically over the M workgroups of
// that interval, and a round number is the transmitted state.
//
// Round 0 labels every vertex with its own id. Every later round lowers
// each vertex's label to the smallest label among its neighbours (atomic
// minimum) and marks the round as changed when one dropped. The single
// step of the barrier ends the kernel after a round that changed nothing:
// the labels then agree across every arc, so each component carries one
// label, and since labels only ever move between vertices of a component
// and its smallest vertex keeps its own id, that label is the smallest id
// of the component -- whatever the schedule, the kills and the forks.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "coop_device.hpp"
#include "coop_internal.h"

using namespace coop;

namespace {

template <bool Coop>
__device__ void cc_body(const CcArgs& a, bool joiner_grid) {
    __shared__ BarrierLds bar;
    __shared__ uint32_t round_sh, flags_sh;
    Group g(a.ctx, a.cfg, bar);
    if (!coop_start<Coop>(g, joiner_grid)) return;
    if (threadIdx.x == 0) round_sh = coop_joined(g) ? coop_transmit_block(g)[0] : 0u;
    __syncthreads();
    uint32_t round = round_sh;
    for (;;) {
        if (!g.bar.member.alive) {
            // killed (parked launches wait to be forked in again)
            if (!coop_rejoin<Coop>(g)) return;
            if (threadIdx.x == 0) round_sh = coop_transmit_block(g)[0];
            __syncthreads();
            round = round_sh;
            continue;
        }
        const uint32_t id = coop_get_group_id(g), M = coop_get_num_groups(g);
        const uint32_t stride = M * blockDim.x;
        if (round == 0) {
            for (uint32_t v = id * blockDim.x + threadIdx.x; v < a.n; v += stride) a.label[v] = v;
        } else {
            bool dropped = false;
            for (uint32_t v = id * blockDim.x + threadIdx.x; v < a.n; v += stride) {
                const uint32_t lv = __hip_atomic_load(&a.label[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                uint32_t best = lv;
                for (uint32_t e = a.row_ptr[v], end = a.row_ptr[v + 1]; e < end; ++e) {
                    const uint32_t lu = __hip_atomic_load(&a.label[a.col[e]], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                    best = lu < best ? lu : best;
                }
                if (best < lv) {
                    atomicMin(&a.label[v], best);
                    dropped = true;
                }
            }
            if (__any(dropped) && (threadIdx.x & 63) == 0)
                __hip_atomic_store(&a.changed[round & 1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        coop_resizing_global_barrier<Coop>(g, [&](uint32_t, uint32_t) -> uint32_t {
            // single step: end after a round that changed nothing, clear the
            // next round's mark, and transmit the next round number
            if (threadIdx.x == 0) {
                uint32_t* tx = coop_transmit_block(g);
                const uint32_t r = tx[0];
                const bool quiet = r > 0 && __hip_atomic_load(&a.changed[r & 1], __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT) == 0u;
                __hip_atomic_store(&a.changed[(r + 1) & 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                tx[0] = r + 1;
                flags_sh = quiet ? kFlagDone : 0u;
            }
            __syncthreads();
            return flags_sh;
        });
        round += 1;
    }
}

}  // namespace

template <bool Coop>
__global__ void __launch_bounds__(1024) cc_kernel(CcArgs a, int joiner) { cc_body<Coop>(a, joiner != 0); }

namespace coop {

hipError_t launch_cc(const CcArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                     uint32_t lds_bytes, hipStream_t s) {
    auto k = coop ? cc_kernel<true> : cc_kernel<false>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_bytes);
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds_bytes, s, a, joiner_grid ? 1 : 0);
    return hipGetLastError();
}

}  // namespace coop
