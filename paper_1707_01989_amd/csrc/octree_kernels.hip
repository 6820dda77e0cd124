// Work-stealing octree build for gfx950: the paper's second class of
// cooperative kernels (work stealing, section 3.2, and the octree of Table
// 1). Every workgroup owns a task queue (a slot); a task is a cube whose
// points get split into its 8 child cubes. A workgroup pops its own newest
// task, or steals the oldest task of another queue (mutex per queue by
// compare-and-swap), splits the cube with the whole workgroup, records the
// children that are leaves and pushes the others as new tasks.
//
// Cooperative version (section 3.2, "Adapting Work Stealing"): at the top
// of the main loop a workgroup offers itself to the scheduler (offer_kill)
// before it takes a task; it may leave with tasks still in its queue, which
// the others steal. There is no id order to keep, so the workgroup that
// leaves is one whose shader engine holds more than its share of the
// target (kill in any order, Appendix B), and the queue belongs to the
// slot, not to the workgroup: a joiner (request_fork, via a host-launched
// joiner grid) takes any free slot, queue and remaining tasks included.
//
// Cube rules: coordinates have 21 bits; a cube at depth d has side
// 2^(21 - d); its child index is 4 bx + 2 by + bz for bit (20 - d); a cube
// with at most `cap` points, or at depth 21, is a leaf. Splits are stable,
// so the final point order and the leaves do not depend on the schedule.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "traverse.h"

namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t child_of(const uint4 p, uint32_t bit) {
    return (((p.x >> bit) & 1u) << 2) | (((p.y >> bit) & 1u) << 1) | ((p.z >> bit) & 1u);
}

// ------------------------------------------------------- queues (thread 0)

__device__ bool q_lock(OctQueue* q, const Cfg& cfg, OctCtl* ctl) {
    const uint64_t t0 = now_ticks();
    for (uint32_t spins = 0;; ++spins) {
        uint32_t expected = 0;
        if (__hip_atomic_compare_exchange_strong(&q->lock, &expected, 1u, __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return true;
        __builtin_amdgcn_s_sleep(1);
        if ((spins & 255) == 255 && now_ticks() - t0 > cfg.watchdog_ticks) {
            atomicCAS(&ctl->error, 0, kErrTimeout);
            return false;
        }
    }
}

__device__ __forceinline__ void q_unlock(OctQueue* q) {
    __hip_atomic_store(&q->lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Take the newest task (own queue, `newest`) or the oldest (stealing).
__device__ uint32_t q_take(OctQueue* q, bool newest, const Cfg& cfg, OctCtl* ctl) {
    if (ld_relaxed(&q->tail) == ld_relaxed(&q->head)) return kNone;     // empty: no lock
    if (!q_lock(q, cfg, ctl)) return kNone;
    const uint32_t h = ld_relaxed(&q->head), t = ld_relaxed(&q->tail);
    uint32_t id = kNone;
    if (t != h) {
        if (newest) {
            id = q->ring[(t - 1) % kOctQueueCap];
            st_relaxed(&q->tail, t - 1);
        } else {
            id = q->ring[h % kOctQueueCap];
            st_relaxed(&q->head, h + 1);
        }
    }
    q_unlock(q);
    return id;
}

__device__ bool q_push(OctQueue* q, const uint32_t* ids, uint32_t k, const Cfg& cfg, OctCtl* ctl) {
    if (!q_lock(q, cfg, ctl)) return false;
    const uint32_t h = ld_relaxed(&q->head);
    uint32_t t = ld_relaxed(&q->tail);
    bool ok = t - h + k <= kOctQueueCap;
    if (ok) {
        for (uint32_t j = 0; j < k; ++j, ++t) q->ring[t % kOctQueueCap] = ids[j];
        st_relaxed(&q->tail, t);
    }
    q_unlock(q);
    if (!ok) atomicCAS(&ctl->error, 0, kErrInternal);
    return ok;
}

// -------------------------------------------------------- one task (all threads)

struct OctLds {
    uint32_t node[5];          // first, end, depth, code_lo, code_hi
    uint32_t cnt[8];           // points per child
    uint32_t start[8];         // first position of each child
    uint32_t base[8];          // next free position of each child (scatter)
    uint32_t wc[kMaxWaves][8]; // per chunk: points per (wave, child)
    uint32_t woff[kMaxWaves][8];
    uint32_t child_ids[8];     // new tasks
    uint32_t nchild;
    uint32_t copy_first[8], copy_end[8];   // odd-depth leaves to move to buf[0]
    uint32_t ncopy;
    uint32_t task, leave;
};

__device__ void split_task(const OctreeArgs& a, OctLds& L, uint32_t slot) {
    const uint32_t tid = threadIdx.x, nthreads = blockDim.x, w = wave_id(), l = lane_id();
    OctCtl* ctl = a.ctl;
    if (tid == 0) {
        const uint32_t* nd = a.nodes + 8ull * L.task;
        for (int i = 0; i < 5; ++i) L.node[i] = nd[i];
        L.nchild = 0;
        L.ncopy = 0;
    }
    if (tid < 8) L.cnt[tid] = 0;
    __syncthreads();
    const uint32_t first = L.node[0], end = L.node[1], depth = L.node[2];
    const uint64_t code = (uint64_t)L.node[3] | ((uint64_t)L.node[4] << 32);
    const uint32_t count = end - first;
    const uint4* src = a.buf[depth & 1];

    if (count <= a.cap || depth >= kOctMaxDepth) {
        // a leaf task (only the root can be one): its points are in place
        if (tid == 0) {
            const uint32_t k = add_relaxed(&ctl->leaf_count, 1u);
            if (k < a.leaf_cap) {
                uint32_t* lf = a.leaves + 8ull * k;
                lf[0] = first; lf[1] = end; lf[2] = depth; lf[3] = (uint32_t)code; lf[4] = (uint32_t)(code >> 32);
            } else {
                atomicCAS(&ctl->error, 0, kErrInternal);
            }
        }
        if (depth & 1)
            for (uint32_t i = first + tid; i < end; i += nthreads) a.buf[0][i] = a.buf[1][i];
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) add_relaxed(&ctl->outstanding, 0xFFFFFFFFu);
        return;
    }

    const uint32_t bit = (kOctMaxDepth - 1) - depth;
    uint4* dst = a.buf[(depth + 1) & 1];
    // pass 1: points per child (per-wave ballots, one LDS add per wave and child)
    for (uint32_t b = first; b < end; b += nthreads) {
        const uint32_t i = b + tid;
        const uint32_t c = i < end ? child_of(src[i], bit) : 8u;
#pragma unroll
        for (uint32_t cc = 0; cc < 8; ++cc) {
            const uint64_t m = __ballot(c == cc);
            if (l == 0 && m) atomicAdd(&L.cnt[cc], (uint32_t)__popcll(m));
        }
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = first;
        for (int c = 0; c < 8; ++c) {
            L.start[c] = acc;
            L.base[c] = acc;
            acc += L.cnt[c];
        }
    }
    __syncthreads();
    // pass 2: stable scatter, one chunk of blockDim points at a time; inside
    // a chunk the rank of a point among its child's points is (points of
    // earlier waves) + (earlier lanes of its wave)
    const uint32_t nw = num_waves();
    for (uint32_t b = first; b < end; b += nthreads) {
        const uint32_t i = b + tid;
        const bool act = i < end;
        const uint4 p = act ? src[i] : make_uint4(0, 0, 0, 0);
        const uint32_t c = act ? child_of(p, bit) : 8u;
        uint32_t rank = 0;
#pragma unroll
        for (uint32_t cc = 0; cc < 8; ++cc) {
            const uint64_t m = __ballot(c == cc);
            if (l == 0) L.wc[w][cc] = (uint32_t)__popcll(m);
            if (c == cc) rank = mbcnt(m);
        }
        __syncthreads();
        if (tid < 8) {
            uint32_t run = L.base[tid];
            for (uint32_t ww = 0; ww < nw; ++ww) {
                L.woff[ww][tid] = run;
                run += L.wc[ww][tid];
            }
            L.base[tid] = run;
        }
        __syncthreads();
        if (act) dst[L.woff[w][c] + rank] = p;
        __syncthreads();
    }
    // children: leaves are recorded now, the others become tasks
    if (tid == 0) {
        for (uint32_t c = 0; c < 8; ++c) {
            const uint32_t k = L.cnt[c];
            if (!k) continue;
            const uint32_t cf = L.start[c], ce = cf + k, cd = depth + 1;
            const uint64_t cc = (code << 3) | c;
            if (k <= a.cap || cd >= kOctMaxDepth) {
                const uint32_t li = add_relaxed(&ctl->leaf_count, 1u);
                if (li < a.leaf_cap) {
                    uint32_t* lf = a.leaves + 8ull * li;
                    lf[0] = cf; lf[1] = ce; lf[2] = cd; lf[3] = (uint32_t)cc; lf[4] = (uint32_t)(cc >> 32);
                } else {
                    atomicCAS(&ctl->error, 0, kErrInternal);
                }
                if (cd & 1) {
                    L.copy_first[L.ncopy] = cf;
                    L.copy_end[L.ncopy] = ce;
                    ++L.ncopy;
                }
            } else {
                const uint32_t id = add_relaxed(&ctl->node_count, 1u);
                if (id < a.node_cap) {
                    uint32_t* nd = a.nodes + 8ull * id;
                    nd[0] = cf; nd[1] = ce; nd[2] = cd; nd[3] = (uint32_t)cc; nd[4] = (uint32_t)(cc >> 32);
                    L.child_ids[L.nchild++] = id;
                } else {
                    atomicCAS(&ctl->error, 0, kErrInternal);
                }
            }
        }
    }
    __syncthreads();
    // leaves at odd depth sit in buf[1]: move them to the result
    for (uint32_t j = 0; j < L.ncopy; ++j)
        for (uint32_t i = L.copy_first[j] + tid; i < L.copy_end[j]; i += nthreads) a.buf[0][i] = a.buf[1][i];
    // every wave's stores are done before the children are published (the
    // queue's release then writes them back for the thief's XCD)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
        if (L.nchild) q_push(&a.q[slot], L.child_ids, L.nchild, a.cfg, ctl);
        add_relaxed(&ctl->outstanding, L.nchild - 1u);
        add_relaxed(&ctl->tasks, 1u);
    }
}

// ------------------------------------------------------------ the kernel

// The task pattern of the programming model (section 3.2, "Adapting Work
// Stealing"): offer_kill and request_fork at the top of the main loop, the
// queue id (the slot) taken when the workgroup becomes active, not
// transmitted.
template <bool Coop>
__device__ void octree_body(const OctreeArgs& a, bool joiner) {
    __shared__ OctLds L;
    __shared__ BarrierLds bar;
    OctCtl* ctl = a.ctl;
    const uint32_t N = a.cfg.N;
    Group g(a.ctx, a.cfg, bar);
    if (!coop_task_start<Coop>(g, joiner)) return;
    const uint32_t slot = coop_get_group_id(g);
    uint32_t rng = (blockIdx.x + 1) * 0x9E3779B9u ^ (slot << 16);
    uint64_t idle_since = now_ticks();          // thread 0: since it last had a task
    for (;;) {
        if (threadIdx.x == 0) L.leave = (ld_relaxed_i(&ctl->error) || ld_relaxed(&ctl->outstanding) == 0) ? 2u : 0u;
        __syncthreads();
        if (L.leave) {
            // every task is done (or one failed): joiners still waiting go too
            coop_task_leave(g);
            coop_task_finish(g);
            return;
        }
        // offer_kill before taking a task: a workgroup may leave with tasks
        // queued, the others steal them
        if (!coop_offer_kill<Coop>(g)) return;
        coop_request_fork<Coop>(g);
        if (threadIdx.x == 0) {
            uint32_t task = q_take(&a.q[slot], true, a.cfg, ctl);
            for (int attempt = 0; attempt < 8 && task == kNone; ++attempt) {
                rng ^= rng << 13;
                rng ^= rng >> 17;
                rng ^= rng << 5;
                const uint32_t v = rng % N;
                if (v != slot) {
                    task = q_take(&a.q[v], false, a.cfg, ctl);
                    if (task != kNone) add_relaxed(&ctl->steals, 1u);
                }
            }
            if (task != kNone) {
                idle_since = now_ticks();
            } else {
                __builtin_amdgcn_s_sleep(2);
                if (now_ticks() - idle_since > a.cfg.watchdog_ticks) atomicCAS(&ctl->error, 0, kErrTimeout);
            }
            L.task = task;
        }
        __syncthreads();
        if (L.task == kNone) continue;
        split_task(a, L, slot);
        __syncthreads();
    }
}

}  // namespace

template <bool Coop>
__global__ void __launch_bounds__(1024) octree_kernel(OctreeArgs a, int joiner) { octree_body<Coop>(a, joiner != 0); }

// Points into buf[0] as {x, y, z, index}; counters, queues and slots
// cleared; the root cube as node 0 in queue 0.
__global__ void octree_init_kernel(OctreeArgs a, const uint32_t* x, const uint32_t* y, const uint32_t* z) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = tid; i < a.n; i += stride) a.buf[0][i] = make_uint4(x[i], y[i], z[i], (uint32_t)i);
    for (uint64_t s = tid; s < a.cfg.N; s += stride) {
        a.q[s].lock = 0;
        a.q[s].head = 0;
        a.q[s].tail = 0;
    }
    if (tid < sizeof(OctCtl) / 4) reinterpret_cast<uint32_t*>(a.ctl)[tid] = 0;
    __syncthreads();
    if (tid == 0) {
        a.nodes[0] = 0;
        a.nodes[1] = a.n;
        a.nodes[2] = 0;
        a.nodes[3] = 0;
        a.nodes[4] = 0;
        if (a.n) {
            a.q[0].ring[0] = 0;
            a.q[0].tail = 1;
            a.ctl->outstanding = 1;
        }
        a.ctl->node_count = 1;
    }
}

namespace coop {

hipError_t launch_octree_init(const OctreeArgs& a, const uint32_t* x, const uint32_t* y, const uint32_t* z,
                              hipStream_t s) {
    hipLaunchKernelGGL(octree_init_kernel, dim3(1024), dim3(256), 0, s, a, x, y, z);
    return hipGetLastError();
}

hipError_t launch_octree(const OctreeArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                         uint32_t lds_bytes, hipStream_t s) {
    auto k = coop ? octree_kernel<true> : octree_kernel<false>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_bytes);
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds_bytes, s, a, joiner_grid ? 1 : 0);
    return hipGetLastError();
}

}  // namespace coop
