// Internal interface between the host runtime and the kernels of libcoop.
// Not part of the public C ABI (that is include/coop.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "coop_device.hpp"

namespace coop {

// Per-launch work counters and the transmit block, on separate cache lines.
struct alignas(256) Work {
    uint64_t claim;            // input frontier claims: {size:32 (hi) | next:32 (lo)}
    uint64_t _p0[31];
    uint32_t out_tail;         // output frontier length
    uint32_t _p1[63];
    uint32_t heavy_tail;       // heavy strips queued this level
    uint32_t _p2[63];
    uint64_t hclaim;           // heavy strip claims: {count (hi) | next (lo)}
    uint64_t _p3[31];
    // transmit block: state a joining workgroup takes over from workgroup 0
    uint32_t xfer_level;       // level (BFS) / round (SSSP, colouring) of the interval
    uint32_t xfer_root;        // index of the current source
    uint32_t xfer_round;       // rounds over all sources (SSSP queue tags)
    uint32_t levels_total;     // statistics: levels/rounds over all sources
    uint32_t _p4[60];
};

struct TraversalArgs {
    Ctx* ctx;
    Work* work;
    const uint32_t* row_ptr;
    const uint32_t* col;
    const uint32_t* w;         // arc weights (SSSP) or null
    uint32_t n;
    uint32_t heavy_th;         // degree above which a vertex is cut into strips
    uint32_t strip;            // arcs per heavy strip
    uint32_t heavy_cap;        // capacity of `heavy` in strips
    uint4* heavy;              // strips {payload, first arc, length, vertex}
    uint32_t* frontier[2];     // n entries each
    const uint32_t* roots;     // sources, processed one after another
    uint32_t nroots;
    uint32_t out_stride;       // elements between consecutive roots' outputs (0: shared)
};

struct BfsArgs {
    TraversalArgs t;
    uint32_t* bitmap;          // ceil(n/32) words, visited set
    uint32_t* level_out;       // nroots * out_stride (or n) levels
};

struct SsspArgs {
    TraversalArgs t;
    uint32_t* stamp;           // n words: round tag of the last queueing
    int32_t* dist_out;         // nroots * out_stride (or n) distances
};

struct ColorArgs {
    TraversalArgs t;
    uint64_t prio_seed;
    uint32_t* pending;         // n words: undecided higher-key neighbours
    uint32_t* colour_out;      // n colours (COLOR) or null
    uint8_t* in_set_out;       // n flags (MIS) or null
    uint32_t mis;              // 0: greedy colouring, 1: greedy MIS
};

struct CotaskArgs {
    uint64_t busy_ticks;       // how long each workgroup holds its compute unit
    uint32_t* started;         // device counter of started workgroups
    uint32_t* finished;        // device counter of finished workgroups
    uint64_t* host_stamp;      // pinned host words: [0] all started, [1] all done (wall clock)
    uint32_t nwg;
};

struct BarrierBenchArgs {
    Ctx* ctx;
    Work* work;
    uint32_t iters;
};

// Launchers (defined in coop_kernels.hip). Each returns a hipError_t.
hipError_t launch_init_ctx(Ctx* c, Work* w, uint32_t N, uint32_t mode, uint32_t wg_size,
                           uint64_t sched_seed, uint32_t sched_p16, uint64_t watchdog_ticks,
                           uint32_t epoch0_wait, HostCtl* host, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s);
hipError_t launch_bfs(const BfsArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                      uint32_t lds_bytes, hipStream_t s);
hipError_t launch_sssp(const SsspArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                       uint32_t lds_bytes, hipStream_t s);
hipError_t launch_color(const ColorArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                        uint32_t lds_bytes, hipStream_t s);
hipError_t launch_barrier_bench(const BarrierBenchArgs& a, bool coop, bool joiner_grid, uint32_t grid,
                                uint32_t block, uint32_t lds_bytes, hipStream_t s);
hipError_t launch_cotask(const CotaskArgs& a, uint32_t block, uint32_t lds_bytes, hipStream_t s);
uint32_t kernel_lds_bytes();   // LDS the traversal kernels need at least

}  // namespace coop
