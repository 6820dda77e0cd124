// Internal interface between the host runtime and the kernels of libcoop.
// Not part of the public C ABI (that is include/coop.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "coop_device.hpp"

namespace coop {

// Transmit block: the per-level state the master step maintains, which a
// joining workgroup takes over from workgroup 0. Loaded and stored as a
// whole by the master (one batch of loads).
struct Xfer {
    uint32_t level;            // level (BFS) / round (SSSP, colouring) of the interval
    uint32_t root;             // index of the current source
    uint32_t round;            // rounds over all sources (SSSP queue tags)
    uint32_t in_size;          // input queue length (queue engine) / heavy strips (HEAVY)
    uint32_t nf_prev;          // BFS: vertices in the previous frontier
    uint32_t lvl_found;        // BFS: found in the current level before a HEAVY phase
    uint32_t lvl_mf_lo;        // BFS: their degree sum (64-bit, split)
    uint32_t lvl_mf_hi;
    uint32_t m_visited_lo;     // BFS: sum of degrees of visited vertices (current source)
    uint32_t m_visited_hi;
    uint32_t levels_total;     // statistics: levels/rounds over all sources
    uint32_t td_levels;        // BFS levels run top-down
    uint32_t bu_levels;        // BFS levels run bottom-up
    uint32_t heavy_phases;     // HEAVY phases
    uint32_t sum_found;        // BFS: the slots' found / mf sums (low 32 bits) the last master step saw
    uint32_t sum_mf;
};

__host__ __device__ inline uint64_t join64(uint32_t lo, uint32_t hi) { return ((uint64_t)hi << 32) | lo; }

// Register copy of the transmit block for the master step: four 16-byte
// loads issued together, four stores at the end (a struct copy would be
// staged through private memory by the compiler).
struct XferR {
    uint4 a, b, c, d;
    __device__ uint32_t& level() { return a.x; }
    __device__ uint32_t& root() { return a.y; }
    __device__ uint32_t& round() { return a.z; }
    __device__ uint32_t& in_size() { return a.w; }
    __device__ uint32_t& nf_prev() { return b.x; }
    __device__ uint32_t& lvl_found() { return b.y; }
    __device__ uint32_t& lvl_mf_lo() { return b.z; }
    __device__ uint32_t& lvl_mf_hi() { return b.w; }
    __device__ uint32_t& m_visited_lo() { return c.x; }
    __device__ uint32_t& m_visited_hi() { return c.y; }
    __device__ uint32_t& levels_total() { return c.z; }
    __device__ uint32_t& td_levels() { return c.w; }
    __device__ uint32_t& bu_levels() { return d.x; }
    __device__ uint32_t& heavy_phases() { return d.y; }
    __device__ uint32_t& sum_found() { return d.z; }
    __device__ uint32_t& sum_mf() { return d.w; }
};

// Per-launch work counters and the transmit block, on separate cache lines.
struct alignas(256) Work {
    uint32_t out_tail;         // output queue length (queue engine)
    uint32_t _p1[63];
    uint32_t heavy_tail;       // heavy strips queued this level
    uint32_t _p2[63];
    Xfer x;
    uint32_t _p4[64 - sizeof(Xfer) / 4];

    __device__ XferR load_x() const {
        const uint4* p = reinterpret_cast<const uint4*>(&x);
        return XferR{p[0], p[1], p[2], p[3]};
    }
    __device__ void store_x(const XferR& r) {
        uint4* p = reinterpret_cast<uint4*>(&x);
        p[0] = r.a;
        p[1] = r.b;
        p[2] = r.c;
        p[3] = r.d;
    }
};
static_assert(sizeof(Xfer) == 64, "transmit block is four 16-byte words");

// Per-workgroup accumulator slot (one 64-byte line per logical id) of
// uint64 fields, updated with fire-and-forget atomic adds: no shared
// counter on the hot path. The master step reads and clears the per-level
// fields; the cumulative ones are summed by the host after the launch.
constexpr uint32_t kSlotWords = 16;     // 8 uint64 fields
constexpr uint32_t kFlWgHost = 64;      // BFS found-list entries per workgroup (the kernels' kFlWg)
enum SlotField : uint32_t {
    kSlotFound = 0,       // per level: vertices reached / queued
    kSlotMf = 1,          // per level: sum of their degrees (BFS direction rule)
    kSlotArcs = 2,        // cumulative: arcs examined
    kSlotRows = 3,        // cumulative: row ranges read
    kSlotBitmap = 4,      // cumulative: bitmap words streamed
    kSlotFoundAll = 5,    // cumulative: vertices reached / queued
    kSlotEngine = 12,     // serving: shader engine of the team member with this rank (32-bit word)
};

struct TraversalArgs {
    Cfg cfg;
    CtxCore* ctx;              // barrier state (a Ctx for the resizable kernels)
    Work* work;
    uint32_t* slots;           // N x kSlotWords per-workgroup accumulators (zeroed at init)
    const uint32_t* row_ptr;
    const uint32_t* col;
    const uint32_t* w;         // arc weights (SSSP) or null
    uint32_t n;
    uint32_t heavy_th;         // degree above which a vertex is cut into strips
    uint32_t strip;            // arcs per heavy strip
    uint32_t heavy_cap;        // capacity of `heavy` in strips
    uint4* heavy;              // strips {payload, first arc, length, vertex}
    uint32_t* frontier[2];     // queue engine: n entries each
    const uint32_t* roots;     // sources, processed one after another
    uint32_t nroots;
    uint32_t out_stride;       // elements between consecutive roots' outputs (0: shared)
    uint32_t N;                // launch limit (slots)
};

struct BfsArgs {
    TraversalArgs t;
    uint32_t* vis;             // visited bitmap, ceil(n/32) words (+ padding to 64-word blocks)
    uint32_t* fb[3];           // rotating frontier bitmaps: current / next / being cleared
    const uint32_t* deg0;      // vertices without arcs (never expanded, skipped bottom-up)
    uint32_t* level_out;       // nroots * out_stride (or n) levels
    uint32_t words;            // bitmap words, multiple of 64
    uint32_t direction_opt;    // 0: top-down only; 1: switch to bottom-up on large frontiers
    uint32_t alpha, beta;      // switching parameters (Beamer et al.)
    uint64_t total_arcs;
    uint32_t bu_prefetch;      // bottom-up levels stage each block's row ranges in LDS
    const uint32_t* col_bu;    // bottom-up probe order: every list by decreasing neighbour degree,
                               // 16-byte aligned and padded by 4 words (the graph's copy)
    const uint2* first2;       // skewed graphs: per vertex its first two neighbours in probe order
                               // (0xFFFFFFFF: none); null otherwise
    uint32_t* flist;           // N x (1 + kFlWgHost) words: per workgroup the count and first 64 vertices it
                               // found in the last phase; null: no lists
    uint32_t inline_on;        // 1: the master step runs small levels itself (top-down)
    uint32_t arrive_sums;      // 1: a level's found and mf come with the barrier arrivals (the
                               // graph keeps them in range: n < 2^24, arcs < 2^28); 0: the master
                               // step sums the statistics slots
};

struct SsspArgs {
    TraversalArgs t;
    uint32_t* fb[3];           // rotating frontier bitmaps: current / next / being cleared
    uint32_t words;            // bitmap words, multiple of 64
    int32_t* dist_out;         // nroots * out_stride (or n) distances, also the working state
    uint32_t* lowered;         // kMaxXcds flags 64 words apart: a workgroup on that XCD lowered a distance
    uint32_t arrive_sums;      // 1: whether a round lowered anything comes with the barrier arrivals
                               // (then the flags are not used)
};

struct ColorArgs {
    TraversalArgs t;
    uint64_t prio_seed;
    uint32_t* pending;         // n words: undecided higher-key neighbours
    uint32_t* colour_out;      // n colours (COLOR) or null
    uint8_t* in_set_out;       // n flags (MIS) or null
    uint32_t mis;              // 0: greedy colouring, 1: greedy MIS
    uint32_t lanes;            // lanes per frontier vertex in a round: 1, 2, 4 or 8
};

// Lanes per frontier vertex in a colouring / MIS round for a graph of `arcs`
// arcs on `n` vertices: a vertex's list is split over about one lane per
// four arcs of the average degree, at most 8.
inline uint32_t color_lanes(uint64_t arcs, uint32_t n) {
    const uint64_t avg = n ? arcs / n : 0;
    return avg >= 24 ? 8u : avg >= 12 ? 4u : avg >= 6 ? 2u : 1u;
}

struct CotaskArgs {
    uint64_t busy_ticks;       // how long each workgroup holds its compute unit
    uint32_t* started;         // device counter of started co-task workgroups (never reset)
    uint32_t* finished;        // device counter of finished co-task workgroups (never reset)
    uint32_t base;             // workgroups of all earlier co-tasks: both counters reach
                               // base + nwg when this one has started / finished
    uint64_t* host_stamp;      // pinned host words: [0] all started, [1] all done (wall clock),
                               // [2] the resizable launch's M and joiner-grid starts when done
    const uint64_t* release;   // that launch's release word, or null
    const uint32_t* joined;    // that launch's count of started joiner-grid workgroups
    uint32_t nwg;
};

struct BarrierBenchArgs {
    Cfg cfg;
    Ctx* ctx;
    Work* work;
    uint32_t iters;
};

// ------------------------------------------------------------- batched

// Barrier lines and transmit blocks of one instance's team (BFS, then
// colouring), zeroed by the batch init kernel.
struct alignas(256) TeamState {
    CtxCore bfs_ctx;
    Work bfs_work;
    CtxCore col_ctx;
    Work col_work;
};

constexpr uint32_t kBatchBfs = 1u;         // run BFS from bfs.t.roots[0]
constexpr uint32_t kBatchColor = 2u;       // then greedy colouring / MIS (col.mis)

// One instance of a batched launch: complete argument blocks of the two
// algorithms (pointers into the instance's graph, outputs and scratch) and
// its team size. Read through the constant address space, so every field is
// a scalar load.
struct alignas(16) BatchInst {
    BfsArgs bfs;
    ColorArgs col;
    uint32_t team;             // workgroups that run this instance together
    uint32_t ops;              // kBatch* bits
    uint32_t pad[2];
};

// Launch-wide counters of a batched launch.
// Counters of a batched launch (who is active, who left for the scheduler
// and who joined live in the launch context's task state).
struct alignas(256) BatchCtl {
    uint32_t ticket;           // next (instance, rank) entry
    uint32_t _p0[63];
    int32_t error;
    uint32_t left;             // workgroups that left when tickets ran out
    uint32_t _p2[62];
};

struct BatchArgs {
    Cfg cfg;                   // N, mode (kill policy), host target, watchdog, keep = team_max
    Ctx* ctx;                  // launch context: task state (active count, kills, forks)
    const BatchInst* inst;     // `count` descriptors in ticket order
    const uint32_t* first;     // count + 1: first ticket of each instance
    TeamState* teams;          // count team blocks
    BatchCtl* ctl;
    uint32_t count;
    uint32_t team_max;         // largest team: the kill rule keeps at least this many workgroups
};

hipError_t launch_batch_init(TeamState* teams, const BatchInst* inst, uint32_t count, BatchCtl* ctl,
                             hipStream_t s);

// ------------------------------------------------------------- serving

constexpr uint32_t kQueryBfs = 1u;
constexpr uint32_t kQuerySssp = 2u;

// Argument blocks of a query of one resident graph in one slot's state
// (slot-major: desc[slot * graphs + graph]). Written before the server
// kernel starts and never changed while it runs, so they are read through
// the constant address space.
struct alignas(16) ServeDesc {
    BfsArgs bfs;
    SsspArgs sssp;
};

// A published query (one per slot, pinned host memory, written by the host
// before it publishes the query's tickets).
struct alignas(64) ServeReq {
    uint32_t desc;             // ServeDesc index
    uint32_t kind;             // kQueryBfs / kQuerySssp
    uint32_t src;              // source vertex (the team's root list points here)
    uint32_t team;             // workgroups of the team
    uint32_t first;            // first ticket of the team
    uint32_t pad0;
    uint64_t out;              // device pointer: n levels (BFS) or distances (SSSP)
    uint64_t seq;              // query number, echoed in the completion word
    uint32_t pad1[6];
};

// Host-written words of the server (pinned).
struct alignas(64) ServeHost {
    uint32_t ticket_end;       // tickets below this are published
    uint32_t stop;             // 1: leave once no ticket is left
    uint32_t heartbeat;        // advanced by the host's poller about every millisecond
    uint32_t pad[13];
};

// Completion record of a slot (pinned): written by the last member of the
// team to leave the query.
struct alignas(64) ServeDone {
    uint64_t seq;              // query number that finished
    uint64_t t_end;            // device wall clock at completion
    int32_t error;             // the slot's barrier error, if any
    uint32_t pad[11];
};

// Device-side words of the server. Who is active, who left for the
// scheduler and who joined live in the launch context's task state.
struct alignas(256) ServeCtl {
    uint32_t ticket;           // next ticket to draw
    uint32_t _p0[63];
    int32_t error;
    uint32_t left;             // workgroups that left at shutdown
    uint32_t queries;          // queries completed
    uint32_t _p1[61];
    // the relay: one idle workgroup at a time reads the host's words over
    // PCIe and republishes them here, where every other idle workgroup polls
    uint32_t relay;            // 1 while an idle workgroup holds the role
    uint32_t end;              // the host's published ticket end, as relayed
    uint32_t stop;             // the host's stop word, as relayed
    uint32_t beat;             // advanced by the relay at every poll
    uint32_t _p2[60];
};

struct ServeArgs {
    Cfg cfg;                   // N, mode, host target (co-task), watchdog, keep = team_max
    Ctx* ctx;                  // launch context: task state, and the relayed host target (T_seen)
    const ServeDesc* desc;     // slots x graphs descriptors
    TeamState* teams;          // per slot: barrier lines and transmit block
    ServeCtl* ctl;
    ServeHost* host;           // pinned control words
    const ServeReq* req;       // pinned, one per slot
    const uint32_t* owner;     // pinned, ticket -> slot (owner_cap entries)
    ServeDone* done;           // pinned, one per slot
    uint32_t owner_cap;
    uint32_t team_max;         // the kill rule keeps at least this many workgroups
    uint32_t slots;            // query slots (records, completion words)
    uint32_t ndesc;            // descriptors (slots x graphs)
};

// ------------------------------------------------ work-stealing octree

constexpr uint32_t kOctQueueCap = 1024;   // node ids per queue (depth-first use keeps it short)
constexpr uint32_t kOctMaxDepth = 21;     // coordinates have 21 bits

// One task queue (ring of node ids) per slot; a workgroup owns one slot at
// a time. Guarded by `lock` (compare-and-swap mutex): the owner pushes and
// pops at the tail, thieves take from the head.
struct alignas(256) OctQueue {
    uint32_t lock;
    uint32_t head;
    uint32_t tail;
    uint32_t _p[61];
    uint32_t ring[kOctQueueCap];
};

struct alignas(256) OctCtl {
    uint32_t outstanding;      // tasks created and not finished
    uint32_t _p0[63];
    uint32_t node_count;       // nodes allocated (node 0 = root)
    uint32_t leaf_count;
    uint32_t _p1[62];
    int32_t error;
    uint32_t _p2[63];
    uint32_t tasks;            // cubes split
    uint32_t steals;           // tasks taken from another slot's queue
    uint32_t _p3[62];
};

struct OctreeArgs {
    Cfg cfg;                   // N = slots, mode, host target, watchdog
    uint4* buf[2];             // points {x, y, z, index}; depth d reads buf[d & 1]; buf[0] is the result
    uint32_t n, cap;
    uint32_t* nodes;           // 8 words per node {first, end, depth, code_lo, code_hi, -, -, -}
    uint32_t node_cap;
    uint32_t* leaves;          // 8 words per leaf {first, end, depth, code_lo, code_hi, -, -, -}
    uint32_t leaf_cap;
    OctCtl* ctl;
    OctQueue* q;               // N queues, one per slot (the workgroup id of the task pattern)
    Ctx* ctx;                  // launch context: task state (slots, active count, kills, forks)
};

hipError_t launch_octree_init(const OctreeArgs& a, const uint32_t* x, const uint32_t* y, const uint32_t* z,
                              hipStream_t s);

// ------------------------------------- connected components (label propagation)

struct CcArgs {
    Cfg cfg;
    Ctx* ctx;
    const uint32_t* row_ptr;
    const uint32_t* col;
    uint32_t n;
    uint32_t* label;           // n labels (the output)
    uint32_t* changed;         // two round marks, 64 words apart
};
hipError_t launch_cc(const CcArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                     uint32_t lds_bytes, hipStream_t s);
hipError_t launch_octree(const OctreeArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                         uint32_t lds_bytes, hipStream_t s);

hipError_t launch_serve_init(TeamState* teams, uint32_t slots, ServeCtl* ctl, hipStream_t s);
hipError_t launch_serve(const ServeArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                        uint32_t lds_bytes, hipStream_t s);
uint32_t occupancy_serve(bool coop, uint32_t block, uint32_t lds_bytes);
hipError_t launch_batch(const BatchArgs& a, bool coop, bool joiner_grid, uint32_t grid, uint32_t block,
                        uint32_t lds_bytes, hipStream_t s);
// Workgroups of the batched kernel one CU holds at this size (registers, LDS, waves).
uint32_t occupancy_batch(bool coop, uint32_t block, uint32_t lds_bytes);

// Launchers (defined in coop_kernels.hip). Each returns a hipError_t.
hipError_t launch_init_ctx(Ctx* c, Work* w, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s);
// *out = the launch context's error word, in stream order after the launch
hipError_t launch_copy_status(const CtxCore* c, int32_t* out, hipStream_t s);
// Bitmap of vertices without arcs (words: multiple of 64, padding bits set).
// Probe-order copy of `col` (every list by decreasing neighbour degree, ties
// in list order) into `out` (arcs + 4 words); allocates its temporaries and
// waits for `s`.
hipError_t build_degree_order(const uint32_t* row_ptr, const uint32_t* col, uint32_t n, uint64_t arcs,
                              uint32_t max_deg, uint32_t* out, hipStream_t s);
// first2[v] = the first two entries of v's list in `col_bu` (0xFFFFFFFF past
// its end), n entries; waits for `s`.
hipError_t build_first_two(const uint32_t* row_ptr, const uint32_t* col_bu, uint32_t n, uint2* first2,
                           hipStream_t s);
hipError_t launch_deg0_bitmap(const uint32_t* row_ptr, uint32_t n, uint32_t* bits, uint32_t words, hipStream_t s);
// Count (into *bad, cleared first) the column indices that are >= n.
hipError_t launch_check_cols(const uint32_t* col, uint64_t arcs, uint32_t n, uint32_t* bad, hipStream_t s);
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
// out[2g] = XCD, out[2g+1] = shader engine of workgroup g, for `groups`
// one-wave workgroups
hipError_t launch_place_probe(uint32_t* out, uint32_t groups, uint32_t lds_bytes, uint64_t hold_ticks,
                              hipStream_t s);
uint32_t kernel_lds_bytes_for(uint32_t block);   // ... with `block` threads per workgroup

}  // namespace coop
