/*
 * coop.h -- C ABI of libcoop: cooperative kernels for blocking graph
 * traversal on MI355X (gfx950).
 *
 * The programming model is the paper's "cooperative kernels" (Sorensen,
 * Evrard, Donaldson, "Cooperative Kernels: GPU Multitasking for Blocking
 * Algorithms", section 3): a kernel is launched asking for up to N
 * workgroups; the number M of active workgroups may change at resizing
 * global barriers, where the scheduler can take workgroups back
 * (offer_kill) for another task and later give them back (request_fork).
 * The device-side primitives live in coop_device.hpp; this header is the
 * host side.
 *
 * Conventions
 *  - Every function returns COOP_OK (0) or a negative COOP_E_* code; no
 *    exception crosses the ABI.
 *  - Pointers named d_* are device pointers (HBM). They are owned by the
 *    caller and must stay valid until the launch has completed
 *    (coop_wait or a stream synchronisation). The library never frees them.
 *  - Graphs are CSR over uint32: row_ptr[n+1] (row_ptr[0] = 0,
 *    non-decreasing), col[arcs] (< n), optional w[arcs]; undirected graphs
 *    store both arcs of every edge. Self loops and duplicates are allowed
 *    but the traversals treat them like any other arc.
 *  - `stream` is a hipStream_t (0 = the null stream). Launches are
 *    asynchronous on that stream. Handles must be finished with coop_wait,
 *    or passed as NULL, in which case the library reaps them itself.
 *  - A runtime may be used from several threads; calls on one coop_rt are
 *    serialised internally.
 */
#ifndef COOP_H
#define COOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* coop_stream_t;   /* same type as hipStream_t */

typedef struct coop_rt coop_rt;
typedef struct coop_graph coop_graph;
typedef struct coop_handle coop_handle;

/* ------------------------------------------------------------ errors */
enum {
    COOP_OK = 0,
    COOP_E_INVALID = -1,   /* bad argument */
    COOP_E_OOM = -2,       /* device or host allocation failed */
    COOP_E_HIP = -3,       /* a HIP call failed; coop_last_hip_error has it */
    COOP_E_TIMEOUT = -4,   /* barrier watchdog fired (non-residency or deadlock) */
    COOP_E_BUSY = -5,      /* request can never fit (serving) */
    COOP_E_OVERFLOW = -6,  /* a distance does not fit in int32 */
    COOP_E_INTERNAL = -7,  /* internal capacity or consistency error */
    COOP_E_TOO_BIG = -8    /* request exceeds a fixed capacity (coop_bfs_noalloc's scratch) */
};

/* Text for an error code (static storage). */
const char* coop_strerror(int code);

/* ------------------------------------------------------------ runtime */

typedef struct coop_device_info {
    int device;
    uint32_t compute_units;        /* CUs (multiProcessorCount) */
    uint32_t lds_per_cu;           /* bytes of LDS per CU */
    uint32_t max_lds_per_group;    /* bytes a workgroup may allocate */
    uint32_t wall_clock_khz;       /* rate of the device wall clock */
    uint64_t hbm_bytes;            /* global memory size */
    char arch[64];                 /* gcnArchName, e.g. "gfx950:sramecc+:xnack-" */
    uint32_t xcds;                 /* XCDs workgroups are dealt over (from where a probe grid lands) */
    uint32_t shader_engines;       /* shader engines per XCD (same probe) */
} coop_device_info;

/* Create a runtime on `device` (HIP ordinal). The runtime owns its streams,
 * scratch buffers and pinned control words. */
int coop_init(int device, coop_rt** out);
/* Wait for everything the runtime launched, then free it. */
int coop_shutdown(coop_rt* rt);
int coop_device_query(coop_rt* rt, coop_device_info* out);
/* The HIP error behind the last COOP_E_HIP on this runtime (0 if none). */
int coop_last_hip_error(coop_rt* rt);

/* ------------------------------------------------------------- graphs */

/* Wrap caller-owned device CSR arrays (no copy). d_w may be NULL (no
 * weights; SSSP then fails with COOP_E_INVALID). The runtime reads row_ptr
 * once (device to host copy) to size its work queues, and checks the CSR:
 * row_ptr[0] = 0, row_ptr[n] = arcs, row_ptr non-decreasing and every
 * column index < n (one pass over d_col on the device); otherwise
 * COOP_E_INVALID and no graph. */
int coop_graph_wrap(coop_rt* rt, const uint32_t* d_row_ptr, const uint32_t* d_col,
                    const uint32_t* d_w, uint32_t n, uint64_t arcs, coop_graph** out);
int coop_graph_release(coop_graph* g);

/* ----------------------------------------------------------- launches */

enum { COOP_MODE_PLAIN = 0, COOP_MODE_COOP = 1 };

enum {
    COOP_F_PARK_KILLED = 1u,      /* killed workgroups queue again as joiners (test mode) */
    COOP_F_RANDOM_SCHEDULE = 2u,  /* seeded device-side kill/fork schedule */
    COOP_F_HOST_SCHEDULE = 4u,    /* barrier reads the host-written target (coop_set_target) */
    COOP_F_TOP_DOWN_ONLY = 8u,    /* BFS: never switch to bottom-up levels */
    COOP_F_REGULAR_BARRIER = 16u, /* the paper's regular resizing barrier: at most one workgroup
                                     leaves per barrier, instead of the query barrier's W at
                                     once (section 4.2); for gather-time comparisons */
    COOP_F_LEVEL_BARRIERS = 32u,  /* BFS: every level is a phase of all workgroups with its own
                                     barrier; by default a master step runs small levels itself,
                                     top-down (frontier of at most 2048 vertices and 4 arcs per
                                     thread), with the same result */
    COOP_F_TEST_LOSE_ONE = 64u,   /* test of the barrier's bounded wait (coop_barrier_bench only):
                                     the last workgroup leaves after the first barrier without
                                     being killed, as a lost workgroup would, so the others'
                                     waits run out after watchdog_ns and the launch ends with
                                     COOP_E_TIMEOUT (every workgroup exits normally) */
    COOP_F_SLOT_SUMS = 128u       /* BFS: the master step sums every workgroup's statistics slot
                                     for a level's counts; by default (graphs with n < 2^24 and
                                     fewer than 2^28 arcs) the counts come with the barrier
                                     arrivals. SSSP: the master step reads per-XCD flags to learn
                                     whether a round lowered a distance instead of a count on the
                                     arrivals. The same result either way */
};

typedef struct coop_launch_opts {
    uint32_t mode;            /* COOP_MODE_PLAIN (fixed M = grid, all resident) or COOP_MODE_COOP */
    uint32_t num_groups;      /* N requested, at most 2048 (else COOP_E_INVALID); 0 = one per
                                 compute unit x residency, capped at 2048 */
    uint32_t group_size;      /* threads per workgroup: multiple of 64, <= 1024; 0 = 1024 */
    uint32_t lds_bytes;       /* LDS per workgroup; 0 = 96 KiB (one workgroup per CU) */
    uint32_t flags;           /* COOP_F_* */
    uint32_t heavy_threshold; /* degree above which a vertex is split into strips; 0 = 512 */
    uint32_t strip;           /* arcs per strip; 0 = 512 */
    uint32_t startup_wait_ns; /* how long workgroup 0 waits for the grid to register; 0 = 20 us */
    uint64_t sched_seed;      /* COOP_F_RANDOM_SCHEDULE: seed */
    double sched_p;           /* COOP_F_RANDOM_SCHEDULE: P(target changes) per barrier */
    uint64_t watchdog_ns;     /* spin bound of every barrier wait; 0 = 10 s */
    uint64_t* d_trace;        /* optional device buffer: per barrier two words, the device
                                 wall clock when the master step began and (low 48 bits)
                                 when it published, with the published flags in the top
                                 16 bits; NULL = no trace */
    uint32_t trace_cap;       /* barriers d_trace (and d_wgtrace) can hold */
    uint32_t join_window;     /* joiners that may wait for admission at once (at least N,
                                 so that the launch's own late workgroups fit); a joiner
                                 that finds more ahead of it leaves (counted in
                                 coop_stats.join_full); 0 = the ring's 8192 entries
                                 minus the launch's N */
    uint64_t* d_wgtrace;      /* optional device buffer: per barrier e and logical workgroup id,
                                 four device wall-clock stamps at [(e * N + id) * 4 + k]: work
                                 start, work done, barrier arrival, release seen; NULL = off */
    uint32_t bu_alpha;        /* BFS direction rule (Beamer et al.): a top-down level is followed
                                 by a bottom-up one when its frontier's arcs x alpha exceed the
                                 arcs not yet visited; 0 = 48 (Beamer et al. use 14 on CPUs;
                                 a top-down claim here is a random atomic, so bottom-up pays
                                 off sooner) */
    uint32_t bu_beta;         /* ... and a bottom-up level by a top-down one when the frontier x
                                 beta is below n and shrinking; 0 = 24 */
} coop_launch_opts;

/* Fill `o` with the defaults (plain mode). */
void coop_launch_opts_default(coop_launch_opts* o);

typedef struct coop_stats {
    int32_t error;            /* COOP_OK or the kernel's COOP_E_* */
    uint32_t barriers;        /* global barriers executed */
    uint32_t kills;           /* workgroups claimed by the scheduler */
    uint32_t forks;           /* workgroups admitted at barriers */
    uint32_t resizes;         /* barriers at which M changed */
    uint32_t min_groups;      /* smallest M after a barrier */
    uint32_t max_groups;      /* largest M after a barrier */
    uint32_t final_groups;    /* M at the last barrier */
    uint32_t grid;            /* workgroups launched (N) */
    uint32_t levels;          /* BFS levels / SSSP or colouring rounds, over all sources */
    double kernel_ms;         /* persistent kernel time (HIP events) */
    double device_ms;         /* first barrier to end (device wall clock) */
    uint64_t arcs;            /* arcs examined (top-down walks + bottom-up probes) */
    uint64_t rows;            /* vertex row ranges (row_ptr pairs) read */
    uint64_t found;           /* vertices reached (BFS) / queued (SSSP, colouring) */
    uint64_t bitmap_words;    /* BFS frontier/visited bitmap words streamed */
    uint32_t td_levels;       /* BFS levels run top-down */
    uint32_t bu_levels;       /* BFS levels run bottom-up */
    uint32_t heavy_phases;    /* extra phases that walked heavy-vertex strips */
    uint32_t join_full;       /* joiners that found the admission ring full and left */
} coop_stats;

/* BFS (the cooperative graph-traversal kernel of the paper's programming
 * section): level of every vertex from each source, one source after
 * another inside one persistent launch. Levels alternate between top-down
 * (expand the frontier) and bottom-up (unvisited vertices look for a parent
 * in the frontier) by the edge-count rule of Beamer et al. (SC 2012) unless
 * COOP_F_TOP_DOWN_ONLY is set; the result is the same either way. A level
 * small enough for one workgroup runs inside a barrier's master step unless
 * COOP_F_LEVEL_BARRIERS is set (again the same result; fewer barriers).
 * d_roots holds nroots source vertices (device memory). d_level receives, for source r, n levels at
 * d_level + r * out_stride (out_stride = 0: every source overwrites the same
 * n entries). Unreached vertices get 0xFFFFFFFF. The kernel checks each source
 * when it starts it: a source >= n fails the launch with COOP_E_INVALID before
 * anything is written for that source (the outputs of the sources before it
 * are complete). */
int coop_bfs(coop_rt* rt, const coop_graph* g, const uint32_t* d_roots, uint32_t nroots,
             uint32_t* d_level, uint64_t out_stride, const coop_launch_opts* opts,
             coop_stream_t stream, coop_handle** out);

/* coop_bfs for callers that cannot allocate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. The same BFS with
 * the same roots, levels, out_stride and options as coop_bfs; it differs in
 * this:
 *  - Nothing is allocated (no device or pinned memory, no events, no
 *    handle). Every scratch buffer of the launch (context, transmit block,
 *    per-workgroup statistics and found lists, heavy-strip list, visited and
 *    three frontier bitmaps: about n/2 bytes plus 200 KiB at 256
 *    workgroups) lives in one static device array
 *    of COOP_NOALLOC_SCRATCH_BYTES per GPU, whose address coop_init looks up.
 *    A call needing more returns COOP_E_TOO_BIG and enqueues nothing (up to
 *    about 60 million vertices fit).
 *  - The call only enqueues four kernels on `stream` (context clear,
 *    statistics clear, the BFS, a status copy) and returns COOP_OK; the
 *    launch's result code (COOP_OK, COOP_E_INVALID for a source >= n,
 *    COOP_E_TIMEOUT, ...) is written to *d_status, one int32 of caller-owned
 *    device memory, in stream order. No statistics are returned.
 *  - COOP_F_HOST_SCHEDULE is refused (COOP_E_INVALID): its target word
 *    lives in pinned memory. Plain and cooperative launches and the seeded
 *    device schedule (COOP_F_RANDOM_SCHEDULE) work.
 *  - Every call on one GPU uses that GPU's one array, which keeps the last
 *    call's contents (each call clears what must start at zero). Calls that
 *    overlap on one GPU race: calls on different streams, threads or
 *    runtimes of the same GPU must be ordered by the caller; calls on one
 *    stream are ordered already.
 * Other errors: COOP_E_INVALID for arguments coop_bfs refuses or a null
 * d_status, COOP_E_HIP when a launch fails. */
#define COOP_NOALLOC_SCRATCH_BYTES (32u << 20)
int coop_bfs_noalloc(coop_rt* rt, const coop_graph* g, const uint32_t* d_roots, uint32_t nroots,
                     uint32_t* d_level, uint64_t out_stride, const coop_launch_opts* opts,
                     int32_t* d_status, coop_stream_t stream);

/* SSSP by frontier Bellman-Ford (relaxations with atomicMin; a vertex whose
 * distance dropped is queued once for the next round). Distances int32;
 * unreached INT32_MAX; a distance >= INT32_MAX fails with COOP_E_OVERFLOW.
 * Weights are uint32 and must be present in the graph. A source >= n fails
 * the launch with COOP_E_INVALID as in coop_bfs. */
int coop_sssp(coop_rt* rt, const coop_graph* g, const uint32_t* d_roots, uint32_t nroots,
              int32_t* d_dist, uint64_t out_stride, const coop_launch_opts* opts,
              coop_stream_t stream, coop_handle** out);

/* Greedy colouring in priority order (Jones-Plassmann rounds over the
 * priority DAG): vertex v gets the smallest colour unused by its
 * higher-priority neighbours, priority key (h(v), v) with h(v) output v of
 * SplitMix64 seeded with prio_seed, higher first. d_colour: n uint32. */
int coop_color(coop_rt* rt, const coop_graph* g, uint64_t prio_seed, uint32_t* d_colour,
               const coop_launch_opts* opts, coop_stream_t stream, coop_handle** out);

/* Greedy maximal independent set in the same priority order: v is in the set
 * iff no higher-priority neighbour is. d_in_set: n bytes (0/1). */
int coop_mis(coop_rt* rt, const coop_graph* g, uint64_t prio_seed, uint8_t* d_in_set,
             const coop_launch_opts* opts, coop_stream_t stream, coop_handle** out);

/* Connected components by minimum-label propagation: d_label (n uint32,
 * device) receives, for every vertex, the smallest vertex id of its
 * component. One round per resizing-barrier interval (the level-by-level
 * pattern of the paper's section 3.2, "Adapting Graph Traversal"), with
 * the round number as transmitted state; the kernel is written only
 * against the device calls of coop_device.hpp, so it is also the worked
 * example of writing a cooperative kernel with them. Same options, kill /
 * fork schedules and stats as coop_bfs (stats.barriers = rounds + 1). */
int coop_cc(coop_rt* rt, const coop_graph* g, uint32_t* d_label, const coop_launch_opts* opts,
            coop_stream_t stream, coop_handle** out);

/* Generic launch by kernel id with a parameter block (immutable, copied). */
enum { COOP_KERNEL_BFS = 1, COOP_KERNEL_SSSP = 2, COOP_KERNEL_COLOR = 3, COOP_KERNEL_MIS = 4,
       COOP_KERNEL_BARRIER = 5, COOP_KERNEL_BATCH = 6 /* handles of coop_batch_run only */,
       COOP_KERNEL_SERVE = 7 /* the launch inside a coop_server */,
       COOP_KERNEL_OCTREE = 8 /* handles of coop_octree only */,
       COOP_KERNEL_CC = 9 /* as coop_cc; d_out = labels */ };
typedef struct coop_params {
    const coop_graph* graph;
    const uint32_t* d_roots;
    uint32_t nroots;
    uint64_t out_stride;
    uint64_t prio_seed;
    uint32_t barrier_iters;   /* COOP_KERNEL_BARRIER: barriers to run */
    void* d_out;              /* levels / distances / colours / set flags */
} coop_params;
int coop_launch(coop_rt* rt, int kernel_id, const coop_params* params, const coop_launch_opts* opts,
                coop_stream_t stream, coop_handle** out);

/* Wait for a launch, fill `stats` (nullable), free the handle. Returns the
 * kernel's error code (COOP_OK, COOP_E_TIMEOUT, COOP_E_OVERFLOW, ...). */
int coop_wait(coop_handle* h, coop_stats* stats);

/* ---------------------------------------------------------- scheduler */

/* Number of workgroups launched for this handle (N). */
uint32_t coop_handle_groups(const coop_handle* h);

/* Scheduler target for a COOP_F_HOST_SCHEDULE launch: at its next resizing
 * barrier the kernel keeps min(max(1, target), N) workgroups (the paper's
 * `query`): surplus workgroups leave (their CUs become free), and waiting
 * joiners are admitted while M < target. The leavers are chosen by shader
 * engine: every engine keeps at most (its share of the resident slots) -
 * ceil((N - target) / engines) workgroups, because the other kernel's
 * workgroups are dealt over the engines round-robin; the regular barrier
 * (COOP_F_REGULAR_BARRIER) lets one leave per barrier, from the engine that
 * owes most. Non-blocking host store. */
int coop_set_target(coop_handle* h, uint32_t target);

/* Give workgroups back: launch `count` joiner workgroups for this handle on
 * the runtime's joiner stream (they register and are admitted at the next
 * barrier, as forks). Usually preceded by coop_set_target(h, N). */
int coop_fork_groups(coop_handle* h, uint32_t count);

/* ----------------------------------------------------------- co-tasks */

typedef struct coop_cotask_cfg {
    uint32_t groups;          /* workgroups the co-task needs (one per CU) */
    uint32_t lds_bytes;       /* LDS per co-task workgroup; 0 = 96 KiB */
    uint64_t busy_ns;         /* how long each workgroup holds its CU */
    uint64_t period_ns;       /* injector: one co-task per period */
    uint32_t max_tasks;       /* injector: stop after this many (0 = until stopped) */
} coop_cotask_cfg;

typedef struct coop_cotask_stats {
    uint32_t count;           /* co-tasks completed */
    double latency_p50_ms;    /* request -> co-task end (host clock) */
    double latency_p99_ms;
    double latency_max_ms;
    double gather_p50_ms;     /* request -> all co-task workgroups running */
    double gather_p99_ms;
    double gather_max_ms;
    double busy_mean_ms;      /* co-task run time on the device */
    double setup_max_ms;      /* injector: longest period start -> request (host API calls) */
    double restore_max_ms;    /* injector: longest co-task end -> workgroups forked back */
    uint32_t late_periods;    /* injector: periods that started more than one period late */
    uint32_t reserved;
} coop_cotask_stats;

/* Work-stealing octree build (the paper's work-stealing class of cooperative
 * kernels, section 3.2 "Adapting Work Stealing"; the octree of Table 1).
 * Points: n coordinates per axis in d_x, d_y, d_z (device, each < 2^21).
 * A cube at depth d has side 2^(21 - d); its points are split stably into
 * its 8 child cubes (child = 4 bx + 2 by + bz for bit 20 - d) until a cube
 * holds at most `cap` points or reaches depth 21 (a leaf). Tasks are cubes
 * to split, kept in one queue per workgroup slot (mutex per queue); idle
 * workgroups steal. In a cooperative launch a workgroup offers itself to
 * the scheduler before each task and may leave with tasks queued (they are
 * stolen); joiner grids (coop_fork_groups) take free slots.
 * Outputs: d_out (4n words, 16-byte aligned) = the points in final order as
 * {x, y, z, input index}; d_leaves (8 words per leaf, room for leaf_cap) =
 * {first, end, depth, code_lo, code_hi, -, -, -} in no particular order
 * (sort by first), code = the child indices from the root, 3 bits per
 * level. Both are the same under any schedule. coop_wait's stats: rows =
 * leaves written (COOP_E_INVALID if more than leaf_cap were needed),
 * levels = cubes split, arcs = tasks stolen, found = n, kills / forks /
 * min_groups / max_groups = workgroups that left / joined and the range of
 * active workgroups. Errors: COOP_E_INVALID, COOP_E_OOM, COOP_E_TIMEOUT
 * (watchdog), COOP_E_HIP. */
int coop_octree(coop_rt* rt, const uint32_t* d_x, const uint32_t* d_y, const uint32_t* d_z, uint32_t n,
                uint32_t cap, uint32_t* d_out, uint32_t* d_leaves, uint32_t leaf_cap,
                const coop_launch_opts* opts, coop_stream_t stream, coop_handle** out);

/* Several cooperative launches at once (the paper's prototype ran one
 * cooperative kernel at a time; its scheduler contexts were designed for
 * several, section 4). coop_share_start starts a host thread that every
 * period_us (0 = 200) gives each added launch its weighted share of the
 * resident workgroups as its scheduler target (at least 1; the remainder
 * goes to the oldest launch) and forks joiners for a launch whose share
 * grew, e.g. when another one ended. A launch's workgroups that the
 * hardware has not started yet start on the compute units the others free
 * at their barriers. Launches must be cooperative with COOP_F_HOST_SCHEDULE;
 * coop_wait detaches a launch. The sharer and the co-task injector exclude
 * each other (COOP_E_BUSY). Errors: COOP_E_INVALID (bad handle or weight 0,
 * launch added twice, sharer not running), COOP_E_BUSY; coop_share_stop
 * returns the first error of a fork it issued. */
typedef struct coop_share_stats {
    uint32_t launches;        /* launches added since coop_share_start */
    uint32_t target_updates;  /* target changes made */
    uint32_t fork_calls;      /* joiner grids launched for grown shares */
    uint32_t reserved;
} coop_share_stats;

int coop_share_start(coop_rt* rt, uint32_t period_us);
int coop_share_add(coop_rt* rt, coop_handle* h, uint32_t weight);
int coop_share_stop(coop_rt* rt, coop_share_stats* out);

/* Run one co-task now on `stream` and wait for it (blocking). latency_ms /
 * gather_ms (nullable) get request->end and request->all-running times. */
int coop_cotask_run(coop_rt* rt, const coop_cotask_cfg* cfg, coop_stream_t stream,
                    double* latency_ms, double* gather_ms);

/* Start a host thread that, every period, asks the cooperative launch `h`
 * for cfg->groups workgroups (target = N - groups), runs the co-task on the
 * runtime's co-task stream, then restores the target and forks the
 * workgroups back. For BFS, SSSP, colouring, MIS and barrier launches the
 * co-task's last workgroup reports the launch's M, and the injector forks
 * N - M joiners less those of earlier forks not yet started; for the other
 * kinds it forks groups + engines - 1 (the engine-balanced kill can take up
 * to engines - 1 more than asked; joiners beyond the target's room leave at
 * once). h may be NULL (co-tasks only). One injector per runtime. */
int coop_injector_start(coop_rt* rt, coop_handle* h, const coop_cotask_cfg* cfg);
/* Stop the injector thread and return its statistics. */
int coop_injector_stop(coop_rt* rt, coop_cotask_stats* out);

/* ------------------------------------------------------------ batched */

/* Batched persistent launch: many independent graph instances in ONE
 * launch, each run by a team of workgroups with a barrier of its own (the
 * paper's level-synchronous loop per instance, not one global barrier for
 * all). Instances are ordered largest first; team size =
 * clamp(ceil((arcs + n) / team_arcs), 1, team_max). In COOP mode a
 * workgroup between two instances is where the scheduler may take it
 * (offer_kill: COOP_F_HOST_SCHEDULE target, or COOP_F_RANDOM_SCHEDULE with
 * probability sched_p per instance boundary; never fewer than team_max
 * workgroups stay) and where joiner workgroups from coop_fork_groups enter.
 * Results never depend on team sizes or on the kill/fork schedule. */
#define COOP_BATCH_BFS   1u   /* BFS levels from bfs_root */
#define COOP_BATCH_COLOR 2u   /* then greedy colouring (as coop_color) */
#define COOP_BATCH_MIS   4u   /* or greedy MIS (as coop_mis); not with COLOR */

typedef struct coop_batch_item {
    const coop_graph* graph;  /* resident graph (coop_graph_wrap) */
    uint32_t ops;             /* COOP_BATCH_* bits, at least one */
    uint32_t bfs_root;        /* BFS source, < n */
    uint64_t prio_seed;       /* colouring / MIS priority seed */
    uint32_t* d_level;        /* BFS: n levels (device, caller-owned) */
    uint32_t* d_colour;       /* COLOR: n colours */
    uint8_t* d_in_set;        /* MIS: n flags */
} coop_batch_item;

/* Tunable schedule of a batched launch (what coop_batch_autotune picks). */
typedef struct coop_tune {
    uint32_t group_size;      /* threads per workgroup, multiple of 64, <= 1024; 0 = 1024 */
    uint32_t num_groups;      /* launch limit N; 0 = all resident workgroups at this size */
    uint64_t team_arcs;       /* work (arcs + vertices) per team member; 0 = 2^20 */
    uint32_t team_max;        /* largest team; 0 = max(1, N / 8); must be <= N */
    uint32_t direction_opt;   /* BFS: 1 = direction-optimising, 0 = top-down only */
    uint32_t heavy_threshold; /* as coop_launch_opts; 0 = 512 */
    uint32_t strip;           /* as coop_launch_opts; 0 = 512 */
} coop_tune;

/* Defaults (what an untuned batch runs with). */
void coop_tune_default(coop_tune* t);

/* Launch `count` instances (items copied; graphs and outputs must stay
 * valid until coop_wait). opts: mode, flags (HOST/RANDOM schedule),
 * sched_seed/sched_p, watchdog_ns; its group and size fields are ignored in
 * favour of `tune` (NULL = defaults). coop_wait's stats sum over instances:
 * barriers = team barriers, levels = BFS levels, arcs/rows/found/bitmap
 * words; kills/forks = workgroups that left/entered between instances;
 * min/max_groups = fewest/most active workgroups. Errors: COOP_E_INVALID
 * (bad item, team_max > N), COOP_E_OOM. */
int coop_batch_run(coop_rt* rt, const coop_batch_item* items, uint32_t count, const coop_tune* tune,
                   const coop_launch_opts* opts, coop_stream_t stream, coop_handle** out);

/* Autotuner: coordinate search (two passes) over group size, workgroup
 * count (0.5, 0.75, 1 and 2 per compute unit), team work, team cap (N/16 ..
 * N/2), BFS direction rule, heavy-vertex threshold and strip, timing each
 * candidate (median of `reps` runs, HIP events) on the calibration subset
 * items[0], items[stride], ... (stride 0 or 1 = all items); a candidate is
 * taken if it is 2% faster. The result is cached, keyed by the device model
 * and the batch's shape (count, sum of n, sum of arcs, largest instance,
 * the union of the items' ops, the launch mode); a later call with the same
 * key returns the cached tune without timing (default_ms = -1). With a
 * subset (stride > 1) the winner is timed once more on the whole batch
 * against the default tune and kept only if it is 2% faster there, so the
 * result is never a schedule that only suits the smaller subset; best_ms
 * and default_ms (nullable) are then the whole batch's times, else the
 * subset's. Outputs of the timed items are overwritten. Not part of the
 * method of the paper: it picks the schedule of the batched launch. */
int coop_batch_autotune(coop_rt* rt, const coop_batch_item* items, uint32_t count, uint32_t stride,
                        uint32_t reps, const coop_launch_opts* opts, coop_stream_t stream, coop_tune* best,
                        double* best_ms, double* default_ms);

/* The autotuner's cache as a text file (a header line, then one line per
 * entry: the key, the schedule and its time), so a tune survives the
 * process. save writes every cached entry; load adds the file's entries to
 * the cache (a malformed file adds none and returns COOP_E_INVALID); both
 * report the cache's size in *entries (nullable). clear empties the cache.
 * No GPU is needed. */
int coop_tune_cache_save(const char* path, uint32_t* entries);
int coop_tune_cache_load(const char* path, uint32_t* entries);
void coop_tune_cache_clear(void);

/* ------------------------------------------------------------ serving */

/* A query server: ONE persistent cooperative launch that runs BFS and SSSP
 * queries on resident graphs as they are submitted (continuous batching).
 * Each query gets a slot of HBM state (the budget decides how many slots
 * exist) and a team of workgroups sized to its graph; queries that arrive
 * while others run are admitted as soon as a slot frees up and run beside
 * them. With COOP_F_HOST_SCHEDULE the server's launch honours
 * coop_set_target on coop_server_handle(): workgroups leave between queries
 * and teams give up members at their barriers, never below team_max
 * workgroups in total; coop_fork_groups brings workgroups back. A query's
 * result never depends on what else runs or on the schedule. */
typedef struct coop_server coop_server;
enum { COOP_QUERY_BFS = 1, COOP_QUERY_SSSP = 2 };

typedef struct coop_server_cfg {
    uint32_t mode;            /* COOP_MODE_PLAIN or COOP_MODE_COOP */
    uint32_t flags;           /* COOP_F_HOST_SCHEDULE */
    uint32_t num_groups;      /* launch limit N; 0 = all resident workgroups but one per shader
                                 engine, so that the host's copies (which run as small kernels)
                                 and other kernels always find a compute unit while the server
                                 stays resident */
    uint32_t group_size;      /* 0 = 1024 */
    uint32_t max_queries;     /* slots; 0 = as many as the budget holds, at most 1024 */
    uint32_t team_max;        /* largest team, <= N; 0 = max(1, N / 4) */
    uint64_t team_arcs_bfs;   /* team = clamp(ceil((arcs + n) / team_arcs), 1, team_max); 0 = 2^22 */
    uint64_t team_arcs_sssp;  /* likewise for SSSP queries; 0 = 2^22 */
    uint32_t direction_opt;   /* BFS: 1 = direction-optimising, 0 = top-down only */
    uint32_t heavy_threshold; /* 0 = 512 */
    uint32_t strip;           /* 0 = 512 */
    uint32_t reserved;
    uint64_t watchdog_ns;     /* barrier spin bound, and how long idle workgroups wait without
                                 the host's heartbeat (its poller thread) before they leave
                                 with COOP_E_TIMEOUT; 0 = 10 s */
} coop_server_cfg;

typedef struct coop_serve_stats {
    uint64_t submitted;       /* queries submitted */
    uint64_t completed;       /* queries finished */
    uint64_t count_bfs, count_sssp;        /* finished, by kind */
    double latency_p50_ms[2]; /* submit -> completion seen by the host; [0] BFS, [1] SSSP */
    double latency_p99_ms[2];
    double wait_p50_ms;       /* submit -> admitted into a slot */
    double wait_p99_ms;
    uint64_t slot_bytes;      /* HBM state per slot */
    uint32_t slots;           /* query slots */
    uint32_t in_flight;       /* queries in slots now */
    uint32_t queued;          /* queries waiting for a slot */
    uint32_t kills;           /* workgroups that left for the scheduler */
    uint32_t forks;           /* joiner workgroups that entered */
    uint32_t min_groups;      /* fewest active workgroups */
    uint32_t max_groups;      /* most active workgroups */
    int32_t error;            /* first error (COOP_OK if none) */
} coop_serve_stats;

void coop_server_cfg_default(coop_server_cfg* cfg);

/* Start a server over `ngraphs` resident graphs (they must outlive it; SSSP
 * queries need weights). hbm_budget: bytes of device memory for query
 * state; slots = min(max_queries, budget / slot_bytes), where slot_bytes
 * covers either kind of query on the largest graph. Errors: COOP_E_INVALID,
 * COOP_E_BUSY (the budget holds no slot), COOP_E_OOM, COOP_E_HIP. The launch
 * runs on a stream of the server's own. */
int coop_server_create(coop_rt* rt, const coop_graph* const* graphs, uint32_t ngraphs, uint64_t hbm_budget,
                       const coop_server_cfg* cfg, coop_server** out);

/* Queue a query: BFS levels (uint32, n) or SSSP distances (int32, n) of
 * `g` (one of the server's graphs) from `src` into d_out (device memory,
 * caller-owned, untouched until the query completes). Never blocks: the
 * query waits in the host queue until a slot is free. *ticket identifies it.
 * Errors: COOP_E_INVALID (unknown graph, bad kind or source, SSSP without
 * weights), COOP_E_BUSY (the server has no slot at all). */
int coop_server_submit(coop_server* s, const coop_graph* g, int kind, uint32_t src, void* d_out,
                       uint64_t* ticket);

/* done = 1 once the query's results are in d_out; latency_ms (nullable)
 * then gets submit -> completion. Returns the query's error code. */
int coop_server_poll(coop_server* s, uint64_t ticket, int* done, double* latency_ms);

/* Block until the query completes (or timeout_ms passes: COOP_E_TIMEOUT). */
int coop_server_wait(coop_server* s, uint64_t ticket, double timeout_ms, double* latency_ms);

int coop_server_stats(coop_server* s, coop_serve_stats* out);

/* The server's persistent launch, for coop_set_target / coop_fork_groups /
 * coop_injector_start (not for coop_wait). */
coop_handle* coop_server_handle(coop_server* s);

/* Finish queued queries, stop the launch, free everything. */
int coop_server_destroy(coop_server* s);

/* ------------------------------------------------------ measurements */

/* Global-barrier latency: a persistent launch that does `iters` barriers
 * and nothing else. ns_per_barrier from the device wall clock. Cooperative
 * launches only: a plain one (opts NULL or COOP_MODE_PLAIN) is refused with
 * COOP_E_INVALID, because one such launch once waited out its watchdog and
 * the cause has not been shown (plain launches of the traversals, which
 * use the same barrier, are not affected). */
int coop_barrier_bench(coop_rt* rt, const coop_launch_opts* opts, uint32_t iters,
                       coop_stream_t stream, double* ns_per_barrier, coop_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* COOP_H */
