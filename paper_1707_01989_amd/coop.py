"""Python binding of libcoop (include/coop.h): argument marshalling only.

Every computation runs in the HIP kernels of ``libcoop.so``. There is no
fallback: if the library is missing, loading raises ``CoopLibraryMissing``.
Device buffers are torch tensors on the GPU (``data_ptr()``), streams are
``torch.cuda.Stream`` objects or raw ``hipStream_t`` integers.

The functions keep the C names (``coop_init``, ``coop_bfs``, ...). A small
``Runtime`` class bundles a runtime with tensor allocation for convenience.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

from . import build as _build

COOP_OK = 0
COOP_E_INVALID = -1
COOP_E_OOM = -2
COOP_E_HIP = -3
COOP_E_TIMEOUT = -4
COOP_E_BUSY = -5
COOP_E_OVERFLOW = -6
COOP_E_INTERNAL = -7
COOP_E_TOO_BIG = -8
COOP_NOALLOC_SCRATCH_BYTES = 32 << 20

COOP_MODE_PLAIN = 0
COOP_MODE_COOP = 1
COOP_F_PARK_KILLED = 1
COOP_F_RANDOM_SCHEDULE = 2
COOP_F_HOST_SCHEDULE = 4
COOP_F_TOP_DOWN_ONLY = 8
COOP_F_REGULAR_BARRIER = 16
COOP_F_LEVEL_BARRIERS = 32
COOP_F_TEST_LOSE_ONE = 64
COOP_F_SLOT_SUMS = 128
COOP_KERNEL_OCTREE = 8
COOP_KERNEL_CC = 9

COOP_KERNEL_BFS = 1
COOP_KERNEL_SSSP = 2
COOP_KERNEL_COLOR = 3
COOP_KERNEL_MIS = 4
COOP_KERNEL_BARRIER = 5
COOP_KERNEL_BATCH = 6

COOP_KERNEL_SERVE = 7

COOP_BATCH_BFS = 1
COOP_BATCH_COLOR = 2
COOP_BATCH_MIS = 4

COOP_QUERY_BFS = 1
COOP_QUERY_SSSP = 2

UNREACHED_LEVEL = 0xFFFFFFFF
UNREACHED_DIST = 0x7FFFFFFF

# every symbol include/coop.h declares (checked by the ABI test)
EXPORTS = [
    "coop_strerror", "coop_launch_opts_default", "coop_init", "coop_shutdown", "coop_device_query",
    "coop_last_hip_error", "coop_graph_wrap", "coop_graph_release", "coop_bfs", "coop_bfs_noalloc", "coop_sssp",
    "coop_cc", "coop_color", "coop_mis", "coop_launch", "coop_wait", "coop_handle_groups", "coop_set_target",
    "coop_fork_groups", "coop_cotask_run", "coop_injector_start", "coop_injector_stop",
    "coop_share_start", "coop_share_add", "coop_share_stop", "coop_octree",
    "coop_barrier_bench", "coop_tune_default", "coop_batch_run", "coop_batch_autotune",
    "coop_tune_cache_save", "coop_tune_cache_load", "coop_tune_cache_clear",
    "coop_server_cfg_default", "coop_server_create", "coop_server_submit", "coop_server_poll",
    "coop_server_wait", "coop_server_stats", "coop_server_handle", "coop_server_destroy",
]


class CoopLibraryMissing(RuntimeError):
    pass


class CoopError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.coop_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} ({code})")


class coop_launch_opts(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_uint32), ("num_groups", ctypes.c_uint32), ("group_size", ctypes.c_uint32),
        ("lds_bytes", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("heavy_threshold", ctypes.c_uint32),
        ("strip", ctypes.c_uint32), ("startup_wait_ns", ctypes.c_uint32), ("sched_seed", ctypes.c_uint64),
        ("sched_p", ctypes.c_double), ("watchdog_ns", ctypes.c_uint64),
        ("d_trace", ctypes.c_void_p), ("trace_cap", ctypes.c_uint32), ("join_window", ctypes.c_uint32),
        ("d_wgtrace", ctypes.c_void_p), ("bu_alpha", ctypes.c_uint32), ("bu_beta", ctypes.c_uint32),
    ]


class coop_stats(ctypes.Structure):
    _fields_ = [
        ("error", ctypes.c_int32), ("barriers", ctypes.c_uint32), ("kills", ctypes.c_uint32),
        ("forks", ctypes.c_uint32), ("resizes", ctypes.c_uint32), ("min_groups", ctypes.c_uint32),
        ("max_groups", ctypes.c_uint32), ("final_groups", ctypes.c_uint32), ("grid", ctypes.c_uint32),
        ("levels", ctypes.c_uint32), ("kernel_ms", ctypes.c_double), ("device_ms", ctypes.c_double),
        ("arcs", ctypes.c_uint64), ("rows", ctypes.c_uint64), ("found", ctypes.c_uint64),
        ("bitmap_words", ctypes.c_uint64), ("td_levels", ctypes.c_uint32), ("bu_levels", ctypes.c_uint32),
        ("heavy_phases", ctypes.c_uint32), ("join_full", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class coop_device_info(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int), ("compute_units", ctypes.c_uint32), ("lds_per_cu", ctypes.c_uint32),
        ("max_lds_per_group", ctypes.c_uint32), ("wall_clock_khz", ctypes.c_uint32),
        ("hbm_bytes", ctypes.c_uint64), ("arch", ctypes.c_char * 64), ("xcds", ctypes.c_uint32),
        ("shader_engines", ctypes.c_uint32),
    ]


class coop_params(ctypes.Structure):
    _fields_ = [
        ("graph", ctypes.c_void_p), ("d_roots", ctypes.c_void_p), ("nroots", ctypes.c_uint32),
        ("out_stride", ctypes.c_uint64), ("prio_seed", ctypes.c_uint64), ("barrier_iters", ctypes.c_uint32),
        ("d_out", ctypes.c_void_p),
    ]


class coop_cotask_cfg(ctypes.Structure):
    _fields_ = [
        ("groups", ctypes.c_uint32), ("lds_bytes", ctypes.c_uint32), ("busy_ns", ctypes.c_uint64),
        ("period_ns", ctypes.c_uint64), ("max_tasks", ctypes.c_uint32),
    ]


class coop_share_stats(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_uint32), ("target_updates", ctypes.c_uint32), ("fork_calls", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class coop_cotask_stats(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_uint32), ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
        ("latency_max_ms", ctypes.c_double), ("gather_p50_ms", ctypes.c_double),
        ("gather_p99_ms", ctypes.c_double), ("gather_max_ms", ctypes.c_double),
        ("busy_mean_ms", ctypes.c_double), ("setup_max_ms", ctypes.c_double),
        ("restore_max_ms", ctypes.c_double), ("late_periods", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class coop_batch_item(ctypes.Structure):
    _fields_ = [
        ("graph", ctypes.c_void_p), ("ops", ctypes.c_uint32), ("bfs_root", ctypes.c_uint32),
        ("prio_seed", ctypes.c_uint64), ("d_level", ctypes.c_void_p), ("d_colour", ctypes.c_void_p),
        ("d_in_set", ctypes.c_void_p),
    ]


class coop_tune(ctypes.Structure):
    _fields_ = [
        ("group_size", ctypes.c_uint32), ("num_groups", ctypes.c_uint32), ("team_arcs", ctypes.c_uint64),
        ("team_max", ctypes.c_uint32), ("direction_opt", ctypes.c_uint32), ("heavy_threshold", ctypes.c_uint32),
        ("strip", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class coop_server_cfg(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("num_groups", ctypes.c_uint32),
        ("group_size", ctypes.c_uint32), ("max_queries", ctypes.c_uint32), ("team_max", ctypes.c_uint32),
        ("team_arcs_bfs", ctypes.c_uint64), ("team_arcs_sssp", ctypes.c_uint64),
        ("direction_opt", ctypes.c_uint32), ("heavy_threshold", ctypes.c_uint32), ("strip", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32), ("watchdog_ns", ctypes.c_uint64),
    ]


class coop_serve_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("count_bfs", ctypes.c_uint64),
        ("count_sssp", ctypes.c_uint64), ("latency_p50_ms", ctypes.c_double * 2),
        ("latency_p99_ms", ctypes.c_double * 2), ("wait_p50_ms", ctypes.c_double), ("wait_p99_ms", ctypes.c_double),
        ("slot_bytes", ctypes.c_uint64), ("slots", ctypes.c_uint32), ("in_flight", ctypes.c_uint32),
        ("queued", ctypes.c_uint32), ("kills", ctypes.c_uint32), ("forks", ctypes.c_uint32),
        ("min_groups", ctypes.c_uint32), ("max_groups", ctypes.c_uint32), ("error", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if isinstance(v, ctypes.Array) else v
        return d


_lib = None
VP = ctypes.c_void_p
VPP = ctypes.POINTER(ctypes.c_void_p)


def library_path() -> str:
    return _build.COOP_SO


def load_library():
    """Load libcoop.so (build it first with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise CoopLibraryMissing(f"{path} not found: build the HIP library first")
    lib = ctypes.CDLL(path)
    i32, u32, u64 = ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "coop_strerror": (ctypes.c_char_p, [i32]),
        "coop_launch_opts_default": (None, [ctypes.POINTER(coop_launch_opts)]),
        "coop_init": (i32, [i32, VPP]),
        "coop_shutdown": (i32, [VP]),
        "coop_device_query": (i32, [VP, ctypes.POINTER(coop_device_info)]),
        "coop_last_hip_error": (i32, [VP]),
        "coop_graph_wrap": (i32, [VP, VP, VP, VP, u32, u64, VPP]),
        "coop_graph_release": (i32, [VP]),
        "coop_bfs": (i32, [VP, VP, VP, u32, VP, u64, ctypes.POINTER(coop_launch_opts), VP, VPP]),
        "coop_bfs_noalloc": (i32, [VP, VP, VP, u32, VP, u64, ctypes.POINTER(coop_launch_opts), VP, VP]),
        "coop_sssp": (i32, [VP, VP, VP, u32, VP, u64, ctypes.POINTER(coop_launch_opts), VP, VPP]),
        "coop_color": (i32, [VP, VP, u64, VP, ctypes.POINTER(coop_launch_opts), VP, VPP]),
        "coop_cc": (i32, [VP, VP, VP, ctypes.POINTER(coop_launch_opts), VP, VPP]),
        "coop_mis": (i32, [VP, VP, u64, VP, ctypes.POINTER(coop_launch_opts), VP, VPP]),
        "coop_launch": (i32, [VP, i32, ctypes.POINTER(coop_params), ctypes.POINTER(coop_launch_opts), VP, VPP]),
        "coop_wait": (i32, [VP, ctypes.POINTER(coop_stats)]),
        "coop_handle_groups": (u32, [VP]),
        "coop_set_target": (i32, [VP, u32]),
        "coop_fork_groups": (i32, [VP, u32]),
        "coop_cotask_run": (i32, [VP, ctypes.POINTER(coop_cotask_cfg), VP,
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "coop_injector_start": (i32, [VP, VP, ctypes.POINTER(coop_cotask_cfg)]),
        "coop_injector_stop": (i32, [VP, ctypes.POINTER(coop_cotask_stats)]),
        "coop_share_start": (i32, [VP, u32]),
        "coop_octree": (i32, [VP, VP, VP, VP, u32, u32, VP, VP, u32, ctypes.POINTER(coop_launch_opts), VP, VPP]),
        "coop_share_add": (i32, [VP, VP, u32]),
        "coop_share_stop": (i32, [VP, ctypes.POINTER(coop_share_stats)]),
        "coop_barrier_bench": (i32, [VP, ctypes.POINTER(coop_launch_opts), u32, VP,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(coop_stats)]),
        "coop_tune_default": (None, [ctypes.POINTER(coop_tune)]),
        "coop_server_cfg_default": (None, [ctypes.POINTER(coop_server_cfg)]),
        "coop_server_create": (i32, [VP, ctypes.POINTER(ctypes.c_void_p), u32, u64, ctypes.POINTER(coop_server_cfg),
                                     VPP]),
        "coop_server_submit": (i32, [VP, VP, i32, u32, VP, ctypes.POINTER(ctypes.c_uint64)]),
        "coop_server_poll": (i32, [VP, u64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]),
        "coop_server_wait": (i32, [VP, u64, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
        "coop_server_stats": (i32, [VP, ctypes.POINTER(coop_serve_stats)]),
        "coop_server_handle": (VP, [VP]),
        "coop_server_destroy": (i32, [VP]),
        "coop_batch_run": (i32, [VP, ctypes.POINTER(coop_batch_item), u32, ctypes.POINTER(coop_tune),
                                 ctypes.POINTER(coop_launch_opts), VP, VPP]),
        "coop_tune_cache_save": (i32, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint32)]),
        "coop_tune_cache_load": (i32, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint32)]),
        "coop_tune_cache_clear": (None, []),
        "coop_batch_autotune": (i32, [VP, ctypes.POINTER(coop_batch_item), u32, u32, u32,
                                      ctypes.POINTER(coop_launch_opts), VP, ctypes.POINTER(coop_tune),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, where: str) -> int:
    if rc != COOP_OK:
        raise CoopError(rc, where)
    return rc


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(s) -> Optional[int]:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def make_opts(mode: int = COOP_MODE_PLAIN, **kw) -> coop_launch_opts:
    o = coop_launch_opts()
    load_library().coop_launch_opts_default(ctypes.byref(o))
    o.mode = mode
    for k, v in kw.items():
        setattr(o, k, v)
    return o


# ----------------------------------------------------------- C-named calls

def coop_strerror(code: int) -> str:
    return load_library().coop_strerror(code).decode()


def coop_init(device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load_library().coop_init(device, ctypes.byref(h)), "coop_init")
    return h.value


def coop_shutdown(rt: int) -> None:
    _check(load_library().coop_shutdown(rt), "coop_shutdown")


def coop_device_query(rt: int) -> dict:
    info = coop_device_info()
    _check(load_library().coop_device_query(rt, ctypes.byref(info)), "coop_device_query")
    d = {k: getattr(info, k) for k, _ in info._fields_}
    d["arch"] = info.arch.decode()
    return d


def coop_graph_wrap(rt: int, row_ptr, col, w, n: int, arcs: int) -> int:
    g = ctypes.c_void_p()
    _check(load_library().coop_graph_wrap(rt, _ptr(row_ptr), _ptr(col), _ptr(w), n, arcs, ctypes.byref(g)),
           "coop_graph_wrap")
    return g.value


def coop_graph_release(g: int) -> None:
    _check(load_library().coop_graph_release(g), "coop_graph_release")


def _handle_out(keep: bool):
    return ctypes.c_void_p() if keep else None


def coop_bfs(rt, g, roots, nroots, level, out_stride=0, opts=None, stream=None, keep=True):
    h = _handle_out(keep)
    rc = load_library().coop_bfs(rt, g, _ptr(roots), nroots, _ptr(level), out_stride,
                                 ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                 ctypes.byref(h) if keep else None)
    _check(rc, "coop_bfs")
    return h.value if keep else None


def coop_bfs_noalloc(rt, g, roots, nroots, level, out_stride=0, opts=None, status=None, stream=None):
    """Enqueue only; the launch's result code lands in `status` (one int32
    on the device)."""
    rc = load_library().coop_bfs_noalloc(rt, g, _ptr(roots), nroots, _ptr(level), out_stride,
                                         ctypes.byref(opts) if opts is not None else None, _ptr(status),
                                         _stream(stream))
    _check(rc, "coop_bfs_noalloc")


def coop_sssp(rt, g, roots, nroots, dist, out_stride=0, opts=None, stream=None, keep=True):
    h = _handle_out(keep)
    rc = load_library().coop_sssp(rt, g, _ptr(roots), nroots, _ptr(dist), out_stride,
                                  ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                  ctypes.byref(h) if keep else None)
    _check(rc, "coop_sssp")
    return h.value if keep else None


def coop_cc(rt, g, label, opts=None, stream=None, keep=True):
    h = _handle_out(keep)
    rc = load_library().coop_cc(rt, g, _ptr(label), ctypes.byref(opts) if opts is not None else None,
                                _stream(stream), ctypes.byref(h) if keep else None)
    _check(rc, "coop_cc")
    return h.value if keep else None


def coop_color(rt, g, prio_seed, colour, opts=None, stream=None, keep=True):
    h = _handle_out(keep)
    rc = load_library().coop_color(rt, g, prio_seed & (2**64 - 1), _ptr(colour),
                                   ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                   ctypes.byref(h) if keep else None)
    _check(rc, "coop_color")
    return h.value if keep else None


def coop_mis(rt, g, prio_seed, in_set, opts=None, stream=None, keep=True):
    h = _handle_out(keep)
    rc = load_library().coop_mis(rt, g, prio_seed & (2**64 - 1), _ptr(in_set),
                                 ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                 ctypes.byref(h) if keep else None)
    _check(rc, "coop_mis")
    return h.value if keep else None


def coop_launch(rt, kernel_id, params: coop_params, opts=None, stream=None, keep=True):
    h = _handle_out(keep)
    rc = load_library().coop_launch(rt, kernel_id, ctypes.byref(params),
                                    ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                    ctypes.byref(h) if keep else None)
    _check(rc, "coop_launch")
    return h.value if keep else None


def coop_wait(h: int) -> tuple[int, dict]:
    """Returns (rc, stats). rc is the kernel's own code; it is not raised."""
    st = coop_stats()
    rc = load_library().coop_wait(h, ctypes.byref(st))
    return rc, st.as_dict()


def coop_handle_groups(h: int) -> int:
    return int(load_library().coop_handle_groups(h))


def coop_set_target(h: int, target: int) -> None:
    _check(load_library().coop_set_target(h, target), "coop_set_target")


def coop_fork_groups(h: int, count: int) -> None:
    _check(load_library().coop_fork_groups(h, count), "coop_fork_groups")


def coop_cotask_run(rt, groups, busy_ns, lds_bytes=0, stream=None) -> tuple[float, float]:
    cfg = coop_cotask_cfg(groups=groups, lds_bytes=lds_bytes, busy_ns=busy_ns, period_ns=0, max_tasks=0)
    lat, gat = ctypes.c_double(), ctypes.c_double()
    _check(load_library().coop_cotask_run(rt, ctypes.byref(cfg), _stream(stream), ctypes.byref(lat),
                                          ctypes.byref(gat)), "coop_cotask_run")
    return lat.value, gat.value


def coop_injector_start(rt, h, groups, busy_ns, period_ns, max_tasks=0, lds_bytes=0) -> None:
    cfg = coop_cotask_cfg(groups=groups, lds_bytes=lds_bytes, busy_ns=busy_ns, period_ns=period_ns,
                          max_tasks=max_tasks)
    _check(load_library().coop_injector_start(rt, h, ctypes.byref(cfg)), "coop_injector_start")


def coop_injector_stop(rt) -> tuple[int, dict]:
    st = coop_cotask_stats()
    rc = load_library().coop_injector_stop(rt, ctypes.byref(st))
    return rc, st.as_dict()


def coop_octree(rt, x, y, z, n, cap, out, leaves, leaf_cap, opts=None, stream=None, keep=True):
    """Work-stealing octree build; x, y, z, out (n x 4), leaves (leaf_cap x 8)
    are device tensors. Returns the launch handle (wait with coop_wait)."""
    h = ctypes.c_void_p()
    _check(load_library().coop_octree(rt, _ptr(x), _ptr(y), _ptr(z), n, cap, _ptr(out), _ptr(leaves), leaf_cap,
                                      ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                      ctypes.byref(h) if keep else None), "coop_octree")
    return h.value


def coop_share_start(rt, period_us=0) -> None:
    _check(load_library().coop_share_start(rt, period_us), "coop_share_start")


def coop_share_add(rt, h, weight=1) -> None:
    _check(load_library().coop_share_add(rt, h, weight), "coop_share_add")


def coop_share_stop(rt) -> tuple[int, dict]:
    st = coop_share_stats()
    rc = load_library().coop_share_stop(rt, ctypes.byref(st))
    return rc, st.as_dict()


def coop_barrier_bench(rt, iters, opts=None, stream=None) -> tuple[float, dict]:
    ns = ctypes.c_double()
    st = coop_stats()
    _check(load_library().coop_barrier_bench(rt, ctypes.byref(opts) if opts is not None else None, iters,
                                             _stream(stream), ctypes.byref(ns), ctypes.byref(st)),
           "coop_barrier_bench")
    return ns.value, st.as_dict()


def coop_tune_default() -> coop_tune:
    t = coop_tune()
    load_library().coop_tune_default(ctypes.byref(t))
    return t


def make_tune(**kw) -> coop_tune:
    t = coop_tune_default()
    for k, v in kw.items():
        setattr(t, k, v)
    return t


def _items_array(items):
    arr = (coop_batch_item * len(items))()
    for i, it in enumerate(items):
        arr[i] = it
    return arr


def coop_batch_run(rt, items, tune=None, opts=None, stream=None, keep=True):
    """items: sequence of coop_batch_item (device pointers must stay alive until coop_wait)."""
    arr = _items_array(items)
    h = _handle_out(keep)
    rc = load_library().coop_batch_run(rt, arr, len(items), ctypes.byref(tune) if tune is not None else None,
                                       ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                       ctypes.byref(h) if keep else None)
    _check(rc, "coop_batch_run")
    return h.value if keep else None


def coop_batch_autotune(rt, items, stride=1, reps=3, opts=None, stream=None) -> tuple[coop_tune, float, float]:
    arr = _items_array(items)
    best = coop_tune()
    bms, dms = ctypes.c_double(), ctypes.c_double()
    _check(load_library().coop_batch_autotune(rt, arr, len(items), stride, reps,
                                              ctypes.byref(opts) if opts is not None else None, _stream(stream),
                                              ctypes.byref(best), ctypes.byref(bms), ctypes.byref(dms)),
           "coop_batch_autotune")
    return best, bms.value, dms.value


def coop_tune_cache_save(path: str) -> int:
    n = ctypes.c_uint32()
    _check(load_library().coop_tune_cache_save(os.fsencode(path), ctypes.byref(n)), "coop_tune_cache_save")
    return n.value


def coop_tune_cache_load(path: str) -> int:
    n = ctypes.c_uint32()
    _check(load_library().coop_tune_cache_load(os.fsencode(path), ctypes.byref(n)), "coop_tune_cache_load")
    return n.value


def coop_tune_cache_clear() -> None:
    load_library().coop_tune_cache_clear()


def coop_server_cfg_default() -> coop_server_cfg:
    c = coop_server_cfg()
    load_library().coop_server_cfg_default(ctypes.byref(c))
    return c


def make_server_cfg(**kw) -> coop_server_cfg:
    c = coop_server_cfg_default()
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def coop_server_create(rt, graphs, hbm_budget, cfg=None) -> int:
    arr = (ctypes.c_void_p * len(graphs))(*graphs)
    s = ctypes.c_void_p()
    _check(load_library().coop_server_create(rt, arr, len(graphs), int(hbm_budget),
                                             ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(s)),
           "coop_server_create")
    return s.value


def coop_server_submit(srv, graph, kind, src, out) -> int:
    t = ctypes.c_uint64()
    _check(load_library().coop_server_submit(srv, graph, kind, src, _ptr(out), ctypes.byref(t)), "coop_server_submit")
    return t.value


def coop_server_poll(srv, ticket) -> tuple[int, bool, float]:
    done, lat = ctypes.c_int(), ctypes.c_double()
    rc = load_library().coop_server_poll(srv, ticket, ctypes.byref(done), ctypes.byref(lat))
    return rc, bool(done.value), lat.value


def coop_server_wait(srv, ticket, timeout_ms=60000.0) -> tuple[int, float]:
    lat = ctypes.c_double()
    rc = load_library().coop_server_wait(srv, ticket, timeout_ms, ctypes.byref(lat))
    return rc, lat.value


def coop_server_stats(srv) -> dict:
    st = coop_serve_stats()
    _check(load_library().coop_server_stats(srv, ctypes.byref(st)), "coop_server_stats")
    return st.as_dict()


def coop_server_handle(srv) -> int:
    return load_library().coop_server_handle(srv)


def coop_server_destroy(srv) -> int:
    return load_library().coop_server_destroy(srv)


# ------------------------------------------------------------- convenience

class DeviceGraph:
    """A graph resident in HBM (torch tensors) wrapped for libcoop."""

    def __init__(self, rt: "Runtime", g, device="cuda"):
        import torch
        self.rt = rt
        self.n = g.n
        self.arcs = g.arcs
        self.row_ptr = torch.from_numpy(g.row_ptr.view("int32")).to(device)
        self.col = torch.from_numpy(g.col.view("int32")).to(device) if g.arcs else \
            torch.zeros(1, dtype=torch.int32, device=device)
        self.w = torch.from_numpy(g.w.view("int32")).to(device) if g.w is not None and g.arcs else None
        self.handle = coop_graph_wrap(rt.rt, self.row_ptr, self.col, self.w, g.n, g.arcs)

    def release(self):
        if self.handle:
            coop_graph_release(self.handle)
            self.handle = None


class Runtime:
    def __init__(self, device: int = 0):
        self.rt = coop_init(device)
        self.info = coop_device_query(self.rt)

    def close(self):
        if self.rt:
            coop_shutdown(self.rt)
            self.rt = None

    def graph(self, g) -> DeviceGraph:
        return DeviceGraph(self, g)

    def _roots(self, roots):
        import numpy as np
        import torch
        r = np.ascontiguousarray(np.asarray(roots, dtype=np.uint32).reshape(-1))
        return torch.from_numpy(r.view("int32")).cuda()

    def octree(self, x, y, z, cap: int, opts=None, stream=None):
        """Work-stealing octree of host (numpy) points: returns (rc, points
        uint32[n, 4] in final order {x, y, z, index}, leaves uint32[k, 5]
        {first, end, depth, code_lo, code_hi} sorted by first, stats)."""
        import numpy as np
        import torch
        n = len(x)
        dx, dy, dz = (torch.from_numpy(np.ascontiguousarray(v, dtype=np.uint32).view(np.int32)).cuda()
                      for v in (x, y, z))
        out = torch.empty((max(n, 1), 4), dtype=torch.int32, device="cuda")
        leaf_cap = max(1, n)
        leaves = torch.empty((leaf_cap, 8), dtype=torch.int32, device="cuda")
        h = coop_octree(self.rt, dx, dy, dz, n, cap, out, leaves, leaf_cap, opts, stream)
        rc, st = coop_wait(h)
        pts = out.cpu().numpy().view(np.uint32)[:n]
        lv = leaves.cpu().numpy().view(np.uint32)[: min(st["rows"], leaf_cap), :5]
        lv = lv[np.argsort(lv[:, 0], kind="stable")]
        return rc, pts, lv, st

    def bfs(self, dg: DeviceGraph, roots, opts=None, stream=None, out=None):
        import torch
        rt = self._roots(roots)
        k = rt.numel()
        if out is None:
            out = torch.empty(k * dg.n, dtype=torch.int32, device="cuda")
        h = coop_bfs(self.rt, dg.handle, rt, k, out, dg.n if k > 1 else 0, opts, stream)
        rc, st = coop_wait(h)
        return rc, out.view(k, dg.n) if k > 1 else out, st

    def sssp(self, dg: DeviceGraph, roots, opts=None, stream=None, out=None):
        import torch
        rt = self._roots(roots)
        k = rt.numel()
        if out is None:
            out = torch.empty(k * dg.n, dtype=torch.int32, device="cuda")
        h = coop_sssp(self.rt, dg.handle, rt, k, out, dg.n if k > 1 else 0, opts, stream)
        rc, st = coop_wait(h)
        return rc, out.view(k, dg.n) if k > 1 else out, st

    def color(self, dg: DeviceGraph, prio_seed: int, opts=None, stream=None):
        import torch
        out = torch.empty(dg.n, dtype=torch.int32, device="cuda")
        h = coop_color(self.rt, dg.handle, prio_seed, out, opts, stream)
        rc, st = coop_wait(h)
        return rc, out, st

    def batch_items(self, dgs, ops=COOP_BATCH_BFS | COOP_BATCH_COLOR, roots=None, seeds=None):
        """Items and output tensors for a batch over DeviceGraphs `dgs`
        (BFS root 0 and priority seed = index unless given)."""
        import torch
        items, outs = [], []
        for i, dg in enumerate(dgs):
            lv = torch.empty(dg.n, dtype=torch.int32, device="cuda") if ops & COOP_BATCH_BFS else None
            cl = torch.empty(dg.n, dtype=torch.int32, device="cuda") if ops & COOP_BATCH_COLOR else None
            ms = torch.empty(dg.n, dtype=torch.uint8, device="cuda") if ops & COOP_BATCH_MIS else None
            items.append(coop_batch_item(graph=dg.handle, ops=ops, bfs_root=int(roots[i]) if roots is not None else 0,
                                         prio_seed=(int(seeds[i]) if seeds is not None else i) & (2**64 - 1),
                                         d_level=_ptr(lv), d_colour=_ptr(cl), d_in_set=_ptr(ms)))
            outs.append({"level": lv, "colour": cl, "in_set": ms})
        return items, outs

    def batch(self, items, tune=None, opts=None, stream=None):
        h = coop_batch_run(self.rt, items, tune, opts, stream)
        return coop_wait(h)

    def cc(self, dg: DeviceGraph, opts=None, stream=None):
        import torch
        out = torch.empty(dg.n, dtype=torch.int32, device="cuda")
        h = coop_cc(self.rt, dg.handle, out, opts, stream)
        rc, st = coop_wait(h)
        return rc, out, st

    def mis(self, dg: DeviceGraph, prio_seed: int, opts=None, stream=None):
        import torch
        out = torch.empty(dg.n, dtype=torch.uint8, device="cuda")
        h = coop_mis(self.rt, dg.handle, prio_seed, out, opts, stream)
        rc, st = coop_wait(h)
        return rc, out, st
