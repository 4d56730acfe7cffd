"""ctypes binding of librpq (include/rpq.h). Argument marshalling only: every
step of a query runs in the library's HIP kernels.

The library must have been built (``paper_2412_10287_amd.build.build()``); if
``librpq.so`` is missing, importing this module raises, so nothing can fall
back to another implementation.

Two layers:
* the raw entry points under their C names (``rpq_graph_load``, ...), with
  ctypes argument types set, in ``lib``;
* thin helpers ``Graph`` / ``NFA`` that hold handles and convert numpy arrays.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# The in-tree build; RPQ_LIB names another build of the same library (for
# instance to compare two builds in one process environment).
LIB_PATH = os.environ.get("RPQ_LIB") or os.path.join(HERE, "librpq.so")

RPQ_OK, RPQ_PENDING = 0, 1
RPQ_EINVAL, RPQ_ENOMEM, RPQ_EDEVICE, RPQ_EAGAIN, RPQ_ENOTFOUND, RPQ_ETIMEDOUT = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "RPQ_OK", 1: "RPQ_PENDING", -1: "RPQ_EINVAL", -2: "RPQ_ENOMEM", -3: "RPQ_EDEVICE",
                -4: "RPQ_EAGAIN", -5: "RPQ_ENOTFOUND", -6: "RPQ_ETIMEDOUT"}

OUT_DEVICE, COUNTERS, KERNEL_TIMING, FORCE_PUSH, FORCE_PULL, HOST_LOOP, GRAPH_LEVELS, RARE_END = \
    1, 2, 4, 8, 16, 32, 64, 128

EXPORTS = ("rpq_bitmap_words", "rpq_graph_load", "rpq_graph_free", "rpq_graph_info", "rpq_set_option",
           "rpq_get_option", "rpq_nfa_load", "rpq_nfa_free", "rpq_single_source", "rpq_single_destination",
           "rpq_single_source_lengths", "rpq_source_set", "rpq_multi_source", "rpq_multi_source_noalloc",
           "rpq_submit", "rpq_submit_deadline", "rpq_poll",
           "rpq_autotune", "rpq_last_error")

TUNE_PLAIN, TUNE_STACKED = 0, 1


class rpq_tuning(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int64), ("alpha", ctypes.c_int64), ("beta", ctypes.c_int64),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double), ("candidates", ctypes.c_int32),
                ("handoff_edges", ctypes.c_int64)]


class rpq_stats(ctypes.Structure):
    _fields_ = [
        ("level_counts", ctypes.POINTER(ctypes.c_int64)),
        ("level_cap", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("push_levels", ctypes.c_int32),
        ("pull_levels", ctypes.c_int32),
        ("visited_pairs", ctypes.c_int64),
        ("product_edges", ctypes.c_int64),
        ("scans", ctypes.c_int64),
        ("scanned_edges", ctypes.c_int64),
        ("alg_bytes", ctypes.c_int64),
        ("active", ctypes.c_int64),
        ("device_ms", ctypes.c_double),
        ("expand_ms", ctypes.c_double),
        ("expand_launches", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("level_us", ctypes.POINTER(ctypes.c_double)),
        ("level_frontier", ctypes.POINTER(ctypes.c_int64)),
        ("level_edges", ctypes.POINTER(ctypes.c_int64)),
        ("level_select_us", ctypes.POINTER(ctypes.c_double)),
        ("updates", ctypes.c_int64),
        ("latency_ms", ctypes.c_double),
        ("plan", ctypes.c_int32),
    ]

_LEVEL_FIELDS = ("level_counts", "level_cap", "level_us", "level_frontier", "level_edges", "level_select_us")


class RPQError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def load_library(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("librpq.so is not built (%s); run paper_2412_10287_amd.build.build()" % path)
    L = ctypes.CDLL(path)
    P, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "rpq_bitmap_words": (i64, [i32]),
        "rpq_graph_load": (ctypes.c_int, [i32, i32, P, P, P, ctypes.POINTER(P)]),
        "rpq_graph_free": (ctypes.c_int, [P]),
        "rpq_graph_info": (ctypes.c_int, [P, ctypes.c_char_p, ctypes.POINTER(i64)]),
        "rpq_set_option": (ctypes.c_int, [P, ctypes.c_char_p, i64]),
        "rpq_get_option": (ctypes.c_int, [P, ctypes.c_char_p, ctypes.POINTER(i64)]),
        "rpq_nfa_load": (ctypes.c_int, [i32, i32, P, P, P, P, i32, P, i32, ctypes.POINTER(P)]),
        "rpq_nfa_free": (ctypes.c_int, [P]),
        "rpq_single_source": (ctypes.c_int, [P, P, i32, P, u32, ctypes.POINTER(rpq_stats)]),
        "rpq_single_destination": (ctypes.c_int, [P, P, i32, P, u32, ctypes.POINTER(rpq_stats)]),
        "rpq_single_source_lengths": (ctypes.c_int, [P, P, i32, P, u32, ctypes.POINTER(rpq_stats)]),
        "rpq_source_set": (ctypes.c_int, [P, P, P, i32, P, u32, ctypes.POINTER(rpq_stats)]),
        "rpq_multi_source": (ctypes.c_int, [P, P, P, i32, P, u32, ctypes.POINTER(rpq_stats)]),
        "rpq_multi_source_noalloc": (ctypes.c_int, [P, P, P, i32, P, u32, ctypes.POINTER(rpq_stats)]),
        "rpq_submit": (ctypes.c_int, [P, P, i32, ctypes.POINTER(u64)]),
        "rpq_submit_deadline": (ctypes.c_int, [P, P, i32, i64, ctypes.POINTER(u64)]),
        "rpq_poll": (ctypes.c_int, [P, u64, P, u32, ctypes.POINTER(rpq_stats), i64]),
        "rpq_autotune": (ctypes.c_int, [P, i32, P, P, i32, ctypes.POINTER(rpq_tuning)]),
        "rpq_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = load_library()

# The HIP runtime librpq itself links (the system ROCm one). Device buffers for
# RPQ_OUT_DEVICE results come from it, so no second runtime enters the process.
_hip = ctypes.CDLL("libamdhip64.so.7", mode=ctypes.RTLD_GLOBAL)
_hip.hipMalloc.restype = ctypes.c_int
_hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
_hip.hipFree.restype = ctypes.c_int
_hip.hipFree.argtypes = [ctypes.c_void_p]
_hip.hipMemcpy.restype = ctypes.c_int
_hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
_hip.hipMemset.restype = ctypes.c_int
_hip.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
_hip.hipDeviceSynchronize.restype = ctypes.c_int
_HIP_D2H = 2
_HIP_D2D = 3


# Handles still open. At interpreter exit they are all closed by an atexit
# handler, graphs first (which joins their served paths' scheduler threads and
# waits for outstanding tickets), while the HIP runtime and ctypes are fully
# alive; objects that reach the finalizer later (for instance kept by a
# reference cycle) are left to the process exit instead of calling into the
# library from a half-torn-down interpreter.
_live_graphs = weakref.WeakSet()
_live_nfas = weakref.WeakSet()
_live_buffers = weakref.WeakSet()


def _close_all():
    for group in (_live_graphs, _live_buffers, _live_nfas):
        for obj in list(group):
            try:
                obj.close(drain=True) if group is _live_graphs else obj.close()
            except Exception:
                pass


atexit.register(_close_all)


class DeviceBuffer:
    """A zeroed device allocation of ``nbytes`` (plumbing for RPQ_OUT_DEVICE)."""

    def __init__(self, nbytes: int):
        self.nbytes = int(nbytes)
        p = ctypes.c_void_p()
        if _hip.hipMalloc(ctypes.byref(p), max(self.nbytes, 1)) != 0:
            raise MemoryError("hipMalloc of %d bytes failed" % self.nbytes)
        self.ptr = p.value
        _live_buffers.add(self)
        if _hip.hipMemset(ctypes.c_void_p(self.ptr), 0, self.nbytes) != 0:
            raise RuntimeError("hipMemset failed")

    def to_host(self, dtype=np.uint64) -> np.ndarray:
        out = np.empty(self.nbytes // np.dtype(dtype).itemsize, dtype=dtype)
        if _hip.hipMemcpy(ctypes.c_void_p(out.ctypes.data), ctypes.c_void_p(self.ptr), self.nbytes, _HIP_D2H) != 0:
            raise RuntimeError("hipMemcpy failed")
        return out

    def copy_from(self, other: "DeviceBuffer"):
        """Device-to-device copy of min(sizes) bytes (used to calibrate traffic counters)."""
        n = min(self.nbytes, other.nbytes)
        if _hip.hipMemcpy(ctypes.c_void_p(self.ptr), ctypes.c_void_p(other.ptr), n, _HIP_D2D) != 0:
            raise RuntimeError("hipMemcpy failed")

    def close(self):
        if getattr(self, "ptr", None):
            _hip.hipFree(ctypes.c_void_p(self.ptr))
            self.ptr = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may be gone at exit)
        if not _finalizing():
            self.close()


def device_synchronize():
    if _hip.hipDeviceSynchronize() != 0:
        raise RuntimeError("hipDeviceSynchronize failed")


def last_error() -> str:
    return lib.rpq_last_error().decode(errors="replace")


def check(status: int) -> int:
    if status < 0:
        raise RPQError(status, last_error())
    return status


def _p(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def bitmap_words(num_vertices: int) -> int:
    return int(lib.rpq_bitmap_words(num_vertices))


_SCALAR_FIELDS = frozenset(k for k, _ in rpq_stats._fields_ if k not in _LEVEL_FIELDS)
_LEVEL_ARRAYS = {"level_counts": np.int64, "level_us": np.float64, "level_frontier": np.int64,
                 "level_edges": np.int64, "level_select_us": np.float64}


class Stats:
    """Statistics of one call: the fields of rpq_stats as attributes (levels,
    push_levels, pull_levels, visited_pairs, product_edges, scans,
    scanned_edges, alg_bytes, active, device_ms, expand_ms, expand_launches,
    batch, updates, latency_ms, plan), read from the C struct when accessed, and the per-level arrays
    level_counts, level_us, level_frontier, level_edges, level_select_us
    (empty unless the call asked for them with level_cap)."""

    __slots__ = ("_s", "_lv", "_cache")

    def __init__(self, s: Optional[rpq_stats] = None, lv: Optional[dict] = None):
        self._s = s if s is not None else rpq_stats()
        self._lv = lv
        self._cache = {}

    @classmethod
    def from_c(cls, s: rpq_stats, lv: Optional[dict]):
        return cls(s, lv)

    def __getattr__(self, k):
        if k in _SCALAR_FIELDS:
            return getattr(self._s, k)
        if k in _LEVEL_ARRAYS:
            c = self._cache
            if k not in c:
                if self._lv is None:
                    c[k] = np.zeros(0, _LEVEL_ARRAYS[k])
                else:
                    a = self._lv[k]
                    c[k] = a[:min(a.size, max(self._s.levels, 0))].copy()
            return c[k]
        raise AttributeError(k)

    def __repr__(self):
        return "Stats(%s)" % ", ".join("%s=%r" % (k, getattr(self._s, k)) for k, _ in rpq_stats._fields_
                                       if k in _SCALAR_FIELDS)


def _stats_struct(level_cap: int):
    """An rpq_stats with per-level output buffers of level_cap entries."""
    st = rpq_stats()
    lv = None
    if level_cap > 0:
        lv = {"level_counts": np.zeros(level_cap, dtype=np.int64),
              "level_us": np.zeros(level_cap, dtype=np.float64),
              "level_frontier": np.zeros(level_cap, dtype=np.int64),
              "level_edges": np.zeros(level_cap, dtype=np.int64),
              "level_select_us": np.zeros(level_cap, dtype=np.float64)}
        st.level_counts = lv["level_counts"].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        st.level_us = lv["level_us"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        st.level_frontier = lv["level_frontier"].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        st.level_edges = lv["level_edges"].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        st.level_select_us = lv["level_select_us"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        st.level_cap = level_cap
    return st, lv


class NFA:
    """Handle on rpq_nfa_load's tables. ``nfa`` is any object with the fields
    num_states, num_labels, sym_ptr, frm, to, start, final (per-symbol COO)."""

    def __init__(self, nfa):
        self.num_states = int(nfa.num_states)
        sp = np.ascontiguousarray(nfa.sym_ptr, dtype=np.int64)
        fr = np.ascontiguousarray(nfa.frm, dtype=np.int32)
        to = np.ascontiguousarray(nfa.to, dtype=np.int32)
        st = np.ascontiguousarray(nfa.start, dtype=np.int32)
        fi = np.ascontiguousarray(nfa.final, dtype=np.int32)
        h = ctypes.c_void_p()
        check(lib.rpq_nfa_load(self.num_states, int(nfa.num_labels), _p(sp), _p(fr), _p(to), _p(st),
                               int(st.size), _p(fi), int(fi.size), ctypes.byref(h)))
        self.h = h
        _live_nfas.add(self)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib.rpq_nfa_free(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may be gone at exit)
        if not _finalizing():
            self.close()


class Graph:
    """Handle on a device-resident graph store built by rpq_graph_load."""

    def __init__(self, g):
        self.num_vertices = int(g.num_vertices)
        self.num_labels = int(g.num_labels)
        lp = np.ascontiguousarray(g.label_ptr, dtype=np.int64)
        s = np.ascontiguousarray(g.src, dtype=np.int32)
        d = np.ascontiguousarray(g.dst, dtype=np.int32)
        h = ctypes.c_void_p()
        check(lib.rpq_graph_load(self.num_vertices, self.num_labels, _p(lp), _p(s), _p(d), ctypes.byref(h)))
        self.h = h
        self.words = bitmap_words(self.num_vertices)
        self._tickets = set()  # submitted and not yet collected by poll
        _live_graphs.add(self)

    def close(self, drain: bool = False):
        """rpq_graph_free. With drain, first waits for the answers of tickets
        still outstanding (rpq_graph_free refuses while any is pending)."""
        if getattr(self, "h", None) is None or not self.h.value:
            return
        if drain:
            scratch = np.empty(self.words, dtype=np.uint64)
            for t in list(self._tickets):
                lib.rpq_poll(self.h, ctypes.c_uint64(t), _p(scratch), 0, None, -1)
            self._tickets.clear()
        check(lib.rpq_graph_free(self.h))
        self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may be gone at exit)
        if not _finalizing():
            self.close()

    def info(self, key: str) -> int:
        v = ctypes.c_int64()
        check(lib.rpq_graph_info(self.h, key.encode(), ctypes.byref(v)))
        return v.value

    def set_option(self, key: str, value: int):
        check(lib.rpq_set_option(self.h, key.encode(), int(value)))

    def get_option(self, key: str) -> int:
        v = ctypes.c_int64()
        check(lib.rpq_get_option(self.h, key.encode(), ctypes.byref(v)))
        return v.value

    def single_source(self, nfa: NFA, source: int, flags: int = 0, level_cap: int = 0,
                      out: Optional[np.ndarray] = None, out_device_ptr: Optional[int] = None):
        """Returns (bitmap or None, Stats). With out_device_ptr the bitmap goes
        to that device address (RPQ_OUT_DEVICE) and None is returned."""
        st, lc = _stats_struct(level_cap)
        if out_device_ptr is not None:
            check(lib.rpq_single_source(self.h, nfa.h, int(source), ctypes.c_void_p(out_device_ptr),
                                        flags | OUT_DEVICE, ctypes.byref(st)))
            return None, Stats.from_c(st, lc)
        bm = out if out is not None else np.zeros(self.words, dtype=np.uint64)
        check(lib.rpq_single_source(self.h, nfa.h, int(source), _p(bm), flags, ctypes.byref(st)))
        return bm, Stats.from_c(st, lc)

    def single_destination(self, nfa: NFA, target: int, flags: int = 0, level_cap: int = 0):
        """Vertices with a matching walk to `target`: (bitmap, Stats)."""
        st, lc = _stats_struct(level_cap)
        bm = np.zeros(self.words, dtype=np.uint64)
        check(lib.rpq_single_destination(self.h, nfa.h, int(target), _p(bm), flags, ctypes.byref(st)))
        return bm, Stats.from_c(st, lc)

    def single_source_lengths(self, nfa: NFA, source: int, flags: int = 0, level_cap: int = 0,
                              out_device_ptr: Optional[int] = None):
        """Shortest accepted walk length per vertex (-1 where none): (int32
        array or None, Stats). With out_device_ptr the lengths go to that
        device address (RPQ_OUT_DEVICE) and None is returned."""
        st, lc = _stats_struct(level_cap)
        if out_device_ptr is not None:
            check(lib.rpq_single_source_lengths(self.h, nfa.h, int(source), ctypes.c_void_p(out_device_ptr),
                                                flags | OUT_DEVICE, ctypes.byref(st)))
            return None, Stats.from_c(st, lc)
        d = np.empty(self.num_vertices, dtype=np.int32)
        check(lib.rpq_single_source_lengths(self.h, nfa.h, int(source), _p(d), flags, ctypes.byref(st)))
        return d, Stats.from_c(st, lc)

    def source_set(self, nfa: NFA, sources: Sequence[int], flags: int = 0, level_cap: int = 0,
                   out_device_ptr: Optional[int] = None):
        """Vertices reached from any of `sources` (one traversal from
        Q_S x sources): (bitmap or None, Stats)."""
        src = np.ascontiguousarray(sources, dtype=np.int32)
        st, lc = _stats_struct(level_cap)
        if out_device_ptr is not None:
            check(lib.rpq_source_set(self.h, nfa.h, _p(src), int(src.size), ctypes.c_void_p(out_device_ptr),
                                     flags | OUT_DEVICE, ctypes.byref(st)))
            return None, Stats.from_c(st, lc)
        bm = np.zeros(self.words, dtype=np.uint64)
        check(lib.rpq_source_set(self.h, nfa.h, _p(src), int(src.size), _p(bm), flags, ctypes.byref(st)))
        return bm, Stats.from_c(st, lc)

    def multi_source(self, nfa: NFA, sources: Sequence[int], flags: int = 0,
                     out_device_ptr: Optional[int] = None, level_cap: int = 0):
        src = np.ascontiguousarray(sources, dtype=np.int32)
        st, lc = _stats_struct(level_cap)
        if out_device_ptr is not None:
            check(lib.rpq_multi_source(self.h, nfa.h, _p(src), int(src.size), ctypes.c_void_p(out_device_ptr),
                                       flags | OUT_DEVICE, ctypes.byref(st)))
            return None, Stats.from_c(st, lc)
        bm = np.zeros((src.size, self.words), dtype=np.uint64)
        check(lib.rpq_multi_source(self.h, nfa.h, _p(src), int(src.size), _p(bm), flags, ctypes.byref(st)))
        return bm, Stats.from_c(st, lc)

    def multi_source_noalloc(self, nfa: NFA, sources: Sequence[int], flags: int = 0,
                             out_device_ptr: Optional[int] = None, level_cap: int = 0):
        """rpq_multi_source_noalloc: as multi_source, with the call's device
        state in the library's fixed scratch array (no allocation)."""
        src = np.ascontiguousarray(sources, dtype=np.int32)
        st, lc = _stats_struct(level_cap)
        if out_device_ptr is not None:
            check(lib.rpq_multi_source_noalloc(self.h, nfa.h, _p(src), int(src.size), ctypes.c_void_p(out_device_ptr),
                                               flags | OUT_DEVICE, ctypes.byref(st)))
            return None, Stats.from_c(st, lc)
        bm = np.zeros((src.size, self.words), dtype=np.uint64)
        check(lib.rpq_multi_source_noalloc(self.h, nfa.h, _p(src), int(src.size), _p(bm), flags, ctypes.byref(st)))
        return bm, Stats.from_c(st, lc)

    def autotune(self, path: int, nfas: Sequence[NFA], sources: Sequence[int]) -> dict:
        """rpq_autotune: time the candidate settings of `path` (TUNE_PLAIN:
        nfas[i] from sources[i]; TUNE_STACKED: nfas[0] from every source) and
        keep the fastest. Returns the chosen values and times."""
        src = np.ascontiguousarray(sources, dtype=np.int32)
        hs = (ctypes.c_void_p * len(nfas))(*[n.h.value for n in nfas])
        out = rpq_tuning()
        check(lib.rpq_autotune(self.h, int(path), hs, _p(src), int(src.size), ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in rpq_tuning._fields_}

    def signature(self) -> str:
        """A key for per-graph settings: sizes and row counts of the store."""
        return "V%d-L%d-E%d-R%d-%d" % (self.num_vertices, self.num_labels, self.info("num_edges"),
                                       self.info("rows_out"), self.info("rows_in"))

    def submit(self, nfa: NFA, source: int, deadline_us: Optional[int] = None) -> int:
        """Queues a query; with deadline_us, rpq_submit_deadline (dropped with
        RPQ_ETIMEDOUT if it has not started that many microseconds later)."""
        t = ctypes.c_uint64()
        if deadline_us is None:
            check(lib.rpq_submit(self.h, nfa.h, int(source), ctypes.byref(t)))
        else:
            check(lib.rpq_submit_deadline(self.h, nfa.h, int(source), int(deadline_us), ctypes.byref(t)))
        self._tickets.add(t.value)
        return t.value

    def poll(self, ticket: int, timeout_us: int = 0, out_device_ptr: Optional[int] = None):
        """Returns (bitmap, Stats) when finished, None while pending. With
        out_device_ptr the bitmap goes to that device address (RPQ_OUT_DEVICE)
        and (None, Stats) is returned."""
        st, lc = _stats_struct(0)
        if out_device_ptr is not None:
            bm, ptr, fl = None, ctypes.c_void_p(out_device_ptr), OUT_DEVICE
        else:
            bm = np.empty(self.words, dtype=np.uint64)
            ptr, fl = _p(bm), 0
        r = lib.rpq_poll(self.h, ctypes.c_uint64(ticket), ptr, fl, ctypes.byref(st), int(timeout_us))
        if r == RPQ_ETIMEDOUT and b"deadline" in (lib.rpq_last_error() or b""):
            self._tickets.discard(ticket)  # dropped by its start deadline: retired
            check(r)
        if r in (RPQ_PENDING, RPQ_ETIMEDOUT):
            return None
        self._tickets.discard(ticket)
        check(r)
        return bm, Stats.from_c(st, lc)
