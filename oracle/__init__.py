"""Reference oracle for single-source two-way regular path queries.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package. The GPU library never calls it, and
the two share no code: the oracle is plain C (``oracle.c``) driven through
ctypes, plus ``alg2`` (the frontier-free fixpoint of Sec. 4, written with scipy
sparse Boolean products) as a second, independent formulation.

``ssr`` computes the plain definition of single-source reachability (Sec. 2,
the SSR map of Def. 2.6) by breadth-first search over explicit (state, vertex)
pairs of the product automaton (Def. 2.5); the correctness theorem of Sec. 4
makes that set equal to Alg. 1's result.
"""
from __future__ import annotations

import ctypes
import os
import sys
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .build import build as _build, LIB_PATH

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        _build()
    _lib = load_library(LIB_PATH)
    return _lib


def load_library(path: str):
    """Open an oracle shared library (the mutation test opens altered copies)."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.og_new.restype = P
    lib.og_new.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P]
    lib.og_free.restype = None
    lib.og_free.argtypes = [P]
    lib.og_num_edges.restype = ctypes.c_int64
    lib.og_num_edges.argtypes = [P, ctypes.c_int]
    lib.og_ssr.restype = ctypes.c_int32
    lib.og_ssr.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, P, P, ctypes.c_int32,
                           P, ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_int32, P,
                           ctypes.c_int32]
    if hasattr(lib, "og_ssr_from"):
        lib.og_ssr_from.restype = ctypes.c_int32
        lib.og_ssr_from.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, P, P, ctypes.c_int32,
                                    P, ctypes.c_int32, P, ctypes.c_int32, P, P, P, ctypes.c_int32, P,
                                    ctypes.c_int32]
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def word_bytes(num_states: int) -> int:
    """Bytes of one vertex's state word: 1, 2 or 4 for up to 8, 16, 32 states."""
    return 1 if num_states <= 8 else 2 if num_states <= 16 else 4 if num_states <= 32 else 8


@dataclass
class Result:
    bitmap: np.ndarray  # uint64, ceil(V/64)
    levels: int  # number of non-empty frontiers (max distance + 1)
    level_counts: np.ndarray  # |M_n|
    product_edges: int
    scans: int
    scanned_edges: int
    alg_bytes: int
    active: int
    dist: Optional[np.ndarray] = None  # (Q, V) int32
    final: Optional[np.ndarray] = None  # the NFA's final states

    def vertices(self) -> np.ndarray:
        return bitmap_to_vertices(self.bitmap)

    def lengths(self) -> np.ndarray:
        """Per vertex, the length of the shortest accepted walk: the least
        distance of a final state at the vertex, -1 where none (needs the
        distances, keep_dist=True)."""
        if self.dist is None:
            raise ValueError("lengths need keep_dist=True")
        V = self.dist.shape[1]
        if self.final is None or len(self.final) == 0:
            return np.full(V, -1, np.int32)
        d = self.dist[np.asarray(self.final, dtype=np.int64)].astype(np.int64)
        d[d < 0] = np.iinfo(np.int64).max
        m = d.min(axis=0)
        return np.where(m == np.iinfo(np.int64).max, -1, m).astype(np.int32)


def bitmap_to_vertices(bm: np.ndarray) -> np.ndarray:
    bits = np.unpackbits(bm.view(np.uint8), bitorder="little")
    return np.nonzero(bits)[0].astype(np.int64)


class Graph:
    """Oracle-side graph: its own per-vertex sorted adjacency lists."""

    def __init__(self, g, lib=None):
        lib = lib or _load()
        self._lib = lib
        self.num_vertices = int(g.num_vertices)
        self.num_labels = int(g.num_labels)
        lp = np.ascontiguousarray(g.label_ptr, dtype=np.int64)
        s = np.ascontiguousarray(g.src, dtype=np.int32)
        d = np.ascontiguousarray(g.dst, dtype=np.int32)
        h = lib.og_new(self.num_vertices, self.num_labels, _ptr(lp), _ptr(s), _ptr(d))
        if not h:
            raise ValueError("oracle rejected the graph")
        self._h = ctypes.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._lib.og_free(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # no foreign calls from a half-finalized interpreter (the memory goes
        # with the process); the check is bound at definition, as module
        # globals may already be gone at exit
        if not _finalizing():
            self.close()

    def num_edges(self, inverse: bool = False) -> int:
        return int(self._lib.og_num_edges(self._h, int(inverse)))

    def ssr(self, nfa, source: int, keep_dist: bool = False, level_cap: int = 1 << 16) -> Result:
        return self._run(nfa, [int(source)], keep_dist, level_cap, single=True)

    def ssr_set(self, nfa, sources, keep_dist: bool = False, level_cap: int = 1 << 16) -> Result:
        """The query from the start set V_s = sources (Def. 2.6): one search
        from every pair of Q_S x V_s."""
        return self._run(nfa, [int(s) for s in sources], keep_dist, level_cap, single=False)

    def _run(self, nfa, sources, keep_dist, level_cap, single) -> Result:
        lib = self._lib
        V = self.num_vertices
        Q = int(nfa.num_states)
        bm = np.zeros((V + 63) // 64, dtype=np.uint64)
        lc = np.zeros(level_cap, dtype=np.int64)
        ctr = np.zeros(5, dtype=np.int64)
        dist = np.empty((Q, V), dtype=np.int32) if keep_dist else None
        sp = np.ascontiguousarray(nfa.sym_ptr, dtype=np.int64)
        fr = np.ascontiguousarray(nfa.frm, dtype=np.int32)
        to = np.ascontiguousarray(nfa.to, dtype=np.int32)
        st = np.ascontiguousarray(nfa.start, dtype=np.int32)
        fi = np.ascontiguousarray(nfa.final, dtype=np.int32)
        if single:
            n = lib.og_ssr(self._h, Q, int(nfa.num_labels), _ptr(sp), _ptr(fr), _ptr(to), _ptr(st),
                           int(st.size), _ptr(fi), int(fi.size), sources[0], _ptr(bm), _ptr(dist),
                           _ptr(lc), level_cap, _ptr(ctr), word_bytes(Q))
        else:
            srcs = np.ascontiguousarray(sources, dtype=np.int32)
            n = lib.og_ssr_from(self._h, Q, int(nfa.num_labels), _ptr(sp), _ptr(fr), _ptr(to), _ptr(st),
                                int(st.size), _ptr(fi), int(fi.size), _ptr(srcs), int(srcs.size), _ptr(bm),
                                _ptr(dist), _ptr(lc), level_cap, _ptr(ctr), word_bytes(Q))
        if n < 0:
            raise ValueError("oracle rejected the query")
        return Result(bm, int(n), lc[:min(max(n, 0), level_cap)].copy(), int(ctr[0]), int(ctr[1]),
                      int(ctr[2]), int(ctr[3]), int(ctr[4]), dist, fi.copy())


def ssr(g, nfa, source: int, keep_dist: bool = False, lib=None) -> Result:
    og = Graph(g, lib)
    try:
        return og.ssr(nfa, source, keep_dist)
    finally:
        og.close()
