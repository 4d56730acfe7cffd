"""Brute-force single-source reachability by walk enumeration (test pin).

Independent of both the oracle and the GPU path: it never builds an automaton.
It enumerates two-way walks from the source (Sec. 2, Defs 2.2-2.3: walks may
repeat vertices, the zero-length walk exists, edges may be used backwards with
inverted labels) together with the words they spell (the map omega<->), and
decides membership with the third-party ``regex`` backtracking matcher on the
expression text. Partial matching prunes words that no extension can complete.
Walks that end at the same vertex with the same word have the same futures, so
they are merged.

``min_match_len`` returns, for each vertex, the length of the shortest matching
walk of length <= K (or -1). With K >= |Q|*|V| - 1 for any NFA of |Q| states
accepting the language, this is complete: a shortest witness is a shortest path
in the product graph, which has |Q|*|V| nodes (the termination bound of App. A).
"""
from __future__ import annotations

import numpy as np
import regex as re_mod

from workloads import regex as R

BASE = 0x4E00  # one code point per symbol, far from regex metacharacters


def sym_char(sym: int) -> str:
    return chr(BASE + sym)


def to_pyregex(node, num_labels: int) -> str:
    if isinstance(node, R.Sym):
        return sym_char(R.symbol_of(node, num_labels))
    if isinstance(node, R.Cat):
        return "(?:" + to_pyregex(node.left, num_labels) + to_pyregex(node.right, num_labels) + ")"
    if isinstance(node, R.Alt):
        return "(?:" + to_pyregex(node.left, num_labels) + "|" + to_pyregex(node.right, num_labels) + ")"
    if isinstance(node, R.Star):
        return "(?:" + to_pyregex(node.child, num_labels) + ")*"
    if isinstance(node, R.Plus):
        return "(?:" + to_pyregex(node.child, num_labels) + ")+"
    if isinstance(node, R.Opt):
        return "(?:" + to_pyregex(node.child, num_labels) + ")?"
    raise TypeError(node)


def min_match_len(g, text: str, source: int, K: int, max_pairs: int = 2_000_000) -> np.ndarray:
    L = g.num_labels
    pat = re_mod.compile(to_pyregex(R.parse(text), L))
    # two-way adjacency: v -> list of (symbol, w)
    adj = [[] for _ in range(g.num_vertices)]
    for l in range(L):
        s, d = g.edges_of(l)
        for a, b in zip(s.tolist(), d.tolist()):
            adj[a].append((l, b))  # forward use of (a -> b)
            adj[b].append((L + l, a))  # backward use of (a -> b), inverted label
    best = np.full(g.num_vertices, -1, dtype=np.int64)
    layer = {(source, "")}
    total = 0
    for k in range(K + 1):
        nxt = set()
        for v, w in layer:
            if best[v] < 0 and pat.fullmatch(w):
                best[v] = k
        if k == K:
            break
        for v, w in layer:
            for sym, u in adj[v]:
                w2 = w + sym_char(sym)
                if (u, w2) in nxt:
                    continue
                if pat.fullmatch(w2, partial=True) is None:
                    continue
                nxt.add((u, w2))
        total += len(nxt)
        if total > max_pairs:
            raise RuntimeError("brute force too large")
        layer = nxt
        if not layer:
            break
    return best


def reach_bitmap(best: np.ndarray) -> np.ndarray:
    V = best.size
    words = np.zeros((V + 63) // 64, dtype=np.uint64)
    for v in np.nonzero(best >= 0)[0]:
        words[v >> 6] |= np.uint64(1) << np.uint64(v & 63)
    return words
