"""The explicit product automaton of an NFA and a graph (Def. 2.5), built as a
networkx multigraph, and the work counters read off it.

This is an independent second construction for the oracle's counters: the
oracle never builds the product, it searches it implicitly over its own
adjacency lists. Here every product edge is materialised:

    (q, v) --a--> (q', w)   iff   q --a--> q' in the NFA  and  v --a--> w in the
                                  two-way graph (for a = l^-, w --l--> v),

one keyed edge per symbol, so two symbols joining the same pair of nodes give
two edges (the product-edge count sums over symbols). Levels come from
networkx's breadth-first distances from the start pairs Q_S x {source}.
Small graphs only.
"""
from __future__ import annotations

from collections import defaultdict

import networkx as nx
import numpy as np


def used_symbols(g, nfa):
    """Symbols with a transition whose label some edge of the graph carries."""
    counts = g.label_counts()
    out = set()
    for _, s, _ in nfa.triples():
        lab = s if s < nfa.num_labels else s - nfa.num_labels
        if lab < g.num_labels and counts[lab] > 0:
            out.add(s)
    return out


def graph_edges(g):
    """Distinct (src, dst) pairs per label."""
    return {l: set(zip(*(x.tolist() for x in g.edges_of(l)))) for l in range(g.num_labels)}


def product(g, nfa):
    """MultiDiGraph over (q, v) with one edge per (symbol, transition, graph edge)."""
    NL = nfa.num_labels
    E = graph_edges(g)
    pg = nx.MultiDiGraph()
    for q, s, q2 in set(nfa.triples()):
        lab, inv = (s, False) if s < NL else (s - NL, True)
        if lab >= g.num_labels:
            continue
        for a, b in E[lab]:
            v, w = (b, a) if inv else (a, b)
            pg.add_edge((q, v), (q2, w), key=s)
    return pg


def levels(pg, nfa, source):
    """Breadth-first distance of every product node reachable from the start
    pairs (start pairs at distance 0)."""
    starts = {(int(q), int(source)) for q in nfa.start}
    if not starts:
        return {}
    hub = ("hub",)
    h = nx.DiGraph(pg)
    h.add_nodes_from(starts)
    for st in starts:
        h.add_edge(hub, st)
    d = nx.single_source_shortest_path_length(h, hub)
    d.pop(hub)
    return {k: v - 1 for k, v in d.items()}


def counters(g, nfa, source, word_bytes):
    """(product_edges, scans, scanned_edges, alg_bytes, active, level_counts)
    read off the explicit product, with the byte model of the single-query
    path: 2w + 8 per active (level, vertex), 8 per scan, 4 + w per scanned
    edge, ceil(V/8) for the result."""
    pg = product(g, nfa)
    dist = levels(pg, nfa, source)
    pe = sum(pg.out_degree(node) for node in dist if node in pg)
    succ_nonempty = defaultdict(set)  # symbol -> states with a transition on it
    for q, s, _ in nfa.triples():
        succ_nonempty[s].add(q)
    used = used_symbols(g, nfa)
    groups = defaultdict(set)  # (level, v) -> states first reached there
    for (q, v), n in dist.items():
        groups[(n, v)].add(q)
    scans = scanned = 0
    byt = (2 * word_bytes + 8) * len(groups)
    for (n, v), S in groups.items():
        for s in used:
            if not (S & succ_nonempty[s]):
                continue
            targets = set()
            for q in S:
                if (q, v) not in pg:
                    continue
                for _, (q2, w), key in pg.out_edges((q, v), keys=True):
                    if key == s:
                        targets.add(w)
            scans += 1
            scanned += len(targets)
            byt += 8 + (4 + word_bytes) * len(targets)
    byt += (g.num_vertices + 7) // 8
    nlev = max(dist.values()) + 1 if dist else 0
    lc = np.zeros(nlev, np.int64)
    for n in dist.values():
        lc[n] += 1
    return pe, scans, scanned, byt, len(groups), lc
