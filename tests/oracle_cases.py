"""Shared small cases and pin checks for the oracle tests (and the mutation
test, which re-runs them against deliberately broken copies of the oracle)."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

from workloads import graphs as G
from workloads import regex as R
import brute


def tiny_graph(rng, nv=None, ne=None, nl=None):
    nv = int(rng.integers(2, 5)) if nv is None else nv
    ne = int(rng.integers(1, 7)) if ne is None else ne
    nl = int(rng.integers(1, 4)) if nl is None else nl
    s = rng.integers(0, nv, size=ne)
    d = rng.integers(0, nv, size=ne)
    l = rng.integers(0, nl, size=ne)
    # occasionally give an edge a second label, or repeat an entry
    if ne and rng.random() < 0.5:
        i = int(rng.integers(0, ne))
        s = np.append(s, s[i]); d = np.append(d, d[i]); l = np.append(l, (l[i] + 1) % nl)
    if ne and rng.random() < 0.3:
        i = int(rng.integers(0, ne))
        s = np.append(s, s[i]); d = np.append(d, d[i]); l = np.append(l, l[i])
    return G.from_triples(nv, nl, s, d, l, dedupe=False)


def tiny_expr(rng, nl, max_leaves=3):
    k = int(rng.integers(1, max_leaves + 1))
    return R.to_string(R.random_ast(rng, k, lambda r: r.integers(0, nl), 0.5,
                                    p_unary=0.4, unary=("star", "plus")))


def check_brute(ssr_fn, rng, n_cases=60):
    """ssr_fn(graph, nfa, source) -> (bitmap, dist (Q, V), levels). Compares the full
    result (complete bound) or the per-vertex shortest matching length."""
    checked_full = 0
    for _ in range(n_cases):
        g = tiny_graph(rng)
        text = tiny_expr(rng, g.num_labels)
        nfa = R.compile_regex(text, g.num_labels)
        src = int(rng.integers(0, g.num_vertices))
        bm, dist, _ = ssr_fn(g, nfa, src)
        K = nfa.num_states * g.num_vertices - 1
        try:
            best = brute.min_match_len(g, text, src, K, max_pairs=300_000)
            complete = True
        except RuntimeError:
            K = 6
            best = brute.min_match_len(g, text, src, K)
            complete = False
        fin = dist[nfa.final] if nfa.final.size else np.full((1, g.num_vertices), -1)
        fin = np.where(fin < 0, np.iinfo(np.int32).max, fin).min(axis=0)
        mine = np.where(fin <= K, fin, -1)
        assert np.array_equal(mine, best), (text, src, mine, best)
        if complete:
            checked_full += 1
            assert np.array_equal(bm, brute.reach_bitmap(best)), (text, src)
    return checked_full


def bitmap_of(vertices, nv):
    words = np.zeros((nv + 63) // 64, dtype=np.uint64)
    for v in np.asarray(vertices, dtype=np.int64):
        words[v >> 6] |= np.uint64(1) << np.uint64(v & 63)
    return words


def label_matrix(g, labels, inverse=()):
    V = g.num_vertices
    m = sp.csr_matrix((V, V), dtype=np.int8)
    for l in labels:
        s, d = g.edges_of(l)
        m = m + sp.csr_matrix((np.ones(s.size, np.int8), (s, d)), shape=(V, V))
    for l in inverse:
        s, d = g.edges_of(l)
        m = m + sp.csr_matrix((np.ones(s.size, np.int8), (d, s)), shape=(V, V))
    m.data[:] = 1
    return m


def bfs_set(m, src):
    return csg.breadth_first_order(m, src, directed=True, return_predecessors=False)


def check_special(ssr_fn, rng, g):
    """Queries whose answer a library routine gives directly."""
    V, L = g.num_vertices, g.num_labels
    for _ in range(6):
        a, b = (int(x) for x in rng.choice(L, size=2, replace=False))
        s = int(rng.integers(0, V))
        Ga = label_matrix(g, [a])
        # a*: plain a-reachability, source included (zero-length walk)
        assert np.array_equal(ssr_fn(g, R.compile_regex("%d*" % a, L), s)[0],
                              bitmap_of(bfs_set(Ga, s), V)), ("a*", a, s)
        # a+: one a-step, then a*
        nb = Ga.indices[Ga.indptr[s]:Ga.indptr[s + 1]]
        want = set()
        for u in nb:
            want |= set(bfs_set(Ga, int(u)).tolist())
        assert np.array_equal(ssr_fn(g, R.compile_regex("%d+" % a, L), s)[0],
                              bitmap_of(sorted(want), V)), ("a+", a, s)
        # (a|^a)*: weakly connected component of s under label a
        ncomp, lab = csg.connected_components(Ga, directed=True, connection="weak")
        assert np.array_equal(ssr_fn(g, R.compile_regex("(%d|^%d)*" % (a, a), L), s)[0],
                              bitmap_of(np.nonzero(lab == lab[s])[0], V)), ("(a|^a)*", a, s)
        # (a|b)*: reachability over the union of the two labels
        Gab = label_matrix(g, [a, b])
        assert np.array_equal(ssr_fn(g, R.compile_regex("(%d|%d)*" % (a, b), L), s)[0],
                              bitmap_of(bfs_set(Gab, s), V)), ("(a|b)*", a, b, s)
        # ^b*: reachability against the b-edges
        Gbt = label_matrix(g, [], [b])
        assert np.array_equal(ssr_fn(g, R.compile_regex("(^%d)*" % b, L), s)[0],
                              bitmap_of(bfs_set(Gbt, s), V)), ("^b*", b, s)
    # every label both ways: weak component of s in the whole graph
    s = int(rng.integers(0, V))
    allq = "(" + "|".join("%d|^%d" % (l, l) for l in range(L)) + ")*"
    ncomp, lab = csg.connected_components(label_matrix(g, range(L)), directed=True,
                                          connection="weak")
    assert np.array_equal(ssr_fn(g, R.compile_regex(allq, L), s)[0],
                          bitmap_of(np.nonzero(lab == lab[s])[0], V))


def check_grid(ssr_fn, side, rng, n=5):
    """Closed forms on a grid without shortcuts: east=0, north=1, west=2,
    south=3; vertex id y*side + x."""
    g = G.grid(side, 0.0, 0)
    for i in range(n):
        x0, y0 = (0, 0) if i == 0 else (int(rng.integers(0, side)), int(rng.integers(0, side)))
        s = y0 * side + x0
        bm, _, lv = ssr_fn(g, R.compile_regex("(0|1)*", 4), s)
        want = [y * side + x for y in range(y0, side) for x in range(x0, side)]
        assert np.array_equal(bm, bitmap_of(want, side * side))
        # one level per Manhattan distance 0 .. (side-1-x0)+(side-1-y0)
        assert lv == (side - 1 - x0) + (side - 1 - y0) + 1
        # (0|^2)* 3: east moves (forward east or backward west) then one step south
        bm2 = ssr_fn(g, R.compile_regex("(0|^2)* 3", 4), s)[0]
        want2 = [(y0 - 1) * side + x for x in range(x0, side)] if y0 > 0 else []
        assert np.array_equal(bm2, bitmap_of(want2, side * side))


def python_counters(g, nfa, dist, word_bytes):
    """Work counters recomputed from the distances, slowly and separately:
    product edges out of reached pairs, scans (level, vertex, symbol with a
    non-empty successor set, with or without neighbours), graph edges
    scanned, algorithmic bytes, active (level, vertex) pairs."""
    V, L, NL = g.num_vertices, g.num_labels, nfa.num_labels
    deg = {}
    for l in range(L):
        s, d = g.edges_of(l)
        pairs = set(zip(s.tolist(), d.tolist()))
        fw = np.zeros(V, np.int64)
        bw = np.zeros(V, np.int64)
        for a, b in pairs:
            fw[a] += 1
            bw[b] += 1
        deg[("f", l)] = fw
        deg[("b", l)] = bw
    succ = {}
    present = g.label_counts() > 0
    for a, s, b in nfa.triples():
        lab = s if s < NL else s - NL
        if lab < L and present[lab]:
            succ.setdefault(s, {}).setdefault(a, set()).add(b)
    pe = scans = scanned = 0
    byt = 0
    active = 0
    for v in range(V):
        levels = {}
        for q in range(nfa.num_states):
            if dist[q, v] >= 0:
                levels.setdefault(int(dist[q, v]), set()).add(q)
        for n, S in levels.items():
            active += 1
            byt += 2 * word_bytes + 8
            for s, tab in succ.items():
                d = int(deg[("f", s) if s < NL else ("b", s - NL)][v])
                img = set()
                for q in S:
                    img |= tab.get(q, set())
                    pe += len(tab.get(q, ())) * d
                if img:
                    scans += 1
                    scanned += d
                    byt += 8 + (4 + word_bytes) * d
    byt += (V + 7) // 8
    return pe, scans, scanned, byt, active


def check_counters_product(ctr_fn, rng, n_cases=80):
    """ctr_fn(graph, nfa, source) -> (product_edges, scans, scanned_edges,
    alg_bytes, active, level_counts). Compared with the same quantities read
    off the explicit product automaton (product_graph.py) on tiny graphs."""
    import product_graph as PG
    from oracle import word_bytes
    for _ in range(n_cases):
        g = tiny_graph(rng, nv=int(rng.integers(2, 7)), ne=int(rng.integers(1, 12)))
        text = tiny_expr(rng, g.num_labels, max_leaves=4)
        nfa = R.compile_regex(text, g.num_labels)
        src = int(rng.integers(0, g.num_vertices))
        got = ctr_fn(g, nfa, src)
        want = PG.counters(g, nfa, src, word_bytes(nfa.num_states))
        assert tuple(got[:5]) == tuple(want[:5]), (text, src, got[:5], want[:5])
        assert np.array_equal(np.asarray(got[5]), want[5]), (text, src)


def check_counters_star(ctr_fn, rng, g, n=6):
    """Closed form for a*: the Glushkov automaton has the start state 0 and
    the state 1 after an a, with 0 -a-> 1 and 1 -a-> 1. The reached pairs are
    (0, s) and (1, v) for v in the a+ reach of s, each with one successor per
    a-edge, so product edges = d_a(s) + sum over that reach of d_a(v). Every
    reached pair is its own (level, vertex) and its own scan (state 1 can
    meet (0, s) at s only at a later level)."""
    V, L = g.num_vertices, g.num_labels
    for _ in range(n):
        a = int(rng.integers(0, L))
        s = int(rng.integers(0, V))
        Ga = label_matrix(g, [a])
        deg = np.diff(Ga.indptr).astype(np.int64)
        plus = set()
        for u in Ga.indices[Ga.indptr[s]:Ga.indptr[s + 1]]:
            plus |= set(bfs_set(Ga, int(u)).tolist())
        plus = np.array(sorted(plus), dtype=np.int64)
        pe = int(deg[s] + deg[plus].sum())
        k = 1 + plus.size
        w = 1
        want = (pe, k, pe, (2 * w + 8) * k + 8 * k + (4 + w) * pe + (V + 7) // 8, k)
        got = ctr_fn(g, R.compile_regex("%d*" % a, L), s)
        assert tuple(got[:5]) == want, ("a*", a, s, got[:5], want)


def grid_star_counters(side, x0, y0):
    """Closed form of the counters of (0|1)* from (x0, y0) on the grid without
    shortcuts (east = 0, north = 1). The Glushkov automaton has the start
    state and one state per occurrence, each state with one successor per
    symbol; (1, v) is reached iff v lies east of the source column, (2, v)
    iff north of the source row, all pairs of v at its Manhattan distance.
    With X = side-1-x0 and Y = side-1-y0, the quadrant has (X+1)(Y+1)
    vertices and X(Y+1) + Y(X+1) edges inside it."""
    X, Y = side - 1 - x0, side - 1 - y0
    pe = (X > 0) + (Y > 0) + max(X - 1, 0) * (Y + 1) + X * Y + X * Y + (X + 1) * max(Y - 1, 0)
    active = (X + 1) * (Y + 1)
    scans = X * (Y + 1) + Y * (X + 1)  # one scan per (vertex, direction) with an edge
    # scans without neighbours: the symbols of the top row (north) and right
    # column (east) of the quadrant
    scans += (X + 1) + (Y + 1)
    scanned = X * (Y + 1) + Y * (X + 1)
    w = 1
    byt = (2 * w + 8) * active + 8 * scans + (4 + w) * scanned + (side * side + 7) // 8
    return pe, scans, scanned, byt, active


def check_counters_grid(ctr_fn, side, rng, n=4):
    g = G.grid(side, 0.0, 0)
    for i in range(n):
        x0, y0 = (0, 0) if i == 0 else (int(rng.integers(0, side)), int(rng.integers(0, side)))
        got = ctr_fn(g, R.compile_regex("(0|1)*", 4), y0 * side + x0)
        want = grid_star_counters(side, x0, y0)
        assert tuple(got[:5]) == want, ("grid", x0, y0, got[:5], want)


def stacked_counters(g, nfa, sources, dists):
    """Work counters of one stacked pass over the sources (levels in lockstep),
    from each source's oracle distances dists[b] (Q x V): scans, scanned
    edges, active (level, vertex) pairs, algorithmic bytes and the
    (edge, transition, non-zero 64-bit source word) updates. The frontier
    column of v at level n holds bit b of state q's row iff dist_b(q, v) = n;
    W = 4 x its non-zero 32-bit words (source b in word b // 32 of its row).
    Bytes: 2W + 8 per active (n, v), 8 per scan, 4 + W per scanned edge, and
    ceil(V/8) per source for the results."""
    V, L, NL, Q = g.num_vertices, g.num_labels, nfa.num_labels, nfa.num_states
    B = len(sources)
    D = np.stack([np.asarray(d) for d in dists])  # (B, Q, V)
    present = g.label_counts() > 0
    succ = {}
    for a, s, b in nfa.triples():
        lab = s if s < NL else s - NL
        if lab < L and present[lab]:
            succ.setdefault(s, {}).setdefault(a, set()).add(b)
    deg = {}
    for s in succ:
        lab, inv = (s, False) if s < NL else (s - NL, True)
        src, dst = g.edges_of(lab)
        pairs = np.unique(np.stack([src, dst], 1), axis=0) if src.size else np.zeros((0, 2), np.int64)
        deg[s] = np.bincount(pairs[:, 1 if inv else 0], minlength=V).astype(np.int64)
    scans = scanned = byt = active = upd = 0
    w32 = np.arange(B) // 32
    w64 = np.arange(B) // 64
    for v in range(V):
        col = D[:, :, v]  # (B, Q)
        for n in np.unique(col[col >= 0]):
            hit = col == n  # (B, Q)
            S = set(np.nonzero(hit.any(axis=0))[0].tolist())
            W = 4 * sum(np.unique(w32[hit[:, q]]).size for q in range(Q))
            nz64 = {q: np.unique(w64[hit[:, q]]).size for q in S}
            active += 1
            byt += 2 * W + 8
            for s, tab in succ.items():
                img = set()
                for q in S:
                    img |= tab.get(q, set())
                if not img:
                    continue
                d = int(deg[s][v])
                scans += 1
                scanned += d
                byt += 8 + (4 + W) * d
                upd += d * sum(len(tab.get(q, ())) * nz64[q] for q in S)
    byt += B * ((V + 7) // 8)
    return scans, scanned, active, byt, upd


def check_stacked_counters_product(rng, n_cases=30):
    """stacked_counters fed with the oracle's distances equals the same
    function fed with the explicit product automaton's distances (networkx),
    and for one source its scans, scanned edges and active pairs are the
    single-query ones."""
    import oracle
    import product_graph as PG
    for _ in range(n_cases):
        g = tiny_graph(rng, nv=int(rng.integers(2, 7)), ne=int(rng.integers(1, 12)))
        text = tiny_expr(rng, g.num_labels, max_leaves=4)
        nfa = R.compile_regex(text, g.num_labels)
        B = int(rng.integers(1, 70))
        srcs = rng.integers(0, g.num_vertices, size=B).tolist()
        og = oracle.Graph(g)
        od = [og.ssr(nfa, s, keep_dist=True).dist for s in srcs]
        pd = []
        pg = PG.product(g, nfa)
        for s in srcs:
            d = np.full((nfa.num_states, g.num_vertices), -1, np.int32)
            for (q, v), n in PG.levels(pg, nfa, s).items():
                d[q, v] = n
            pd.append(d)
        a = stacked_counters(g, nfa, srcs, od)
        assert a == stacked_counters(g, nfa, srcs, pd), text
        r = og.ssr(nfa, srcs[0])
        one = stacked_counters(g, nfa, srcs[:1], od[:1])
        assert one[:3] == (r.scans, r.scanned_edges, r.active), text
