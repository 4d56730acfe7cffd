"""Pins of the oracle against what the paper and the mathematics fix, with no
GPU: brute-force walk enumeration with an independent regex matcher, the
frontier-free fixpoint (Alg. 2), library special cases, grid closed forms,
invariants of the query semantics, and the work counters recomputed from the
distances."""
import numpy as np
import pytest

import oracle
from oracle.alg2 import alg2
from workloads import configs as C
from workloads import graphs as G
from workloads import regex as R
import oracle_cases as OC
from nfa_sim import subset_dfa, thompson


def oracle_fn(g, nfa, src):
    r = oracle.ssr(g, nfa, src, keep_dist=True)
    return r.bitmap, r.dist, r.levels


def test_brute_force_tiny():
    rng = np.random.default_rng(11)
    full = OC.check_brute(oracle_fn, rng, n_cases=120)
    assert full >= 60  # most cases run to the complete bound


def test_handworked_golden():
    # hand-derived fixtures; see the file for each case's derivation
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "handworked.txt")
    cases = _read_golden(path)
    assert len(cases) >= 6
    for c in cases:
        g = G.from_triples(c["V"], c["L"], *zip(*c["edges"]), dedupe=False) if c["edges"] else \
            G.from_triples(c["V"], c["L"], [], [], [])
        nfa = R.compile_regex(c["query"], c["L"])
        r = oracle.ssr(g, nfa, c["source"])
        assert r.vertices().tolist() == c["expect"], c
        if "levels" in c:
            assert r.levels == c["levels"], c


def _read_golden(path):
    cases, cur = [], None
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        key, _, val = line.partition(":")
        key, val = key.strip(), val.strip()
        if key == "case":
            cur = {"name": val, "edges": []}
            cases.append(cur)
        elif key == "graph":
            v, l = val.split()
            cur["V"], cur["L"] = int(v), int(l)
        elif key == "edge":
            s, d, l = val.split()
            cur["edges"].append((int(s), int(d), int(l)))
        elif key == "query":
            cur["query"] = val
        elif key == "source":
            cur["source"] = int(val)
        elif key == "expect":
            cur["expect"] = [int(x) for x in val.split()] if val != "-" else []
        elif key == "levels":
            cur["levels"] = int(val)
    return cases


@pytest.mark.parametrize("seed", range(4))
def test_alg2_agrees(seed):
    rng = np.random.default_rng(100 + seed)
    g = G.erdos_renyi(300, 900, 4, 50 + seed)
    og = oracle.Graph(g)
    for _ in range(12):
        text = R.to_string(R.random_ast(rng, int(rng.integers(1, 6)),
                                        lambda r: r.integers(0, 4), 0.4))
        nfa = R.compile_regex(text, 4)
        s = int(rng.integers(0, 300))
        assert np.array_equal(og.ssr(nfa, s).bitmap, alg2(g, nfa, s)), text


def test_alg2_agrees_er_workload():
    w = C.er_workload()
    og = oracle.Graph(w.graph)
    for text, nfa, s in list(zip(w.queries, w.nfas, w.sources))[:8]:
        assert np.array_equal(og.ssr(nfa, int(s)).bitmap, alg2(w.graph, nfa, int(s))), text


def test_library_special_cases():
    rng = np.random.default_rng(5)
    OC.check_special(oracle_fn, rng, G.erdos_renyi(2000, 6000, 5, 3))
    OC.check_special(oracle_fn, rng, G.rmat(11, 4, 6, 1.1, 9))


def test_grid_closed_forms():
    OC.check_grid(oracle_fn, 24, np.random.default_rng(2), n=6)


def _rand_query(rng, L, k=(1, 5)):
    return R.to_string(R.random_ast(rng, int(rng.integers(*k)), lambda r: r.integers(0, L), 0.4))


def test_invariants():
    rng = np.random.default_rng(21)
    L = 3
    g = G.erdos_renyi(400, 1000, L, 77)
    og = oracle.Graph(g)
    V = g.num_vertices
    S = lambda text, s, graph=og: set(graph.ssr(R.compile_regex(text, L), s).vertices().tolist())
    for _ in range(10):
        r1, r2 = _rand_query(rng, L), _rand_query(rng, L)
        s = int(rng.integers(0, V))
        # I4 union
        assert S("(%s)|(%s)" % (r1, r2), s) == S(r1, s) | S(r2, s)
        # I5 concatenation
        mid = S(r1, s)
        want = set()
        for u in mid:
            want |= S(r2, u)
        assert S("(%s) (%s)" % (r1, r2), s) == want
        # I6 star = source plus the plus
        assert S("(%s)*" % r1, s) == {s} | S("(%s)+" % r1, s)
        # I7 language-equivalent automata agree
        node = R.parse(r1)
        gl = R.glushkov(node, L)
        for other in (subset_dfa(gl), thompson(node, L)):
            if other.num_states <= 64:
                assert np.array_equal(og.ssr(other, s).bitmap, og.ssr(gl, s).bitmap)
    # I3 reversal: t in SSR(s, R) iff s in SSR(t, R reversed and inverted)
    for _ in range(4):
        text = _rand_query(rng, L)
        nfa = R.compile_regex(text, L)
        rev = R.reverse_nfa(nfa)
        s = int(rng.integers(0, V))
        fwd = og.ssr(nfa, s).vertices()
        for t in fwd[:15].tolist() + rng.integers(0, V, size=10).tolist():
            assert (t in set(fwd.tolist())) == (s in set(og.ssr(rev, int(t)).vertices().tolist()))
    # I9 empty language (no final states) and the empty word
    empty = R.nfa_from_triples(2, L, [(0, 0, 1)], [0], [])
    assert og.ssr(empty, 5).vertices().size == 0
    assert 7 in S("0*", 7) and 7 in S("(0 1)?", 7)
    # a.a* = a+
    for a in range(L):
        s = int(rng.integers(0, V))
        assert S("%d %d*" % (a, a), s) == S("%d+" % a, s)


def test_monotone_in_edges():
    # I2: adding edges never removes an answer
    rng = np.random.default_rng(8)
    L = 3
    g = G.erdos_renyi(300, 500, L, 4)
    extra_s = rng.integers(0, 300, 200)
    extra_d = rng.integers(0, 300, 200)
    extra_l = rng.integers(0, L, 200)
    lab = np.repeat(np.arange(L), np.diff(g.label_ptr))
    g2 = G.from_triples(300, L, np.concatenate([g.src, extra_s]),
                        np.concatenate([g.dst, extra_d]), np.concatenate([lab, extra_l]))
    o1, o2 = oracle.Graph(g), oracle.Graph(g2)
    for _ in range(15):
        nfa = R.compile_regex(_rand_query(rng, L), L)
        s = int(rng.integers(0, 300))
        a, b = o1.ssr(nfa, s).bitmap, o2.ssr(nfa, s).bitmap
        assert np.array_equal(a & b, a)


def test_level_counts_and_bound():
    rng = np.random.default_rng(3)
    g = G.erdos_renyi(500, 1500, 4, 1)
    og = oracle.Graph(g)
    for _ in range(10):
        nfa = R.compile_regex(_rand_query(rng, 4), 4)
        s = int(rng.integers(0, 500))
        r = og.ssr(nfa, s, keep_dist=True)
        d = r.dist
        assert r.levels <= nfa.num_states * 500  # termination bound of App. A
        assert r.levels == d.max() + 1
        for n in range(r.levels):
            assert r.level_counts[n] == np.count_nonzero(d == n) > 0
        assert r.level_counts[0] == len(set(nfa.start.tolist()))


def test_counters_match_python():
    rng = np.random.default_rng(31)
    g = G.erdos_renyi(200, 700, 3, 12)
    og = oracle.Graph(g)
    for _ in range(8):
        nfa = R.compile_regex(_rand_query(rng, 3), 3)
        s = int(rng.integers(0, 200))
        r = og.ssr(nfa, s, keep_dist=True)
        want = OC.python_counters(g, nfa, r.dist, oracle.word_bytes(nfa.num_states))
        assert (r.product_edges, r.scans, r.scanned_edges, r.alg_bytes, r.active) == want


def oracle_counters(g, nfa, src):
    r = oracle.ssr(g, nfa, src)
    return r.product_edges, r.scans, r.scanned_edges, r.alg_bytes, r.active, r.level_counts


def test_counters_explicit_product_graph():
    # counters and level counts against the explicit product automaton of
    # Def. 2.5 (networkx), on tiny graphs with multi-labelled and repeated edges
    OC.check_counters_product(oracle_counters, np.random.default_rng(41), n_cases=150)


def test_counters_closed_form_star():
    rng = np.random.default_rng(43)
    OC.check_counters_star(oracle_counters, rng, G.erdos_renyi(1500, 5000, 4, 13))
    OC.check_counters_star(oracle_counters, rng, G.rmat(10, 6, 5, 1.1, 17))


def test_counters_closed_form_grid():
    OC.check_counters_grid(oracle_counters, 17, np.random.default_rng(47), n=6)


def test_grid_counter_closed_form_by_hand():
    # the closed form itself, against a count done by hand on a 2 x 2 grid
    # from (0, 0): (0,(0,0)) has an east and a north edge, (1,(1,0)) a north
    # edge, (2,(0,1)) an east edge, the two pairs at (1,1) none: 4 product
    # edges; 4 active vertices, 8 scans (each reached vertex, both symbols),
    # 4 scanned edges
    assert OC.grid_star_counters(2, 0, 0) == (4, 8, 4, 10 * 4 + 8 * 8 + 5 * 4 + 1, 4)


def test_input_edge_cases():
    g = G.from_triples(1, 1, [], [], [])
    og = oracle.Graph(g)
    assert og.ssr(R.compile_regex("0*", 1), 0).vertices().tolist() == [0]
    assert og.ssr(R.compile_regex("0", 1), 0).vertices().tolist() == []
    # self-loop usable both ways; labels beyond the graph's contribute nothing
    g = G.from_triples(2, 1, [0], [0], [0])
    og = oracle.Graph(g)
    nfa = R.compile_regex("0 ^0 1*", 2)
    assert og.ssr(nfa, 0).vertices().tolist() == [0]
    with pytest.raises(ValueError):
        og.ssr(R.compile_regex("0", 1), 2)


def test_stacked_counters_explicit_product_graph():
    OC.check_stacked_counters_product(np.random.default_rng(53), n_cases=40)


def test_lengths_brute_force():
    # the shortest accepted walk per vertex (least distance of a final state
    # at the vertex) equals the brute-force enumeration's shortest matching
    # walk, which never builds an automaton
    import brute
    rng = np.random.default_rng(2024)
    checked = 0
    for _ in range(60):
        g = OC.tiny_graph(rng)
        text = OC.tiny_expr(rng, g.num_labels)
        nfa = R.compile_regex(text, g.num_labels)
        src = int(rng.integers(0, g.num_vertices))
        r = oracle.ssr(g, nfa, src, keep_dist=True)
        try:
            best = brute.min_match_len(g, text, src, nfa.num_states * g.num_vertices - 1, max_pairs=300_000)
        except RuntimeError:
            continue
        assert np.array_equal(r.lengths(), best), (text, src)
        checked += 1
    assert checked >= 30


def test_lengths_grid_manhattan():
    # (0|1)* on the grid without shortcuts: the shortest walk east/north from
    # (x0, y0) to (x, y) has length (x - x0) + (y - y0); -1 outside the
    # upper-right quadrant
    side = 24
    g = G.grid(side, 0.0, 0)
    og = oracle.Graph(g)
    nfa = R.compile_regex("(0|1)*", 4)
    xs, ys = np.meshgrid(np.arange(side), np.arange(side))
    for x0, y0 in ((0, 0), (5, 17), (23, 23), (11, 2)):
        got = og.ssr(nfa, y0 * side + x0, keep_dist=True).lengths()
        want = np.where((xs >= x0) & (ys >= y0), (xs - x0) + (ys - y0), -1).ravel()
        assert np.array_equal(got, want), (x0, y0)


def test_source_set_union_and_nearest_source():
    # a query from a start set V_s (Def. 2.6): the answer is the union of the
    # single-source answers, and a pair's distance is its least distance from
    # any source (breadth-first search from a set); repeats change nothing
    rng = np.random.default_rng(99)
    cases = []
    for _ in range(40):
        g = OC.tiny_graph(rng)
        cases.append((g, R.compile_regex(OC.tiny_expr(rng, g.num_labels), g.num_labels)))
    w = C.er_workload(n=600, m=2400, num_labels=4, n_queries=6)
    cases += [(w.graph, nfa) for nfa in w.nfas]
    for g, nfa in cases:
        og = oracle.Graph(g)
        k = int(rng.integers(1, min(6, g.num_vertices) + 1))
        srcs = [int(x) for x in rng.integers(0, g.num_vertices, size=k)]
        srcs.append(srcs[0])
        got = og.ssr_set(nfa, srcs, keep_dist=True)
        ones = [og.ssr(nfa, s, keep_dist=True) for s in srcs]
        bm = np.zeros_like(got.bitmap)
        for r in ones:
            bm |= r.bitmap
        assert np.array_equal(got.bitmap, bm), nfa.text
        big = np.iinfo(np.int64).max
        d = np.stack([np.where(r.dist < 0, big, r.dist.astype(np.int64)) for r in ones]).min(axis=0)
        d = np.where(d == big, -1, d)
        assert np.array_equal(got.dist, d), nfa.text
        assert got.levels == int(d.max()) + 1
        assert np.array_equal(got.level_counts, np.bincount(d[d >= 0].ravel(), minlength=got.levels))
