"""GPU parity of the two outputs beyond the Boolean answer, through the C ABI:

* rpq_single_source_lengths: the length of the shortest accepted walk per
  vertex, element by element against the oracle's least final-state distance,
  the brute-force enumeration on tiny graphs and the Manhattan distance on the
  grid, in the persistent kernel (automatic, push, pull) and the host loop;
* rpq_source_set: the query from a start set V_s (Def. 2.6), against the
  oracle's search from Q_S x V_s (answer, per-level |M_n|, work counters),
  for sets that fit a small level and sets that start on the whole grid."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from workloads import configs as C
from workloads import graphs as G
from workloads import regex as R
import oracle_cases as OC

MODES = {"auto": 0, "push": 8, "pull": 16, "hostloop": 32, "hostloop-pull": 32 | 16, "graph": 64,
         "graph-pull": 64 | 16}


@pytest.fixture(scope="module")
def rpq():
    from paper_2412_10287_amd import rpq as mod
    return mod


def _lengths_all_modes(rpq, gg, nfa, s, want, tag):
    nh = rpq.NFA(nfa)
    for name, fl in MODES.items():
        d, st = gg.single_source_lengths(nh, int(s), flags=fl, level_cap=4096)
        assert np.array_equal(d, want), (tag, nfa.text, int(s), name)
        bm, _ = gg.single_source(nh, int(s), flags=fl)
        assert np.array_equal(OC.bitmap_of(np.nonzero(d >= 0)[0].tolist(), gg.num_vertices), bm), (tag, name)


def test_lengths_tiny_brute(rpq):
    import brute
    rng = np.random.default_rng(31)
    checked = 0
    for case in range(40):
        g = OC.tiny_graph(rng)
        text = OC.tiny_expr(rng, g.num_labels)
        nfa = R.compile_regex(text, g.num_labels)
        src = int(rng.integers(0, g.num_vertices))
        want = oracle.ssr(g, nfa, src, keep_dist=True).lengths()
        try:
            best = brute.min_match_len(g, text, src, nfa.num_states * g.num_vertices - 1, max_pairs=300_000)
            assert np.array_equal(best, want)
            checked += 1
        except RuntimeError:
            pass
        print("case", case, text, src, flush=True)
        _lengths_all_modes(rpq, rpq.Graph(g), nfa, src, want, case)
    assert checked >= 15


def test_lengths_er_and_rmat(rpq):
    w = C.er_workload()
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    for nfa, s in zip(w.nfas, w.sources):
        _lengths_all_modes(rpq, gg, nfa, s, og.ssr(nfa, int(s), keep_dist=True).lengths(), "er")
    w = C.rmat_workload(scale=17, edge_factor=16, num_labels=16, n_per_template=2)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    gg.set_option("pull_alpha", 4)  # switch directions inside the automatic runs
    for nfa, s in zip(w.nfas, w.sources):
        print("rmat17", nfa.text, int(s), flush=True)
        _lengths_all_modes(rpq, gg, nfa, s, og.ssr(nfa, int(s), keep_dist=True).lengths(), "rmat17")
    # wide state words (2 and 4 bytes)
    rng = np.random.default_rng(8)
    for leaves in (12, 25):
        nfa = R.glushkov(R.random_ast(rng, leaves, lambda r: r.integers(0, 16), 0.3), 16)
        s = int(w.sources[0])
        _lengths_all_modes(rpq, gg, nfa, s, og.ssr(nfa, s, keep_dist=True).lengths(), "wide")


def test_lengths_grid_manhattan_and_device_output(rpq):
    side = 96
    g = G.grid(side, 0.0, 0)
    gg = rpq.Graph(g)
    nh = rpq.NFA(R.compile_regex("(0|1)*", 4))
    xs, ys = np.meshgrid(np.arange(side), np.arange(side))
    out = rpq.DeviceBuffer(4 * side * side)
    for x0, y0 in ((0, 0), (40, 7), (95, 95)):
        want = np.where((xs >= x0) & (ys >= y0), (xs - x0) + (ys - y0), -1).ravel().astype(np.int32)
        for name, fl in MODES.items():
            d, st = gg.single_source_lengths(nh, y0 * side + x0, flags=fl)
            assert np.array_equal(d, want), (x0, y0, name)
        gg.single_source_lengths(nh, y0 * side + x0, out_device_ptr=out.ptr)
        assert np.array_equal(out.to_host(np.int32), want), (x0, y0)
    out.close()


def _check_set(rpq, gg, og, nfa, srcs, tag):
    want = og.ssr_set(nfa, srcs)
    nh = rpq.NFA(nfa)
    for name, fl in MODES.items():
        bm, st = gg.source_set(nh, srcs, flags=fl | rpq.COUNTERS, level_cap=4096)
        assert np.array_equal(bm, want.bitmap), (tag, nfa.text, len(srcs), name)
        assert np.array_equal(st.level_counts, want.level_counts), (tag, nfa.text, len(srcs), name)
        assert (st.product_edges, st.scans, st.scanned_edges, st.active, st.alg_bytes) == \
            (want.product_edges, want.scans, want.scanned_edges, want.active, want.alg_bytes), (tag, name)


def test_source_sets(rpq):
    rng = np.random.default_rng(5)
    for case in range(20):
        g = OC.tiny_graph(rng)
        nfa = R.compile_regex(OC.tiny_expr(rng, g.num_labels), g.num_labels)
        srcs = [int(x) for x in rng.integers(0, g.num_vertices, size=int(rng.integers(1, 5)))]
        _check_set(rpq, rpq.Graph(g), oracle.Graph(g), nfa, srcs, case)
    w = C.rmat_workload(scale=14, edge_factor=16, num_labels=16, n_per_template=1)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    V = w.graph.num_vertices
    for k in (1, 3, 100, 511, 512, 513, 3000):
        # up to 512 start vertices the first levels run in one workgroup;
        # more start on the whole grid; repeats are merged
        srcs = [int(x) for x in rng.integers(0, V, size=k)] + [0, 0]
        for nfa in w.nfas:
            print("set", k, nfa.text, flush=True)
            _check_set(rpq, gg, og, nfa, srcs, k)
    # the whole vertex set, with the empty word accepted (every vertex)
    nfa = R.compile_regex("0*", 16)
    _check_set(rpq, gg, og, nfa, list(range(V)), "all")
    bm, _ = gg.source_set(rpq.NFA(nfa), list(range(V)))
    assert int(sum(bin(int(x)).count("1") for x in bm)) == V
    # a single source equals rpq_single_source
    for nfa, s in zip(w.nfas, w.sources):
        a, sa = gg.source_set(rpq.NFA(nfa), [int(s)], level_cap=512)
        b, sb = gg.single_source(rpq.NFA(nfa), int(s), level_cap=512)
        assert np.array_equal(a, b) and np.array_equal(sa.level_counts, sb.level_counts)


def test_source_set_errors(rpq):
    g = G.erdos_renyi(100, 300, 2, 1)
    gg = rpq.Graph(g)
    nh = rpq.NFA(R.compile_regex("0*", 2))
    for bad in ([], [100], [3, -1]):
        with pytest.raises(rpq.RPQError) as e:
            gg.source_set(nh, bad)
        assert e.value.status == rpq.RPQ_EINVAL
    with pytest.raises(rpq.RPQError):
        gg.single_source_lengths(nh, 100)
    bm, _ = gg.source_set(nh, [0, 5])
    assert np.array_equal(bm, oracle.Graph(g).ssr_set(R.compile_regex("0*", 2), [0, 5]).bitmap)
