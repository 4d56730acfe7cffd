"""GPU parity: the HIP path (through the C ABI) against the oracle, bit-exact,
on the same seeded inputs. Results are sets, so the tolerance is zero bits;
per-level frontier sizes |M_n| and the algorithmic counters must match too."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from workloads import configs as C
from workloads import graphs as G
from workloads import regex as R
import oracle_cases as OC


@pytest.fixture(scope="module")
def rpq():
    from paper_2412_10287_amd import rpq as mod
    return mod


MODES = {"auto": 0, "push": 8, "pull": 16, "hostloop": 32, "hostloop-pull": 32 | 16, "graph": 64,
         "graph-pull": 64 | 16}


def _run(rpq, gg, nfa_h, src, flags=0, level_cap=0):
    bm, st = gg.single_source(nfa_h, src, flags=flags, level_cap=level_cap)
    return bm, st


def test_first_light(rpq):
    # a few tiny cases per mode, host-driven levels first; prints each case
    rng = np.random.default_rng(5)
    for case in range(4):
        g = OC.tiny_graph(rng)
        text = OC.tiny_expr(rng, g.num_labels)
        nfa = R.compile_regex(text, g.num_labels)
        src = int(rng.integers(0, g.num_vertices))
        want = oracle.ssr(g, nfa, src)
        gg = rpq.Graph(g)
        print("persistent grid", gg.info("persistent_grid"), "occupancy api blocks/CU",
              gg.info("occupancy_blocks_per_cu"), flush=True)
        nh = rpq.NFA(nfa)
        for name in ("hostloop", "hostloop-pull", "auto", "push", "pull"):
            print("case", case, text, "source", src, "mode", name, flush=True)
            bm, st = _run(rpq, gg, nh, src, MODES[name], level_cap=64)
            assert np.array_equal(bm, want.bitmap), (case, text, src, name)


def test_tiny_graphs_all_modes(rpq):
    rng = np.random.default_rng(99)
    for case in range(60):
        g = OC.tiny_graph(rng)
        text = OC.tiny_expr(rng, g.num_labels)
        nfa = R.compile_regex(text, g.num_labels)
        src = int(rng.integers(0, g.num_vertices))
        want = oracle.ssr(g, nfa, src)
        gg = rpq.Graph(g)
        nh = rpq.NFA(nfa)
        for name, fl in MODES.items():
            bm, st = _run(rpq, gg, nh, src, fl, level_cap=64)
            assert np.array_equal(bm, want.bitmap), (case, text, src, name)
            assert st.levels == want.levels, (case, text, name)
            assert np.array_equal(st.level_counts, want.level_counts), (case, text, name)


def test_er_workload(rpq):
    w = C.er_workload()
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    for text, nfa, s in zip(w.queries, w.nfas, w.sources):
        want = og.ssr(nfa, int(s))
        nh = rpq.NFA(nfa)
        for name, fl in MODES.items():
            bm, st = _run(rpq, gg, nh, int(s), fl | rpq.COUNTERS, level_cap=4096)
            assert np.array_equal(bm, want.bitmap), (text, name)
            assert np.array_equal(st.level_counts, want.level_counts), (text, name)
            assert st.visited_pairs == int(want.level_counts.sum())
            assert (st.product_edges, st.scans, st.scanned_edges, st.active, st.alg_bytes) == \
                (want.product_edges, want.scans, want.scanned_edges, want.active, want.alg_bytes), (text, name)


def test_rmat_small_templates(rpq):
    w = C.rmat_workload(scale=14, edge_factor=16, num_labels=16, n_per_template=6)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    switched = 0
    for text, nfa, s in zip(w.queries, w.nfas, w.sources):
        want = og.ssr(nfa, int(s))
        nh = rpq.NFA(nfa)
        for name, fl in MODES.items():
            bm, st = _run(rpq, gg, nh, int(s), fl, level_cap=4096)
            assert np.array_equal(bm, want.bitmap), (text, name)
            assert np.array_equal(st.level_counts, want.level_counts), (text, name)
        # direction switching on: push->pull->push within one traversal
        for alpha, beta in ((4, 24), (30, 4), (1000, 2)):
            gg.set_option("pull_alpha", alpha)
            gg.set_option("pull_beta", beta)
            for fl in (0, rpq.HOST_LOOP):
                bm, st = _run(rpq, gg, nh, int(s), fl, level_cap=4096)
                assert np.array_equal(bm, want.bitmap), (text, alpha, beta, fl)
                assert np.array_equal(st.level_counts, want.level_counts), (text, alpha, beta, fl)
                switched += st.push_levels > 0 and st.pull_levels > 0
        gg.set_option("pull_alpha", 0)
    assert switched > 0


def test_wide_state_words(rpq):
    # 9..16 states use 2-byte words, 17..32 states 4-byte words
    rng = np.random.default_rng(4)
    g = G.rmat(12, 8, 6, 1.1, 21)
    og = oracle.Graph(g)
    gg = rpq.Graph(g)
    for leaves in (9, 12, 15, 20, 26, 31):
        ast = R.random_ast(rng, leaves, lambda r: r.integers(0, 6), 0.3)
        nfa = R.glushkov(ast, 6)
        assert nfa.num_states == leaves + 1
        nh = rpq.NFA(nfa)
        for s in rng.integers(0, g.num_vertices, size=3):
            want = og.ssr(nfa, int(s))
            for name, fl in MODES.items():
                bm, st = _run(rpq, gg, nh, int(s), fl, level_cap=4096)
                assert np.array_equal(bm, want.bitmap), (leaves, name)
                assert np.array_equal(st.level_counts, want.level_counts), (leaves, name)


def test_long_chain_runs_of_small_levels(rpq):
    # a path of 5000 vertices: 5000 levels of one vertex each, all small, so
    # the levels run in workgroup 0 in runs of at most 2048 (three runs);
    # a second label hangs a star off the middle so one level is large
    n = 5000
    src = list(range(n - 1)) + [2500] * 3000
    dst = list(range(1, n)) + [n + i for i in range(3000)]
    lab = [0] * (n - 1) + [1] * 3000
    g = G.from_triples(n + 3000, 2, np.array(src), np.array(dst), np.array(lab))
    gg = rpq.Graph(g)
    og = oracle.Graph(g)
    for text in ("0*", "(0|1)*", "0* 1"):
        nfa = R.compile_regex(text, 2)
        want = og.ssr(nfa, 0)
        for name in ("auto", "push", "pull"):
            bm, st = _run(rpq, gg, rpq.NFA(nfa), 0, MODES[name], level_cap=8192)
            assert np.array_equal(bm, want.bitmap), (text, name)
            assert np.array_equal(st.level_counts, want.level_counts), (text, name)


def test_small_level_handoffs(rpq):
    # Workgroup 0 runs small levels from the start of a query and hands a
    # level to the grid once it is too large. Here the hand-off happens
    # (a) at level 0, from a hub with 20000 out-edges (more push edges than a
    # small level may have), and (b) at level 1, where 1000 vertices with
    # three labelled out-edges each give 3000 items (more than one LDS tile
    # holds) but only 3000 edges.
    hub, m = 0, 1000
    src = [hub] * 20000 + [hub] * m
    dst = [1 + m + i for i in range(20000)] + [1 + i for i in range(m)]
    lab = [3] * 20000 + [0] * m
    base = 1 + m + 20000
    for i in range(m):
        for k in (1, 2, 3):
            src.append(1 + i)
            dst.append(base + (3 * i + k) % 4000)
            lab.append(k)
    g = G.from_triples(base + 4000, 4, np.array(src), np.array(dst), np.array(lab))
    gg = rpq.Graph(g)
    og = oracle.Graph(g)
    for text in ("3", "3*", "(3|0)+", "0 (1|2|3)", "0 (1|2|3) ^3", "(0|1|2|3)*"):
        nfa = R.compile_regex(text, 4)
        want = og.ssr(nfa, hub)
        for name in ("auto", "push", "pull", "hostloop"):
            bm, st = _run(rpq, gg, rpq.NFA(nfa), hub, MODES[name], level_cap=64)
            assert np.array_equal(bm, want.bitmap), (text, name)
            assert np.array_equal(st.level_counts, want.level_counts), (text, name)
            assert st.levels == want.levels, (text, name)


def test_fused_mid_size_levels(rpq):
    # With 2^17 vertices, levels of 1025 to 4096 candidates after a push level
    # are fused: each workgroup pushes its own items, and rounds beyond its
    # budget (hubs of this R-MAT graph) are pushed over the grid after the
    # barrier. Wide state words (11 and 19 states) take the same path.
    w = C.rmat_workload(scale=17, edge_factor=16, num_labels=16, n_per_template=3)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    extra = ["(0|1|2|3|4|5|6|7|8|9)*", "(0|^1|2|^3|4|5|6|7|8|9|10|11|12|13|14|15|^0|1 2)*"]
    cases = list(zip(w.queries, w.nfas, w.sources))
    cases += [(t, R.compile_regex(t, 16), int(w.sources[k])) for k, t in enumerate(extra)]
    for text, nfa, s in cases:
        want = og.ssr(nfa, int(s))
        nh = rpq.NFA(nfa)
        for name in ("auto", "push"):
            bm, st = _run(rpq, gg, nh, int(s), MODES[name] | rpq.COUNTERS, level_cap=4096)
            assert np.array_equal(bm, want.bitmap), (text, name)
            assert np.array_equal(st.level_counts, want.level_counts), (text, name)
            assert (st.product_edges, st.scans, st.scanned_edges, st.active, st.alg_bytes) == \
                (want.product_edges, want.scans, want.scanned_edges, want.active, want.alg_bytes), (text, name)
            bm2, st2 = _run(rpq, gg, nh, int(s), MODES[name])
            assert np.array_equal(bm2, want.bitmap), (text, name)
            assert st2.visited_pairs == int(want.level_counts.sum()), (text, name)


def test_grid_closed_forms_gpu(rpq):
    side = 48
    g = G.grid(side, 0.0, 0)
    gg = rpq.Graph(g)

    def fn(graph, nfa, s):
        bm, st = gg.single_source(rpq.NFA(nfa), s)
        return bm, None, st.levels

    OC.check_grid(fn, side, np.random.default_rng(3), n=4)


def test_special_cases_gpu(rpq):
    g = G.erdos_renyi(3000, 9000, 5, 3)
    gg = rpq.Graph(g)

    def fn(graph, nfa, s):
        bm, st = gg.single_source(rpq.NFA(nfa), s)
        return bm, None, st.levels

    OC.check_special(fn, np.random.default_rng(17), g)


def test_edge_cases(rpq):
    # isolated source, empty start set, no final states, labels missing from the
    # graph, self-loops, a single vertex
    g = G.from_triples(5, 2, [0, 1, 1, 3], [1, 1, 2, 3], [0, 0, 1, 0])
    gg = rpq.Graph(g)
    og = oracle.Graph(g)
    cases = [R.compile_regex(t, 4) for t in ["0*", "0+", "(0|^0)*", "3*", "3", "^3 0", "1 ^1", "0 0 0 0"]]
    cases.append(R.nfa_from_triples(2, 2, [(0, 0, 1)], [], [1]))
    cases.append(R.nfa_from_triples(2, 2, [(0, 0, 1)], [0], []))
    for nfa in cases:
        nh = rpq.NFA(nfa)
        for s in range(5):
            want = og.ssr(nfa, s)
            for name, fl in MODES.items():
                bm, st = _run(rpq, gg, nh, s, fl, level_cap=64)
                assert np.array_equal(bm, want.bitmap), (nfa.text, s, name)
                assert st.levels == want.levels
    one = rpq.Graph(G.from_triples(1, 1, [], [], []))
    bm, _ = one.single_source(rpq.NFA(R.compile_regex("0*", 1)), 0)
    assert bm.tolist() == [1]


def test_errors(rpq):
    g = G.erdos_renyi(100, 300, 2, 1)
    gg = rpq.Graph(g)
    nh = rpq.NFA(R.compile_regex("0*", 2))
    with pytest.raises(rpq.RPQError) as e:
        gg.single_source(nh, 100)
    assert e.value.status == rpq.RPQ_EINVAL
    with pytest.raises(rpq.RPQError):
        gg.single_source(nh, 0, flags=rpq.FORCE_PUSH | rpq.FORCE_PULL)
    with pytest.raises(rpq.RPQError):
        gg.set_option("no_such_option", 1)
    # still usable after errors
    bm, _ = gg.single_source(nh, 0)
    assert np.array_equal(bm, oracle.ssr(g, R.compile_regex("0*", 2), 0).bitmap)


def test_repeat_is_stable(rpq):
    # all device updates are idempotent ORs; repeated runs (different atomic
    # interleavings) must give identical sets and level counts
    w = C.rmat_workload(scale=13, edge_factor=16, num_labels=8, n_per_template=2)
    gg = rpq.Graph(w.graph)
    for nfa, s in zip(w.nfas, w.sources):
        nh = rpq.NFA(nfa)
        first, st0 = gg.single_source(nh, int(s), level_cap=1024)
        for _ in range(5):
            bm, st = gg.single_source(nh, int(s), level_cap=1024)
            assert np.array_equal(bm, first)
            assert np.array_equal(st.level_counts, st0.level_counts)
        # without per-level outputs |P| comes from the kernel's own sum
        bm, st = gg.single_source(nh, int(s))
        assert np.array_equal(bm, first)
        assert st.visited_pairs == int(st0.level_counts.sum()) and st.levels == st0.levels


def test_cooperative_launch_option(rpq):
    # the persistent kernel started with hipLaunchCooperativeKernel and with
    # an ordinary launch (the default) gives the oracle's answers either way
    w = C.rmat_workload(scale=13, edge_factor=16, num_labels=8, n_per_template=2)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    assert gg.get_option("cooperative_launch") == 0
    with pytest.raises(rpq.RPQError):
        gg.set_option("cooperative_launch", 2)
    for coop in (1, 0):
        gg.set_option("cooperative_launch", coop)
        for nfa, s in zip(w.nfas, w.sources):
            want = og.ssr(nfa, int(s))
            bm, st = gg.single_source(rpq.NFA(nfa), int(s), level_cap=1024)
            assert np.array_equal(bm, want.bitmap), coop
            assert np.array_equal(st.level_counts, want.level_counts), coop


def test_query_constant_cache(rpq):
    # automata over most of the 128 symbols (constant blocks of about 36 KB,
    # beyond the LDS copy) from 160 handles, queried twice in opposite
    # orders: the device cache of query constants fills, starts over and
    # serves repeats; every answer stays the oracle's
    L = 64
    g = G.erdos_renyi(3000, 20000, L, seed=5)
    og = oracle.Graph(g)
    gg = rpq.Graph(g)
    rng = np.random.default_rng(7)
    cases = []
    for k in range(160):
        syms = rng.permutation(2 * L)
        tr = [(0, int(a), 1) for a in syms[:100]] + [(1, int(a), 1) for a in syms[100:128]]
        tr += [(1, int(a), 2) for a in rng.choice(2 * L, size=20, replace=False)]
        nfa = R.nfa_from_triples(3, L, tr, [0], [2])
        cases.append((nfa, rpq.NFA(nfa), int(rng.integers(0, 3000))))
    want = [og.ssr(nfa, s).bitmap for nfa, _, s in cases]
    for order in (list(range(len(cases))), list(reversed(range(len(cases))))):
        for i in order:
            _, nh, s = cases[i]
            bm, _ = gg.single_source(nh, s)
            assert np.array_equal(bm, want[i]), i


def test_single_destination(rpq):
    # SDR(t) = { s : t in SSR(s) } (Sec. 2), checked by running the oracle's
    # single-source query from every vertex; the GPU runs the reversed,
    # inverted automaton from t (Sec. 4)
    rng = np.random.default_rng(21)
    for case in range(6):
        g = G.erdos_renyi(120, 420, 3, 100 + case)
        og = oracle.Graph(g)
        gg = rpq.Graph(g)
        text = OC.tiny_expr(rng, g.num_labels, max_leaves=4)
        nfa = R.compile_regex(text, g.num_labels)
        nh = rpq.NFA(nfa)
        reach = np.stack([og.ssr(nfa, s).bitmap for s in range(g.num_vertices)])
        for t in rng.integers(0, g.num_vertices, size=4):
            t = int(t)
            col = (reach[:, t >> 6] >> np.uint64(t & 63)) & np.uint64(1)
            want = OC.bitmap_of(np.nonzero(col)[0].tolist(), g.num_vertices)
            for fl in (0, 8, 16):
                bm, _ = gg.single_destination(nh, t, flags=fl)
                assert np.array_equal(bm, want), (text, t, fl)


def test_autotune_keeps_answers(rpq):
    # the tuner times its candidates and keeps one; answers under the kept
    # settings are still the oracle's, on both tuned paths
    w = C.rmat_workload(scale=12, edge_factor=8, num_labels=8, n_per_template=2)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    nh = [rpq.NFA(n) for n in w.nfas]
    srcs = [int(s) for s in w.sources]
    rec = gg.autotune(rpq.TUNE_PLAIN, nh, srcs)
    assert rec["candidates"] >= 22 and rec["best_ms"] <= rec["default_ms"] + 1e-9
    assert gg.get_option("pull_alpha") == rec["alpha"] and gg.get_option("persistent_grid") == rec["grid"]
    for h, n, s in zip(nh, w.nfas, srcs):
        bm, _ = gg.single_source(h, s)
        assert np.array_equal(bm, og.ssr(n, s).bitmap)
    rec = gg.autotune(rpq.TUNE_STACKED, nh[:1], srcs * 3)
    assert gg.get_option("stacked_alpha") == rec["alpha"]
    # the second stage times the hand-off thresholds other than the kept one
    assert rec["candidates"] == 19 + 3 and rec["handoff_edges"] in (0, 1 << 20, 1 << 22, 1 << 24)
    assert gg.get_option("stacked_handoff_edges") == rec["handoff_edges"]
    assert rec["best_ms"] <= rec["default_ms"] + 1e-9
    bms, _ = gg.multi_source(nh[0], srcs * 3)
    for i, s in enumerate(srcs * 3):
        assert np.array_equal(bms[i], og.ssr(w.nfas[0], s).bitmap)


def test_rare_end_plan(rpq):
    # the rare-end plan (one stacked traversal of the reversed automaton from
    # every candidate endpoint, reporting only whether each reaches the
    # source) returns the forward traversal's answer: forced, and chosen
    # automatically under rare_end_max; queries ending in rare labels, in
    # inverse labels, accepting the empty word, and with no candidates
    g = G.rmat(12, 8, 16, 1.3, 77)
    og = oracle.Graph(g)
    gg = rpq.Graph(g)
    counts = g.label_counts()
    rare = [int(l) for l in np.argsort(counts)[:6]]
    common = [int(l) for l in np.argsort(counts)[-3:]]
    rng = np.random.default_rng(19)
    texts = ["%d* %d" % (common[0], rare[0]), "(%d|%d)* ^%d" % (common[0], common[1], rare[1]),
             "%d+ (%d|%d)" % (common[2], rare[2], rare[3]), "%d*" % rare[4], "%d ^%d*" % (common[1], rare[5]),
             "(%d|^%d)* %d" % (common[0], common[0], rare[0]), "15 14", "^%d" % rare[2]]
    used = 0
    for text in texts:
        nfa = R.compile_regex(text, 16)
        nh = rpq.NFA(nfa)
        for s in rng.integers(0, g.num_vertices, size=6):
            want = og.ssr(nfa, int(s)).bitmap
            try:
                bm, st = gg.single_source(nh, int(s), flags=rpq.RARE_END)
            except rpq.RPQError as e:
                assert e.status == rpq.RPQ_EINVAL and "candidate" in str(e), (text, str(e))
                continue
            assert st.plan == 1, text
            assert np.array_equal(bm, want), (text, int(s))
            used += 1
            out = rpq.DeviceBuffer(8 * gg.words)
            gg.single_source(nh, int(s), flags=rpq.RARE_END, out_device_ptr=out.ptr)
            assert np.array_equal(out.to_host(), want), (text, int(s))
            out.close()
    assert used >= 20
    # automatic choice: the same answers, plan 1 exactly when few candidates
    gg.set_option("rare_end_max", 300)
    for text in texts:
        nfa = R.compile_regex(text, 16)
        nh = rpq.NFA(nfa)
        s = int(rng.integers(0, g.num_vertices))
        bm, st = gg.single_source(nh, s)
        assert np.array_equal(bm, og.ssr(nfa, s).bitmap), text
        bm2, st2 = gg.single_source(nh, s, level_cap=64)  # per-level outputs: always forward
        assert st2.plan == 0 and np.array_equal(bm2, bm)
    gg.set_option("rare_end_max", 0)
    with pytest.raises(rpq.RPQError):
        gg.single_source(rpq.NFA(R.compile_regex(texts[0], 16)), 0, flags=rpq.RARE_END | rpq.COUNTERS)
