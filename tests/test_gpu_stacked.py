"""GPU parity of the stacked multi-source path (rpq_multi_source): each
source's bitmap equals the oracle's, for batch sizes that use 1, 2, 4, 8 and 16
64-bit words per state row, with repeated sources and NFAs of 1..32 states, in
the push direction, the pull direction and with the automatic switch; the
per-level frontier sizes summed over sources equal the oracle's |M_n| sums."""
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


# direction modes of the stacked kernel: automatic switch, push only, pull
# from level 0 (pull needs at most 8 states; wider automata always push)
STACK_MODES = {"auto": 0, "push": 8, "pull": 16}


def _check(rpq, gg, og, nfa, srcs, flags=0):
    """Every source's bitmap equals the oracle's; the level count, |P| and the
    per-level |M_n| (summed over sources) too, when one launch holds the batch."""
    bms, st = gg.multi_source(rpq.NFA(nfa), srcs, flags=flags, level_cap=4096)
    lv, pairs = 0, 0
    lc = np.zeros(4096, np.int64)
    for i, s in enumerate(srcs):
        r = og.ssr(nfa, int(s))
        assert np.array_equal(bms[i], r.bitmap), (nfa.text, i, int(s), flags)
        lv = max(lv, r.levels)
        pairs += int(r.level_counts.sum())
        lc[:len(r.level_counts)] += r.level_counts
    assert st.levels == lv, (nfa.text, flags)
    assert st.visited_pairs == pairs, (nfa.text, flags)
    if len(srcs) <= gg.get_option("max_batch"):
        assert np.array_equal(st.level_counts, lc[:lv]), (nfa.text, flags)
    return st


@pytest.mark.parametrize("B", [1, 5, 64, 65, 130, 256, 513, 1000])
def test_batch_sizes(rpq, B):
    g = G.rmat(12, 8, 6, 1.1, 31)
    gg = rpq.Graph(g)
    og = oracle.Graph(g)
    rng = np.random.default_rng(B)
    srcs = rng.integers(0, g.num_vertices, size=B)
    if B > 3:
        srcs[1] = srcs[2]
    gg.set_option("max_batch", 1024)
    for name, fl in STACK_MODES.items():
        print("B", B, "mode", name, flush=True)
        _check(rpq, gg, og, R.compile_regex("(0|^1)* 2 3*", 6), srcs, fl)


def test_direction_thresholds(rpq):
    # the automatic switch at several thresholds, including pull at almost
    # every level (alpha large, beta 1) and a switch back to push
    g = G.rmat(13, 8, 4, 1.1, 5)
    gg = rpq.Graph(g)
    og = oracle.Graph(g)
    srcs = np.random.default_rng(4).integers(0, g.num_vertices, size=150)
    nfa = R.compile_regex("(0|1)* ^2 (3|0)*", 4)
    seen = set()
    for alpha, beta in ((1, 24), (4, 24), (64, 1), (1000, 1), (2, 1000)):
        gg.set_option("stacked_alpha", alpha)
        gg.set_option("stacked_beta", beta)
        st = _check(rpq, gg, og, nfa, srcs)
        seen.add((st.push_levels > 0, st.pull_levels > 0))
    assert (True, True) in seen  # some setting mixed both directions


def test_hubs_pull_heavy(rpq):
    # stars far above the pull pass's light-row bound: a hub with 1499 in-edges
    # of label 0 and 1500 out-edges of label 1, plus random edges
    rng = np.random.default_rng(11)
    n, hub = 3000, 7
    src = list(rng.integers(0, n, 6000))
    dst = list(rng.integers(0, n, 6000))
    lab = list(rng.integers(0, 3, 6000))
    src += list(range(1, 1500)) + [hub] * 1500
    dst += [hub] * 1499 + list(range(1500, 3000))
    lab += [0] * 1499 + [1] * 1500
    g = G.from_triples(n, 3, np.array(src), np.array(dst), np.array(lab))
    gg = rpq.Graph(g)
    og = oracle.Graph(g)
    srcs = rng.integers(0, n, size=100)
    for text in ("(0|1)*", "0 ^0 1*", "(^1|2)* 0", "(0|^0|1|^1|2)*"):
        nfa = R.compile_regex(text, 3)
        for name, fl in STACK_MODES.items():
            print(text, name, flush=True)
            _check(rpq, gg, og, nfa, srcs, fl)


def test_state_counts_and_templates(rpq):
    rng = np.random.default_rng(7)
    w = C.rmat_workload(scale=13, edge_factor=16, num_labels=8, n_per_template=2)
    gg = rpq.Graph(w.graph)
    og = oracle.Graph(w.graph)
    srcs = rng.integers(0, w.graph.num_vertices, size=70)
    for nfa in w.nfas:
        for fl in STACK_MODES.values():
            _check(rpq, gg, og, nfa, srcs, fl)
    for leaves in (1, 4, 7, 12, 20, 31):
        nfa = R.glushkov(R.random_ast(rng, leaves, lambda r: r.integers(0, 8), 0.3), 8)
        for fl in STACK_MODES.values():
            _check(rpq, gg, og, nfa, srcs[:40], fl)


def test_er_and_tiny(rpq):
    w = C.er_workload()
    gg = rpq.Graph(w.graph)
    og = oracle.Graph(w.graph)
    for nfa in w.nfas:
        _check(rpq, gg, og, nfa, w.sources)
    rng = np.random.default_rng(3)
    for _ in range(20):
        g = OC.tiny_graph(rng)
        nfa = R.compile_regex(OC.tiny_expr(rng, g.num_labels), g.num_labels)
        gg, og = rpq.Graph(g), oracle.Graph(g)
        for fl in STACK_MODES.values():
            _check(rpq, gg, og, nfa, list(range(g.num_vertices)) * 2, fl)


def test_grid_batch(rpq):
    side = 40
    g = G.grid(side, 0.0, 0)
    gg = rpq.Graph(g)
    srcs = [0, side * side - 1, 5 * side + 7, 17 * side + 3]
    for fl in STACK_MODES.values():
        bms, st = gg.multi_source(rpq.NFA(R.compile_regex("(0|1)*", 4)), srcs, flags=fl, level_cap=256)
        assert st.levels == 2 * side - 1  # from the corner (0, 0)
        assert len(st.level_us) == st.levels and (st.level_us > 0).all()
        for i, s in enumerate(srcs):
            x0, y0 = s % side, s // side
            want = OC.bitmap_of([y * side + x for y in range(y0, side) for x in range(x0, side)], side * side)
            assert np.array_equal(bms[i], want)


def test_long_chain_batch(rpq):
    # 3000 levels of a path with 64 sources along it: runs of small levels
    # in workgroup 0 (at most 2048 per run) and the grid-wide levels between
    n = 3000
    g = G.from_triples(n, 1, np.arange(n - 1), np.arange(1, n), np.zeros(n - 1, dtype=np.int64))
    gg = rpq.Graph(g)
    og = oracle.Graph(g)
    srcs = list(range(0, 64 * 7, 7))
    nfa = R.compile_regex("0*", 1)
    for name, fl in STACK_MODES.items():
        bms, st = gg.multi_source(rpq.NFA(nfa), srcs, flags=fl, level_cap=4096)
        assert st.levels == n  # from vertex 0 along the whole path
        for i, s in enumerate(srcs):
            assert np.array_equal(bms[i], og.ssr(nfa, s).bitmap), (name, s)


def test_repeat_and_device_output(rpq):
    g = G.rmat(11, 8, 4, 1.1, 2)
    gg = rpq.Graph(g)
    nfa = rpq.NFA(R.compile_regex("0 (1|^2)*", 4))
    srcs = np.arange(0, 300, 3)
    first, _ = gg.multi_source(nfa, srcs)
    for _ in range(3):
        again, _ = gg.multi_source(nfa, srcs)
        assert np.array_equal(again, first)
    out = rpq.DeviceBuffer(8 * len(srcs) * gg.words)
    gg.multi_source(nfa, srcs, out_device_ptr=out.ptr)
    assert np.array_equal(out.to_host().reshape(len(srcs), gg.words), first)
    # single queries into the same device buffer
    for i, s in enumerate(srcs[:5]):
        gg.single_source(nfa, int(s), out_device_ptr=out.ptr + 8 * i * gg.words)
    assert np.array_equal(out.to_host().reshape(len(srcs), gg.words)[:5], first[:5])


@pytest.mark.parametrize("B", [5, 130, 1000])
def test_phase_kernel_handoff(rpq, B):
    # push levels with at least stacked_handoff_edges edges (and V/16) run as
    # separate phase kernels, and the persistent kernel resumes after them:
    # threshold 1 hands off every level of at least V/16 edges. Answers,
    # level counts and |P| against the oracle, for both thresholds, an
    # automaton of more than 8 states, and the allocation-free entry point
    g = G.rmat(12, 8, 6, 1.1, 31)
    gg = rpq.Graph(g)
    og = oracle.Graph(g)
    rng = np.random.default_rng(B)
    srcs = rng.integers(0, g.num_vertices, size=B)
    gg.set_option("max_batch", 1024)
    wide = R.glushkov(R.random_ast(rng, 14, lambda r: r.integers(0, 6), 0.3), 6)
    for thr in (1, 0):
        gg.set_option("stacked_handoff_edges", thr)
        for nfa in (R.compile_regex("(0|^1)* 2 3*", 6), wide):
            for name, fl in STACK_MODES.items():
                print("B", B, "threshold", thr, nfa.text, name, flush=True)
                _check(rpq, gg, og, nfa, srcs, fl)
    gg.set_option("stacked_handoff_edges", 1)
    nfa = R.compile_regex("(0|^1)* 2 3*", 6)
    a, sa = gg.multi_source_noalloc(rpq.NFA(nfa), [int(x) for x in srcs[:256]], level_cap=64)
    for i, s in enumerate(srcs[:256]):
        assert np.array_equal(a[i], og.ssr(nfa, int(s)).bitmap), i
    gg.close()


def test_batched_counters(rpq):
    # the stacked call's work counters with RPQ_COUNTERS follow the batched
    # model, recomputed here from each source's oracle distances: scans over
    # the union of the sources' frontier states, scanned edges, active
    # (level, vertex) pairs, algorithmic bytes (word-granular columns) and
    # word updates; product edges are the oracle's summed over the sources
    g = G.rmat(10, 8, 5, 1.1, 77)
    gg = rpq.Graph(g)
    og = oracle.Graph(g)
    rng = np.random.default_rng(12)
    texts = ["(0|^1)* 2 3*", "0 ^1 (2|4)*", "(0|1|2|3|4)+"]
    nfas = [R.compile_regex(t, 5) for t in texts]
    nfas.append(R.glushkov(R.random_ast(rng, 14, lambda r: r.integers(0, 5), 0.3), 5))  # > 8 states
    for nfa in nfas:
        for B, maxb in ((1, 1024), (40, 1024), (100, 1024), (300, 1024), (300, 128)):
            # a call of more than max_batch sources runs in batches of
            # max_batch, each its own lockstep pass; the counters add up
            gg.set_option("max_batch", maxb)
            srcs = [int(x) for x in rng.integers(0, g.num_vertices, size=B)]
            res = [og.ssr(nfa, s, keep_dist=True) for s in srcs]
            want = np.zeros(5, np.int64)
            for b0 in range(0, B, maxb):
                want += OC.stacked_counters(g, nfa, srcs[b0:b0 + maxb], [r.dist for r in res[b0:b0 + maxb]])
            scans, scanned, active, byt, upd = (int(x) for x in want)
            pe = sum(int(r.product_edges) for r in res)
            for name, fl in STACK_MODES.items():
                # with the phase kernels on every large level (threshold 1)
                # and without (0): the counters add up the same
                for thr in (1, 0):
                    print(nfa.text, B, maxb, name, thr, flush=True)
                    gg.set_option("stacked_handoff_edges", thr)
                    bms, st = gg.multi_source(rpq.NFA(nfa), srcs, flags=fl | rpq.COUNTERS)
                    for i, r in enumerate(res):
                        assert np.array_equal(bms[i], r.bitmap), (nfa.text, B, name, i)
                    got = (st.scans, st.scanned_edges, st.active, st.alg_bytes, st.updates, st.product_edges)
                    assert got == (scans, scanned, active, byt, upd, pe), (nfa.text, B, maxb, name, thr, got)
