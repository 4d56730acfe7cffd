"""rpq_multi_source_noalloc through the C ABI against rpq_multi_source (the
same traversal with allocated state): bit-identical answers and equal
statistics on two calls in a row, the second with a smaller input, to host
and to device memory; a call too large for the fixed array fails cleanly and
the next call still works. The answers are also the oracle's."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from workloads import graphs as G
from workloads import regex as R


@pytest.fixture(scope="module")
def rpq():
    from paper_2412_10287_amd import rpq as mod
    return mod


def _both(rpq, gg, og, nfa, srcs, flags):
    nh = rpq.NFA(nfa)
    want, sw = gg.multi_source(nh, srcs, flags=flags | rpq.COUNTERS, level_cap=1024)
    got, sg = gg.multi_source_noalloc(nh, srcs, flags=flags | rpq.COUNTERS, level_cap=1024)
    assert np.array_equal(got, want), (nfa.text, len(srcs), flags)
    for k in ("levels", "push_levels", "pull_levels", "visited_pairs", "product_edges", "scans", "scanned_edges",
              "active", "alg_bytes", "updates", "batch"):
        assert getattr(sg, k) == getattr(sw, k), (k, nfa.text, len(srcs))
    assert np.array_equal(sg.level_counts, sw.level_counts)
    for i, s in enumerate(srcs[:8]):
        assert np.array_equal(got[i], og.ssr(nfa, int(s)).bitmap), (nfa.text, int(s))
    # device output: the answers go straight to the caller's buffer
    out = rpq.DeviceBuffer(8 * len(srcs) * gg.words)
    gg.multi_source_noalloc(nh, srcs, flags=flags, out_device_ptr=out.ptr)
    assert np.array_equal(out.to_host().reshape(len(srcs), gg.words), want)
    out.close()


def test_noalloc_matches_allocating_path(rpq):
    rng = np.random.default_rng(2)
    big = G.rmat(12, 8, 6, 1.1, 41)
    small = G.erdos_renyi(700, 2800, 6, 9)
    nfas = [R.compile_regex("(0|^1)* 2 3*", 6),
            R.glushkov(R.random_ast(rng, 14, lambda r: r.integers(0, 6), 0.3), 6)]  # 15 states
    for round_ in range(2):
        # first call: 4096 vertices, 1000 sources (16 words per row); second:
        # 700 vertices, 70 sources
        for g, B in ((big, 1000), (small, 70)):
            gg, og = rpq.Graph(g), oracle.Graph(g)
            gg.set_option("max_batch", 1024)
            srcs = [int(x) for x in rng.integers(0, g.num_vertices, size=B)]
            for nfa in nfas:
                for fl in (0, 8, 16):
                    print("round", round_, "V", g.num_vertices, "B", B, nfa.text, "flags", fl, flush=True)
                    _both(rpq, gg, og, nfa, srcs, fl)
            gg.close()


def test_noalloc_too_large_fails_cleanly(rpq):
    # 2^19 vertices with 1000 sources (16 words per row) need 400 MB of
    # rows: RPQ_EINVAL before any device work; a call of 3 sources (36 MB)
    # then still works
    n = 1 << 19
    g = G.from_triples(n, 1, np.array([0, 1]), np.array([1, 2]), np.array([0, 0]))
    gg = rpq.Graph(g)
    gg.set_option("max_batch", 1024)
    nh = rpq.NFA(R.compile_regex("0*", 1))
    with pytest.raises(rpq.RPQError) as e:
        gg.multi_source_noalloc(nh, list(range(1000)))
    assert e.value.status == rpq.RPQ_EINVAL and "scratch" in str(e.value)
    bm, st = gg.multi_source_noalloc(nh, [0, 1, 5])
    want, _ = gg.multi_source(nh, [0, 1, 5])
    assert np.array_equal(bm, want)
