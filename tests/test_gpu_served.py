"""GPU parity of the served path (rpq_submit / rpq_poll) and rpq_multi_source:
every result equals the oracle's bit for bit, and the same query gives the same
bitmap alone and inside a mix of concurrently admitted queries."""
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from workloads import configs as C
from workloads import graphs as G
from workloads import regex as R


@pytest.fixture(scope="module")
def rpq():
    from paper_2412_10287_amd import rpq as mod
    return mod


def _submit_all(gg, nfas, sources):
    return [gg.submit(n, int(s)) for n, s in zip(nfas, sources)]


def _poll_all(gg, tickets):
    out = []
    for t in tickets:
        r = gg.poll(t, timeout_us=-1)
        assert r is not None
        out.append(r)
    return out


def test_served_er_vs_oracle_and_alone(rpq):
    w = C.er_workload()
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    nh = [rpq.NFA(n) for n in w.nfas]
    want = [og.ssr(n, int(s)) for n, s in zip(w.nfas, w.sources)]
    mixed = _poll_all(gg, _submit_all(gg, nh, w.sources))
    for (bm, st), wr, text in zip(mixed, want, w.queries):
        assert np.array_equal(bm, wr.bitmap), text
        assert st.levels == wr.levels, text
        assert st.visited_pairs == int(wr.level_counts.sum()), text
    # alone = in the mix
    for h, s, (bm_mix, _) in zip(nh, w.sources, mixed):
        bm, _ = _poll_all(gg, [gg.submit(h, int(s))])[0]
        assert np.array_equal(bm, bm_mix)


def test_served_rmat_templates_small_slots(rpq):
    w = C.rmat_workload(scale=14, edge_factor=16, num_labels=16, n_per_template=8)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    gg.set_option("max_slots", 3)  # most requests wait for a free slot
    nh = [rpq.NFA(n) for n in w.nfas]
    res = _poll_all(gg, _submit_all(gg, nh, w.sources))
    for (bm, st), n, s, text in zip(res, w.nfas, w.sources, w.queries):
        r = og.ssr(n, int(s))
        assert np.array_equal(bm, r.bitmap), text
        assert st.levels == r.levels, text


def test_served_mixed_state_counts(rpq):
    # NFAs from 1 to 32 states in one mix (state words of 1, 2 and 4 bytes on
    # the plain path; 4-byte words in the served engine)
    rng = np.random.default_rng(12)
    g = G.rmat(12, 8, 6, 1.1, 5)
    og = oracle.Graph(g)
    gg = rpq.Graph(g)
    nfas, srcs = [], []
    for leaves in (1, 2, 3, 5, 8, 12, 15, 20, 26, 31):
        ast = R.random_ast(rng, leaves, lambda r: r.integers(0, 6), 0.3)
        nfas.append(R.glushkov(ast, 6))
        srcs.append(int(rng.integers(0, g.num_vertices)))
    nh = [rpq.NFA(n) for n in nfas]
    res = _poll_all(gg, _submit_all(gg, nh, srcs))
    for (bm, st), n, s in zip(res, nfas, srcs):
        assert np.array_equal(bm, og.ssr(n, s).bitmap)
        plain, _ = gg.single_source(rpq.NFA(n), s)
        assert np.array_equal(bm, plain)


def test_multi_source_equals_single(rpq):
    g = G.rmat(13, 8, 4, 1.1, 8)
    gg = rpq.Graph(g)
    og = oracle.Graph(g)
    nfa = R.compile_regex("(0|^1)* 2", 4)
    nh = rpq.NFA(nfa)
    srcs = np.random.default_rng(3).integers(0, g.num_vertices, size=40)
    srcs[5] = srcs[6]  # repeated source
    bms, st = gg.multi_source(nh, srcs)
    assert st.batch == 40
    for i, s in enumerate(srcs):
        assert np.array_equal(bms[i], og.ssr(nfa, int(s)).bitmap)


def test_concurrent_submitters(rpq):
    w = C.er_workload(n=3000, m=12000, num_labels=4, n_queries=24)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    nh = [rpq.NFA(n) for n in w.nfas]
    results = {}

    def worker(k):
        for i in range(k, len(nh), 3):
            t = gg.submit(nh[i], int(w.sources[i]))
            results[i] = gg.poll(t, timeout_us=-1)

    ths = [threading.Thread(target=worker, args=(k,)) for k in range(3)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    for i, (n, s) in enumerate(zip(w.nfas, w.sources)):
        assert np.array_equal(results[i][0], og.ssr(n, int(s)).bitmap)


def test_poll_semantics(rpq):
    g = G.erdos_renyi(500, 2000, 2, 1)
    gg = rpq.Graph(g)
    nh = rpq.NFA(R.compile_regex("(0|1)*", 2))
    t = gg.submit(nh, 0)
    r = gg.poll(t, timeout_us=-1)
    assert r is not None
    with pytest.raises(rpq.RPQError) as e:
        gg.poll(t, timeout_us=0)  # retired
    assert e.value.status == rpq.RPQ_ENOTFOUND
    empty = rpq.NFA(R.nfa_from_triples(2, 2, [(0, 0, 1)], [], [1]))
    bm, _ = gg.poll(gg.submit(empty, 3), timeout_us=-1)
    assert not bm.any()
    with pytest.raises(rpq.RPQError):
        gg.submit(nh, 500)


def test_result_pool_backpressure_and_device_output(rpq):
    # two slots give four result-pool entries: twelve queries submitted before
    # any poll must wait for entries and slots, then every answer arrives, in
    # any poll order, to host or device memory
    w = C.er_workload(n=2000, m=9000, num_labels=4, n_queries=12)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    gg.set_option("max_slots", 2)
    nh = [rpq.NFA(n) for n in w.nfas]
    tickets = [gg.submit(h, int(s)) for h, s in zip(nh, w.sources)]
    out = rpq.DeviceBuffer(8 * gg.words)
    for i in reversed(range(len(tickets))):
        want = og.ssr(w.nfas[i], int(w.sources[i])).bitmap
        if i % 2:
            r = gg.poll(tickets[i], timeout_us=30_000_000)
            assert r is not None, i  # a stalled scheduler times out instead of hanging
            bm = r[0]
        else:
            r = gg.poll(tickets[i], timeout_us=30_000_000, out_device_ptr=out.ptr)
            assert r is not None, i
            bm = out.to_host()
        assert np.array_equal(bm, want), i


def test_large_query_cap(rpq):
    # every finished query counts as large (threshold 0), so after the first
    # finishes at most two run at once; answers are unchanged and all arrive
    w = C.rmat_workload(scale=13, edge_factor=16, num_labels=8, n_per_template=6)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    gg.set_option("large_query_pairs", 0)
    gg.set_option("large_query_slots", 2)
    gg.set_option("serve_promote_pairs", 0)  # the large-period cap, not promotion
    assert gg.get_option("large_query_slots") == 2
    nh = [rpq.NFA(n) for n in w.nfas]
    for rnd in range(2):
        res = _poll_all(gg, _submit_all(gg, nh, w.sources))
        for (bm, st), n, s, text in zip(res, w.nfas, w.sources, w.queries):
            r = og.ssr(n, int(s))
            assert np.array_equal(bm, r.bitmap), (rnd, text)
            assert st.levels == r.levels, (rnd, text)
        if rnd == 1:
            assert max(st.batch for _, st in res) <= 2


def test_same_nfa_requests_run_as_stacked_groups(rpq):
    # 80 requests of one NFA handle, submitted together with a few others:
    # waiting requests of one NFA run as stacked groups (serve_stack_min 16),
    # the rest through the slots; every answer equals the oracle's
    w = C.rmat_workload(scale=13, edge_factor=16, num_labels=8, n_per_template=2)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    gg.set_option("serve_stack_min", 16)
    gg.set_option("max_batch", 64)
    gg.set_option("max_slots", 2)  # most requests wait, so groups form
    assert gg.get_option("serve_stack_min") == 16
    shared = rpq.NFA(w.nfas[1])
    others = [rpq.NFA(n) for n in w.nfas]
    srcs = np.random.default_rng(8).integers(0, w.graph.num_vertices, size=80)
    tickets = [(gg.submit(o, int(s)), n, int(s)) for o, n, s in zip(others, w.nfas, w.sources)]
    tickets += [(gg.submit(shared, int(s)), w.nfas[1], int(s)) for s in srcs]
    grouped = 0
    for t, n, s in reversed(tickets):
        bm, st = gg.poll(t, timeout_us=60_000_000)
        assert np.array_equal(bm, og.ssr(n, s).bitmap), s
        grouped += st.batch > 2
    print("answers from stacked groups:", grouped)
    assert grouped > 0


def test_burst_gathers_into_one_group(rpq):
    # a burst of one NFA's requests waits for the rest of the burst (the
    # serve_group_wait_us window, here long enough for Python's submits) and
    # runs as one stacked group of max_batch; with the window off the slots
    # may take the first requests; every answer equals the oracle's
    w = C.rmat_workload(scale=13, edge_factor=16, num_labels=8, n_per_template=1)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    for bad in (-1, 1_000_001):
        with pytest.raises(rpq.RPQError) as e:
            gg.set_option("serve_group_wait_us", bad)
        assert e.value.status == rpq.RPQ_EINVAL
    gg.set_option("serve_group_wait_us", 200_000)
    assert gg.get_option("serve_group_wait_us") == 200_000
    gg.set_option("max_batch", 64)
    nh = rpq.NFA(w.nfas[0])
    srcs = [int(x) for x in np.random.default_rng(12).integers(0, w.graph.num_vertices, size=64)]
    for window in (200_000, 0):
        gg.set_option("serve_group_wait_us", window)
        tickets = [(gg.submit(nh, s), s) for s in srcs]
        batches = []
        for t, s in tickets:
            bm, st = gg.poll(t, timeout_us=60_000_000)
            assert np.array_equal(bm, og.ssr(w.nfas[0], s).bitmap), (window, s)
            batches.append(st.batch)
        print("window", window, "batches", sorted(set(batches)), flush=True)
        if window:
            assert all(b == 64 for b in batches)


@pytest.mark.parametrize("lanes", [0, 2, 3])
def test_large_queries_run_alone(rpq, lanes):
    # threshold 0: after the first answer every query counts as large, and
    # with large_query_slots 0 the rest run through the single-query kernel:
    # one at a time in the scheduler thread (lanes 0), or on `lanes`
    # executors side by side, each with its own state (three lanes share
    # the co-resident workgroups); answers and level counts are unchanged
    w = C.rmat_workload(scale=13, edge_factor=16, num_labels=8, n_per_template=4)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    gg.set_option("large_query_pairs", 0)
    gg.set_option("large_query_slots", 0)
    gg.set_option("serve_lanes", lanes)
    gg.set_option("serve_promote_pairs", 0)  # large periods, not promotion
    nh = [rpq.NFA(n) for n in w.nfas]
    for rnd in range(2):
        res = _poll_all(gg, _submit_all(gg, nh, w.sources))
        for (bm, st), n, s, text in zip(res, w.nfas, w.sources, w.queries):
            r = og.ssr(n, int(s))
            assert np.array_equal(bm, r.bitmap), (rnd, text)
            assert st.levels == r.levels and st.visited_pairs == int(r.level_counts.sum()), (rnd, text)
        if rnd == 1:
            assert all(st.batch == 1 for _, st in res)
    assert gg.info("serve_lanes") == lanes
    gg.close()


def test_lanes_with_plain_calls_and_pull(rpq):
    # every served query moves from its slot to a lane after its first level
    # (promotion threshold 1 pair) while the same handle answers plain calls
    # from another thread (up to three persistent grids wanting the GPU),
    # with the pull direction on
    w = C.rmat_workload(scale=14, edge_factor=16, num_labels=8, n_per_template=3)
    og = oracle.Graph(w.graph)
    want = [og.ssr(n, int(s)).bitmap for n, s in zip(w.nfas, w.sources)]
    gg = rpq.Graph(w.graph)
    gg.set_option("serve_promote_pairs", 1)
    gg.set_option("serve_lanes", 2)
    gg.set_option("pull_alpha", 2)
    nh = [rpq.NFA(n) for n in w.nfas]
    errors = []

    def plain():
        try:
            for _ in range(3):
                for h, s, b in zip(nh, w.sources, want):
                    bm, _ = gg.single_source(h, int(s))
                    if not np.array_equal(bm, b):
                        errors.append(("plain", int(s)))
        except Exception as e:  # reported below
            errors.append(repr(e))

    th = threading.Thread(target=plain)
    th.start()
    for rnd in range(3):
        res = _poll_all(gg, _submit_all(gg, nh, w.sources))
        for i, (bm, _) in enumerate(res):
            if not np.array_equal(bm, want[i]):
                errors.append(("served", rnd, i))
    th.join(timeout=240)
    assert not th.is_alive()
    assert not errors, errors[:5]
    gg.close()


def test_memory_budget_admission(rpq):
    # budgets that hold one or two slots (each slot costs about 144 KB of
    # state and query constants on this 3000-vertex graph, plus about 88 KB
    # shared): the engine admits that many queries at once, the rest wait in
    # the queue, and every answer is the oracle's; a budget below one slot
    # fails every ticket with RPQ_ENOMEM and the handle can still be freed
    w = C.er_workload(n=3000, m=12000, num_labels=4, n_queries=24)
    og = oracle.Graph(w.graph)
    want = [og.ssr(n, int(s)).bitmap for n, s in zip(w.nfas, w.sources)]
    for budget, lo, hi in ((500 << 10, 1, 2), (300 << 10, 1, 1)):
        gg = rpq.Graph(w.graph)
        gg.set_option("serve_stack_min", 0)
        gg.set_option("mem_budget", budget)
        nh = [rpq.NFA(n) for n in w.nfas]
        tickets = [gg.submit(h, int(s)) for h, s in zip(nh, w.sources)]
        got = [gg.poll(t, timeout_us=30_000_000) for t in tickets]
        slots = gg.info("serve_slots")
        print("budget", budget, "slots", slots, flush=True)
        assert lo <= slots <= hi, (budget, slots)
        for i, r in enumerate(got):
            assert r is not None and np.array_equal(r[0], want[i]), (budget, i)
        gg.close()
    gg = rpq.Graph(w.graph)
    gg.set_option("mem_budget", 200 << 10)
    nh = rpq.NFA(w.nfas[0])
    # the engine starts with the first submit; its failure reaches that
    # ticket's poll, or the submit itself when the engine failed first
    with pytest.raises(rpq.RPQError) as e:
        t = gg.submit(nh, int(w.sources[0]))
        gg.poll(t, timeout_us=30_000_000)
    assert e.value.status in (rpq.RPQ_ENOMEM, rpq.RPQ_EDEVICE) and "budget" in str(e.value)
    gg.close()


def test_submit_deadline(rpq):
    # one slot, so requests queue behind each other: with a 1 us deadline to
    # start, queued requests are dropped (RPQ_ETIMEDOUT, ticket retired) and
    # the ones that started return the oracle's answer; with a long deadline
    # every request completes
    w = C.rmat_workload(scale=14, edge_factor=16, num_labels=8, n_per_template=4)
    og = oracle.Graph(w.graph)
    want = [og.ssr(n, int(s)).bitmap for n, s in zip(w.nfas, w.sources)]
    gg = rpq.Graph(w.graph)
    gg.set_option("max_slots", 1)
    gg.set_option("serve_stack_min", 0)
    nh = [rpq.NFA(n) for n in w.nfas]
    tickets = [gg.submit(h, int(s), deadline_us=1) for h, s in zip(nh, w.sources)]
    expired = done = 0
    for i, t in enumerate(tickets):
        try:
            r = gg.poll(t, timeout_us=30_000_000)
        except rpq.RPQError as e:
            assert e.status == rpq.RPQ_ETIMEDOUT and "deadline" in str(e), str(e)
            expired += 1
            with pytest.raises(rpq.RPQError) as e2:
                gg.poll(t, timeout_us=0)
            assert e2.value.status == rpq.RPQ_ENOTFOUND
            continue
        assert r is not None and np.array_equal(r[0], want[i]), i
        done += 1
    print("expired", expired, "done", done)
    assert expired >= 1 and expired + done == len(tickets)
    tickets = [gg.submit(h, int(s), deadline_us=60_000_000) for h, s in zip(nh, w.sources)]
    for i, t in enumerate(tickets):
        r = gg.poll(t, timeout_us=60_000_000)
        assert r is not None and np.array_equal(r[0], want[i]), i
    gg.close()


@pytest.mark.parametrize("threshold", [1, 2000, 0])
def test_promotion_to_lanes(rpq, threshold):
    # a slot query whose reached pairs pass serve_promote_pairs moves to a
    # lane and starts over there; answers, level counts and |P| stay the
    # oracle's, and promoted answers carry batch 1 (threshold 0: never)
    w = C.rmat_workload(scale=13, edge_factor=16, num_labels=8, n_per_template=4)
    og = oracle.Graph(w.graph)
    gg = rpq.Graph(w.graph)
    gg.set_option("serve_promote_pairs", threshold)
    gg.set_option("serve_stack_min", 0)
    nh = [rpq.NFA(n) for n in w.nfas]
    for rnd in range(2):
        res = _poll_all(gg, _submit_all(gg, nh, w.sources))
        alone = 0
        for (bm, st), n, s, text in zip(res, w.nfas, w.sources, w.queries):
            r = og.ssr(n, int(s))
            assert np.array_equal(bm, r.bitmap), (threshold, rnd, text)
            assert st.levels == r.levels and st.visited_pairs == int(r.level_counts.sum()), (threshold, text)
            alone += st.batch == 1
        print("threshold", threshold, "round", rnd, "promoted", alone, "of", len(res))
        if threshold == 1:
            assert alone >= len(res) // 2
    assert gg.info("serve_lanes") == (2 if threshold else 0)
    gg.close()
