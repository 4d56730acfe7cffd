"""Persistent launches from several graph handles at once: threads query two
handles (plain single-source and stacked multi-source calls, whose grids fill
the GPU and wait at grid barriers) concurrently; the launches of one process
take their workgroups from a per-device budget of co-resident workgroups
(grids that fit together run side by side, the others wait), so none waits
at a barrier for workgroups another grid holds, and every answer is the
oracle's."""
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from workloads import configs as C


@pytest.fixture(scope="module")
def rpq():
    from paper_2412_10287_amd import rpq as mod
    return mod


def test_two_handles_concurrent(rpq):
    wa = C.rmat_workload(scale=14, edge_factor=16, num_labels=8, n_per_template=2)
    wb = C.er_workload()
    work = []
    for w in (wa, wb):
        og = oracle.Graph(w.graph)
        want = [og.ssr(n, int(s)).bitmap for n, s in zip(w.nfas, w.sources)]
        work.append((w, rpq.Graph(w.graph), want))
    errors = []

    def plain(w, gg, want, rounds):
        try:
            hs = [rpq.NFA(n) for n in w.nfas]
            for _ in range(rounds):
                for h, s, b in zip(hs, w.sources, want):
                    bm, _ = gg.single_source(h, int(s))
                    if not np.array_equal(bm, b):
                        errors.append(("plain", w.name, int(s)))
        except Exception as e:  # reported below
            errors.append(repr(e))

    def stacked(w, gg, want, rounds):
        try:
            h = rpq.NFA(w.nfas[0])
            srcs = [int(w.sources[0])] * 3 + [int(s) for s in w.sources[1:]]
            for _ in range(rounds):
                bms, _ = gg.multi_source(h, [int(w.sources[0])] * 3)
                for b in bms:
                    if not np.array_equal(b, want[0]):
                        errors.append(("stacked", w.name))
                gg.multi_source(h, srcs)
        except Exception as e:
            errors.append(repr(e))

    ths = []
    for w, gg, want in work:
        ths.append(threading.Thread(target=plain, args=(w, gg, want, 4)))
        ths.append(threading.Thread(target=stacked, args=(w, gg, want, 6)))
    for t in ths:
        t.start()
    for t in ths:
        t.join(timeout=240)
        assert not t.is_alive()
    assert not errors, errors[:5]
