"""The C-ABI library loads, exports every function include/rpq.h declares, and
rejects invalid arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "rpq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rpq_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def rpq():
    from paper_2412_10287_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_2412_10287_amd import rpq as mod
    return mod


def test_exports_match_header(rpq):
    decl = _declared()
    assert len(decl) >= 13
    assert sorted(rpq.EXPORTS) == decl
    for name in decl:
        assert hasattr(rpq.lib, name)


def test_nfa_validation(rpq):
    lib = rpq.lib
    h = ctypes.c_void_p()
    sp = np.array([0, 1, 1, 1, 1], dtype=np.int64)
    fr = np.array([0], dtype=np.int32)
    to = np.array([1], dtype=np.int32)
    st = np.array([0], dtype=np.int32)
    fi = np.array([1], dtype=np.int32)
    P = lambda a: ctypes.c_void_p(a.ctypes.data)
    assert lib.rpq_nfa_load(2, 2, P(sp), P(fr), P(to), P(st), 1, P(fi), 1, ctypes.byref(h)) == 0
    assert lib.rpq_nfa_free(h) == 0
    # too many states, bad state ids, decreasing sym_ptr, NULL out
    assert lib.rpq_nfa_load(33, 2, P(sp), P(fr), P(to), P(st), 1, P(fi), 1, ctypes.byref(h)) == rpq.RPQ_EINVAL
    assert "num_states" in rpq.last_error()
    bad = np.array([5], dtype=np.int32)
    assert lib.rpq_nfa_load(2, 2, P(sp), P(fr), P(bad), P(st), 1, P(fi), 1, ctypes.byref(h)) == rpq.RPQ_EINVAL
    assert lib.rpq_nfa_load(2, 2, P(sp), P(fr), P(to), P(bad), 1, P(fi), 1, ctypes.byref(h)) == rpq.RPQ_EINVAL
    dec = np.array([0, 1, 0, 1, 1], dtype=np.int64)
    assert lib.rpq_nfa_load(2, 2, P(dec), P(fr), P(to), P(st), 1, P(fi), 1, ctypes.byref(h)) == rpq.RPQ_EINVAL
    assert lib.rpq_nfa_load(2, 2, P(sp), P(fr), P(to), P(st), 1, P(fi), 1, None) == rpq.RPQ_EINVAL


def test_graph_validation(rpq):
    lib = rpq.lib
    h = ctypes.c_void_p()
    P = lambda a: ctypes.c_void_p(a.ctypes.data)
    lp = np.array([0, 2], dtype=np.int64)
    s = np.array([0, 1], dtype=np.int32)
    d = np.array([1, 5], dtype=np.int32)
    assert lib.rpq_graph_load(3, 1, P(lp), P(s), P(d), ctypes.byref(h)) == rpq.RPQ_EINVAL
    assert "out of range" in rpq.last_error()
    assert lib.rpq_graph_load(0, 1, P(lp), P(s), P(d), ctypes.byref(h)) == rpq.RPQ_EINVAL
    bad = np.array([1, 2], dtype=np.int64)
    assert lib.rpq_graph_load(3, 1, P(bad), P(s), P(d), ctypes.byref(h)) == rpq.RPQ_EINVAL
    assert lib.rpq_bitmap_words(64) == 1 and lib.rpq_bitmap_words(65) == 2


def test_query_argument_checks(rpq):
    lib = rpq.lib
    out = np.zeros(4, dtype=np.uint64)
    assert lib.rpq_single_source(None, None, 0, ctypes.c_void_p(out.ctypes.data), 0, None) == rpq.RPQ_EINVAL
    assert lib.rpq_multi_source(None, None, None, 0, None, 0, None) == rpq.RPQ_EINVAL
    assert lib.rpq_single_destination(None, None, 0, ctypes.c_void_p(out.ctypes.data), 0, None) == rpq.RPQ_EINVAL
    tun = rpq.rpq_tuning()
    assert lib.rpq_autotune(None, 0, None, None, 1, ctypes.byref(tun)) == rpq.RPQ_EINVAL
    t = ctypes.c_uint64()
    assert lib.rpq_submit(None, None, 0, ctypes.byref(t)) == rpq.RPQ_EINVAL
    assert lib.rpq_poll(None, 1, None, 0, None, 0) == rpq.RPQ_EINVAL


def test_tuning_cache_roundtrip(rpq, tmp_path):
    # the persisted-settings layer (no GPU): a stand-in graph records what the
    # tuner is asked and which options are applied
    from paper_2412_10287_amd import autotune

    class FakeGraph:
        def __init__(self):
            self.options, self.tuned = {}, 0

        def signature(self):
            return "V10-L2-E20-R5-5"

        def autotune(self, path, nfas, sources):
            self.tuned += 1
            return {"grid": 64, "alpha": 4, "beta": 24, "best_ms": 1.0, "default_ms": 2.0, "candidates": 22}

        def set_option(self, key, value):
            self.options[key] = value

    cache = str(tmp_path / "tuning.json")
    g1 = FakeGraph()
    r1 = autotune.tune(g1, rpq.TUNE_PLAIN, [], [], cache=cache)
    assert not r1["cached"] and g1.tuned == 1
    g2 = FakeGraph()
    r2 = autotune.tune(g2, rpq.TUNE_PLAIN, [], [], cache=cache)
    assert r2["cached"] and g2.tuned == 0
    assert g2.options == {"persistent_grid": 64, "pull_alpha": 4, "pull_beta": 24}
    g3 = FakeGraph()
    g3.autotune = lambda path, nfas, sources: {"grid": 0, "alpha": 0, "beta": 24, "best_ms": 1.0, "default_ms": 1.5,
                                               "candidates": 22, "handoff_edges": 1 << 22}
    autotune.tune(g3, rpq.TUNE_STACKED, [], [], cache=cache)  # another path: measured again
    assert g3.options == {}
    g4 = FakeGraph()
    r4 = autotune.tune(g4, rpq.TUNE_STACKED, [], [], cache=cache)
    assert r4["cached"] and g4.tuned == 0
    assert g4.options == {"stacked_alpha": 0, "stacked_beta": 24, "stacked_handoff_edges": 1 << 22}
    # the C struct and its ctypes mirror agree on the new field's place
    assert rpq.rpq_tuning.handoff_edges.offset == 48 and ctypes.sizeof(rpq.rpq_tuning) == 56


def test_library_links_roctx(rpq):
    # the named host ranges (one per C-ABI call, per host-driven level, per
    # stacked batch and served step) come from the roctx library
    import shutil
    import subprocess
    if not shutil.which("readelf"):
        pytest.skip("no readelf")
    out = subprocess.run(["readelf", "-d", rpq.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert "librocprofiler-sdk-roctx" in out
