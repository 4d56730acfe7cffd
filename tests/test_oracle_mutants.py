"""The oracle's pins catch plausible mistakes.

Each case copies ``oracle.c``, plants one mistake by a textual replacement
(a dropped inverse rule, a transposed operand, a wrong target state, Alg. 1's
empty initial visited set taken literally, a wrong label range, start states
read as final ones, and in the work counters: successors counted per group
of states, a wrong state-word width, scans only where neighbours exist),
builds the copy with gcc into a temporary directory, and runs the CPU pins
against it. Every mutant must fail at least one pin. The real
oracle is never modified."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import oracle_cases as OC
from test_oracle import _read_golden
from workloads import graphs as G
from workloads import regex as R

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "no-inverse": ("int inv = s >= nfa_nl;\n            int32_t l = inv ? s - nfa_nl : s;",
                   "int inv = 0;\n            int32_t l = s >= nfa_nl ? s - nfa_nl : s;"),
    "transposed-inverse": ("const int32_t *nb = inv ? g->in_nbr : g->out_nbr;",
                           "const int32_t *nb = inv ? g->out_nbr : g->in_nbr;"),
    "stay-in-state": ("int32_t q2 = ttgt[t];", "int32_t q2 = q;"),
    "literal-empty-visited": ("if (dist[(int64_t)fin[i] * nv + v] >= 0)",
                              "if (dist[(int64_t)fin[i] * nv + v] > 0)"),
    "label-range-off-by-one": ("if (lb[mid] <= l) x = mid + 1;", "if (lb[mid] <= l + 1) x = mid + 1;"),
    "start-as-final": ("if (dist[(int64_t)fin[i] * nv + v] >= 0)",
                       "if (dist[(int64_t)start[i % nstart] * nv + v] >= 0)"),
    "first-neighbour-only": ("for (int64_t k = lo; k < hi; k++) {\n                int64_t c2",
                             "for (int64_t k = lo; k < hi && k < lo + 1; k++) {\n                int64_t c2"),
    # work counters: successors counted once per group of states instead of
    # once per state; a 4-byte state word whatever the automaton's size; a
    # scan counted only where the vertex has neighbours
    "counter-per-group-successors": (
        "prod_edges += (int64_t)__builtin_popcountll(succ[(int64_t)u * nq + q]) * deg;\n",
        "\n"),
    "counter-word-width": ("bytes += 8 + (4 + word_bytes) * deg;", "bytes += 8 + (4 + 4) * deg;"),
    "counter-scan-needs-neighbours": ("if (img) {\n                        scans++;",
                                      "if (img && deg) {\n                        scans++;"),
}
# the per-group mutant also counts the group's image once per scan
_PG_OLD = "if (img) {\n                        scans++;"
_PG_NEW = "if (img) {\n                        prod_edges += (int64_t)__builtin_popcountll(img) * deg;\n" \
          "                        scans++;"


def _build_mutant(name, tmp):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, name
    if name == "counter-per-group-successors":
        assert text.count(_PG_OLD) == 1
        text = text.replace(_PG_OLD, _PG_NEW)
    path_c = os.path.join(tmp, name + ".c")
    path_so = os.path.join(tmp, name + ".so")
    open(path_c, "w").write(text.replace(old, new))
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", path_c, "-o", path_so],
                   check=True)
    return oracle.load_library(path_so)


def _pins(lib):
    def fn(g, nfa, src):
        r = oracle.ssr(g, nfa, src, keep_dist=True, lib=lib)
        return r.bitmap, r.dist, r.levels

    rng = np.random.default_rng(1)
    for c in _read_golden(os.path.join(os.path.dirname(__file__), "golden", "handworked.txt")):
        g = G.from_triples(c["V"], c["L"], *zip(*c["edges"]), dedupe=False)
        r = oracle.ssr(g, R.compile_regex(c["query"], c["L"]), c["source"], lib=lib)
        assert r.vertices().tolist() == c["expect"]
    OC.check_brute(fn, rng, n_cases=40)
    OC.check_special(fn, rng, G.erdos_renyi(500, 1500, 4, 3))
    OC.check_grid(fn, 12, rng, n=3)

    def ctr(g, nfa, src):
        r = oracle.ssr(g, nfa, src, lib=lib)
        return r.product_edges, r.scans, r.scanned_edges, r.alg_bytes, r.active, r.level_counts

    OC.check_counters_product(ctr, rng, n_cases=40)
    OC.check_counters_star(ctr, rng, G.erdos_renyi(500, 1500, 4, 3))
    OC.check_counters_grid(ctr, 9, rng, n=2)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(name, tmp)
        with pytest.raises(AssertionError):
            _pins(lib)


def test_unmutated_copy_passes():
    with tempfile.TemporaryDirectory() as tmp:
        path_so = os.path.join(tmp, "same.so")
        subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", SRC, "-o", path_so],
                       check=True)
        _pins(oracle.load_library(path_so))
