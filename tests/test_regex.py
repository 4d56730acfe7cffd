"""The expression front end: parser round trip, and Glushkov automata accept
exactly the words the expression denotes (checked against the third-party
``regex`` matcher on every word up to a length bound)."""
import itertools

import numpy as np
import pytest
import regex as re_mod

from workloads import regex as R
from brute import to_pyregex, sym_char
from nfa_sim import accepts, subset_dfa, thompson

L = 3


def _words(syms, k):
    for n in range(k + 1):
        yield from itertools.product(syms, repeat=n)


def _check_language(text, nfa, k=5):
    node = R.parse(text)
    pat = re_mod.compile(to_pyregex(node, L))
    syms = sorted(set(R.symbol_of(s, L) for s in R.leaves(node))) + [2 * L - 1]
    for w in _words(syms, k):
        want = pat.fullmatch("".join(sym_char(s) for s in w)) is not None
        assert accepts(nfa, w) == want, (text, w)


EXPRS = ["0", "^1", "0*", "0+", "0 1", "0|1", "(0|1)*", "0 ^1 2*", "^0 1*", "(0 1)*",
         "(0|^0)*", "0? 1", "((0 1)|2)+ ^2", "0/1/2", "^^0", "(0*)*", "(0|1)+ 2 (^1)*"]


@pytest.mark.parametrize("text", EXPRS)
def test_glushkov_language(text):
    nfa = R.compile_regex(text, L)
    assert nfa.num_states == len(R.leaves(R.parse(text))) + 1
    _check_language(text, nfa)


@pytest.mark.parametrize("text", EXPRS)
def test_equivalent_constructions(text):
    node = R.parse(text)
    g = R.glushkov(node, L)
    for other in (subset_dfa(g), thompson(node, L)):
        for w in _words(sorted(set(R.symbol_of(s, L) for s in R.leaves(node))), 4):
            assert accepts(g, w) == accepts(other, w)


def test_roundtrip_and_errors():
    rng = np.random.default_rng(7)
    for _ in range(50):
        ast = R.random_ast(rng, int(rng.integers(1, 8)), lambda r: r.integers(0, L), 0.5)
        assert R.parse(R.to_string(ast)) == ast
    for bad in ["", "(", "0|", "^(0 1)", "a", "0)", "*"]:
        with pytest.raises(R.ParseError):
            R.parse(bad)
    with pytest.raises(ValueError):
        R.compile_regex("5", L)


def test_reverse_nfa_language():
    # reversal of Sec. 4: the reversed automaton accepts the reversed word with
    # every symbol inverted
    for text in EXPRS:
        n = R.compile_regex(text, L)
        r = R.reverse_nfa(n)
        syms = sorted(set(R.symbol_of(s, L) for s in R.leaves(R.parse(text))))
        inv = lambda s: s - L if s >= L else s + L
        for w in _words(syms, 4):
            assert accepts(n, w) == accepts(r, tuple(inv(s) for s in reversed(w)))


def test_templates():
    assert R.instantiate("a ^b c*", [5, 17, 3]) == "5 ^17 3*"
    sizes = [R.compile_regex(R.instantiate(t, [0, 1, 2]), 3).num_states for t in R.TEMPLATES]
    assert sizes == [2, 3, 3, 3, 4]
