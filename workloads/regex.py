"""Regular expressions over labels and inverse labels, and their compilation to
epsilon-free NFAs.

This is the query front end, not part of the traversal method: the method takes
an NFA (Sec. 2, Def. 2.4: states, transitions carrying symbols of the two-way
alphabet, start set, final set). The paper compiles its queries to minimized
DFAs (Sec. 5.2); results depend only on the accepted language, so any
epsilon-free NFA serves. Here Glushkov's position automaton is used: one state
per label occurrence plus an initial state, every transition into a position
carrying that position's symbol.

Symbol encoding shared by every consumer: with ``num_labels`` = L, symbol
``s < L`` is the forward label ``s`` and ``s >= L`` is the inverse of label
``s - L`` (Sec. 2: the inverse alphabet, with ``(a^-)^- = a``).

Grammar (whitespace or '/' concatenates; '^' inverts one label)::

    alt  := cat ('|' cat)*
    cat  := post (('/' | ' ') post)*
    post := atom ('*' | '+' | '?')*
    atom := LABEL | '^' LABEL | '(' alt ')'
    LABEL := decimal label id
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple, Union

import numpy as np


# --------------------------------------------------------------------------- AST
@dataclass(frozen=True)
class Sym:
    label: int
    inv: bool = False


@dataclass(frozen=True)
class Cat:
    left: "Node"
    right: "Node"


@dataclass(frozen=True)
class Alt:
    left: "Node"
    right: "Node"


@dataclass(frozen=True)
class Star:
    child: "Node"


@dataclass(frozen=True)
class Plus:
    child: "Node"


@dataclass(frozen=True)
class Opt:
    child: "Node"


Node = Union[Sym, Cat, Alt, Star, Plus, Opt]


def to_string(n: Node) -> str:
    """Fully parenthesised text form that ``parse`` reads back."""
    if isinstance(n, Sym):
        return ("^" if n.inv else "") + str(n.label)
    if isinstance(n, Cat):
        return "(" + to_string(n.left) + " " + to_string(n.right) + ")"
    if isinstance(n, Alt):
        return "(" + to_string(n.left) + "|" + to_string(n.right) + ")"
    if isinstance(n, Star):
        return "(" + to_string(n.child) + ")*"
    if isinstance(n, Plus):
        return "(" + to_string(n.child) + ")+"
    if isinstance(n, Opt):
        return "(" + to_string(n.child) + ")?"
    raise TypeError(n)


def leaves(n: Node) -> List[Sym]:
    if isinstance(n, Sym):
        return [n]
    if isinstance(n, (Cat, Alt)):
        return leaves(n.left) + leaves(n.right)
    return leaves(n.child)


def symbol_of(s: Sym, num_labels: int) -> int:
    return s.label + (num_labels if s.inv else 0)


# ------------------------------------------------------------------------ parser
class ParseError(ValueError):
    pass


def parse(text: str) -> Node:
    toks = _tokenize(text)
    pos = [0]

    def peek() -> Optional[str]:
        return toks[pos[0]] if pos[0] < len(toks) else None

    def take() -> str:
        t = peek()
        if t is None:
            raise ParseError("unexpected end of expression: %r" % text)
        pos[0] += 1
        return t

    def p_alt() -> Node:
        n = p_cat()
        while peek() == "|":
            take()
            n = Alt(n, p_cat())
        return n

    def p_cat() -> Node:
        n = p_post()
        while True:
            t = peek()
            if t == "/":
                take()
                n = Cat(n, p_post())
            elif t is not None and (t == "(" or t == "^" or t.isdigit()):
                n = Cat(n, p_post())
            else:
                return n

    def p_post() -> Node:
        n = p_atom()
        while peek() in ("*", "+", "?"):
            op = take()
            n = Star(n) if op == "*" else Plus(n) if op == "+" else Opt(n)
        return n

    def p_atom() -> Node:
        t = take()
        if t == "(":
            n = p_alt()
            if take() != ")":
                raise ParseError("missing ')' in %r" % text)
            return n
        if t == "^":
            inv = True
            while peek() == "^":  # (a^-)^- = a
                take()
                inv = not inv
            t = take()
            if not t.isdigit():
                raise ParseError("'^' must precede a label in %r" % text)
            return Sym(int(t), inv)
        if t.isdigit():
            return Sym(int(t), False)
        raise ParseError("unexpected token %r in %r" % (t, text))

    n = p_alt()
    if peek() is not None:
        raise ParseError("trailing input %r in %r" % (peek(), text))
    return n


def _tokenize(text: str) -> List[str]:
    out: List[str] = []
    i = 0
    while i < len(text):
        c = text[i]
        if c.isspace():
            i += 1
            continue
        if c.isdigit():
            j = i
            while j < len(text) and text[j].isdigit():
                j += 1
            out.append(text[i:j])
            i = j
            continue
        if c in "|/*+?()^":
            out.append(c)
            i += 1
            continue
        raise ParseError("bad character %r in %r" % (c, text))
    if not out:
        raise ParseError("empty expression")
    return out


# ----------------------------------------------------------------------- NFA
@dataclass
class NFA:
    """Epsilon-free NFA in per-symbol COO form.

    Transitions of symbol ``s`` are ``(frm[i] -> to[i])`` for
    ``i in [sym_ptr[s], sym_ptr[s+1])``: the per-symbol Boolean transition
    matrices of Sec. 3 in coordinate form. ``sym_ptr`` has ``2*num_labels+1``
    entries (forward symbols first, then inverse symbols).
    """

    num_states: int
    num_labels: int
    sym_ptr: np.ndarray  # int64, 2L+1
    frm: np.ndarray  # int32
    to: np.ndarray  # int32
    start: np.ndarray  # int32
    final: np.ndarray  # int32
    text: str = ""

    def triples(self) -> List[Tuple[int, int, int]]:
        out = []
        for s in range(2 * self.num_labels):
            for i in range(int(self.sym_ptr[s]), int(self.sym_ptr[s + 1])):
                out.append((int(self.frm[i]), s, int(self.to[i])))
        return out


def nfa_from_triples(num_states: int, num_labels: int,
                     triples: Sequence[Tuple[int, int, int]],
                     start: Sequence[int], final: Sequence[int],
                     text: str = "") -> NFA:
    """Build the per-symbol COO form from ``(from, symbol, to)`` triples."""
    nsym = 2 * num_labels
    tr = sorted(set((int(s), int(a), int(b)) for a, s, b in triples))
    for s, a, b in tr:
        if not (0 <= s < nsym and 0 <= a < num_states and 0 <= b < num_states):
            raise ValueError("transition out of range: %r" % ((a, s, b),))
    counts = np.zeros(nsym + 1, dtype=np.int64)
    for s, _, _ in tr:
        counts[s + 1] += 1
    sym_ptr = np.cumsum(counts).astype(np.int64)
    frm = np.array([a for _, a, _ in tr], dtype=np.int32)
    to = np.array([b for _, _, b in tr], dtype=np.int32)
    return NFA(num_states, num_labels, sym_ptr, frm, to,
               np.array(sorted(set(start)), dtype=np.int32),
               np.array(sorted(set(final)), dtype=np.int32), text)


def glushkov(node: Node, num_labels: int, text: str = "") -> NFA:
    """Glushkov (position) automaton of ``node``.

    State 0 is initial; state i >= 1 is the i-th label occurrence (left to
    right). Transitions: 0 -> p for p in First, p -> p' for p' in Follow(p),
    each labelled with the symbol of the target position. Finals: Last, plus 0
    when the empty word is accepted.
    """
    syms: List[int] = []

    def number(n: Node):
        # returns (nullable, first, last) over position ids; fills follow
        if isinstance(n, Sym):
            if n.label >= num_labels or n.label < 0:
                raise ValueError("label %d outside [0,%d)" % (n.label, num_labels))
            syms.append(symbol_of(n, num_labels))
            p = len(syms)
            follow[p] = set()
            return False, {p}, {p}
        if isinstance(n, Cat):
            n1, f1, l1 = number(n.left)
            n2, f2, l2 = number(n.right)
            for p in l1:
                follow[p] |= f2
            return (n1 and n2, f1 | f2 if n1 else set(f1), l1 | l2 if n2 else set(l2))
        if isinstance(n, Alt):
            n1, f1, l1 = number(n.left)
            n2, f2, l2 = number(n.right)
            return n1 or n2, f1 | f2, l1 | l2
        if isinstance(n, (Star, Plus)):
            n1, f1, l1 = number(n.child)
            for p in l1:
                follow[p] |= f1
            return (True if isinstance(n, Star) else n1), f1, l1
        if isinstance(n, Opt):
            n1, f1, l1 = number(n.child)
            return True, f1, l1
        raise TypeError(n)

    follow: dict = {}
    nullable, first, last = number(node)
    triples = [(0, syms[p - 1], p) for p in first]
    for p, fs in follow.items():
        for p2 in fs:
            triples.append((p, syms[p2 - 1], p2))
    finals = set(last) | ({0} if nullable else set())
    return nfa_from_triples(len(syms) + 1, num_labels, triples, [0], sorted(finals),
                            text or to_string(node))


def compile_regex(text: str, num_labels: int) -> NFA:
    return glushkov(parse(text), num_labels, text)


def reverse_nfa(n: NFA) -> NFA:
    """The reversed two-way automaton of Sec. 4 (single-destination by reversal):
    every transition is turned around and its symbol inverted, start and final
    sets swap. It accepts the reversed, inverted language."""
    L = n.num_labels
    tr = []
    for a, s, b in n.triples():
        inv = s - L if s >= L else s + L
        tr.append((b, inv, a))
    return nfa_from_triples(n.num_states, L, tr, n.final.tolist(), n.start.tolist(),
                            "rev(" + n.text + ")")


# ----------------------------------------------------------- random expressions
def random_ast(rng: np.random.Generator, n_leaves: int, pick_label, p_inv: float,
               ops=("cat", "alt"), p_unary: float = 0.35,
               unary=("star", "plus")) -> Node:
    """Random expression with exactly ``n_leaves`` label occurrences.

    ``pick_label(rng)`` draws a label id; each leaf is inverted with
    probability ``p_inv``; every node is wrapped in a Kleene star / plus with
    probability ``p_unary``.
    """
    def build(k: int) -> Node:
        if k == 1:
            n: Node = Sym(int(pick_label(rng)), bool(rng.random() < p_inv))
        else:
            k1 = int(rng.integers(1, k))
            op = ops[int(rng.integers(0, len(ops)))]
            a, b = build(k1), build(k - k1)
            n = Cat(a, b) if op == "cat" else Alt(a, b)
        if rng.random() < p_unary:
            u = unary[int(rng.integers(0, len(unary)))]
            n = Star(n) if u == "star" else Plus(n)
        return n

    return build(n_leaves)


# The five query templates of the plain single-query workload; letters are
# distinct labels filled in per query.
TEMPLATES = ("a*", "a b*", "(a|b)+", "^a b*", "a ^b c*")


def instantiate(template: str, labels: Sequence[int]) -> str:
    out = template
    for ch, lab in zip("abc", labels):
        out = out.replace(ch, str(int(lab)))
    return out


def template_arity(template: str) -> int:
    return sum(1 for ch in "abc" if ch in template)
