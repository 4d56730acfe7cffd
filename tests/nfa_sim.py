"""Test helpers over NFAs in per-symbol COO form: word acceptance by state-set
simulation, subset construction, Thompson construction with epsilon closure.
Used only to check the expression compiler and the language-equivalence
invariant; never by the oracle or the GPU path."""
from __future__ import annotations

from typing import Dict, FrozenSet, List, Tuple

from workloads import regex as R


def accepts(nfa: R.NFA, word) -> bool:
    cur = set(int(q) for q in nfa.start)
    tr = nfa.triples()
    for s in word:
        cur = {b for (a, sym, b) in tr if sym == s and a in cur}
        if not cur:
            return False
    return bool(cur & set(int(q) for q in nfa.final))


def subset_dfa(nfa: R.NFA) -> R.NFA:
    """Deterministic automaton of the same language (reachable subsets only)."""
    tr = nfa.triples()
    syms = sorted(set(s for _, s, _ in tr))
    start = frozenset(int(q) for q in nfa.start)
    ids: Dict[FrozenSet[int], int] = {start: 0}
    order: List[FrozenSet[int]] = [start]
    out: List[Tuple[int, int, int]] = []
    i = 0
    while i < len(order):
        S = order[i]
        for s in syms:
            T = frozenset(b for (a, sym, b) in tr if sym == s and a in S)
            if not T:
                continue
            if T not in ids:
                ids[T] = len(order)
                order.append(T)
            out.append((ids[S], s, ids[T]))
        i += 1
    fin = set(int(q) for q in nfa.final)
    finals = [ids[S] for S in order if S & fin]
    return R.nfa_from_triples(len(order), nfa.num_labels, out, [0], finals, "dfa(" + nfa.text + ")")


def thompson(node, num_labels: int) -> R.NFA:
    """Thompson construction, then epsilon closure to an epsilon-free NFA."""
    eps: List[Tuple[int, int]] = []
    trans: List[Tuple[int, int, int]] = []
    cnt = [0]

    def new():
        cnt[0] += 1
        return cnt[0] - 1

    def build(n):
        if isinstance(n, R.Sym):
            a, b = new(), new()
            trans.append((a, R.symbol_of(n, num_labels), b))
            return a, b
        if isinstance(n, R.Cat):
            a1, b1 = build(n.left)
            a2, b2 = build(n.right)
            eps.append((b1, a2))
            return a1, b2
        if isinstance(n, R.Alt):
            a, b = new(), new()
            a1, b1 = build(n.left)
            a2, b2 = build(n.right)
            eps.extend([(a, a1), (a, a2), (b1, b), (b2, b)])
            return a, b
        if isinstance(n, (R.Star, R.Plus, R.Opt)):
            a, b = new(), new()
            a1, b1 = build(n.child)
            eps.extend([(a, a1), (b1, b)])
            if not isinstance(n, R.Opt):
                eps.append((b1, a1))
            if not isinstance(n, R.Plus):
                eps.append((a, b))
            return a, b
        raise TypeError(n)

    s0, f0 = build(node)
    nst = cnt[0]
    clo = []
    for q in range(nst):
        seen = {q}
        stack = [q]
        while stack:
            x = stack.pop()
            for a, b in eps:
                if a == x and b not in seen:
                    seen.add(b)
                    stack.append(b)
        clo.append(seen)
    # q --s--> r if some p in closure(q) has p --s--> r; final if closure hits f0
    out = []
    for q in range(nst):
        for (p, s, r) in trans:
            if p in clo[q]:
                out.append((q, s, r))
    finals = [q for q in range(nst) if f0 in clo[q]]
    return R.nfa_from_triples(nst, num_labels, out, [s0], finals, "thompson")
