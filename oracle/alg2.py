"""Second reference: the frontier-free fixpoint of Sec. 4 (Alg. 2), written with
scipy sparse products and clipped to the Boolean semiring.

TEST INFRASTRUCTURE (see the package docstring). It is a different formulation
from ``oracle.c`` (matrix fixpoint versus explicit pair search) and is used only
to cross-check it on small graphs.

Steps, in the paper's notation: the per-symbol NFA matrices N^a and graph
matrices G^a are built (Sec. 3, Defs 3.7-3.8, with G^{a^-} = (G^a)^T); P starts
as the start states at the source; then P <- P + sum_a (N^a)^T P G^a over the
symbols both alphabets share, until P stops changing; the answer is F P, F the
final-state row.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _bool(m):
    m = sp.csr_matrix(m)
    m.data = np.ones_like(m.data)
    m.eliminate_zeros()
    return m


def alg2(g, nfa, source: int, max_iter: int | None = None) -> np.ndarray:
    """Returns the reachable-vertex bitmap (uint64 words, LSB first)."""
    V, L = g.num_vertices, g.num_labels
    Q, NL = nfa.num_states, nfa.num_labels
    G = {}
    for l in range(L):
        s, d = g.edges_of(l)
        if s.size:
            G[l] = _bool(sp.coo_matrix((np.ones(s.size, np.int64), (s, d)), shape=(V, V)))
    N = {}
    for s in range(2 * NL):
        a, b = int(nfa.sym_ptr[s]), int(nfa.sym_ptr[s + 1])
        if b > a:
            N[s] = _bool(sp.coo_matrix((np.ones(b - a, np.int64), (nfa.frm[a:b], nfa.to[a:b])),
                                       shape=(Q, Q)))
    P = sp.lil_matrix((Q, V), dtype=np.int64)
    for q in nfa.start:
        P[int(q), source] = 1
    P = _bool(P)
    it = 0
    while True:
        acc = P.copy()
        for s, Ns in N.items():
            l = s if s < NL else s - NL
            if l >= L or l not in G:
                continue  # symbol absent from the graph's alphabet
            Gs = G[l] if s < NL else G[l].T.tocsr()
            acc = acc + (Ns.T @ P) @ Gs
        acc = _bool(acc)
        if (acc != P).nnz == 0:
            break
        P = acc
        it += 1
        if max_iter is not None and it > max_iter:
            raise RuntimeError("fixpoint did not settle")
    F = np.zeros(Q, dtype=np.int64)
    F[nfa.final] = 1
    reach = (sp.csr_matrix(F) @ P).toarray().ravel() > 0
    words = np.zeros((V + 63) // 64, dtype=np.uint64)
    idx = np.nonzero(reach)[0]
    np.bitwise_or.at(words, idx >> 6, (np.uint64(1) << (idx & 63).astype(np.uint64)))
    return words
