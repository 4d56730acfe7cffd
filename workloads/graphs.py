"""Seeded synthetic edge-labelled graphs (Sec. 2, Def. 2.1) in per-label COO form.

A graph is ``LabeledGraph(V, L, label_ptr, src, dst)``: the edges carrying label
``l`` are ``(src[i] -> dst[i])`` for ``i in [label_ptr[l], label_ptr[l+1])``.
An edge with several labels appears once per label. Vertex ids are 0-based.

Nothing here evaluates a query; these are inputs only. All generators take an
explicit seed and use numpy's PCG64 ``default_rng``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class LabeledGraph:
    num_vertices: int
    num_labels: int
    label_ptr: np.ndarray  # int64, L+1
    src: np.ndarray  # int32
    dst: np.ndarray  # int32
    name: str = ""

    @property
    def num_edges(self) -> int:
        return int(self.label_ptr[-1])

    def label_counts(self) -> np.ndarray:
        return np.diff(self.label_ptr)

    def edges_of(self, l: int):
        a, b = int(self.label_ptr[l]), int(self.label_ptr[l + 1])
        return self.src[a:b], self.dst[a:b]


def from_triples(num_vertices: int, num_labels: int, src, dst, lab, dedupe: bool = True,
                 name: str = "") -> LabeledGraph:
    """Group ``(src, dst, label)`` triples by label (and optionally dedupe)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    lab = np.asarray(lab, dtype=np.int64)
    if src.size:
        assert src.min() >= 0 and src.max() < num_vertices
        assert dst.min() >= 0 and dst.max() < num_vertices
        assert lab.min() >= 0 and lab.max() < num_labels
    bits = max(1, int(num_vertices - 1).bit_length())
    if 2 * bits + max(1, int(num_labels - 1).bit_length()) > 63:
        raise ValueError("graph too large for 64-bit edge keys")
    key = (lab << np.int64(2 * bits)) | (src << np.int64(bits)) | dst
    key = np.unique(key) if dedupe else np.sort(key, kind="stable")
    mask = np.int64((1 << bits) - 1)
    d = (key & mask).astype(np.int32)
    s = ((key >> np.int64(bits)) & mask).astype(np.int32)
    l = (key >> np.int64(2 * bits))
    counts = np.bincount(l, minlength=num_labels).astype(np.int64)
    ptr = np.zeros(num_labels + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return LabeledGraph(num_vertices, num_labels, ptr, s, d, name)


def zipf_labels(rng: np.random.Generator, m: int, num_labels: int, s: float) -> np.ndarray:
    """Label of each of ``m`` edges, P(label = l) proportional to (l+1)^-s."""
    w = 1.0 / np.arange(1, num_labels + 1, dtype=np.float64) ** s
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(m)
    return np.minimum(np.searchsorted(cdf, u, side="right"), num_labels - 1).astype(np.int64)


def erdos_renyi(n: int, m: int, num_labels: int, seed: int) -> LabeledGraph:
    """G(n, m) directed: ``m`` distinct ordered pairs, no self-loops, each with
    one label drawn uniformly from [0, num_labels)."""
    rng = np.random.default_rng(seed)
    if m > n * (n - 1):
        raise ValueError("too many edges")
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        s = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        d = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        ok = s != d
        k = s[ok] * n + d[ok]
        # keep first occurrences in draw order so the result is seed-stable
        allk = np.concatenate([keys, k])
        _, first = np.unique(allk, return_index=True)
        keys = allk[np.sort(first)][:m]
    src = keys // n
    dst = keys % n
    lab = rng.integers(0, num_labels, size=m, dtype=np.int64)
    return from_triples(n, num_labels, src, dst, lab, name="er-%d-%d-%d" % (n, m, num_labels))


def rmat(scale: int, edge_factor: int, num_labels: int, zipf_s: float, seed: int,
         abcd=(0.57, 0.19, 0.19, 0.05)) -> LabeledGraph:
    """R-MAT (Chakrabarti, Zhan, Faloutsos 2004): 2^scale vertices,
    edge_factor * 2^scale generated edges; quadrant probabilities ``abcd`` per
    bit; a seeded vertex permutation; Zipf labels; per-label dedupe."""
    rng = np.random.default_rng(seed)
    n = 1 << scale
    m = edge_factor * n
    a, b, c, _ = abcd
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    chunk = 1 << 22
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        s = np.zeros(hi - lo, dtype=np.int64)
        d = np.zeros(hi - lo, dtype=np.int64)
        for bit in range(scale):
            u = rng.random(hi - lo)
            right = (u >= a) & (u < a + b) | (u >= a + b + c)  # quadrants b, d
            down = u >= a + b  # quadrants c, d
            s |= down.astype(np.int64) << bit
            d |= right.astype(np.int64) << bit
        src[lo:hi] = s
        dst[lo:hi] = d
    perm = rng.permutation(n).astype(np.int64)
    src = perm[src]
    dst = perm[dst]
    lab = zipf_labels(rng, m, num_labels, zipf_s)
    return from_triples(n, num_labels, src, dst, lab,
                        name="rmat-%d-%d-L%d" % (scale, edge_factor, num_labels))


def chung_lu(n: int, m: int, gamma: float, num_labels: int, zipf_s: float, seed: int,
             i0: float = 10.0) -> LabeledGraph:
    """Directed Chung-Lu graph with power-law expected degrees.

    Vertex i (before a random relabelling) has in- and out-weight proportional
    to (i + i0)^(-1/(gamma-1)); each of ``m`` edges picks its source by the
    out-weights and its destination by the in-weights, independently, under
    independent seeded permutations. Labels Zipf(s); per-label dedupe.
    """
    rng = np.random.default_rng(seed)
    w = (np.arange(n, dtype=np.float64) + i0) ** (-1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    perm_s = rng.permutation(n).astype(np.int32)
    perm_d = rng.permutation(n).astype(np.int32)
    src = np.empty(m, dtype=np.int64)
    dst = np.empty(m, dtype=np.int64)
    chunk = 1 << 24
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        src[lo:hi] = perm_s[np.minimum(np.searchsorted(cdf, rng.random(hi - lo)), n - 1)]
        dst[lo:hi] = perm_d[np.minimum(np.searchsorted(cdf, rng.random(hi - lo)), n - 1)]
    del cdf, w
    lab = zipf_labels(rng, m, num_labels, zipf_s)
    return from_triples(n, num_labels, src, dst, lab,
                        name="chunglu-%d-%d-L%d" % (n, m, num_labels))


def chung_lu_fast(n: int, m: int, gamma: float, num_labels: int, zipf_s: float, seed: int,
                  i0: float = 10.0) -> LabeledGraph:
    """Directed Chung-Lu graph for large sizes, without sorting.

    Per-label edge counts are drawn from the Zipf(s) multinomial, so edges are
    produced already grouped by label. Endpoints are drawn by inverting the
    CDF of the continuous weight density (x + i0)^(-1/(gamma-1)) on [0, n)
    (the continuous counterpart of ``chung_lu``'s discrete weights), then
    relabelled by independent seeded permutations for sources and targets.
    Duplicate (src, dst, label) entries are kept: consumers merge them.
    """
    rng = np.random.default_rng(seed)
    w = 1.0 / np.arange(1, num_labels + 1, dtype=np.float64) ** zipf_s
    counts = rng.multinomial(m, w / w.sum()).astype(np.int64)
    ptr = np.zeros(num_labels + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    beta = 1.0 / (gamma - 1.0)
    a = 1.0 - beta
    x0, x1 = i0 ** a, (n + i0) ** a
    perm_s = rng.permutation(n).astype(np.int32)
    perm_d = rng.permutation(n).astype(np.int32)
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    chunk = 1 << 24
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        for out, perm in ((src, perm_s), (dst, perm_d)):
            u = rng.random(hi - lo)
            x = (x0 + u * (x1 - x0)) ** (1.0 / a) - i0
            idx = np.minimum(x.astype(np.int64), n - 1)
            out[lo:hi] = perm[idx]
    return LabeledGraph(n, num_labels, ptr, src, dst, name="chunglu-%d-%d-L%d" % (n, m, num_labels))


GRID_E, GRID_N, GRID_W, GRID_S = 0, 1, 2, 3


def grid(side: int, shortcut_frac: float, seed: int) -> LabeledGraph:
    """side x side grid, vertex id = y*side + x. Directed edges to the four
    neighbours, labelled by direction: east=0, north=1 (y+1), west=2, south=3
    (y-1). Plus ``shortcut_frac`` * (grid edges) uniformly random (u, v) pairs
    with uniform labels in [0, 4)."""
    rng = np.random.default_rng(seed)
    ids = np.arange(side * side, dtype=np.int64)
    x = ids % side
    y = ids // side
    parts_s, parts_d, parts_l = [], [], []
    for lab, ok, delta in ((GRID_E, x < side - 1, 1), (GRID_N, y < side - 1, side),
                           (GRID_W, x > 0, -1), (GRID_S, y > 0, -side)):
        s = ids[ok]
        parts_s.append(s)
        parts_d.append(s + delta)
        parts_l.append(np.full(s.size, lab, dtype=np.int64))
    m_grid = sum(p.size for p in parts_s)
    k = int(round(shortcut_frac * m_grid))
    if k:
        parts_s.append(rng.integers(0, side * side, size=k, dtype=np.int64))
        parts_d.append(rng.integers(0, side * side, size=k, dtype=np.int64))
        parts_l.append(rng.integers(0, 4, size=k, dtype=np.int64))
    return from_triples(side * side, 4, np.concatenate(parts_s), np.concatenate(parts_d),
                        np.concatenate(parts_l),
                        name="grid-%d-sc%g" % (side, shortcut_frac))


def out_degree(g: LabeledGraph) -> np.ndarray:
    return np.bincount(g.src, minlength=g.num_vertices).astype(np.int64)


def in_degree(g: LabeledGraph) -> np.ndarray:
    return np.bincount(g.dst, minlength=g.num_vertices).astype(np.int64)
