"""The five seeded workloads (graph, queries, sources) and small variants.

Seeds follow ``s_i = 1000*config + i``: graph i=1, queries i=2, sources i=3,
arrivals i=4. ``scale`` shrinks a workload for tests while keeping its shape.

* er      -- Erdos-Renyi 10k vertices / 50k edges / 8 uniform labels; 16 random
             expressions of <= 4 label occurrences; uniform sources.
* rmat    -- R-MAT scale 20, edge factor 16, (0.57, 0.19, 0.19, 0.05), 64 Zipf(1.1)
             labels; 100 queries, 20 per template, labels drawn in proportion to
             their edge counts; sources in proportion to out-degree.
* kg      -- Chung-Lu 20M vertices / 200M edges, gamma 2.1, 1000 Zipf(1.2) labels;
             one random expression with 3..11 occurrences (4..12 states);
             sources in proportion to out-degree.
* serve   -- the kg graph; templates plus random expressions of 1..31 occurrences,
             leaf inversion p=0.3, Poisson arrivals.
* grid    -- 4096^2 grid, direction labels, 1% shortcuts (and a no-shortcut variant);
             (0|1)* and (0|^2)* 3; uniform sources plus the corner (0,0).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import graphs as G
from . import regex as R


@dataclass
class Workload:
    name: str
    graph: G.LabeledGraph
    queries: List[str]  # expression text, one per query
    sources: np.ndarray  # int32, one per query (plain) or per batch slot
    nfas: List[R.NFA] = field(default_factory=list)
    arrivals_s: Optional[np.ndarray] = None

    def compile(self):
        self.nfas = [R.compile_regex(q, self.graph.num_labels) for q in self.queries]
        return self


def seed(config: int, i: int) -> int:
    return 1000 * config + i


def degree_weighted_sources(rng, g: G.LabeledGraph, k: int) -> np.ndarray:
    deg = G.out_degree(g).astype(np.float64)
    p = deg / deg.sum()
    return rng.choice(g.num_vertices, size=k, p=p).astype(np.int32)


def er_workload(n: int = 10_000, m: int = 50_000, num_labels: int = 8,
                n_queries: int = 16, max_leaves: int = 4, cfg: int = 1) -> Workload:
    g = G.erdos_renyi(n, m, num_labels, seed(cfg, 1))
    rq = np.random.default_rng(seed(cfg, 2))
    qs = []
    for _ in range(n_queries):
        k = int(rq.integers(1, max_leaves + 1))
        ast = R.random_ast(rq, k, lambda r: r.integers(0, num_labels), p_inv=0.5)
        qs.append(R.to_string(ast))
    rs = np.random.default_rng(seed(cfg, 3))
    src = rs.integers(0, n, size=n_queries).astype(np.int32)
    return Workload("er-%d-%d-L%d" % (n, m, num_labels), g, qs, src).compile()


def template_queries(rng, label_counts: np.ndarray, n_per_template: int,
                     templates=R.TEMPLATES) -> List[str]:
    p = label_counts.astype(np.float64)
    p = p / p.sum()
    out = []
    for t in templates:
        k = R.template_arity(t)
        for _ in range(n_per_template):
            labs = rng.choice(len(p), size=k, replace=False, p=p)
            out.append(R.instantiate(t, labs))
    return out


def rmat_workload(scale: int = 20, edge_factor: int = 16, num_labels: int = 64,
                  n_per_template: int = 20, cfg: int = 2) -> Workload:
    g = G.rmat(scale, edge_factor, num_labels, 1.1, seed(cfg, 1))
    rq = np.random.default_rng(seed(cfg, 2))
    qs = template_queries(rq, g.label_counts(), n_per_template)
    rs = np.random.default_rng(seed(cfg, 3))
    src = degree_weighted_sources(rs, g, len(qs))
    return Workload("rmat-%d-%d-L%d" % (scale, edge_factor, num_labels), g, qs, src).compile()


def kg_graph(n: int = 20_000_000, m: int = 200_000_000, num_labels: int = 1000,
             cfg: int = 3) -> G.LabeledGraph:
    return G.chung_lu_fast(n, m, 2.1, num_labels, 1.2, seed(cfg, 1))


def kg_query(rng, g: G.LabeledGraph, min_leaves: int = 3, max_leaves: int = 11,
             p_inv: float = 0.3) -> str:
    p = g.label_counts().astype(np.float64)
    p /= p.sum()
    k = int(rng.integers(min_leaves, max_leaves + 1))
    ast = R.random_ast(rng, k, lambda r: r.choice(len(p), p=p), p_inv=p_inv)
    return R.to_string(ast)


def kg_workload(n: int = 20_000_000, m: int = 200_000_000, num_labels: int = 1000,
                batch: int = 256, cfg: int = 3) -> Workload:
    g = kg_graph(n, m, num_labels, cfg)
    rq = np.random.default_rng(seed(cfg, 2))
    q = kg_query(rq, g)
    rs = np.random.default_rng(seed(cfg, 3))
    src = degree_weighted_sources(rs, g, batch)
    return Workload("kg-%d-%d-L%d" % (n, m, num_labels), g, [q], src).compile()


def serve_queries(g: G.LabeledGraph, n_queries: int, rate_qps: float, cfg: int = 4):
    """Mixed query stream: half template queries, half random expressions with
    1..31 occurrences (2..32 states), leaf inversion p=0.3; degree-weighted
    sources; Poisson arrival times (seconds)."""
    rq = np.random.default_rng(seed(cfg, 2))
    qs = []
    lc = g.label_counts().astype(np.float64)
    for i in range(n_queries):
        if rq.random() < 0.5:
            t = R.TEMPLATES[int(rq.integers(0, len(R.TEMPLATES)))]
            labs = rq.choice(len(lc), size=R.template_arity(t), replace=False, p=lc / lc.sum())
            qs.append(R.instantiate(t, labs))
        else:
            qs.append(kg_query(rq, g, 1, 31, 0.3))
    rs = np.random.default_rng(seed(cfg, 3))
    src = degree_weighted_sources(rs, g, n_queries)
    ra = np.random.default_rng(seed(cfg, 4))
    arr = np.cumsum(ra.exponential(1.0 / rate_qps, size=n_queries))
    return qs, src, arr


GRID_QUERIES = ("(0|1)*", "(0|^2)* 3")


def grid_workload(side: int = 4096, shortcut_frac: float = 0.01, batch: int = 64,
                  cfg: int = 5) -> Workload:
    g = G.grid(side, shortcut_frac, seed(cfg, 1))
    rs = np.random.default_rng(seed(cfg, 3))
    src = np.concatenate([[0], rs.integers(0, side * side, size=batch - 1)]).astype(np.int32)
    return Workload("grid-%d-sc%g" % (side, shortcut_frac), g, list(GRID_QUERIES), src).compile()
