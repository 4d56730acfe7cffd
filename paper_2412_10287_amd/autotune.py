"""Persisted autotuning: the settings rpq_autotune chose for a graph, kept in a
JSON file keyed by the graph's signature (sizes and row counts of its store)
and the tuned path, so later runs on the same graph skip the measurement.

The measurement itself runs in the library (rpq_autotune); this module only
stores and re-applies its result through rpq_set_option.
"""
from __future__ import annotations

import json
import os
from typing import Optional, Sequence

from . import rpq

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rpq_mi355x", "tuning.json")
_KEYS = {rpq.TUNE_PLAIN: ("persistent_grid", "pull_alpha", "pull_beta"),
         rpq.TUNE_STACKED: (None, "stacked_alpha", "stacked_beta")}


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def apply(graph: "rpq.Graph", path: int, chosen: dict):
    grid_key, a_key, b_key = _KEYS[path]
    if grid_key:
        graph.set_option(grid_key, int(chosen["grid"]))
    graph.set_option(a_key, int(chosen["alpha"]))
    graph.set_option(b_key, int(chosen["beta"]))
    if path == rpq.TUNE_STACKED and "handoff_edges" in chosen:
        graph.set_option("stacked_handoff_edges", int(chosen["handoff_edges"]))


def tune(graph: "rpq.Graph", path: int, nfas: Sequence["rpq.NFA"], sources: Sequence[int],
         cache: Optional[str] = DEFAULT_CACHE, retune: bool = False) -> dict:
    """Apply the cached settings for (graph, path) or measure them with
    rpq_autotune on the given sample and cache the result. Returns the record
    (chosen values, times, whether it came from the cache)."""
    key = "%s/%s" % (graph.signature(), "plain" if path == rpq.TUNE_PLAIN else "stacked")
    table = _load(cache) if cache else {}
    if not retune and key in table:
        rec = dict(table[key])
        apply(graph, path, rec)
        rec["cached"] = True
        return rec
    rec = graph.autotune(path, nfas, sources)
    rec["cached"] = False
    if cache:
        table[key] = {k: v for k, v in rec.items() if k != "cached"}
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        tmp = cache + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return rec
