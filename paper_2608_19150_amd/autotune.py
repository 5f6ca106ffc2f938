"""Tile autotuner for the batched sweep.

The batched sweep's tile is the workgroup size: how many cells of a
generation one velocity's workgroup has in flight (the rest of a wider
generation is walked in further passes).  Small workgroups leave more room
per CU for other velocities' workgroups (more velocities in flight), large
ones cover wide generations in one pass; the best choice depends on the
instances' generation widths and element types, so it is measured: each
candidate times a few real sweeps of the batch (`bgk_batch_time_sweep`) and
the fastest is kept in a JSON cache keyed by the batch's shape.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import Batch

CANDIDATES = (64, 128, 192, 256)


def default_cache_path():
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "bgktgs", "autotune.json")


def batch_key(solvers):
    """A key for the batch's shape: dimension, element order, cells and
    velocities of every instance (order-independent)."""
    parts = sorted(f"{s.dag.dim}:{s.dag.order}:{s.dag.n_cells}:{s.dag.n_v}" for s in solvers)
    return hashlib.sha256(";".join(parts).encode()).hexdigest()[:16]


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_sweep_threads(solvers, fs, *, candidates=CANDIDATES, reps=3, cache_path=None,
                       use_cache=True):
    """Returns (best_threads, {threads: ms per sweep}).  `fs` are the
    instances' current states (read only)."""
    path = cache_path or default_cache_path()
    key = batch_key(solvers)
    table = _load(path) if use_cache else {}
    if use_cache and key in table:
        entry = table[key]
        return int(entry["threads"]), {int(k): v for k, v in entry["ms"].items()}
    probe = Batch(solvers, graph=False)
    probe.time_sweep(fs, candidates[0], reps=1)      # warm-up
    ms = {int(t): probe.time_sweep(fs, t, reps=reps) for t in candidates}
    best = min(ms, key=ms.get)
    table[key] = {"threads": best, "ms": {str(k): v for k, v in ms.items()}}
    _store(path, table)
    return best, ms


def autotuned_batch(solvers, fs, *, graph=True, chunk_iters=4, cache_path=None, **kw):
    """A Batch whose sweep workgroup size was chosen by tune_sweep_threads."""
    best, ms = tune_sweep_threads(solvers, fs, cache_path=cache_path, **kw)
    return Batch(solvers, graph=graph, chunk_iters=chunk_iters, sweep_threads=best), best, ms
