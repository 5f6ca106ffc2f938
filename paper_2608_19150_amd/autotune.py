"""Tile autotuners for the sweep.

Single-instance sweeps (tune_sweep_walk): the tile is the walk, i.e. how
many velocities a workgroup serves and how many cells of a generation each
has in flight: the workgroup walk (one velocity per workgroup of 64-256
threads) or the packed walk (64/L velocities per 64-lane workgroup, L
lanes each).  Narrow generations favour packing, wide ones the workgroup
walk; each candidate times real sweeps of the caller's inputs
(`tgs_sweep`) and the fastest is kept in a JSON cache keyed by the DAG's
shape, then set on the DAG (`tgs_dag_set_walk`; every walk gives the same
results bit for bit).

Batched sweeps (tune_batch_walk): the same two walks over every instance's
velocities at once.  With the workgroup walk the tile is the workgroup
size: how many cells of a generation one velocity's workgroup has in flight
(the rest of a wider generation is walked in further passes); small
workgroups leave more room per CU for other velocities' workgroups, large
ones cover wide generations in one pass.  With the packed walk 64/L
velocities of one instance share a 64-lane workgroup, which suits the
narrow generations of small instances once the batch has velocities enough
to fill the GPU.  Each candidate times a few real sweeps of the batch
(`bgk_batch_time_sweep`) and the fastest is kept in a JSON cache keyed by
the batch's shape (tune_sweep_threads: the workgroup sizes alone).
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import torch

from . import Batch, tgs_sweep

CANDIDATES = (64, 128, 192, 256)
BATCH_WALK_CANDIDATES = tuple(("wg", t) for t in (64, 128, 256)) + tuple(
    ("packed", l) for l in (4, 8, 16, 32))
WALK_CANDIDATES = tuple(("wg", t) for t in (64, 128, 192, 256)) + tuple(
    ("packed", l) for l in (2, 4, 8, 16, 32))


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


def tune_batch_walk(solvers, fs, *, candidates=BATCH_WALK_CANDIDATES, reps=3, cache_path=None,
                    use_cache=True):
    """Returns ((kind, value), {(kind, value): ms per sweep}) for the batched
    sweep: ("wg", threads) or ("packed", lanes).  `fs` are the instances'
    current states (read only)."""
    path = cache_path or default_cache_path()
    key = "batchwalk:" + batch_key(solvers)
    table = _load(path) if use_cache else {}
    if use_cache and key in table:
        kind, val = table[key]["best"]
        return (kind, int(val)), {(k.split(":")[0], int(k.split(":")[1])): v
                                  for k, v in table[key]["ms"].items()}
    probe = Batch(solvers, graph=False)
    probe.time_sweep(fs, 128, reps=1)      # warm-up
    ms = {}
    for kind, val in candidates:
        if kind == "wg":
            ms[(kind, val)] = probe.time_sweep(fs, val, reps=reps)
        else:
            ms[(kind, val)] = probe.time_sweep(fs, 128, reps=reps, lanes=val)
    best = min(ms, key=ms.get)
    table[key] = {"best": list(best), "ms": {f"{k}:{v}": t for (k, v), t in ms.items()}}
    _store(path, table)
    return best, ms


def batch_walk_kwargs(best):
    """Batch keyword arguments for a tune_batch_walk choice."""
    kind, val = best
    return {"sweep_threads": val} if kind == "wg" else {"sweep_lanes": val}


def autotuned_batch(solvers, fs, *, graph=True, chunk_iters=4, cache_path=None, **kw):
    """A Batch whose sweep walk was chosen by tune_batch_walk."""
    best, ms = tune_batch_walk(solvers, fs, cache_path=cache_path, **kw)
    return (Batch(solvers, graph=graph, chunk_iters=chunk_iters, **batch_walk_kwargs(best)),
            best, ms)


def dag_key(dag):
    """A key for a single instance's sweep shape: element type, cells,
    velocities and the generation counts (which fix the walk's chain)."""
    _, G = dag.generations()
    G = np.asarray(G)
    parts = f"{dag.dim}:{dag.order}:{dag.n_cells}:{dag.n_v}:{int(G.sum())}:{int(G.max())}"
    return "walk:" + hashlib.sha256(parts.encode()).hexdigest()[:16]


def time_sweep(dag, sweep_kw, reps=3):
    """Median milliseconds of `reps` tgs_sweep calls with the DAG's current
    walk (one untimed call first)."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    tgs_sweep(dag, **sweep_kw)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        ev[0].record()
        tgs_sweep(dag, **sweep_kw)
        ev[1].record()
        torch.cuda.synchronize()
        ts.append(ev[0].elapsed_time(ev[1]))
    return float(np.median(ts))


def tune_sweep_walk(dag, sweep_kw, *, candidates=WALK_CANDIDATES, reps=3, cache_path=None,
                    use_cache=True):
    """Chooses the single-instance sweep walk by timing `tgs_sweep` with
    `sweep_kw` (q, nu, mcoef, f_out, sigma_shift, boundary data, ...) under
    every candidate, sets the fastest on the DAG and returns
    (best, {candidate: ms}); candidates are ("wg", threads) and
    ("packed", lanes).  Packed walks need FP64 sweeps."""
    path = cache_path or default_cache_path()
    key = dag_key(dag)
    table = _load(path) if use_cache else {}
    if use_cache and key in table:
        kind, val = table[key]["best"]
        _apply(dag, kind, int(val))
        return (kind, int(val)), {tuple(k.split(":")[:1]) + (int(k.split(":")[1]),): v
                                  for k, v in table[key]["ms"].items()}
    ms = {}
    for kind, val in candidates:
        _apply(dag, kind, val)
        ms[(kind, val)] = time_sweep(dag, sweep_kw, reps=reps)
    best = min(ms, key=ms.get)
    _apply(dag, *best)
    table[key] = {"best": list(best), "ms": {f"{k}:{v}": t for (k, v), t in ms.items()}}
    _store(path, table)
    return best, ms


def _apply(dag, kind, val):
    if kind == "wg":
        dag.set_walk(threads=val, lanes=0)
    else:
        dag.set_walk(threads=0, lanes=val)
