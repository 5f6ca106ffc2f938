"""Upwind graphs, depth-first topological order and generations (Sec. 4.1).

For a velocity v_j the mesh induces a directed graph: an edge (a, b) means
cell a shares a facet with cell b and is upwind of it, i.e. v_j.n > 0 on
that facet with n the outward normal of a.  A depth-first search gives a
topological order; an edge into a cell that is still on the DFS stack (a
back edge) closes a cycle and is lagged: the downwind cell then takes that
facet's inflow from the previous Picard iterate.

Readings taken here (design notes A9-A11):
  * a facet with v.n == 0 carries no edge; "zero" is taken as
    |v.n| <= 1e-12 |v| (n the unit normal), so that a tangential facet whose
    computed flux is rounding noise of either sign is classified the same
    way by any implementation (eq. cell-inflow-outflow-boundaries puts such
    a facet in neither the inflow nor the outflow boundary);
  * DFS roots are visited in ascending cell index and children in ascending
    local facet order of the current cell;
  * the generation of a cell is 0 when it has no non-lagged in-edge,
    otherwise 1 + the largest generation among its non-lagged predecessors
    (the longest-path recursion of Sec. 4.1).
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry


TANGENTIAL_TOL = 1e-12


def facet_speeds(geo: Geometry, v: np.ndarray) -> np.ndarray:
    """s[c][k] = v . n_{c,k} (outward unit normal); tangential facets
    (|s| <= 1e-12 |v|) get exactly 0."""
    v = np.asarray(v, dtype=np.float64)
    s = geo.normal @ v
    s[np.abs(s) <= TANGENTIAL_TOL * np.linalg.norm(v)] = 0.0
    return s


def facet_speeds_batch(normals: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Per item i: s[i][k] = V[i] . normals[i][k] with the same tangential rule."""
    s = np.einsum("ikd,id->ik", normals, V)
    s[np.abs(s) <= TANGENTIAL_TOL * np.linalg.norm(V, axis=1)[:, None]] = 0.0
    return s


def dfs_order(geo: Geometry, v: np.ndarray):
    """Return (topological order, lagged[c][k] bool) for velocity v."""
    s = facet_speeds(geo, v)
    n = geo.n_cells
    color = np.zeros(n, dtype=np.int8)      # 0 white, 1 on stack, 2 done
    lagged = np.zeros((n, geo.dim + 1), dtype=bool)
    post = []
    for root in range(n):
        if color[root]:
            continue
        color[root] = 1
        stack = [(root, 0)]
        while stack:
            c, k = stack[-1]
            if k > geo.dim:
                stack.pop()
                color[c] = 2
                post.append(c)
                continue
            stack[-1] = (c, k + 1)
            b = geo.nbr[c, k]
            if b < 0 or not s[c, k] > 0.0:
                continue
            if color[b] == 1:
                lagged[b, geo.nbr_face[c, k]] = True      # back edge: b lags this inflow
            elif color[b] == 0:
                color[b] = 1
                stack.append((b, 0))
    return post[::-1], lagged


def generations(geo: Geometry, v: np.ndarray, lagged: np.ndarray, order=None) -> np.ndarray:
    """gen(b) = 0 without non-lagged in-edges, else 1 + max over predecessors.

    ``order`` must be a topological order of the graph without lagged edges;
    when omitted it is recomputed by a DFS that ignores the lagged edges.
    """
    s = facet_speeds(geo, v)
    if order is None:
        order = _topo_without(geo, s, lagged)
    gen = np.zeros(geo.n_cells, dtype=np.int64)
    done = np.zeros(geo.n_cells, dtype=bool)
    for b in order:
        g = 0
        for k in range(geo.dim + 1):
            a = geo.nbr[b, k]
            if a >= 0 and s[b, k] < 0.0 and not lagged[b, k]:
                if not done[a]:
                    raise RuntimeError("order is not topological")
                g = max(g, gen[a] + 1)
        gen[b] = g
        done[b] = True
    return gen


def _topo_without(geo: Geometry, s: np.ndarray, lagged: np.ndarray):
    n = geo.n_cells
    color = np.zeros(n, dtype=np.int8)
    post = []
    for root in range(n):
        if color[root]:
            continue
        color[root] = 1
        stack = [(root, 0)]
        while stack:
            c, k = stack[-1]
            if k > geo.dim:
                stack.pop()
                color[c] = 2
                post.append(c)
                continue
            stack[-1] = (c, k + 1)
            b = geo.nbr[c, k]
            if b < 0 or not s[c, k] > 0.0 or lagged[b, geo.nbr_face[c, k]]:
                continue
            if color[b] == 1:
                raise RuntimeError("graph still has a cycle after lagging")
            if color[b] == 0:
                color[b] = 1
                stack.append((b, 0))
    return post[::-1]


def build_all(geo: Geometry, V: np.ndarray, lagged=None):
    """Per-velocity DFS: returns (gen[N_v][N_c], lagged[N_v][N_c][d+1]).

    When ``lagged`` is given (e.g. another implementation's lagging choice on
    a cyclic mesh) it replaces the DFS back edges.
    """
    V = np.asarray(V, dtype=np.float64)
    nv = V.shape[0]
    gens = np.zeros((nv, geo.n_cells), dtype=np.int64)
    lags = np.zeros((nv, geo.n_cells, geo.dim + 1), dtype=bool)
    for j in range(nv):
        if lagged is None:
            order, lag = dfs_order(geo, V[j])
            gens[j] = generations(geo, V[j], lag, order)
        else:
            lag = np.asarray(lagged[j], dtype=bool)
            gens[j] = generations(geo, V[j], lag)
        lags[j] = lag
    return gens, lags
