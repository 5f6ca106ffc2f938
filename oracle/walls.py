"""Wall boundary conditions: bounce-back and specular reflection.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use the oracle; the library never does.

* Sec. "Boundary conditions": besides given inflow data, a boundary point
  can be a bounce-back wall, f_bc(x, v) = f(x, -v), or a reflecting wall,
  f_bc(x, v) = f(x, R_n v) with R_n v = v - 2 (v.n) n.  As the paper
  assumes, the velocity set must be closed under the map (walls normal to a
  coordinate axis and a grid symmetric about 0), so f_bc at a node is the
  value of the distribution at another node of the same set.
* The boundary data are refreshed once per Picard iteration (the boundary
  update is one of the steps of each nonlinear iteration, Sec. "Solver
  performance"): the sweep of iteration l+1 reads the wall data of iterate
  l, so each sweep is still a triangular solve per velocity.  In the sweep
  the data enter only at facet nodes where v.n < 0, the upwind side.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry

INFLOW, BOUNCE_BACK, REFLECT = 0, 1, 2


def wall_map(V, normal, kind: int) -> np.ndarray:
    """Index j' of T v_j for every velocity j (T = -I or R_n), found by
    searching the whole set; raises if some image is not a node."""
    V = np.asarray(V, dtype=np.float64)
    if kind == BOUNCE_BACK:
        W = -V
    elif kind == REFLECT:
        n = np.asarray(normal, dtype=np.float64)
        n = n / np.linalg.norm(n)
        W = V - 2.0 * (V @ n)[:, None] * n[None, :]
    else:
        raise ValueError(kind)
    scale = max(1.0, float(np.abs(V).max()))
    jj = np.empty(V.shape[0], dtype=np.int64)
    for j in range(V.shape[0]):
        d = np.abs(V - W[j]).max(axis=1)
        jj[j] = int(np.argmin(d))
        if d[jj[j]] > 1e-9 * scale:
            raise ValueError("the velocity set is not closed under the wall map")
    return jj


def wall_values(geo: Geometry, V, f, kinds, gbc) -> np.ndarray:
    """Boundary data for one sweep: ``gbc`` [n_bfaces][n_fp][N_v] with the
    rows of every wall facet replaced by the distribution ``f``
    [N_c][N_p][N_v] at the mapped velocity, at the same facet node."""
    kinds = np.asarray(kinds)
    g = np.array(gbc, dtype=np.float64, copy=True)
    cache = {}
    for c in range(geo.n_cells):
        for k in range(geo.dim + 1):
            bf = geo.bface[c, k]
            if bf < 0 or kinds[bf] == INFLOW:
                continue
            key = (int(kinds[bf]), tuple(np.round(geo.normal[c, k], 12)))
            if key not in cache:
                cache[key] = wall_map(V, geo.normal[c, k], int(kinds[bf]))
            fn = geo.ref["face_nodes"][k]
            g[bf] = f[c][np.ix_(fn, cache[key])]
    return g


def boundary_kinds(geo: Geometry, rule) -> np.ndarray:
    """Kind of every boundary facet from ``rule(midpoint, unit normal)``."""
    kinds = np.zeros(geo.bnode_x.shape[0], dtype=np.int8)
    for c in range(geo.n_cells):
        for k in range(geo.dim + 1):
            bf = geo.bface[c, k]
            if bf >= 0:
                kinds[bf] = rule(geo.bnode_x[bf].mean(axis=0), geo.normal[c, k])
    return kinds
