"""Physical cells, faces and node maps for a simplicial mesh.

Sec. 3.1: the DG space is built cell by cell from an affine map
x = x_0 + J xi of the reference simplex; the upwind flux of eq. def-F needs,
for every facet of every cell, the outward unit normal, the facet measure and
the neighbour across it (eq. cell-inflow-outflow-boundaries).

This module computes those quantities directly: facet normals from edge
vectors (2D: a rotated edge; 3D: a cross product), oriented away from the
cell centroid; interior facets matched by their sorted vertex tuple; the
neighbour's node at each facet node matched by physical coordinates.

Reading (A9 of the design notes): each interior facet stores one unit normal,
that of its lower-indexed cell; the other cell uses its negation, so the
upwind test v.n is exactly antisymmetric across a facet.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import factorial

import numpy as np

from .refel import reference


@dataclass
class Geometry:
    dim: int
    order: int
    n_cells: int
    n_p: int
    n_fp: int
    ref: dict
    det: np.ndarray         # |det J|            [n_cells]
    vol: np.ndarray         # |K|                [n_cells]
    jinv: np.ndarray        # J^{-1}             [n_cells][dim][dim]
    nbr: np.ndarray         # neighbour cell or -1        [n_cells][dim+1]
    nbr_face: np.ndarray    # neighbour's facet index     [n_cells][dim+1]
    normal: np.ndarray      # outward unit normal         [n_cells][dim+1][dim]
    area: np.ndarray        # facet measure               [n_cells][dim+1]
    nbr_node: np.ndarray    # neighbour local node at each facet node [n_cells][dim+1][n_fp]
    bface: np.ndarray       # boundary facet id or -1     [n_cells][dim+1]
    bnode_x: np.ndarray     # coordinates of boundary facet nodes [n_bfaces][n_fp][dim]
    node_x: np.ndarray      # DG node coordinates         [n_cells][n_p][dim]


def _facet_normal(pts: np.ndarray, dim: int) -> tuple[np.ndarray, float]:
    """Unnormalised-then-normalised normal and measure of a facet given its vertices."""
    if dim == 2:
        t = pts[1] - pts[0]
        length = float(np.hypot(t[0], t[1]))
        return np.array([t[1], -t[0]]) / length, length
    a = pts[1] - pts[0]
    b = pts[2] - pts[0]
    c = np.cross(a, b)
    nc = float(np.linalg.norm(c))
    return c / nc, 0.5 * nc


def build(vert: np.ndarray, cells: np.ndarray, order: int) -> Geometry:
    vert = np.asarray(vert, dtype=np.float64)
    cells = np.asarray(cells, dtype=np.int64)
    n_cells, nv = cells.shape
    dim = nv - 1
    ref = reference(dim, order)
    n_p, n_fp = ref["n_p"], ref["n_fp"]

    X = vert[cells]                                   # [c][d+1][d]
    J = np.stack([X[:, k + 1] - X[:, 0] for k in range(dim)], axis=2)  # columns
    det = np.abs(np.linalg.det(J))
    jinv = np.linalg.inv(J)
    vol = det / factorial(dim)
    node_x = np.einsum("pk,ckd->cpd", ref["node_bary"], X)

    # facet matching by sorted vertex tuple; facet k is opposite local vertex k
    owner = {}
    nbr = -np.ones((n_cells, dim + 1), dtype=np.int64)
    nbr_face = -np.ones((n_cells, dim + 1), dtype=np.int64)
    for c in range(n_cells):
        for k in range(dim + 1):
            key = tuple(sorted(int(cells[c, i]) for i in range(dim + 1) if i != k))
            if key in owner:
                c0, k0 = owner.pop(key)
                nbr[c, k], nbr_face[c, k] = c0, k0
                nbr[c0, k0], nbr_face[c0, k0] = c, k
            else:
                owner[key] = (c, k)

    normal = np.zeros((n_cells, dim + 1, dim))
    area = np.zeros((n_cells, dim + 1))
    centroid = X.mean(axis=1)
    for c in range(n_cells):
        for k in range(dim + 1):
            if nbr[c, k] >= 0 and nbr[c, k] < c:
                continue  # the lower-indexed cell owns the facet normal
            fv = X[c, [i for i in range(dim + 1) if i != k]]
            n, a = _facet_normal(fv, dim)
            if np.dot(n, fv.mean(axis=0) - centroid[c]) < 0.0:
                n = -n
            normal[c, k] = n
            area[c, k] = a
            if nbr[c, k] >= 0:
                c1, k1 = nbr[c, k], nbr_face[c, k]
                normal[c1, k1] = -n
                area[c1, k1] = a

    # neighbour node at each facet node, matched by coordinates
    nbr_node = -np.ones((n_cells, dim + 1, n_fp), dtype=np.int64)
    bface = -np.ones((n_cells, dim + 1), dtype=np.int64)
    bx = []
    for c in range(n_cells):
        for k in range(dim + 1):
            fn = ref["face_nodes"][k]
            if nbr[c, k] < 0:
                bface[c, k] = len(bx)
                bx.append(node_x[c, fn])
                continue
            c1 = nbr[c, k]
            for p, a in enumerate(fn):
                dist = np.linalg.norm(node_x[c1] - node_x[c, a], axis=1)
                b = int(np.argmin(dist))
                if dist[b] > 1e-10:
                    raise RuntimeError("non-conforming facet")
                nbr_node[c, k, p] = b
    bnode_x = np.array(bx).reshape(-1, n_fp, dim)
    return Geometry(dim, order, n_cells, n_p, n_fp, ref, det, vol, jinv, nbr, nbr_face,
                    normal, area, nbr_node, bface, bnode_x, node_x)
