"""The per-cell upwind DG solve and the transport sweep (Sec. 4, Sec. 4.1).

Eq. bgk-ss-picard, tested against phi_a on cell K with f = sum_b f_b phi_b:

  -(f, v.grad phi_a)_K + sum_{outflow facets} (v.n)(f, phi_a)_e + (sigma f, phi_a)_K
      = (nu M + q, phi_a)_K + sum_{inflow facets} |v.n| (fhat, phi_a)_e

Readings (design notes A2, A6, A8): both the current and the lagged inflow
enter the right-hand side with +|v.n| (the sign printed on the non-lagged
term is a typo; eq. bgk-ss-inflow-outflow fixes it); sigma, nu, M and q are
collocated at the DG nodes, so (sigma f, phi_a)_K = (M_K diag(sigma) f)_a and
(nu M + q, phi_a)_K = (M_K (nu*M + q))_a; boundary inflow values are nodal at
the boundary facet nodes.

With the reference matrices of ``refel`` this is

  A = |K| mass diag(sigma) - |det J| sum_beta (J^{-1} v)_beta stiff_beta
      + sum_{k: s_k > 0} s_k |e_k| face_mass_k
  b = |K| mass (nu*M + q) + sum_{k: s_k < 0} |s_k| |e_k| face_mass_k fhat_k

and the cell's nodal values are A^{-1} b (LAPACK, partial pivoting).

Array layout used throughout the oracle: nodal fields are [cell][node] and
phase-space fields are [cell][node][velocity].
"""
from __future__ import annotations

import numpy as np

from .dag import facet_speeds, facet_speeds_batch
from .geometry import Geometry


def cell_matrices(geo: Geometry, cells: np.ndarray, V: np.ndarray, sigma: np.ndarray):
    """Batched A for items (cells[i], V[i]); sigma[i] holds the cell's nodal sigma."""
    ref = geo.ref
    vt = np.einsum("iab,ib->ia", geo.jinv[cells], V)                     # J^{-1} v
    A = geo.vol[cells, None, None] * ref["mass"][None] * sigma[:, None, :]
    A = A - geo.det[cells, None, None] * np.einsum("ib,bxy->ixy", vt, ref["stiff"])
    s = facet_speeds_batch(geo.normal[cells], V)
    for k in range(geo.dim + 1):
        w = np.where(s[:, k] > 0.0, s[:, k], 0.0) * geo.area[cells, k]
        A = A + w[:, None, None] * ref["face_mass"][k][None]
    return A, s


def _solve_items(geo, cells, jj, V, sigma, nu, Mv, q, gbc, f_prev, f_out, lagged):
    """Assemble and solve the cell systems for items (cells[i], velocity jj[i])."""
    ref = geo.ref
    Vi = V[jj]
    A, s = cell_matrices(geo, cells, Vi, sigma[cells])
    src = nu[cells] * Mv[cells, :, jj] + q[cells, :, jj]                  # [i][p]
    b = geo.vol[cells, None] * np.einsum("xy,iy->ix", ref["mass"], src)
    for k in range(geo.dim + 1):
        inflow = s[:, k] < 0.0
        if not np.any(inflow):
            continue
        fn = ref["face_nodes"][k]
        fhat = np.zeros((cells.shape[0], geo.n_p))
        nb = geo.nbr[cells, k]
        interior = inflow & (nb >= 0)
        bnd = inflow & (nb < 0)
        if np.any(interior):
            ii = np.nonzero(interior)[0]
            lag = lagged[jj[ii], cells[ii], k] if lagged is not None else np.zeros(ii.size, bool)
            for p, a in enumerate(fn):
                nn = geo.nbr_node[cells[ii], k, p]
                cur = f_out[nb[ii], nn, jj[ii]]
                if np.any(lag):
                    old = f_prev[nb[ii], nn, jj[ii]]
                    cur = np.where(lag, old, cur)
                fhat[ii, a] = cur
        if np.any(bnd):
            ii = np.nonzero(bnd)[0]
            bf = geo.bface[cells[ii], k]
            for p, a in enumerate(fn):
                fhat[ii, a] = gbc[bf, p, jj[ii]]
        w = np.where(inflow, -s[:, k], 0.0) * geo.area[cells, k]
        b = b + w[:, None] * np.einsum("xy,iy->ix", ref["face_mass"][k], fhat)
    x = np.linalg.solve(A, b[:, :, None])[:, :, 0]
    f_out[cells, :, jj] = x


def sweep(geo: Geometry, V, sigma, nu, Mv, q, gbc, gens, lagged=None, f_prev=None):
    """One transport sweep over all velocities, generation by generation.

    For g = 0, 1, ... every (velocity j, cell K) with gen_j(K) = g is solved;
    all of them only need inflow from generations < g (or lagged/boundary
    data), which is the topological-generation sweep of Sec. 4.1.

    V [N_v][d]; sigma, nu [N_c][N_p]; Mv, q [N_c][N_p][N_v];
    gbc [n_bfaces][n_fp][N_v]; gens [N_v][N_c]; lagged [N_v][N_c][d+1] bool;
    f_prev [N_c][N_p][N_v] (needed when lagged facets exist).
    """
    V = np.asarray(V, dtype=np.float64)
    f_out = np.full((geo.n_cells, geo.n_p, V.shape[0]), np.nan)
    if lagged is not None and not np.any(lagged):
        lagged = None
    if lagged is not None and f_prev is None:
        raise ValueError("lagged facets need f_prev")
    gmax = int(gens.max())
    jj_all, cc_all = np.nonzero(np.ones_like(gens, dtype=bool))
    gflat = gens[jj_all, cc_all]
    order = np.argsort(gflat, kind="stable")
    bounds = np.searchsorted(gflat[order], np.arange(gmax + 2))
    for g in range(gmax + 1):
        sel = order[bounds[g]:bounds[g + 1]]
        _solve_items(geo, cc_all[sel], jj_all[sel], V, sigma, nu, Mv, q, gbc, f_prev, f_out,
                     lagged)
    return f_out


def sweep_in_order(geo: Geometry, V, sigma, nu, Mv, q, gbc, orders, lagged=None, f_prev=None):
    """The same sweep, one cell at a time, visiting each velocity's cells in
    the given topological order (e.g. the DFS reverse post-order)."""
    V = np.asarray(V, dtype=np.float64)
    f_out = np.full((geo.n_cells, geo.n_p, V.shape[0]), np.nan)
    for j in range(V.shape[0]):
        for c in orders[j]:
            _solve_items(geo, np.array([c]), np.array([j]), V, sigma, nu, Mv, q, gbc, f_prev,
                         f_out, lagged)
    return f_out


def dense_solve(geo: Geometry, v, sigma, nu, Mv_j, q_j, gbc_j, lagged_j=None, f_prev_j=None):
    """Solve eq. bgk-ss-picard for one velocity as one global linear system.

    Every cell's rows are assembled with the neighbour coupling of its
    non-lagged inflow facets in the matrix (no ordering is used at all);
    boundary and lagged inflow go to the right-hand side.  On small meshes
    this pins the sweep, which must reproduce it to rounding.
    Fields here are for one velocity: Mv_j, q_j [N_c][N_p], gbc_j [n_bf][n_fp].
    """
    ref = geo.ref
    n_p = geo.n_p
    N = geo.n_cells * n_p
    G = np.zeros((N, N))
    rhs = np.zeros(N)
    v = np.asarray(v, dtype=np.float64)
    s_all = facet_speeds(geo, v)
    for c in range(geo.n_cells):
        A, _ = cell_matrices(geo, np.array([c]), v[None], sigma[[c]])
        r0 = c * n_p
        G[r0:r0 + n_p, r0:r0 + n_p] += A[0]
        rhs[r0:r0 + n_p] += geo.vol[c] * ref["mass"] @ (nu[c] * Mv_j[c] + q_j[c])
        for k in range(geo.dim + 1):
            s = s_all[c, k]
            if not s < 0.0:
                continue
            fm = -s * geo.area[c, k] * ref["face_mass"][k]
            fn = ref["face_nodes"][k]
            nb = geo.nbr[c, k]
            if nb < 0:
                val = np.zeros(n_p)
                val[fn] = gbc_j[geo.bface[c, k]]
                rhs[r0:r0 + n_p] += fm @ val
            elif lagged_j is not None and lagged_j[c, k]:
                val = np.zeros(n_p)
                val[fn] = f_prev_j[nb, geo.nbr_node[c, k]]
                rhs[r0:r0 + n_p] += fm @ val
            else:
                for p, a in enumerate(fn):
                    col = nb * n_p + geo.nbr_node[c, k, p]
                    G[r0:r0 + n_p, col] -= fm[:, a]
    return np.linalg.solve(G, rhs).reshape(geo.n_cells, n_p)
