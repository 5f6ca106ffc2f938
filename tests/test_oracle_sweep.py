"""Oracle pins: upwind graphs, generations and the transport sweep.

* The sweep must equal a dense global solve of the same DG system
  (eq. bgk-ss-picard assembled without any ordering).
* Longest-path generations are unique on a DAG: the DFS-based oracle must
  equal brute-force longest paths, and a closed form on a structured mesh.
* Spatially uniform data gives f = (nu M + q)/sigma exactly (fluxes cancel).
* Manufactured steady transport converges at order k+1 (the DG order the
  north star asks for in free streaming).
"""
import math

import numpy as np
import pytest

import problems as P
from oracle import dag, geometry, transport


def _random_inputs(geo, nv, seed):
    rng = np.random.default_rng(seed)
    sig = rng.uniform(1.0, 3.0, (geo.n_cells, geo.n_p))
    nu = rng.uniform(0.0, 1.0, sig.shape)
    Mv = rng.uniform(0.0, 1.0, (geo.n_cells, geo.n_p, nv))
    q = rng.uniform(0.0, 1.0, Mv.shape)
    gbc = rng.uniform(0.0, 1.0, (geo.bnode_x.shape[0], geo.n_fp, nv))
    return sig, nu, Mv, q, gbc


@pytest.mark.parametrize("dim,order,n_side,n1", [(2, 1, 4, 4), (2, 2, 3, 4), (3, 1, 2, 3)])
def test_sweep_equals_dense_global_solve(dim, order, n_side, n1):
    pr = P.small_problem(dim=dim, order=order, n_side=n_side, n_1d=n1)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, order)
    V = pr.vgrid.v
    gens, lags = dag.build_all(geo, V)
    assert not lags.any()                     # Delaunay meshes: no cycles
    sig, nu, Mv, q, gbc = _random_inputs(geo, V.shape[0], 11)
    f = transport.sweep(geo, V, sig, nu, Mv, q, gbc, gens)
    for j in range(V.shape[0]):
        fd = transport.dense_solve(geo, V[j], sig, nu, Mv[:, :, j], q[:, :, j], gbc[:, :, j])
        assert np.abs(fd - f[:, :, j]).max() <= 1e-13 * np.abs(fd).max()


def test_dfs_order_sweep_equals_generation_sweep():
    pr = P.small_problem(n_side=4, n_1d=5, order=2)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 2)
    V = pr.vgrid.v
    gens, _ = dag.build_all(geo, V)
    orders = [dag.dfs_order(geo, V[j])[0] for j in range(V.shape[0])]
    sig, nu, Mv, q, gbc = _random_inputs(geo, V.shape[0], 3)
    f1 = transport.sweep(geo, V, sig, nu, Mv, q, gbc, gens)
    f2 = transport.sweep_in_order(geo, V, sig, nu, Mv, q, gbc, orders)
    assert np.abs(f1 - f2).max() <= 1e-14 * np.abs(f1).max()


def _brute_longest(geo, v, lagged):
    s = dag.facet_speeds(geo, v)
    gen = np.zeros(geo.n_cells, dtype=np.int64)
    for _ in range(geo.n_cells + 1):           # Bellman-Ford style relaxation
        changed = False
        for b in range(geo.n_cells):
            for k in range(geo.dim + 1):
                a = geo.nbr[b, k]
                if a >= 0 and s[b, k] < 0 and not lagged[b, k] and gen[a] + 1 > gen[b]:
                    gen[b] = gen[a] + 1
                    changed = True
        if not changed:
            return gen
    raise AssertionError("cycle")


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_generations_equal_brute_force(seed):
    pr = P.small_problem(n_side=5, n_1d=6, seed=seed)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 1)
    V = pr.vgrid.v
    gens, lags = dag.build_all(geo, V)
    for j in range(V.shape[0]):
        np.testing.assert_array_equal(gens[j], _brute_longest(geo, V[j], lags[j]))
        counts = np.bincount(gens[j])
        assert counts.sum() == geo.n_cells and np.all(counts > 0)


def test_generations_structured_closed_form():
    """Right-triangle mesh, cells (lower, upper) per lattice square (i, j).
    For v1 > v2 > 0 the upper triangle of square (i, j) is in generation 2i and
    the lower one in 2i + 1; for v2 > v1 > 0, lower 2j and upper 2j + 1."""
    n = 6
    mesh = P.structured_square_mesh(n)
    geo = geometry.build(mesh.vert, mesh.cells, 1)
    for v, fn in (((1.0, 0.4), lambda i, j, up: 2 * i + (0 if up else 1)),
                  ((0.3, 0.9), lambda i, j, up: 2 * j + (1 if up else 0))):
        order, lag = dag.dfs_order(geo, np.array(v))
        gen = dag.generations(geo, np.array(v), lag, order)
        for i in range(n):
            for j in range(n):
                c = 2 * (i * n + j)
                assert gen[c] == fn(i, j, False)
                assert gen[c + 1] == fn(i, j, True)


def random_lagged_set(geo, V, frac, seed):
    """Mark a random subset of each velocity's interior inflow facets as lagged.

    Any subset of in-edges may be lagged (Sec. 4: the lagged part of the
    inflow boundary is a free partition); removing edges keeps the graph
    acyclic."""
    rng = np.random.default_rng(seed)
    lag = np.zeros((V.shape[0], geo.n_cells, geo.dim + 1), dtype=bool)
    for j in range(V.shape[0]):
        s = dag.facet_speeds(geo, V[j])
        cand = (s < 0) & (geo.nbr >= 0)
        lag[j] = cand & (rng.uniform(size=cand.shape) < frac)
    return lag


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1)])
def test_lagged_sweep_equals_dense_with_lagged_inflow(dim, order):
    pr = P.small_problem(dim=dim, order=order, n_side=3, n_1d=4)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, order)
    V = pr.vgrid.v
    lags = random_lagged_set(geo, V, 0.3, 4)
    gens, _ = dag.build_all(geo, V, lagged=lags)
    sig, nu, Mv, q, gbc = _random_inputs(geo, V.shape[0], 5)
    f_prev = np.random.default_rng(9).uniform(0, 1, (geo.n_cells, geo.n_p, V.shape[0]))
    f = transport.sweep(geo, V, sig, nu, Mv, q, gbc, gens, lags, f_prev)
    for j in range(V.shape[0]):
        fd = transport.dense_solve(geo, V[j], sig, nu, Mv[:, :, j], q[:, :, j], gbc[:, :, j],
                                   lags[j], f_prev[:, :, j])
        assert np.abs(fd - f[:, :, j]).max() <= 1e-13 * np.abs(fd).max()
        np.testing.assert_array_equal(gens[j], _brute_longest(geo, V[j], lags[j]))


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1)])
def test_uniform_data_closed_form(dim, order):
    pr = P.small_problem(dim=dim, order=order, n_side=3, n_1d=4)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, order)
    V = pr.vgrid.v
    nv = V.shape[0]
    gens, _ = dag.build_all(geo, V)
    rng = np.random.default_rng(2)
    mj, qj = rng.uniform(0, 1, nv), rng.uniform(0, 1, nv)
    sigma, nu = 1.7, 0.4
    Mv = np.broadcast_to(mj, (geo.n_cells, geo.n_p, nv)).copy()
    q = np.broadcast_to(qj, Mv.shape).copy()
    exact = (nu * mj + qj) / sigma
    gbc = np.broadcast_to(exact, (geo.bnode_x.shape[0], geo.n_fp, nv)).copy()
    f = transport.sweep(geo, V, np.full((geo.n_cells, geo.n_p), sigma),
                        np.full((geo.n_cells, geo.n_p), nu), Mv, q, gbc, gens)
    assert np.abs(f - exact).max() <= 1e-14 * exact.max() * 4


def _manufactured_error(dim, order, n_side, v):
    """Steady v.grad f + sigma f = s with f_ex smooth, inflow = f_ex; L2 error."""
    if dim == 2:
        mesh = P.jittered_square_mesh(n_side, 0.2, 40 + n_side)
        fex = lambda x: np.sin(1.3 * x[:, 0] + 0.4) * np.cos(0.9 * x[:, 1]) + 2.0  # noqa: E731
        grad = lambda x: np.stack([1.3 * np.cos(1.3 * x[:, 0] + 0.4) * np.cos(0.9 * x[:, 1]),  # noqa: E731
                                   -0.9 * np.sin(1.3 * x[:, 0] + 0.4) * np.sin(0.9 * x[:, 1])], 1)
    else:
        mesh = P.jittered_cube_mesh(n_side, 0.15, 40 + n_side)
        fex = lambda x: np.sin(x[:, 0] + 0.5 * x[:, 1]) + np.cos(0.7 * x[:, 2]) + 2.0  # noqa: E731
        grad = lambda x: np.stack([np.cos(x[:, 0] + 0.5 * x[:, 1]),  # noqa: E731
                                   0.5 * np.cos(x[:, 0] + 0.5 * x[:, 1]),
                                   -0.7 * np.sin(0.7 * x[:, 2])], 1)
    geo = geometry.build(mesh.vert, mesh.cells, order)
    v = np.asarray(v, dtype=float)
    sigma = 1.0
    xs = geo.node_x.reshape(-1, dim)
    src = (grad(xs) @ v + sigma * fex(xs)).reshape(geo.n_cells, geo.n_p, 1)
    gbc = fex(geo.bnode_x.reshape(-1, dim)).reshape(-1, geo.n_fp, 1)
    order_, lag = dag.dfs_order(geo, v)
    gens = dag.generations(geo, v, lag, order_)[None]
    f = transport.sweep(geo, v[None], np.full((geo.n_cells, geo.n_p), sigma),
                        np.zeros((geo.n_cells, geo.n_p)), np.zeros_like(src), src, gbc, gens)
    e = f[:, :, 0] - fex(xs).reshape(geo.n_cells, geo.n_p)
    err2 = np.einsum("c,cp,pq,cq->", geo.vol, e, geo.ref["mass"], e)
    return math.sqrt(err2)


@pytest.mark.parametrize("dim,order,sides,min_slope", [
    (2, 1, (4, 8, 16, 32), 1.8), (2, 2, (4, 8, 16, 32), 2.8), (3, 1, (2, 4, 8), 1.7)])
def test_free_streaming_convergence_order(dim, order, sides, min_slope):
    v = (1.0, 0.7) if dim == 2 else (1.0, 0.6, 0.3)
    errs = [_manufactured_error(dim, order, n, v) for n in sides]
    slopes = [math.log(errs[i] / errs[i + 1], 2) for i in range(len(errs) - 1)]
    assert slopes[-1] >= min_slope, (errs, slopes)
