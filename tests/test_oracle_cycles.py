"""Oracle pins: cycle breaking by DFS back edges (Sec. 4.1, design note A10).

On a non-Delaunay tetrahedral mesh the upwind graph of a velocity can have
cycles; the oracle's DFS lags every back edge (an edge into a cell still on
the stack), and the downwind cell takes that facet's inflow from the
previous Picard iterate.  These tests check that rule against facts that do
not come from the DFS itself, on the committed cyclic mesh (golden fixture):

* the strongly connected components (SciPy, an independent algorithm) say
  which velocities have cycles; the DFS lags something exactly there;
* every lagged facet is an interior inflow facet of the cell that lags it,
  and the edge it carries lies on a cycle (its downwind cell reaches its
  upwind cell in the full graph);
* the graph without the lagged edges is acyclic (SciPy again), and the
  generations are its longest paths (brute-force relaxation);
* the sweep with the lagged facets equals a dense global solve in which the
  lagged facets take the previous iterate;
* a converged step does not depend on which valid set of edges is lagged.
"""
import os

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import breadth_first_order, connected_components

import problems as P
from oracle import dag, geometry, solver, transport

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cyclic_mesh():
    return P.load_mesh_text(os.path.join(GOLDEN, "cyclic_tet_mesh.txt"))


def _edges(geo, v, lagged=None):
    """Directed edges (a, b) with a upwind of b across an interior facet."""
    s = dag.facet_speeds(geo, v)
    b, k = np.nonzero((geo.nbr >= 0) & (s < 0))     # b's inflow facets
    a = geo.nbr[b, k]
    if lagged is not None:
        keep = ~lagged[b, k]
        a, b, k = a[keep], b[keep], k[keep]
    return a, b, k


def _graph(n, a, b):
    return coo_matrix((np.ones(len(a)), (a, b)), shape=(n, n)).tocsr()


def _acyclic(n, a, b):
    ncomp, _ = connected_components(_graph(n, a, b), directed=True, connection="strong")
    return ncomp == n


def _brute_longest(geo, v, lagged):
    a, b, _ = _edges(geo, v, lagged)
    gen = np.zeros(geo.n_cells, dtype=np.int64)
    for _ in range(geo.n_cells + 1):
        new = gen.copy()
        np.maximum.at(new, b, gen[a] + 1)
        if np.array_equal(new, gen):
            return gen
        gen = new
    raise AssertionError("no fixed point: the graph has a cycle")


@pytest.fixture(scope="module")
def setup():
    m = cyclic_mesh()
    geo = geometry.build(m.vert, m.cells, 1)
    vg = P.tensor_velocity_grid(6, 6.0, 3)
    return geo, vg


def test_fixture_is_a_valid_tiling(setup):
    geo, _ = setup
    assert geo.n_cells == 218
    assert abs(geo.vol.sum() - 1.0) < 1e-12
    assert geo.vol.min() > 0
    # every facet interior or on the cube's boundary
    bx = geo.bnode_x.reshape(-1, 3)
    on_face = np.any(np.isclose(bx, 0.0) | np.isclose(bx, 1.0), axis=1)
    assert on_face.all()


def test_dfs_lags_exactly_where_cycles_are(setup):
    geo, vg = setup
    n_cyclic = 0
    for v in vg.v:
        a, b, _ = _edges(geo, v)
        cyclic = not _acyclic(geo.n_cells, a, b)
        order, lag = dag.dfs_order(geo, v)
        assert lag.any() == cyclic
        n_cyclic += cyclic
    assert n_cyclic == 62


def test_lagged_edges_lie_on_cycles_and_break_them(setup):
    geo, vg = setup
    n_lagged = 0
    for v in vg.v:
        order, lag = dag.dfs_order(geo, v)
        if not lag.any():
            continue
        s = dag.facet_speeds(geo, v)
        a_all, b_all, _ = _edges(geo, v)
        G = _graph(geo.n_cells, a_all, b_all)
        for b, k in zip(*np.nonzero(lag)):
            assert geo.nbr[b, k] >= 0 and s[b, k] < 0      # an interior inflow facet of b
            a = geo.nbr[b, k]
            reach = breadth_first_order(G, b, directed=True, return_predecessors=False)
            assert a in reach                                # b ~> a: a -> b closes a cycle
            n_lagged += 1
        a, b, _ = _edges(geo, v, lag)
        assert _acyclic(geo.n_cells, a, b)
        gen = dag.generations(geo, v, lag, order)
        np.testing.assert_array_equal(gen, _brute_longest(geo, v, lag))
        pos = np.empty(geo.n_cells, dtype=np.int64)
        pos[np.asarray(order)] = np.arange(geo.n_cells)
        assert np.all(pos[a] < pos[b])                       # the DFS order is topological
    assert n_lagged > 62


def test_sweep_with_back_edges_equals_dense_solve(setup):
    geo, vg = setup
    V = vg.v
    gens, lags = dag.build_all(geo, V)
    assert lags.any()
    rng = np.random.default_rng(17)
    nv = V.shape[0]
    sig = rng.uniform(1.0, 3.0, (geo.n_cells, geo.n_p))
    nu = rng.uniform(0.0, 1.0, sig.shape)
    Mv = rng.uniform(0.0, 1.0, (geo.n_cells, geo.n_p, nv))
    q = rng.uniform(0.0, 1.0, Mv.shape)
    gbc = rng.uniform(0.0, 1.0, (geo.bnode_x.shape[0], geo.n_fp, nv))
    f_prev = rng.uniform(0.0, 1.0, Mv.shape)
    f = transport.sweep(geo, V, sig, nu, Mv, q, gbc, gens, lags, f_prev)
    for j in np.nonzero(lags.reshape(nv, -1).any(axis=1))[0][:12]:
        fd = transport.dense_solve(geo, V[j], sig, nu, Mv[:, :, j], q[:, :, j], gbc[:, :, j],
                                   lags[j], f_prev[:, :, j])
        assert np.abs(fd - f[:, :, j]).max() <= 1e-13 * np.abs(fd).max()
        # f_prev really enters: changing it at a lagged facet's upwind cell moves f
        b, k = [int(x) for x in np.argwhere(lags[j])[0]]
        fp2 = f_prev[:, :, j].copy()
        fp2[geo.nbr[b, k]] += 1.0
        fd2 = transport.dense_solve(geo, V[j], sig, nu, Mv[:, :, j], q[:, :, j], gbc[:, :, j],
                                    lags[j], fp2)
        assert np.abs(fd2[b] - fd[b]).max() > 1e-6


def _scc_lag_set(geo, V):
    """Another valid lagged set: every in-edge of a cell from another cell of
    its own strongly connected component (a superset of what is needed)."""
    lags = np.zeros((V.shape[0], geo.n_cells, geo.dim + 1), dtype=bool)
    for j, v in enumerate(V):
        a, b, k = _edges(geo, v)
        _, lab = connected_components(_graph(geo.n_cells, a, b), directed=True,
                                      connection="strong")
        same = lab[a] == lab[b]
        lags[j, b[same], k[same]] = True
    return lags


@pytest.mark.parametrize("mode,n1", [("DIRECT", 4), ("MATCHED", 8)])
def test_converged_step_does_not_depend_on_the_lagged_set(setup, mode, n1):
    """(MATCHED runs on a grid fine enough that no node falls back to DIRECT:
    a held fallback depends on the iterates, so with fallbacks two lagged
    sets can settle on different fixed points.)"""
    geo, _ = setup
    vg = P.tensor_velocity_grid(n1, 6.0, 3)
    V, w = vg.v, vg.w
    st = P.planar_riemann_state(3, seed=5, width=0.15)
    f0 = solver.initial_condition(geo, V, st)
    g = solver.boundary_values(geo, V, st)
    dt = solver.explicit_dt(geo, V, 10.0)
    gens0, lag0 = dag.build_all(geo, V)
    alt = _scc_lag_set(geo, V)
    assert alt.sum() > lag0.sum() > 0
    gens1, lag1 = dag.build_all(geo, V, lagged=alt)
    f_a, st_a = solver.bgk_step(geo, V, w, f0, g, dt, gens0, lag0, tau=1e-13, mode=mode, L=6.0)
    f_b, st_b = solver.bgk_step(geo, V, w, f0, g, dt, gens1, lag1, tau=1e-13, mode=mode, L=6.0)
    assert st_a["fallbacks"] == 0 and st_b["fallbacks"] == 0
    assert st_b["iters"][0] > st_a["iters"][0]        # more lagging, slower iteration
    assert np.abs(f_b - f_a).max() <= 1e-10 * np.abs(f_a).max()
