"""Degenerate inputs of the method and invalid inputs of the C ABI.

One-cell meshes (every facet on the boundary), a single velocity, velocities
exactly tangential to facets (v.n = 0 gives no DAG edge) including v = 0
(every cell its own generation 0), checked against the oracle; and the
errors build_mesh_dag reports for malformed meshes and velocity sets."""
import numpy as np
import pytest

import problems as P
from oracle import dag as odag
from oracle import geometry, kinetic, solver, transport

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2608_19150_amd as B

TOL64 = 1e-12


def rel(x, ref):
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def _inputs(geo, nv, seed):
    rng = np.random.default_rng(seed)
    q = rng.uniform(0.0, 1.0, (geo.n_cells, geo.n_p, nv))
    nu = rng.uniform(0.1, 2.0, (geo.n_cells, geo.n_p))
    prim = np.concatenate([rng.uniform(0.2, 1.5, (geo.n_cells, geo.n_p, 1)),
                           rng.uniform(-0.5, 0.5, (geo.n_cells, geo.n_p, geo.dim)),
                           rng.uniform(0.6, 1.4, (geo.n_cells, geo.n_p, 1))], axis=-1)
    return q, nu, prim


def _check_sweep(pr, d, seed, shift=9.0, qscale=2.0):
    """GPU sweep through the C ABI against the oracle sweep."""
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    V = pr.vgrid.v
    q, nu, prim = _inputs(geo, V.shape[0], seed)
    gen, _ = d.generations()
    ogen, olag = odag.build_all(geo, V)
    np.testing.assert_array_equal(gen, ogen)
    mcoef = B.maxwellian_coef_from_primitive(B._dev(prim.reshape(-1, geo.dim + 2)), geo.dim)
    bc = B.state_coefficients(d, pr.state, "boundary")
    qg = d.pack(B._dev(q))
    fo = torch.empty_like(qg)
    B.tgs_sweep(d, q=qg, nu=B._dev(nu.reshape(-1)), mcoef=mcoef, f_out=fo, sigma_shift=shift,
                q_scale=qscale, bc_coef=bc)
    f_gpu = d.unpack(fo).cpu().numpy()
    coef = kinetic.direct_coefficients(prim[..., 0], prim[..., 1:-1], prim[..., -1])
    Mv = kinetic.coef_values(coef, V)
    g = solver.boundary_values(geo, V, pr.state)
    f_ref = transport.sweep(geo, V, nu + shift, nu, Mv, qscale * q, g, ogen, olag)
    assert rel(f_gpu, f_ref) <= TOL64
    return geo, ogen


ONE_CELL = {
    2: (np.array([[0.0, 0.0], [1.0, 0.1], [0.3, 0.8]]), np.array([[0, 1, 2]], dtype=np.int32)),
    3: (np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1], [0.3, 0.2, 0.8]]),
        np.array([[0, 1, 2, 3]], dtype=np.int32)),
}


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1)])
def test_one_cell_mesh_sweep_and_step_match_oracle(dim, order):
    vert, cells = ONE_CELL[dim]
    # smooth data: a Sod jump inside one P2 cell makes a nodal density
    # non-positive, which the method (no limiter) rejects
    pr = P.Problem(P.Mesh(vert, cells), order, P.tensor_velocity_grid(4, 6.0, dim),
                   P.fourier_state(dim, 11))
    d = B.Dag.from_problem(pr)
    geo, ogen = _check_sweep(pr, d, 1)
    assert geo.n_cells == 1 and (ogen == 0).all()
    # a whole backward-Euler step (constant nu, three Picard iterations)
    d2, f, bc, dt = B.problem_setup(pr)
    s = B.Solver(d2, dt=dt, bc_coef=bc, fixed_iters=3)
    s.step(f)
    V, w = pr.vgrid.v, pr.vgrid.w
    gens, lags = odag.build_all(geo, V)
    f0 = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    fref, _ = solver.bgk_step(geo, V, w, f0, g, dt, gens, lags, fixed_iters=3)
    assert rel(d2.unpack(f).cpu().numpy(), fref) <= TOL64


def test_single_velocity_sweep_and_moments_match_oracle():
    base = P.small_problem(dim=2, order=2, n_side=4, n_1d=4)
    V = np.array([[0.7, -0.4]])
    W = np.array([1.5])
    pr = P.Problem(base.mesh, 2, P.VelocityGrid(V, W), base.state)
    d = B.Dag(pr.mesh.vert, pr.mesh.cells, 2, V, W)
    _check_sweep(pr, d, 2)
    f = np.random.default_rng(3).uniform(0, 1, d.f_shape)
    U = B.moments(d, d.pack(B._dev(f))).cpu().numpy().reshape(d.n_cells, d.n_p, -1)
    assert rel(U, kinetic.moments(f, V, W)) <= TOL64


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1)])
def test_tangential_velocities_and_zero_velocity_match_oracle(dim, order):
    """An odd tensor grid holds v = 0, tangential to every facet.  In 2D the
    mesh is the unperturbed lattice, whose axis-aligned and diagonal edges
    are also exactly tangential to families of velocities (a 3D lattice has
    no non-degenerate Delaunay tetrahedrisation, so 3D keeps its jitter)."""
    pr = P.small_problem(dim=dim, order=order, n_side=4 if dim == 2 else 3,
                         n_1d=5 if dim == 2 else 3, jitter=0.0 if dim == 2 else 0.2)
    V = pr.vgrid.v
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    zero = int(np.flatnonzero(np.all(V == 0.0, axis=1))[0])
    tangential = 0
    for j in range(V.shape[0]):
        s = odag.facet_speeds(geo, V[j])
        tangential += int(((s == 0.0) & (geo.nbr >= 0)).sum())
    assert tangential > 0
    if dim == 2:
        assert tangential > 2 * int((geo.nbr >= 0).sum())   # beyond v = 0 alone
    d = B.Dag.from_problem(pr)
    _, ogen = _check_sweep(pr, d, 4)
    assert (ogen[zero] == 0).all()


def _mesh_error(vert, cells, order=1, dim=2, v=None, w=None):
    v = np.array([[0.5] * dim]) if v is None else v
    w = np.array([1.0]) if w is None else w
    with pytest.raises(B.BGKError) as e:
        B.Dag(np.asarray(vert, dtype=np.float64), np.asarray(cells, dtype=np.int32), order, v, w)
    return e.value.code


def test_build_mesh_dag_rejects_malformed_input():
    good_v = [[0, 0], [1, 0], [0, 1], [1, 1]]
    assert _mesh_error(good_v, np.zeros((0, 3))) == B.BGK_E_INVALID            # no cells
    assert _mesh_error(good_v, [[0, 1, 7]]) == B.BGK_E_INVALID                # vertex id
    assert _mesh_error([[0, 0], [1, 0], [2, 0]], [[0, 1, 2]]) == B.BGK_E_INVALID  # zero area
    assert _mesh_error(good_v, [[0, 1, 1]]) == B.BGK_E_INVALID                # repeated vertex
    # a facet shared by three cells
    fan_v = [[0, 0], [1, 0], [0.5, 1], [0.5, -1], [0.5, 0.5]]
    assert _mesh_error(fan_v, [[0, 1, 2], [0, 1, 3], [0, 1, 4]]) == B.BGK_E_INVALID
    assert _mesh_error(good_v, [[0, 1, 2]], order=3) == B.BGK_E_UNSUPPORTED
    cube_v = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]
    assert _mesh_error(cube_v, [[0, 1, 2, 3]], order=2, dim=3) == B.BGK_E_UNSUPPORTED
    assert _mesh_error(good_v, [[0, 1, 2]], v=np.zeros((0, 2)), w=np.zeros(0)) == \
        B.BGK_E_INVALID                                                       # no velocities
