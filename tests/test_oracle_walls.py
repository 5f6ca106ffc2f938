"""Oracle pins: bounce-back and reflecting walls (Sec. "Boundary conditions").

* Maps: on a tensor grid symmetric about 0 (first axis slowest), -v is the
  reversed index and the reflection about axis a reverses tensor index a.
* Wall-flux identities (the proposition on bounce-back and reflection
  moments, at the discrete level): with wall data taken from f itself, the
  upwind mass flux through every wall facet node vanishes, and so does the
  energy flux; a wrong map, weight or node breaks it.
* A uniform Maxwellian drifting parallel to reflecting walls is an exact
  steady state (its reflection is itself); one drifting across them is not.
* A closed box (walls only) conserves total mass and energy over converged
  steps, for reflection, bounce-back and a mix, in 2D and 3D.
* In a reflecting box the phase-space L2 norm does not grow under B-stable
  schemes for streaming and the linear Maxwellian (Prop. linear stability).
"""
import numpy as np
import pytest

import problems as P
from oracle import dag, geometry, kinetic, solver, walls


@pytest.mark.parametrize("n1,dim", [(4, 2), (5, 2), (4, 3)])
def test_wall_maps_are_index_reversals_on_symmetric_tensor_grids(n1, dim):
    vg = P.tensor_velocity_grid(n1, 3.0, dim)
    V = vg.v
    nv = V.shape[0]
    np.testing.assert_array_equal(walls.wall_map(V, None, walls.BOUNCE_BACK),
                                  np.arange(nv)[::-1])
    idx = np.stack(np.unravel_index(np.arange(nv), (n1,) * dim), axis=1)
    for a in range(dim):
        nrm = np.zeros(dim)
        nrm[a] = -1.0 if a % 2 else 1.0
        ref = idx.copy()
        ref[:, a] = n1 - 1 - ref[:, a]
        np.testing.assert_array_equal(walls.wall_map(V, nrm, walls.REFLECT),
                                      np.ravel_multi_index(ref.T, (n1,) * dim))
    gl = P.gl_velocity_grid(3, 3.0, dim)
    np.testing.assert_array_equal(walls.wall_map(gl.v, None, walls.BOUNCE_BACK),
                                  np.arange(gl.v.shape[0])[::-1])
    with pytest.raises(ValueError):
        walls.wall_map(V + 0.1, None, walls.BOUNCE_BACK)


def _box(dim, order=1, n_side=3):
    if dim == 2:
        mesh = P.jittered_square_mesh(n_side, 0.25, 5)
    else:
        mesh = P.jittered_cube_mesh(n_side, 0.2, 5)
    return geometry.build(mesh.vert, mesh.cells, order), mesh


@pytest.mark.parametrize("dim,order,kind", [(2, 1, walls.REFLECT), (2, 2, walls.BOUNCE_BACK),
                                            (3, 1, walls.REFLECT), (3, 1, walls.BOUNCE_BACK)])
def test_wall_flux_identities_with_data_from_f(dim, order, kind):
    geo, _ = _box(dim, order)
    vg = P.tensor_velocity_grid(6 if dim == 2 else 4, 4.0, dim)
    V, w = vg.v, vg.w
    rng = np.random.default_rng(3)
    f = rng.uniform(0.1, 1.0, (geo.n_cells, geo.n_p, V.shape[0]))
    kinds = np.full(geo.bnode_x.shape[0], kind, dtype=np.int8)
    g = walls.wall_values(geo, V, f, kinds, np.zeros((geo.bnode_x.shape[0], geo.n_fp, V.shape[0])))
    e2 = 0.5 * np.sum(V * V, axis=1)
    checked = 0
    for c in range(geo.n_cells):
        for k in range(dim + 1):
            bf = geo.bface[c, k]
            if bf < 0:
                continue
            s = V @ geo.normal[c, k]
            fn = geo.ref["face_nodes"][k]
            fhat = np.where(s[None, :] > 0, f[c, fn, :], g[bf])
            scale = np.abs(w * s * fhat).sum(axis=1).max()
            assert np.abs(fhat @ (w * s)).max() <= 1e-13 * scale
            assert np.abs(fhat @ (w * s * e2)).max() <= 1e-13 * scale * e2.max()
            checked += 1
    assert checked == geo.bnode_x.shape[0]


def _strip_walls(geo):
    return walls.boundary_kinds(geo, lambda x, n: walls.REFLECT if abs(n[1]) > 0.5 else
                                walls.INFLOW)


@pytest.mark.parametrize("u", [(0.4, 0.0), (0.0, 0.4)])
def test_drift_parallel_to_reflecting_walls_is_steady(u):
    mesh = P.rectangle_mesh(6, 2, 0.0, 1.0, 0.0, 0.2)
    geo = geometry.build(mesh.vert, mesh.cells, 1)
    vg = P.tensor_velocity_grid(8, 5.0, 2)
    V, w = vg.v, vg.w
    st = P.uniform_state(1.1, (*u, 0.0), 0.9, dim=2)
    kinds = _strip_walls(geo)
    assert (kinds == walls.REFLECT).sum() == 12
    gens, lags = dag.build_all(geo, V)
    f0 = solver.initial_condition(geo, V, st)
    g = solver.boundary_values(geo, V, st)
    f1, _ = solver.bgk_step(geo, V, w, f0, g, 0.05, gens, lags, nu_const=2.0, tau=1e-13,
                            walls=kinds)
    err = np.abs(f1 - f0).max() / np.abs(f0).max()
    if u[1] == 0.0:
        assert err <= 1e-12
    else:                       # drift through the walls: the reflection changes it
        assert err > 1e-3


@pytest.mark.parametrize("dim,scheme,rule", [
    (2, "BE", "reflect"), (2, "DIRK2", "bounce"), (2, "BE", "mixed"), (3, "BE", "reflect")])
def test_closed_box_conserves_mass_and_energy(dim, scheme, rule):
    geo, _ = _box(dim, 1, 3 if dim == 2 else 2)
    vg = P.tensor_velocity_grid(8 if dim == 2 else 5, 4.0, dim)
    V, w = vg.v, vg.w
    st = P.planar_riemann_state(dim, 12, width=0.3)
    choose = {"reflect": lambda x, n: walls.REFLECT,
              "bounce": lambda x, n: walls.BOUNCE_BACK,
              "mixed": lambda x, n: walls.REFLECT if abs(n[0]) > 0.5 else walls.BOUNCE_BACK}
    kinds = walls.boundary_kinds(geo, choose[rule])
    gens, lags = dag.build_all(geo, V)
    f = solver.initial_condition(geo, V, st)
    g = solver.boundary_values(geo, V, st)        # unused: every facet is a wall
    dt = solver.explicit_dt(geo, V, 10.0)
    E = kinetic.collision_invariants(V) * w[:, None]
    tot = lambda f: np.einsum("c,pq,cqj,jm->m", geo.vol, geo.ref["mass"], f, E)  # noqa: E731
    t0 = tot(f)
    for _ in range(2):
        f, _ = solver.bgk_step(geo, V, w, f, g, dt, gens, lags, scheme=scheme, nu_const=5.0,
                               tau=1e-13, walls=kinds)
    t1 = tot(f)
    assert abs(t1[0] - t0[0]) <= 1e-10 * t0[0]                 # mass
    assert abs(t1[-1] - t0[-1]) <= 1e-10 * t0[-1]              # energy
    # momentum is not conserved: the walls push back
    assert np.abs(t1[1:-1] - t0[1:-1]).max() > 1e-6 * t0[0]


@pytest.mark.parametrize("mode,nu,scheme", [("MATCHED", 0.0, "BE"), ("LINEAR", 5.0, "BE"),
                                            ("LINEAR", 5.0, "BDIRK2"), ("MATCHED", 0.0, "BDIRK2")])
def test_l2_norm_does_not_grow_in_a_reflecting_box(mode, nu, scheme):
    """Prop. linear stability with walls: specular reflection returns through
    the boundary exactly the |v.n| f^2 that leaves (the velocity set is
    closed under the map, with equal weights), so for streaming (nu = 0) or
    the linear Maxwellian a B-stable scheme cannot increase the phase-space
    L2 norm."""
    geo, _ = _box(2, 1, 3)
    vg = P.tensor_velocity_grid(8, 4.0, 2)
    V, w = vg.v, vg.w
    st = P.planar_riemann_state(2, 12, width=0.3)
    kinds = np.full(geo.bnode_x.shape[0], walls.REFLECT, dtype=np.int8)
    gens, lags = dag.build_all(geo, V)
    f = solver.initial_condition(geo, V, st)
    g = solver.boundary_values(geo, V, st)
    dt = solver.explicit_dt(geo, V, 10.0)
    norm = lambda f: np.einsum("c,cpj,pq,cqj,j->", geo.vol, f, geo.ref["mass"], f, w)  # noqa: E731
    prev = norm(f)
    for _ in range(3):
        f, _ = solver.bgk_step(geo, V, w, f, g, dt, gens, lags, scheme=scheme, mode=mode,
                               nu_const=nu, L=vg.L, tau=1e-13, walls=kinds)
        cur = norm(f)
        assert cur <= prev * (1 + 1e-12)
        prev = cur
