"""Bounce-back and reflecting walls through the C ABI, against the oracle.

The boundary update (wall rows of the dense boundary data gathered from an
iterate at the mapped velocities, for the velocities that can enter) is
compared bit for bit; whole steps with
walls (lagged by one Picard iteration, as in the oracle) within 1e-12; a
closed box conserves mass and energy on the GPU; invalid wall sets are
rejected."""
import sys

import numpy as np
import pytest

import problems as P
from oracle import dag as odag
from oracle import geometry, kinetic, solver, walls as owalls

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2608_19150_amd as B

TOL64 = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(x, ref):
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def _mixed(dim):
    if dim == 2:
        return lambda x, n: owalls.REFLECT if abs(n[1]) > 0.5 else owalls.BOUNCE_BACK
    return lambda x, n: (owalls.REFLECT if abs(n[0]) > 0.5 else
                         owalls.BOUNCE_BACK if abs(n[1]) > 0.5 else owalls.INFLOW)


@pytest.mark.parametrize("dim,order,n1", [(2, 1, 6), (2, 2, 5), (3, 1, 4)])
def test_wall_values_equal_oracle_gather(dim, order, n1):
    say("wall values", dim, order, n1)
    pr = P.small_problem(dim=dim, order=order, n_side=4 if dim == 2 else 3, n_1d=n1)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, order)
    V = pr.vgrid.v
    kinds = owalls.boundary_kinds(geo, _mixed(dim))
    assert (kinds != owalls.INFLOW).any()
    d = B.Dag.from_problem(pr)
    w = B.Walls(d, kinds)
    assert w.n_walls == int((kinds != owalls.INFLOW).sum())
    f = np.random.default_rng(20 + dim + order).uniform(0.0, 1.0, d.f_shape)
    bcd = torch.full((d.n_bfaces, d.n_fp, d.n_v), -7.0, dtype=torch.float64, device="cuda")
    B.wall_values(w, d.pack(B._dev(f)), bcd)
    g = bcd.cpu().numpy()
    ref = owalls.wall_values(geo, V, f, kinds, np.full(g.shape, -7.0))
    # entries of velocities that can enter through the facet (v.n <= 0) are
    # gathered; the others, never read by a sweep, stay untouched
    incoming = np.zeros(g.shape, dtype=bool)
    for c in range(geo.n_cells):
        for k in range(dim + 1):
            bf = geo.bface[c, k]
            if bf >= 0:
                incoming[bf] = (V @ geo.normal[c, k] <= 1e-9 * np.linalg.norm(V, axis=1))[None, :]
    np.testing.assert_array_equal(g[incoming], ref[incoming])
    assert (g[~incoming] == -7.0).all()


def _strip(order, state="sod"):
    mesh = P.rectangle_mesh(10, 3, 0.0, 1.0, 0.0, 0.15)
    st = P.sod_state(2) if state == "sod" else P.fourier_state(2, 3)
    return P.Problem(mesh, order, P.tensor_velocity_grid(8, 5.0, 2), st)


def _strip_kinds(geo):
    return owalls.boundary_kinds(geo, lambda x, n: owalls.REFLECT if abs(n[1]) > 0.5 else
                                 owalls.INFLOW)


def _run_both(pr, kinds, steps, **kw):
    d, f, bc, dt = B.problem_setup(pr)
    w = B.Walls(d, kinds)
    s = B.Solver(d, dt=dt, bc_coef=bc, walls=w, **kw)
    st = [s.step(f) for _ in range(steps)]
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    V, wts = pr.vgrid.v, pr.vgrid.w
    gens, lags = odag.build_all(geo, V)
    fr = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    okw = dict(scheme=kw.get("tableau", "BE"), mode=kw.get("mode", "MATCHED"),
               nu_model=kw.get("nu_model", "const"), nu_const=kw.get("nu_const", 1.0),
               kn=kw.get("kn", 1.0), tau=kw.get("tau", 1e-10),
               fixed_iters=kw.get("fixed_iters") or None)
    ost = []
    for _ in range(steps):
        fr, o = solver.bgk_step(geo, V, wts, fr, g, dt, gens, lags, walls=kinds, **okw)
        ost.append(o["iters"])
    return d.unpack(f).cpu().numpy(), fr, [x["iters"] for x in st], ost, geo


@pytest.mark.parametrize("order,tableau", [(1, "BE"), (2, "DIRK2")])
def test_bgk_step_with_reflecting_walls_matches_oracle(order, tableau):
    say("walls step", order, tableau)
    pr = _strip(order, "sod" if order == 1 else "fourier")
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, order)
    kinds = _strip_kinds(geo)
    f, fr, it, oit, _ = _run_both(pr, kinds, 2, tableau=tableau, fixed_iters=3, nu_const=2.0)
    assert rel(f, fr) <= TOL64


def test_bgk_step_with_walls_converged_matches_oracle():
    pr = _strip(1)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 1)
    kinds = _strip_kinds(geo)
    f, fr, it, oit, _ = _run_both(pr, kinds, 2, tau=1e-10, nu_const=5.0)
    assert it == oit
    assert rel(f, fr) <= TOL64


def test_bgk_step_3d_mixed_walls_matches_oracle():
    say("walls 3d")
    pr = P.small_problem(dim=3, order=1, n_side=3, n_1d=4, state="fourier", nu_model="kn",
                         kn=0.1)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 1)
    kinds = owalls.boundary_kinds(geo, _mixed(3))
    f, fr, _, _, _ = _run_both(pr, kinds, 2, fixed_iters=3, nu_model="kn", kn=0.1)
    assert rel(f, fr) <= TOL64


@pytest.mark.parametrize("kind", [owalls.REFLECT, owalls.BOUNCE_BACK])
def test_closed_box_conserves_mass_and_energy_on_gpu(kind):
    pr = P.Problem(P.jittered_square_mesh(4, 0.25, 5), 1, P.tensor_velocity_grid(8, 4.0, 2),
                   P.planar_riemann_state(2, 12, width=0.3))
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 1)
    kinds = np.full(geo.bnode_x.shape[0], kind, dtype=np.int8)
    d, f, bc, dt = B.problem_setup(pr)
    s = B.Solver(d, dt=dt, bc_coef=bc, walls=B.Walls(d, kinds), tau=1e-13, nu_const=5.0)
    V, w = pr.vgrid.v, pr.vgrid.w
    E = kinetic.collision_invariants(V) * w[:, None]

    def tot():
        fc = d.unpack(f).cpu().numpy()
        return np.einsum("c,pq,cqj,jm->m", geo.vol, geo.ref["mass"], fc, E)

    t0 = tot()
    for _ in range(3):
        s.step(f)
    t1 = tot()
    assert abs(t1[0] - t0[0]) <= 1e-10 * t0[0]
    assert abs(t1[-1] - t0[-1]) <= 1e-10 * t0[-1]


def test_walls_validation():
    pr = _strip(1)
    d = B.Dag.from_problem(pr)
    good = np.zeros(d.n_bfaces, dtype=np.int8)

    def code(fn):
        with pytest.raises(B.BGKError) as e:
            fn()
        return e.value.code

    with pytest.raises(ValueError):
        B.Walls(d, good[:-1])
    bad = good.copy()
    bad[0] = 5
    assert code(lambda: B.Walls(d, bad)) == B.BGK_E_INVALID
    # a velocity set not closed under -v
    shifted = B.Dag(pr.mesh.vert, pr.mesh.cells, 1, pr.vgrid.v + 0.1, pr.vgrid.w)
    assert code(lambda: B.Walls(shifted, np.ones(shifted.n_bfaces, dtype=np.int8))) == \
        B.BGK_E_INVALID
    # walls of another DAG, and batched stepping with walls
    d2, f0, bc, dt = B.problem_setup(pr)
    other = B.Walls(d, good)
    assert code(lambda: B.Solver(d2, dt=dt, bc_coef=bc, walls=other)) == B.BGK_E_INVALID
    s = B.Solver(d2, dt=dt, bc_coef=bc, walls=B.Walls(d2, good))
    assert code(lambda: B.Batch([s])) == B.BGK_E_UNSUPPORTED


@pytest.mark.parametrize("mode,nu,tableau", [("MATCHED", 0.0, "BE"), ("LINEAR", 50.0, "BE"),
                                             ("LINEAR", 50.0, "BDIRK2"),
                                             ("MATCHED", 0.0, "BDIRK2")])
def test_l2_norm_does_not_grow_in_a_reflecting_box_on_gpu(mode, nu, tableau):
    """Prop. linear stability: in a closed reflecting box the boundary terms
    cancel, so B-stable steps of streaming or the linear Maxwellian do not
    increase the phase-space L2 norm."""
    pr = P.Problem(P.jittered_square_mesh(8, 0.25, 9), 1, P.tensor_velocity_grid(10, 5.0, 2),
                   P.planar_riemann_state(2, 13, width=0.2))
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 1)
    d, f, bc, dt = B.problem_setup(pr)
    s = B.Solver(d, dt=dt, bc_coef=bc, tableau=tableau, tau=1e-13, mode=mode, nu_const=nu,
                 walls=B.Walls(d, np.full(d.n_bfaces, owalls.REFLECT, dtype=np.int8)))
    w = pr.vgrid.w

    def norm():
        fc = d.unpack(f).cpu().numpy()
        return np.einsum("c,cpj,pq,cqj,j->", geo.vol, fc, geo.ref["mass"], fc, w)

    prev = norm()
    for _ in range(4):
        s.step(f)
        cur = norm()
        assert cur <= prev * (1 + 1e-12)
        prev = cur


def test_bgk_step_with_walls_and_lagged_facets_matches_oracle():
    """Walls on a DAG with lagged facets: the solver keeps the previous
    iterate in a second buffer, and the wall data come from it."""
    pr = _strip(1)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 1)
    V, w = pr.vgrid.v, pr.vgrid.w
    kinds = _strip_kinds(geo)
    rng = np.random.default_rng(31)
    lag = np.zeros((V.shape[0], geo.n_cells), dtype=np.uint8)
    lags = np.zeros((V.shape[0], geo.n_cells, 3), dtype=bool)
    for j in range(V.shape[0]):
        sp = odag.facet_speeds(geo, V[j])
        pick = (sp < 0) & (geo.nbr >= 0) & (rng.uniform(size=sp.shape) < 0.3)
        lags[j] = pick
        lag[j] = (pick * (1 << np.arange(3))[None, :]).sum(axis=1)
    d, f, bc, dt = B.problem_setup(pr, lagged=lag)
    assert d.n_lagged > 0
    s = B.Solver(d, dt=dt, bc_coef=bc, walls=B.Walls(d, kinds), fixed_iters=3, nu_const=2.0)
    for _ in range(2):
        s.step(f)
    gens, olags = odag.build_all(geo, V, lagged=lags)
    np.testing.assert_array_equal(olags, lags)
    fr = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    for _ in range(2):
        fr, _ = solver.bgk_step(geo, V, w, fr, g, dt, gens, olags, nu_const=2.0, fixed_iters=3,
                                walls=kinds)
    assert rel(d.unpack(f).cpu().numpy(), fr) <= TOL64
