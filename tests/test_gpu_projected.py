"""The Q2 velocity space and the conservative projection of the Maxwellian
(Sec. 3.2, App. B) through the C ABI, against the oracle.

The projected Maxwellian of seeded moments (including drifts that put mass
in the extended first and last cells) matches the oracle's erf closed forms
and reproduces the moments exactly; whole steps in PROJECTED mode match the
oracle's Picard iteration with the projected Maxwellian; malformed Q2 grids
and modes that need one are rejected."""
import sys

import numpy as np
import pytest

import problems as P
from oracle import dag as odag
from oracle import geometry, kinetic, solver, velocity

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


def _gl_problem(dim, order, n_side, vcells, L=6.0, state="fourier", **kw):
    base = P.small_problem(dim=dim, order=order, n_side=n_side, n_1d=4, state=state)
    return P.Problem(base.mesh, order, P.gl_velocity_grid(vcells, L, dim), base.state, **kw)


def _moments_of(prim, dim):
    n, u, th = prim[:, 0], prim[:, 1:-1], prim[:, -1]
    return np.concatenate([n[:, None], n[:, None] * u,
                           (0.5 * n * (dim * th + np.sum(u * u, axis=1)))[:, None]], axis=1)


def _seeded_prim(n_nodes, dim, seed, L):
    rng = np.random.default_rng(seed)
    prim = np.concatenate([rng.uniform(0.2, 1.5, (n_nodes, 1)),
                           rng.uniform(-0.5 * L, 0.5 * L, (n_nodes, dim)),
                           rng.uniform(0.3, 2.0, (n_nodes, 1))], axis=1)
    # a few nodes drifting to the edge of the box: their Gaussians reach far
    # into the extended first and last cells
    prim[:4, 1] = [0.97 * L, -0.97 * L, 0.9 * L, -0.6 * L]
    prim[:4, -1] = [1.0, 2.0, 3.0, 0.5]
    return prim


# vcells = 1: the only cell is both the first and the last (extended to
# both infinities); vcells = 2: every cell is an end cell
@pytest.mark.parametrize("dim,order,vcells", [(2, 1, 5), (2, 2, 4), (3, 1, 3), (2, 1, 1),
                                              (3, 1, 2)])
def test_projected_maxwellian_matches_oracle_and_conserves_moments(dim, order, vcells):
    say("projected maxwellian", dim, order, vcells)
    L = 6.0
    pr = _gl_problem(dim, order, 3, vcells, L)
    d = B.Dag.from_problem(pr)
    assert d.dg_cells == vcells and d.n_v == (3 * vcells) ** dim
    prim = _seeded_prim(d.n_nodes, dim, 40 + dim + order, L)
    U = _moments_of(prim, dim)
    coef, nu, Md, status = B.maxwellian(d, B._dev(U), mode="PROJECTED", nu_model="kn", kn=0.1,
                                        dense=True)
    assert int(status[0]) == 0 and int(status[1]) == 0
    # the coefficients are the primitive variables
    assert rel(coef.cpu().numpy(), prim) <= 1e-13
    M = Md.cpu().numpy()
    ref = velocity.projected_maxwellian(prim[:, 0], prim[:, 1:-1], prim[:, -1], vcells, L)
    assert rel(M, ref) <= TOL64
    # exact conservation (App. B): the discrete moments of P M equal U
    V, w = pr.vgrid.v, pr.vgrid.w
    Um = kinetic.moments(M[:, None, :], V, w)[:, 0, :]
    assert np.abs(Um - U).max() <= 1e-12 * np.abs(U).max()
    np.testing.assert_allclose(nu.cpu().numpy(),
                               kinetic.collision_frequency(U, dim, "kn", kn=0.1), rtol=1e-14)


# a Sod jump inside P2 cells makes nodal densities non-positive (no
# limiter), so the P2 case runs the smooth Fourier state
@pytest.mark.parametrize("dim,order,tableau,nu_model,state", [(2, 1, "BE", "const", "sod"),
                                                              (2, 2, "DIRK2", "kn", "fourier"),
                                                              (3, 1, "BE", "kn", "sod")])
def test_bgk_step_projected_fixed_iterations_matches_oracle(dim, order, tableau, nu_model, state):
    say("bgk_step projected", dim, order, tableau, nu_model, state)
    vcells = 4 if dim == 2 else 3
    pr = _gl_problem(dim, order, 4 if dim == 2 else 3, vcells, state=state, nu_model=nu_model,
                     kn=0.1, tableau=tableau)
    d, f, bc, dt = B.problem_setup(pr)
    s = B.Solver(d, dt=dt, bc_coef=bc, tableau=tableau, fixed_iters=3, mode="PROJECTED",
                 nu_model=nu_model, nu_const=1.0, kn=0.1)
    for _ in range(2):
        s.step(f)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, order)
    V, w = pr.vgrid.v, pr.vgrid.w
    gens, lags = odag.build_all(geo, V)
    fr = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    for _ in range(2):
        fr, _ = solver.bgk_step(geo, V, w, fr, g, dt, gens, lags, scheme=tableau,
                                mode="PROJECTED", nu_model=nu_model, nu_const=1.0, kn=0.1,
                                fixed_iters=3, L=pr.vgrid.L, vcells=vcells)
    assert rel(d.unpack(f).cpu().numpy(), fr) <= TOL64


def test_bgk_step_projected_converged_matches_oracle():
    say("bgk_step projected converged")
    pr = _gl_problem(2, 2, 4, 4, state="fourier", nu_model="kn", kn=0.05)
    d, f, bc, dt = B.problem_setup(pr)
    s = B.Solver(d, dt=dt, bc_coef=bc, tau=1e-10, mode="PROJECTED", nu_model="kn", kn=0.05)
    st = [s.step(f) for _ in range(3)]
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 2)
    V, w = pr.vgrid.v, pr.vgrid.w
    gens, lags = odag.build_all(geo, V)
    fr = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    ost = []
    for _ in range(3):
        fr, o = solver.bgk_step(geo, V, w, fr, g, dt, gens, lags, mode="PROJECTED",
                                nu_model="kn", kn=0.05, tau=1e-10, L=pr.vgrid.L, vcells=4)
        ost.append(o["iters"])
    assert [x["iters"] for x in st] == ost
    assert rel(d.unpack(f).cpu().numpy(), fr) <= TOL64


def test_projected_mode_and_q2_grid_validation():
    pr = _gl_problem(2, 1, 3, 4)
    vg = pr.vgrid
    mesh = pr.mesh

    def dag(**kw):
        args = dict(n_1d=len(vg.nodes_1d), nodes_1d=vg.nodes_1d, weights_1d=vg.weights_1d,
                    L=vg.L, dg_cells=vg.dg_cells)
        args.update(kw)
        v, w = args.pop("v", vg.v), args.pop("w", vg.w)
        return B.Dag(mesh.vert, mesh.cells, 1, v, w, **args)

    def code(fn):
        with pytest.raises(B.BGKError) as e:
            fn()
        return e.value.code

    assert dag().dg_cells == 4
    assert code(lambda: dag(dg_cells=5)) == B.BGK_E_INVALID         # n_1d != 3 dg_cells
    assert code(lambda: dag(dg_cells=-2)) == B.BGK_E_INVALID        # not positive
    assert code(lambda: dag(L=6.5)) == B.BGK_E_INVALID              # nodes of another box
    # equispaced nodes declared as a Q2 grid
    eq = P.tensor_velocity_grid(12, vg.L, 2)
    assert code(lambda: dag(v=eq.v, w=eq.w, nodes_1d=eq.nodes_1d,
                            weights_1d=eq.weights_1d)) == B.BGK_E_INVALID
    # PROJECTED needs the Q2 space: in the Maxwellian call and in the solver
    plain = B.Dag.from_problem(P.small_problem(dim=2, order=1, n_side=3, n_1d=6))
    U = B._dev(_moments_of(_seeded_prim(plain.n_nodes, 2, 1, 6.0), 2))
    assert code(lambda: B.maxwellian(plain, U, mode="PROJECTED")) == B.BGK_E_INVALID
    bc = torch.zeros((1, 4), dtype=torch.float64, device="cuda")
    assert code(lambda: B.Solver(plain, dt=0.1, bc_coef=bc, mode="PROJECTED")) == B.BGK_E_INVALID
    # batched stepping has no projected Maxwellian
    d2, f0, bc2, dt = B.problem_setup(pr)
    s = B.Solver(d2, dt=dt, bc_coef=bc2, mode="PROJECTED")
    assert code(lambda: B.Batch([s])) == B.BGK_E_UNSUPPORTED


def test_fp32_refined_projected_steps_with_walls_match_fp64_oracle_moments():
    """The FP32 correction sweep on the paper-literal set-up (Q2 velocities,
    projected Maxwellian, reflecting walls): converged moments equal the
    FP64 oracle's (tau = 1e-13) within the FP32 form's 1e-9."""
    from oracle import walls as owalls
    base = P.sod_strip_problem(3, 10.0)
    mesh = P.rectangle_mesh(16, 2, -1.0, 1.0, -P.SOD_STRIP_HALF_HEIGHT, P.SOD_STRIP_HALF_HEIGHT)
    pr = P.Problem(mesh, 1, base.vgrid, base.state, nu_const=10.0)
    d, f, bc, _ = B.problem_setup(pr)
    kinds = P.sod_strip_wall_kinds(B.boundary_facet_midpoints(d))
    s = B.Solver(d, dt=P.SOD_STRIP_DT, bc_coef=bc, walls=B.Walls(d, kinds), tau=1e-12,
                 mode="PROJECTED", nu_const=10.0, precision=B.TGS_FP32_CORRECTION)
    for _ in range(2):
        s.step(f)
    geo = geometry.build(mesh.vert, mesh.cells, 1)
    V, w = pr.vgrid.v, pr.vgrid.w
    okinds = owalls.boundary_kinds(geo, lambda x, n: owalls.REFLECT if abs(n[1]) > 0.5 else
                                   owalls.INFLOW)
    gens, lags = odag.build_all(geo, V)
    fr = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    for _ in range(2):
        fr, _ = solver.bgk_step(geo, V, w, fr, g, P.SOD_STRIP_DT, gens, lags, mode="PROJECTED",
                                nu_const=10.0, tau=1e-13, L=7.0, vcells=3, walls=okinds)
    U = kinetic.moments(d.unpack(f).cpu().numpy(), V, w).reshape(-1, 4)
    Uref = kinetic.moments(fr, V, w).reshape(-1, 4)
    err = 0.0
    for sl in (slice(0, 1), slice(1, 3), slice(3, 4)):
        den = max(np.linalg.norm(Uref[:, sl]), np.linalg.norm(Uref[:, 0]))
        err = max(err, np.linalg.norm(U[:, sl] - Uref[:, sl]) / den)
    assert err <= 1e-9, err
