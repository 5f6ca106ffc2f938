"""Parity at the benchmark sizes, in the launch configuration bench.py times
(library-chosen workgroup size and ring, factorised Maxwellian tables, the
pipelined walk): every velocity and node is computed on the GPU, and the
oracle recomputes a sample one by one - whole velocities of the sweep over
the full mesh, single nodes of the moment reduction and the Maxwellian.

Workloads: ~200k graded P2 triangles x 32^2 velocities (the 2D workload),
the same mesh on 30^2- and 33^2-node Q2 velocity spaces with the projected
Maxwellian, and ~55k P1 tetrahedra x 16^3 velocities (the 3D workload)."""
import gc

import numpy as np
import pytest

import problems as P
from oracle import dag as odag
from oracle import geometry, kinetic, solver, transport, velocity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2608_19150_amd as B

TOL64 = 1e-12


def rel(x, ref):
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def _release():
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _nodal_inputs(n_nodes, dim, seed):
    """Seeded per-node nu and primitive (n, u, theta)."""
    rng = np.random.default_rng(seed)
    nu = rng.uniform(0.1, 2.0, n_nodes)
    prim = np.concatenate([rng.uniform(0.2, 1.5, (n_nodes, 1)),
                           rng.uniform(-0.5, 0.5, (n_nodes, dim)),
                           rng.uniform(0.6, 1.4, (n_nodes, 1))], axis=1)
    return nu, prim


@pytest.mark.parametrize("workload,sample", [("2d", (0, 311, 528, 777, 1023)),
                                             ("3d", (0, 1365, 2050, 4095))])
def test_full_size_sweep_matches_oracle_on_sampled_velocities(workload, sample):
    pr = P.config_c2(316) if workload == "2d" else P.config_c3(kn=1e-2)
    d = B.Dag.from_problem(pr)
    assert d.n_cells > 5e4 and d.n_v >= 1024
    nu, prim = _nodal_inputs(d.n_nodes, d.dim, 9100)
    gen = torch.Generator(device="cuda").manual_seed(9101)
    q = torch.rand(d.f_shape, dtype=torch.float64, device="cuda", generator=gen)
    js = np.array(sample)
    jt = torch.as_tensor(js, device="cuda")
    q_s = q[..., jt].cpu().numpy()
    qg = d.pack(q)
    del q
    mcoef = B.maxwellian_coef_from_primitive(B._dev(prim), d.dim)
    bc = B.state_coefficients(d, pr.state, "boundary")
    fo = torch.empty_like(qg)
    B.tgs_sweep(d, q=qg, nu=B._dev(nu), mcoef=mcoef, f_out=fo, sigma_shift=41.0, q_scale=3.0,
                bc_coef=bc)
    del qg
    f_s = d.unpack(fo)[..., jt].cpu().numpy()
    del fo, mcoef, bc, d
    _release()
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    V = pr.vgrid.v[js]
    gens, lags = odag.build_all(geo, V)
    assert not lags.any()
    nn = nu.reshape(geo.n_cells, geo.n_p)
    pp = prim.reshape(geo.n_cells, geo.n_p, -1)
    coef = kinetic.direct_coefficients(pp[..., 0], pp[..., 1:-1], pp[..., -1])
    Mv = kinetic.coef_values(coef, V)
    g = solver.boundary_values(geo, V, pr.state)
    f_ref = transport.sweep(geo, V, nn + 41.0, nn, Mv, 3.0 * q_s, g, gens)
    assert rel(f_s, f_ref) <= TOL64


def test_full_size_moments_and_maxwellian_match_oracle_on_sampled_nodes():
    pr = P.config_c2(316)
    d = B.Dag.from_problem(pr)
    V, w = pr.vgrid.v, pr.vgrid.w
    rng = np.random.default_rng(9200)
    cells = np.sort(rng.choice(d.n_cells, 400, replace=False))
    gen = torch.Generator(device="cuda").manual_seed(9201)
    f = torch.rand(d.f_shape, dtype=torch.float64, device="cuda", generator=gen)
    f_s = f[torch.as_tensor(cells, device="cuda")].cpu().numpy()
    fg = d.pack(f)
    del f
    U = B.moments(d, fg).cpu().numpy().reshape(d.n_cells, d.n_p, -1)
    del fg
    assert rel(U[cells], kinetic.moments(f_s, V, w)) <= TOL64
    # Maxwellian of seeded realizable moments at every node (n, n u,
    # n (d theta + |u|^2) / 2 from a seeded (n, u, theta))
    _, prim = _nodal_inputs(d.n_nodes, d.dim, 9202)
    n, u, th = prim[:, 0], prim[:, 1:-1], prim[:, -1]
    Um = np.concatenate([n[:, None], n[:, None] * u,
                         (0.5 * n * (d.dim * th + np.sum(u * u, axis=1)))[:, None]], axis=1)
    coef, nu, _, status = B.maxwellian(d, B._dev(Um), mode="MATCHED", nu_model="kn", kn=1e-2)
    assert int(status[1]) == 0
    nodes = np.sort(rng.choice(d.n_nodes, 2000, replace=False))
    ref, nfb = kinetic.matched_coefficients(Um[nodes], V, w)
    assert nfb == 0 and int(status[0]) == 0
    assert rel(coef.cpu().numpy()[nodes], ref) <= TOL64
    nu_ref = kinetic.collision_frequency(Um[nodes], d.dim, "kn", kn=1e-2)
    assert rel(nu.cpu().numpy()[nodes], nu_ref) <= 1e-14
    del coef, nu, d
    _release()


def test_batched_workload_instances_at_full_size_equal_single_instance_steps():
    """Instances of the batched workload at their own sizes (the two largest
    meshes, the largest velocity grid and the stiffest Kn among the 64),
    stepped together in the benchmark's batch configuration (hipGraph chunks
    of 4 iterations, 64-thread sweeps) and one by one through bgk_step: the
    same f bit for bit, with the same iteration counts."""
    probs = P.config_c4_instances()
    size = [p.mesh.n_cells * (3 if p.order == 1 else 6) * p.vgrid.n_v for p in probs]
    pick = set(np.argsort(size)[-2:].tolist())
    pick.add(int(np.argmax([p.vgrid.n_v for p in probs])))
    pick.add(int(np.argmin([p.kn for p in probs])))
    picked = [probs[i] for i in sorted(pick)]

    def setup(pr):
        d, f0, bc, dt = B.problem_setup(pr)
        s = B.Solver(d, dt=dt, bc_coef=bc, tableau=pr.tableau, tau=pr.tau, mode="MATCHED",
                     nu_model=pr.nu_model, kn=pr.kn)
        return s, f0

    ref, ref_iters = [], []
    for pr in picked:
        s, f = setup(pr)
        ref_iters.append(s.step(f)["iters"])
        ref.append(f.cpu())
        del s, f
        _release()
    pairs = [setup(pr) for pr in picked]
    batch = B.Batch([p[0] for p in pairs], graph=True, chunk_iters=4, sweep_threads=64)
    st = batch.step([p[1] for p in pairs])
    for i, x in enumerate(st):
        assert x["status"] == 0 and x["iters"] == ref_iters[i], (i, x, ref_iters[i])
        assert torch.equal(pairs[i][1].cpu(), ref[i]), i
    del batch, pairs
    _release()


@pytest.mark.parametrize("vcells", [10, 11])
def test_full_size_projected_step_matches_oracle_on_sampled_velocities(vcells):
    """One Picard iteration of a backward-Euler step on the 2D workload's mesh
    with the Q2 velocity space in PROJECTED mode (10 cells per axis: the
    benchmarked 30^2 nodes; 11: 33^2 nodes, more sweep workgroups than stay
    resident at once), from seeded moments: projected-Maxwellian tables at
    full size feed the pipelined sweep; the oracle recomputes whole sampled
    velocities from the same moments, its 1-D erf projections and its sweep."""
    base = P.config_c2_q2(316, vcells)
    pr = P.Problem(base.mesh, 2, base.vgrid, base.state, nu_model="kn", kn=1e-2, tableau="BE",
                   cfl=base.cfl)
    d, f, bc, dt = B.problem_setup(pr)
    n1 = 3 * vcells
    assert d.n_cells > 5e4 and d.n_v == n1 * n1 and d.dg_cells == vcells
    _, prim = _nodal_inputs(d.n_nodes, 2, 9300)
    n, u, th = prim[:, 0], prim[:, 1:-1], prim[:, -1]
    Um = np.concatenate([n[:, None], n[:, None] * u,
                         (0.5 * n * (2 * th + np.sum(u * u, axis=1)))[:, None]], axis=1)
    s = B.Solver(d, dt=dt, bc_coef=bc, tableau="BE", fixed_iters=1, mode="PROJECTED",
                 nu_model="kn", kn=1e-2)
    assert s.step(f, U_guess=B._dev(Um))["iters"] == [1]
    js = np.array([0, 7 * n1 + 3, (n1 // 2) * n1 + n1 // 2, 21 * n1 + 8, n1 * n1 - 1])
    f_s = d.unpack(f)[..., torch.as_tensor(js, device="cuda")].cpu().numpy()
    del s, f, bc, d
    _release()
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    V = pr.vgrid.v[js]
    gens, lags = odag.build_all(geo, V)
    assert not lags.any()
    # projected Maxwellian at the sampled velocities: n (2 pi theta)^-1 times
    # the two axes' 1-D projections at the sample's tensor indices
    p0 = velocity.project_gaussian_1d(u[:, 0], th, vcells, 8.0)
    p1 = velocity.project_gaussian_1d(u[:, 1], th, vcells, 8.0)
    Mv = (n / (2.0 * np.pi * th))[:, None] * p0[:, js // n1] * p1[:, js % n1]
    Mv = Mv.reshape(geo.n_cells, geo.n_p, -1)
    nu = kinetic.collision_frequency(Um, 2, "kn", kn=1e-2).reshape(geo.n_cells, geo.n_p)
    f0 = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    f_ref = transport.sweep(geo, V, nu + 1.0 / dt, nu, Mv, f0 / dt, g, gens)
    assert rel(f_s, f_ref) <= TOL64


def test_strip_full_size_packed_walk_step_matches_oracle_on_sampled_velocities():
    """The narrow-generation strip as benchmarked: 3072 P1 triangles, 192^2
    Q2 velocities (the packed walk the library chooses), reflecting walls,
    projected Maxwellian, nu = 1000: one Picard iteration of a backward-Euler
    step from seeded moments.  The oracle recomputes sampled velocities: the
    walls' data come from the initial state at the mirrored velocities (the
    sample is closed under the mirror, so the oracle's wall update runs on
    it directly)."""
    from oracle import walls as owalls
    pr = P.sod_strip_problem(64, 1000.0)
    d, f, bc, _ = B.problem_setup(pr)
    assert d.sweep_lanes < 64 and d.n_v == 192 * 192
    kinds = P.sod_strip_wall_kinds(B.boundary_facet_midpoints(d))
    _, prim = _nodal_inputs(d.n_nodes, 2, 9400)
    n, u, th = prim[:, 0], prim[:, 1:-1], prim[:, -1]
    Um = np.concatenate([n[:, None], n[:, None] * u,
                         (0.5 * n * (2 * th + np.sum(u * u, axis=1)))[:, None]], axis=1)
    dt = P.SOD_STRIP_DT
    s = B.Solver(d, dt=dt, bc_coef=bc, walls=B.Walls(d, kinds), fixed_iters=1, mode="PROJECTED",
                 nu_const=1000.0)
    assert s.step(f, U_guess=B._dev(Um))["iters"] == [1]
    n1 = 192
    base = np.array([0, 5 * n1 + 17, 96 * n1 + 40, 130 * n1 + 150, n1 * n1 - 1])
    mirror = (base // n1) * n1 + (n1 - 1 - base % n1)        # v_2 -> -v_2
    js = np.unique(np.concatenate([base, mirror]))
    f_s = d.unpack(f)[..., torch.as_tensor(js, device="cuda")].cpu().numpy()
    del s, f, bc, d
    _release()
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 1)
    V = pr.vgrid.v[js]
    okinds = owalls.boundary_kinds(geo, lambda x, nrm: owalls.REFLECT if abs(nrm[1]) > 0.5 else
                                   owalls.INFLOW)
    np.testing.assert_array_equal(okinds, kinds)
    gens, lags = odag.build_all(geo, V)
    f0 = solver.initial_condition(geo, V, pr.state)
    g = owalls.wall_values(geo, V, f0, okinds, solver.boundary_values(geo, V, pr.state))
    p0 = velocity.project_gaussian_1d(u[:, 0], th, 64, 7.0)
    p1 = velocity.project_gaussian_1d(u[:, 1], th, 64, 7.0)
    Mv = ((n / (2.0 * np.pi * th))[:, None] * p0[:, js // n1] * p1[:, js % n1])
    Mv = Mv.reshape(geo.n_cells, geo.n_p, -1)
    nu = np.full((geo.n_cells, geo.n_p), pr.nu_const)
    f_ref = transport.sweep(geo, V, nu + 1.0 / dt, nu, Mv, f0 / dt, g, gens, lags)
    assert rel(f_s, f_ref) <= TOL64


def test_duct_full_size_step_matches_oracle_on_sampled_velocities():
    """The duct as benchmarked: 10,523 P1 tetrahedra x 48^3 = 110,592 Q2
    velocities, bounce-back (x_2) and reflecting (x_3) walls, Maxwellian and
    zero inflow, projected Maxwellian, nu = 1: one Picard iteration of a
    backward-Euler step from seeded moments.  The sample is closed under
    both wall maps (v -> -v and v_3 -> -v_3), so the oracle's wall update
    runs on it directly."""
    from oracle import walls as owalls

    import bench
    pr = P.duct_problem()
    d, walls, bc, f = bench.duct_setup(pr)
    assert d.n_v == 110592
    _, prim = _nodal_inputs(d.n_nodes, 3, 9500)
    n, u, th = prim[:, 0], prim[:, 1:-1], prim[:, -1]
    Um = np.concatenate([n[:, None], n[:, None] * u,
                         (0.5 * n * (3 * th + np.sum(u * u, axis=1)))[:, None]], axis=1)
    dt = P.DUCT_DT
    s = B.Solver(d, dt=dt, bc_coef=bc, walls=walls, fixed_iters=1, mode="PROJECTED",
                 nu_const=pr.nu_const)
    assert s.step(f, U_guess=B._dev(Um))["iters"] == [1]
    del s
    _release()
    n1 = 48
    base = np.array([[0, 0, 0], [24, 23, 24], [30, 10, 40], [5, 33, 17], [47, 20, 26]])
    imgs = [base, n1 - 1 - base, np.stack([base[:, 0], base[:, 1], n1 - 1 - base[:, 2]], 1),
            np.stack([n1 - 1 - base[:, 0], n1 - 1 - base[:, 1], base[:, 2]], 1)]
    idx = np.unique(np.concatenate(imgs), axis=0)
    js = np.ravel_multi_index(idx.T, (n1, n1, n1))
    f_s = d.unpack(f)[..., torch.as_tensor(js, device="cuda")].cpu().numpy()
    kinds, bprim = P.duct_boundary(B.boundary_facet_midpoints(d))
    del f, bc, walls, d
    _release()
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 1)
    V = pr.vgrid.v[js]
    gens, lags = odag.build_all(geo, V)
    f0 = solver.initial_condition(geo, V, pr.state)
    # inflow data: Maxwellian of each boundary facet's state (n = 0: none)
    bx = geo.bnode_x.reshape(-1, 3)
    bp = np.repeat(bprim, geo.n_fp, axis=0)
    g_in = np.where(bp[:, :1] > 0,
                    kinetic.maxwellian_values(np.maximum(bp[:, 0], 1e-300), bp[:, 1:4], bp[:, 4],
                                              V), 0.0).reshape(bx.shape[0] // geo.n_fp,
                                                               geo.n_fp, -1)
    g = owalls.wall_values(geo, V, f0, kinds, g_in)
    p = [velocity.project_gaussian_1d(u[:, a], th, 16, 12.0) for a in range(3)]
    i0, i1, i2 = idx[:, 0], idx[:, 1], idx[:, 2]
    Mv = (n / (2.0 * np.pi * th) ** 1.5)[:, None] * p[0][:, i0] * p[1][:, i1] * p[2][:, i2]
    Mv = Mv.reshape(geo.n_cells, geo.n_p, -1)
    nu = np.full((geo.n_cells, geo.n_p), pr.nu_const)
    f_ref = transport.sweep(geo, V, nu + 1.0 / dt, nu, Mv, f0 / dt, g, gens, lags)
    assert rel(f_s, f_ref) <= TOL64
