"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Error measure (design note A21): max-norm error over the whole array divided
by the max norm of the oracle's array; 1e-12 for every FP64 result.
Generations are integers and must match exactly.
"""
import math
import sys

import numpy as np
import pytest

import problems as P
from oracle import dag as odag
from oracle import geometry, kinetic, solver, transport

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
import paper_2608_19150_amd as B  # noqa: E402

TOL64 = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def _problem(dim, order, n_side, n1, seed=7, state="sod"):
    return P.small_problem(dim=dim, order=order, n_side=n_side, n_1d=n1, seed=seed, state=state)


CASES = [(2, 1, 5, 6), (2, 2, 4, 5), (3, 1, 3, 4)]


@pytest.mark.parametrize("dim,order,n_side,n1", CASES)
def test_generations_match_oracle(dim, order, n_side, n1):
    say("generations", dim, order, n_side, n1)
    pr = _problem(dim, order, n_side, n1)
    d = B.Dag.from_problem(pr)
    gen, G = d.generations()
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, order)
    ogen, olag = odag.build_all(geo, pr.vgrid.v)
    assert not olag.any() and d.n_lagged == 0
    np.testing.assert_array_equal(gen, ogen)
    np.testing.assert_array_equal(G, ogen.max(axis=1) + 1)


def test_generations_c1_match_oracle():
    pr = P.config_c1()
    d = B.Dag.from_problem(pr)
    gen, _ = d.generations()
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 1)
    ogen, _ = odag.build_all(geo, pr.vgrid.v)
    np.testing.assert_array_equal(gen, ogen)


def test_pack_unpack_roundtrip():
    pr = _problem(2, 2, 4, 5)
    d = B.Dag.from_problem(pr)
    x = torch.randn(d.f_shape, dtype=torch.float64, device="cuda")
    y = d.unpack(d.pack(x))
    assert torch.equal(x, y)


def _random_sweep_inputs(pr, seed):
    rng = np.random.default_rng(seed)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    nv = pr.vgrid.n_v
    dim = geo.dim
    q = rng.uniform(0.0, 1.0, (geo.n_cells, geo.n_p, nv))
    nu = rng.uniform(0.1, 2.0, (geo.n_cells, geo.n_p))
    n = rng.uniform(0.2, 1.5, (geo.n_cells, geo.n_p))
    u = rng.uniform(-0.5, 0.5, (geo.n_cells, geo.n_p, dim))
    th = rng.uniform(0.6, 1.4, (geo.n_cells, geo.n_p))
    prim = np.concatenate([n[..., None], u, th[..., None]], axis=-1)
    return geo, q, nu, prim


def _gpu_sweep(d, pr, q, nu, prim, shift, qscale, bc_dense=None, f_prev=None, precision=0):
    qg = d.pack(B._dev(q))
    mcoef = B.maxwellian_coef_from_primitive(B._dev(prim.reshape(-1, d.dim + 2)), d.dim)
    bc = None if bc_dense is not None else B.state_coefficients(d, pr.state, "boundary")
    fo = torch.empty_like(qg)
    fp = d.pack(B._dev(f_prev)) if f_prev is not None else None
    B.tgs_sweep(d, q=qg, nu=B._dev(nu.reshape(-1)), mcoef=mcoef, f_out=fo, sigma_shift=shift,
                q_scale=qscale, bc_coef=bc, bc_dense=None if bc_dense is None else B._dev(bc_dense),
                f_prev=fp, precision=precision)
    return d.unpack(fo).cpu().numpy()


def _oracle_sweep(geo, pr, q, nu, prim, shift, qscale, gens, lags=None, f_prev=None, gbc=None):
    V = pr.vgrid.v
    coef = kinetic.direct_coefficients(prim[..., 0], prim[..., 1:-1], prim[..., -1])
    Mv = kinetic.coef_values(coef, V)
    g = solver.boundary_values(geo, V, pr.state) if gbc is None else gbc
    return transport.sweep(geo, V, nu + shift, nu, Mv, qscale * q, g, gens, lags, f_prev)


@pytest.mark.parametrize("dim,order,n_side,n1", CASES)
def test_sweep_fp64_matches_oracle(dim, order, n_side, n1):
    say("sweep fp64", dim, order, n_side, n1)
    pr = _problem(dim, order, n_side, n1, state="riemann")
    d = B.Dag.from_problem(pr)
    geo, q, nu, prim = _random_sweep_inputs(pr, 3)
    gens, _ = odag.build_all(geo, pr.vgrid.v)
    f_gpu = _gpu_sweep(d, pr, q, nu, prim, 37.0, 2.5)
    f_ref = _oracle_sweep(geo, pr, q, nu, prim, 37.0, 2.5, gens)
    assert rel(f_gpu, f_ref) <= TOL64


@pytest.mark.parametrize("dim,order,n_side,n1", CASES)
def test_sweep_fp64_coefficient_path_matches_oracle(dim, order, n_side, n1):
    """A velocity set given without its tensor structure: the sweep evaluates
    the Maxwellian from the node coefficients (no factorised tables)."""
    pr = _problem(dim, order, n_side, n1, state="riemann")
    d = B.Dag(pr.mesh.vert, pr.mesh.cells, pr.order, pr.vgrid.v, pr.vgrid.w)
    geo, q, nu, prim = _random_sweep_inputs(pr, 13)
    gens, _ = odag.build_all(geo, pr.vgrid.v)
    f_gpu = _gpu_sweep(d, pr, q, nu, prim, 37.0, 2.5)
    f_ref = _oracle_sweep(geo, pr, q, nu, prim, 37.0, 2.5, gens)
    assert rel(f_gpu, f_ref) <= TOL64


def test_sweep_fp64_c1_size_matches_oracle():
    pr = P.config_c1()
    d = B.Dag.from_problem(pr)
    geo, q, nu, prim = _random_sweep_inputs(pr, 4)
    gens, _ = odag.build_all(geo, pr.vgrid.v)
    f_gpu = _gpu_sweep(d, pr, q, nu, prim, 191.0, 191.0)
    f_ref = _oracle_sweep(geo, pr, q, nu, prim, 191.0, 191.0, gens)
    assert rel(f_gpu, f_ref) <= TOL64


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1)])
def test_sweep_bitwise_reproducible_across_runs_and_workgroup_sizes(dim, order):
    """The workgroup size changes which thread solves which cell of a
    generation (and which generations overflow); results are bitwise equal,
    and so are repeated runs."""
    say("sweep reproducibility", dim, order)
    pr = _problem(dim, order, 5 if dim == 2 else 3, 6)
    geo, q, nu, prim = _random_sweep_inputs(pr, 12)
    outs = []
    for T in (64, 128, 192, 256, 192):
        d = B.Dag.from_problem(pr, sweep_threads=T)
        outs.append(_gpu_sweep(d, pr, q, nu, prim, 7.0, 3.0))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


WIDE = [(3, 1, 10, 2), (2, 2, 80, 2), (2, 1, 80, 2)]


@pytest.mark.parametrize("dim,order,n_side,n1", WIDE)
def test_sweep_wide_generations_match_oracle(dim, order, n_side, n1):
    """Generations of 60-110 cells: with 64-thread workgroups a generation
    takes two chunks (the pipelined walk's steps, or the plain walk's second
    pass for P1 triangles); the result matches the oracle and equals the
    256-thread (one chunk per generation) sweep bit for bit."""
    say("sweep wide generations", dim, order, n_side, n1)
    pr = _problem(dim, order, n_side, n1, state="riemann")
    geo, q, nu, prim = _random_sweep_inputs(pr, 21)
    gens, _ = odag.build_all(geo, pr.vgrid.v)
    widest = max(int(np.bincount(g).max()) for g in gens)
    assert 64 < widest <= 256
    outs = []
    for T in (64, 256):
        d = B.Dag.from_problem(pr, sweep_threads=T)
        outs.append(_gpu_sweep(d, pr, q, nu, prim, 37.0, 2.5))
    assert np.array_equal(outs[0], outs[1])
    f_ref = _oracle_sweep(geo, pr, q, nu, prim, 37.0, 2.5, gens)
    assert rel(outs[0], f_ref) <= TOL64


@pytest.mark.parametrize("dim,order,n_side", [(2, 2, 80), (3, 1, 10)])
def test_step_wide_generations_bitwise_across_workgroup_sizes(dim, order, n_side):
    """Whole steps through the solver (factorised tables, pipelined walk) on
    meshes whose generations are wider than 64 cells: 64-, 128- and
    256-thread workgroups give the same f bit for bit."""
    say("step wide generations", dim, order, n_side)
    pr = _problem(dim, order, n_side, 4, state="fourier")
    outs = []
    for T in (64, 128, 256):
        d, f0, bc, dt = B.problem_setup(pr, sweep_threads=T)
        s = B.Solver(d, dt=dt, bc_coef=bc, tableau="DIRK2", fixed_iters=2, mode="MATCHED",
                     nu_model="kn", kn=0.1)
        s.step(f0)
        outs.append(d.unpack(f0).cpu().numpy())
        del s, d, f0
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("dim,order,n_side,n1", WIDE)
def test_sweep_small_ring_matches_oracle(dim, order, n_side, n1):
    """A 64-slot LDS ring with 64-thread workgroups on generations of 60-110
    cells: upwind values older than the ring come from HBM after a workgroup
    fence, and the chunks of a generation wider than the ring are separated
    by barriers.  The FP64 sweep matches the oracle and equals the full-ring
    sweep bit for bit; so does the FP32 correction sweep, whose corrections
    are then read back from HBM."""
    say("sweep small ring", dim, order, n_side, n1)
    pr = _problem(dim, order, n_side, n1, state="riemann")
    geo, q, nu, prim = _random_sweep_inputs(pr, 31)
    gens, _ = odag.build_all(geo, pr.vgrid.v)
    assert max(int(np.bincount(g).max()) for g in gens) > 64
    small = B.Dag.from_problem(pr, sweep_threads=64, ring_slots=64)
    full = B.Dag.from_problem(pr, sweep_threads=64)
    f_small = _gpu_sweep(small, pr, q, nu, prim, 11.0, 2.0)
    assert np.array_equal(f_small, _gpu_sweep(full, pr, q, nu, prim, 11.0, 2.0))
    f_ref = _oracle_sweep(geo, pr, q, nu, prim, 11.0, 2.0, gens)
    assert rel(f_small, f_ref) <= TOL64
    fp = f_ref * (1.0 + 1e-3 * np.random.default_rng(32).standard_normal(f_ref.shape))
    g_small = _gpu_sweep(small, pr, q, nu, prim, 11.0, 2.0, f_prev=fp, precision=1)
    g_full = _gpu_sweep(full, pr, q, nu, prim, 11.0, 2.0, f_prev=fp, precision=1)
    assert np.array_equal(g_small, g_full)


def test_step_small_ring_bitwise_equal_to_full_ring():
    """Whole DIRK2 steps through the solver (tables, pipelined walk) with a
    64-slot ring on generations wider than it equal full-ring steps bit for
    bit."""
    pr = _problem(2, 2, 80, 4, state="fourier")
    outs = []
    for rs in (64, 0):
        d, f0, bc, dt = B.problem_setup(pr, sweep_threads=64, ring_slots=rs)
        s = B.Solver(d, dt=dt, bc_coef=bc, tableau="DIRK2", fixed_iters=2, mode="MATCHED",
                     nu_model="kn", kn=0.1)
        s.step(f0)
        outs.append(d.unpack(f0).cpu().numpy())
        del s, d, f0
    assert np.array_equal(outs[0], outs[1])


def test_dag_rejects_bad_ring_slots():
    pr = _problem(2, 1, 3, 4)
    for bad in (8, 24, 2048):
        with pytest.raises(B.BGKError) as e:
            B.Dag.from_problem(pr, ring_slots=bad)
        assert e.value.code == B.BGK_E_INVALID


def test_sweep_dense_boundary_matches_oracle():
    pr = _problem(2, 2, 3, 4)
    d = B.Dag.from_problem(pr)
    geo, q, nu, prim = _random_sweep_inputs(pr, 5)
    gens, _ = odag.build_all(geo, pr.vgrid.v)
    gbc = np.random.default_rng(6).uniform(0, 1, (geo.bnode_x.shape[0], geo.n_fp, pr.vgrid.n_v))
    f_gpu = _gpu_sweep(d, pr, q, nu, prim, 5.0, 1.0, bc_dense=gbc)
    f_ref = _oracle_sweep(geo, pr, q, nu, prim, 5.0, 1.0, gens, gbc=gbc)
    assert rel(f_gpu, f_ref) <= TOL64


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1)])
def test_sweep_with_lagged_facets_matches_oracle(dim, order):
    say("sweep lagged", dim, order)
    pr = _problem(dim, order, 3, 4)
    geo, q, nu, prim = _random_sweep_inputs(pr, 8)
    V = pr.vgrid.v
    rng = np.random.default_rng(12)
    lags = np.zeros((V.shape[0], geo.n_cells, dim + 1), dtype=bool)
    bits = np.zeros((V.shape[0], geo.n_cells), dtype=np.uint8)
    for j in range(V.shape[0]):
        s = odag.facet_speeds(geo, V[j])
        lags[j] = (s < 0) & (geo.nbr >= 0) & (rng.uniform(size=s.shape) < 0.3)
        for k in range(dim + 1):
            bits[j] |= (lags[j][:, k].astype(np.uint8) << k)
    d = B.Dag.from_problem(pr, lagged=bits)
    assert d.n_lagged == int(lags.sum())
    np.testing.assert_array_equal(d.lagged(), bits)
    gens, _ = odag.build_all(geo, V, lagged=lags)
    gen_gpu, _ = d.generations()
    np.testing.assert_array_equal(gen_gpu, gens)
    f_prev = rng.uniform(0, 1, (geo.n_cells, geo.n_p, V.shape[0]))
    f_gpu = _gpu_sweep(d, pr, q, nu, prim, 3.0, 1.0, f_prev=f_prev)
    f_ref = _oracle_sweep(geo, pr, q, nu, prim, 3.0, 1.0, gens, lags, f_prev)
    assert rel(f_gpu, f_ref) <= TOL64


# then: a few cells with thousands of velocities (64 velocity lanes per cell
# in the moment kernel); 4232 cells with 8281 velocities (the velocity-split
# reduction: chunk sums, then their ordered sum); 22,999 tetrahedra (the
# 256-cell blocks of large tetrahedral meshes)
@pytest.mark.parametrize("dim,order,n_side,n1", CASES + [(2, 2, 3, 48), (3, 1, 2, 14),
                                                         (2, 1, 46, 91), (3, 1, 15, 4)])
def test_moments_and_ratios_match_oracle(dim, order, n_side, n1):
    pr = _problem(dim, order, n_side, n1)
    d = B.Dag.from_problem(pr)
    rng = np.random.default_rng(2)
    f = rng.uniform(0, 1, d.f_shape)
    f_old = f * (1 + 1e-3 * rng.normal(size=f.shape))
    fs = d.pack(B._dev(f))
    U_old = B.moments(d, d.pack(B._dev(f_old)))
    U, ratio = B.moments(d, fs, U_prev=U_old)
    V, w = pr.vgrid.v, pr.vgrid.w
    Uref = kinetic.moments(f, V, w).reshape(-1, dim + 2)
    Uold_ref = kinetic.moments(f_old, V, w).reshape(-1, dim + 2)
    assert rel(U.cpu().numpy(), Uref) <= TOL64
    rref = solver.relative_changes(Uref, Uold_ref, dim)
    rg = ratio.cpu().numpy()
    say("ratios", rg, rref, np.abs(rg - rref))
    # each ratio is a norm of moment differences (here ~1e-5 of the moments)
    # over a norm of moments: moments that agree to 1e-12 of their size give
    # ratios that agree to about 2e-12 in absolute terms, whatever their own
    # size; checked against 1e-13 (the relative error of a 2e-5 ratio is
    # rounding of order 1e-11 and says nothing about the kernel)
    assert np.all(np.abs(rg - rref) <= 1e-13)
    # bitwise reproducible
    U2 = B.moments(d, fs)
    assert torch.equal(U, U2)


@pytest.mark.parametrize("mode", ["DIRECT", "MATCHED", "LINEAR"])
@pytest.mark.parametrize("dim,n1", [(2, 16), (3, 10)])
def test_maxwellian_matches_oracle(mode, dim, n1):
    pr = _problem(dim, 1, 2, n1)
    d = B.Dag.from_problem(pr)
    V, w = pr.vgrid.v, pr.vgrid.w
    rng = np.random.default_rng(4)
    nn = d.n_nodes
    n = rng.uniform(0.1, 1.5, nn)
    u = rng.uniform(-1.0, 1.0, (nn, dim))
    th = rng.uniform(0.5, 2.0, nn)
    f = kinetic.maxwellian_values(n, u, th, V) * (1 + 0.1 * np.cos(V[:, 0]))[None]
    U = kinetic.moments(f, V, w)
    coef, nu, Md, status = B.maxwellian(d, B._dev(U), mode=mode,
                                        nu_model="kn", kn=0.01, dense=True)
    ref, nfb = solver.maxwellian_coefficients(U, V, w, mode, pr.vgrid.L)
    assert nfb == 0 and int(status[0]) == 0 and int(status[1]) == 0
    assert rel(coef.cpu().numpy(), ref) <= 1e-12
    assert rel(Md.cpu().numpy(), kinetic.coef_values(ref, V)) <= 1e-12
    nu_ref = kinetic.collision_frequency(U, dim, "kn", kn=0.01)
    assert rel(nu.cpu().numpy(), nu_ref) <= 1e-14
    if mode == "MATCHED":
        Um = kinetic.moments(Md.cpu().numpy(), V, w)
        assert rel(Um, U) <= 1e-13


def _run_steps(pr, nsteps, *, mode="MATCHED", fixed_iters=0, tau=1e-10, precision=0):
    d, f0, bc, dt = B.problem_setup(pr)
    s = B.Solver(d, dt=dt, bc_coef=bc, tableau=pr.tableau, tau=tau, fixed_iters=fixed_iters,
                 precision=precision, mode=mode, nu_model=pr.nu_model, nu_const=pr.nu_const,
                 kn=pr.kn)
    f = f0
    stats = []
    for _ in range(nsteps):
        stats.append(s.step(f))
    return d, d.unpack(f).cpu().numpy(), stats, dt


def _oracle_steps(pr, nsteps, dt, *, mode="MATCHED", fixed_iters=None, tau=1e-10):
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    V, w = pr.vgrid.v, pr.vgrid.w
    gens, lags = odag.build_all(geo, V)
    f = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    stats = []
    for _ in range(nsteps):
        f, st = solver.bgk_step(geo, V, w, f, g, dt, gens, lags, scheme=pr.tableau, mode=mode,
                                nu_model=pr.nu_model, nu_const=pr.nu_const, kn=pr.kn, tau=tau,
                                fixed_iters=fixed_iters, L=pr.vgrid.L)
        stats.append(st)
    return geo, f, stats


@pytest.mark.parametrize("tableau", ["BE", "DIRK2", "DIRK3"])
def test_steps_chained_through_their_moments_equal_plain_steps(tableau):
    """A step's converged moments (U_out) handed to the next step as its
    initial moments (U_guess) are the moments of f^k that step would compute:
    the chained steps equal plain steps bit for bit."""
    pr = _problem(2, 2, 4, 6, state="fourier")
    outs = []
    for chained in (False, True):
        d, f, bc, dt = B.problem_setup(pr)
        s = B.Solver(d, dt=dt, bc_coef=bc, tableau=tableau, tau=1e-10, mode="MATCHED",
                     nu_model="kn", kn=0.05)
        U = torch.empty((d.n_nodes, d.dim + 2), dtype=torch.float64, device="cuda")
        iters = []
        for k in range(3):
            if chained:
                iters.append(s.step(f, U_guess=U if k else None, U_out=U)["iters"])
            else:
                iters.append(s.step(f)["iters"])
        outs.append((d.unpack(f).cpu().numpy(), iters))
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0], outs[1][0])


def test_bgk_step_c1_fixed_iterations_matches_oracle():
    say("bgk_step c1 fixed")
    pr = P.config_c1()
    d, f, st, dt = _run_steps(pr, 2, fixed_iters=3)
    geo, fref, _ = _oracle_steps(pr, 2, dt, fixed_iters=3)
    assert rel(f, fref) <= TOL64


def test_bgk_step_c1_converged_matches_oracle():
    say("bgk_step c1 converged")
    pr = P.config_c1()
    d, f, st, dt = _run_steps(pr, 5)
    geo, fref, ost = _oracle_steps(pr, 5, dt)
    assert [s["iters"] for s in st] == [s["iters"] for s in ost]
    assert rel(f, fref) <= TOL64


@pytest.mark.parametrize("tableau", ["DIRK2", "DIRK3", "BDIRK2"])
def test_bgk_step_dirk_kn_matches_oracle(tableau):
    say("bgk_step", tableau)
    pr = P.small_problem(order=2, n_side=4, n_1d=8, state="fourier", nu_model="kn", kn=0.05,
                         tableau=tableau)
    d, f, st, dt = _run_steps(pr, 2, fixed_iters=4)
    geo, fref, _ = _oracle_steps(pr, 2, dt, fixed_iters=4)
    assert rel(f, fref) <= TOL64


@pytest.mark.parametrize("state", ["fourier", "sod"])
def test_bgk_step_3d_matches_oracle(state):
    pr = P.small_problem(dim=3, order=1, n_side=3, n_1d=6, state=state, nu_model="kn", kn=0.1)
    d, f, st, dt = _run_steps(pr, 2, fixed_iters=3)
    geo, fref, _ = _oracle_steps(pr, 2, dt, fixed_iters=3)
    assert rel(f, fref) <= TOL64


@pytest.mark.parametrize("kn,nsteps,fixed", [(1.0, 2, None), (1e-2, 2, None), (1e-4, 1, None)])
def test_bgk_step_3d_knudsen_range_matches_oracle(kn, nsteps, fixed):
    """The 3D workload's three Knudsen numbers (nu = n theta^(-1/2) / Kn) at a
    size the oracle runs in seconds: the same smoothed planar Riemann set-up
    (180 P1 tetrahedra, 8^3 velocities on [-6, 6]^3, BE, CFL 10); f within
    1e-12.  Kn = 1 and 1e-2: two steps converged to tau = 1e-10 with equal
    iteration counts.  Kn = 1e-4 is collision-dominated (nu dt ~ 1e2, so
    Picard contracts by about nu dt / (1 + nu dt) per iteration and a step
    needs ~700 iterations, minutes for the oracle): one step of 40 fixed
    iterations."""
    say("bgk_step 3d kn", kn)
    mesh = P.jittered_cube_mesh(3, 0.2, seed=3000)
    pr = P.Problem(mesh, 1, P.tensor_velocity_grid(8, 6.0, 3),
                   P.planar_riemann_state(3, seed=3001, width=0.5), nu_model="kn", kn=kn,
                   tableau="BE", name=f"c3_small_kn{kn:g}")
    d, f, st, dt = _run_steps(pr, nsteps, fixed_iters=fixed or 0)
    geo, fref, ost = _oracle_steps(pr, nsteps, dt, fixed_iters=fixed)
    say("iters", [s["iters"] for s in st], [s["iters"] for s in ost])
    assert [s["iters"] for s in st] == [s["iters"] for s in ost]
    assert rel(f, fref) <= TOL64


def test_nonphysical_state_is_reported_like_the_oracle():
    """A sharp 3D Riemann state on a 6^3 velocity grid drives nodal moments
    non-physical; the oracle raises and the library returns BGK_E_NONPHYSICAL."""
    pr = P.small_problem(dim=3, order=1, n_side=3, n_1d=6, state="riemann", nu_model="kn", kn=0.1)
    with pytest.raises(B.BGKError) as e:
        _run_steps(pr, 2, fixed_iters=3)
    assert e.value.code == B.BGK_E_NONPHYSICAL
    d = B.Dag.from_problem(pr)
    with pytest.raises(solver.NonPhysicalError):
        _oracle_steps(pr, 2, d.explicit_dt(pr.cfl), fixed_iters=3)


def test_matched_fallbacks_stay_direct_like_the_oracle():
    """A sharp oblique Riemann state on an 8-point grid (no v = 0): DG
    undershoot gives some nodes moments no non-negative discrete
    distribution has, so their MATCHED solve fails; they take DIRECT and keep
    it for the stage, on both sides, with equal counts and results."""
    say("matched fallbacks")
    mesh = P.jittered_square_mesh(4, 0.25, seed=7)
    st = P.State("plane", {"normal": np.array([0.8, 0.6]), "center": np.full(2, 0.5),
                           "left": (1.0, (0.0, 0.0, 0.0), 1.0),
                           "right": (0.2, (0.0, 0.0, 0.0), 0.5)})
    pr = P.Problem(mesh, 1, P.tensor_velocity_grid(8, 6.0, 2), st, nu_model="kn", kn=0.5,
                   tableau="BE", name="fallback")
    d, f, gst, dt = _run_steps(pr, 3)
    geo, fref, ost = _oracle_steps(pr, 3, dt)
    assert [s["iters"] for s in gst] == [s["iters"] for s in ost]
    assert [s["fallbacks"] for s in gst] == [s["fallbacks"] for s in ost]
    assert min(s["fallbacks"] for s in ost) > 0
    assert rel(f, fref) <= TOL64


def test_uniform_maxwellian_preserved_on_gpu():
    pr = P.small_problem(n_side=4, n_1d=8, state="uniform")
    d, f0, bc, dt = B.problem_setup(pr)
    f_init = d.unpack(f0).cpu().numpy()
    s = B.Solver(d, dt=dt, bc_coef=bc)
    f = f0
    for _ in range(5):
        st = s.step(f)
        assert st["iters"] == [1]
    assert rel(d.unpack(f).cpu().numpy(), f_init) <= 1e-13


# ---------------------------------------------------------------------------
# FP32 solve with FP64 refinement (defect correction): per sweep the result
# must be within 1e-5 of the FP64 oracle sweep on identical inputs; converged
# moments within 1e-9 of an FP64 oracle run converged to tau = 1e-13.
# ---------------------------------------------------------------------------
TOL32_SWEEP = 1e-5
TOL32_MOMENTS = 1e-9


@pytest.mark.parametrize("dim,order,n_side,n1", CASES)
def test_sweep_fp32_correction_matches_oracle(dim, order, n_side, n1):
    say("sweep fp32c", dim, order, n_side, n1)
    pr = _problem(dim, order, n_side, n1, state="riemann")
    d = B.Dag.from_problem(pr)
    geo, q, nu, prim = _random_sweep_inputs(pr, 13)
    gens, _ = odag.build_all(geo, pr.vgrid.v)
    rng = np.random.default_rng(14)
    f_ref = _oracle_sweep(geo, pr, q, nu, prim, 37.0, 2.5, gens)
    # previous iterate: the answer perturbed by 10% (a Picard iterate, not the solution)
    f_prev = f_ref * (1.0 + 0.1 * rng.uniform(-1, 1, f_ref.shape))
    f_gpu = _gpu_sweep(d, pr, q, nu, prim, 37.0, 2.5, f_prev=f_prev, precision=B.TGS_FP32_CORRECTION)
    err = rel(f_gpu, f_ref)
    assert err <= TOL32_SWEEP, err
    assert err > 1e-13          # the solve really ran in FP32


def _moment_err(U, Uref, dim):
    blocks = [slice(0, 1), slice(1, 1 + dim), slice(1 + dim, 2 + dim)]
    n0 = np.linalg.norm(Uref[:, 0])
    out = []
    for m, sl in enumerate(blocks):
        den = np.linalg.norm(Uref[:, sl])
        if m == 1:
            den = max(den, n0)
        out.append(np.linalg.norm(U[:, sl] - Uref[:, sl]) / den)
    return max(out)


@pytest.mark.parametrize("prob", ["c1", "p2_kn"])
def test_fp32_refined_steps_match_converged_fp64_moments(prob):
    say("fp32 refined steps", prob)
    if prob == "c1":
        pr = P.config_c1()
        nsteps = 2
    else:
        pr = P.small_problem(order=2, n_side=4, n_1d=10, state="fourier", nu_model="kn", kn=0.05,
                             tableau="DIRK2")
        nsteps = 2
    d, f, st, dt = _run_steps(pr, nsteps, tau=1e-12, precision=B.TGS_FP32_CORRECTION)
    geo, fref, _ = _oracle_steps(pr, nsteps, dt, tau=1e-13)
    V, w = pr.vgrid.v, pr.vgrid.w
    U = kinetic.moments(f, V, w).reshape(-1, geo.dim + 2)
    Uref = kinetic.moments(fref, V, w).reshape(-1, geo.dim + 2)
    err = _moment_err(U, Uref, geo.dim)
    assert err <= TOL32_MOMENTS, err
