"""The packed sweep walk (lane groups of 1..32 lanes per velocity; 1 lane is
the paper's thread-per-velocity TS) against the oracle and, bit for bit,
against the workgroup walk; the automatic choice between the walks; whole
steps with walls and lagged facets on the packed walk."""
import sys

import numpy as np
import pytest

import problems as P
from oracle import dag as odag
from oracle import geometry, kinetic, solver, transport, walls as owalls

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2608_19150_amd as B

TOL64 = 1e-12
LANES = [1, 2, 4, 8, 16, 32]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(x, ref):
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def _inputs(pr, seed):
    rng = np.random.default_rng(seed)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    nv, dim = pr.vgrid.n_v, geo.dim
    q = rng.uniform(0.0, 1.0, (geo.n_cells, geo.n_p, nv))
    nu = rng.uniform(0.1, 2.0, (geo.n_cells, geo.n_p))
    prim = np.concatenate([rng.uniform(0.2, 1.5, (geo.n_cells, geo.n_p, 1)),
                           rng.uniform(-0.5, 0.5, (geo.n_cells, geo.n_p, dim)),
                           rng.uniform(0.6, 1.4, (geo.n_cells, geo.n_p, 1))], axis=-1)
    return geo, q, nu, prim


def _sweep(d, pr, q, nu, prim, shift=13.0, qscale=2.0):
    qg = d.pack(B._dev(q))
    mcoef = B.maxwellian_coef_from_primitive(B._dev(prim.reshape(-1, d.dim + 2)), d.dim)
    bc = B.state_coefficients(d, pr.state, "boundary")
    fo = torch.empty_like(qg)
    B.tgs_sweep(d, q=qg, nu=B._dev(nu.reshape(-1)), mcoef=mcoef, f_out=fo, sigma_shift=shift,
                q_scale=qscale, bc_coef=bc)
    return d.unpack(fo).cpu().numpy()


def _oracle(geo, pr, q, nu, prim, gens, shift=13.0, qscale=2.0, V=None):
    V = pr.vgrid.v if V is None else V
    coef = kinetic.direct_coefficients(prim[..., 0], prim[..., 1:-1], prim[..., -1])
    Mv = kinetic.coef_values(coef, V)
    g = solver.boundary_values(geo, V, pr.state)
    return transport.sweep(geo, V, nu + shift, nu, Mv, qscale * q, g, gens)


@pytest.mark.parametrize("dim,order,n_side,n1", [(2, 1, 5, 6), (2, 2, 4, 5), (3, 1, 3, 4)])
@pytest.mark.parametrize("tensor", [True, False])
def test_packed_walk_equals_workgroup_walk_and_oracle(dim, order, n_side, n1, tensor):
    say("packed walk", dim, order, n_side, n1, tensor)
    pr = P.small_problem(dim=dim, order=order, n_side=n_side, n_1d=n1, state="riemann")
    geo, q, nu, prim = _inputs(pr, 70 + dim + order)
    gens, _ = odag.build_all(geo, pr.vgrid.v)
    ref = _oracle(geo, pr, q, nu, prim, gens)

    def dag(**kw):
        if tensor:
            return B.Dag.from_problem(pr, **kw)
        return B.Dag(pr.mesh.vert, pr.mesh.cells, order, pr.vgrid.v, pr.vgrid.w, **kw)

    wg = dag(sweep_lanes=64)
    assert wg.sweep_lanes == 64
    f_wg = _sweep(wg, pr, q, nu, prim)
    assert rel(f_wg, ref) <= TOL64
    for L in LANES:
        d = dag(sweep_lanes=L)
        assert d.sweep_lanes == L
        f = _sweep(d, pr, q, nu, prim)
        assert np.array_equal(f, f_wg), L


def test_automatic_walk_choice():
    # narrow generations (a 256 x 6 strip) with many velocities: packed; the
    # same strip with too few velocities to fill the GPU that way, and a
    # mesh with wide generations: the workgroup walk
    strip = P.sod_strip_problem(32, 1.0)
    assert B.Dag.from_problem(strip).sweep_lanes == 8
    assert B.Dag.from_problem(P.sod_strip_problem(4, 1.0)).sweep_lanes == 64
    wide = P.Problem(P.jittered_square_mesh(60, 0.25, 3), 1, P.tensor_velocity_grid(4, 3.0, 2),
                     P.sod_state(2))
    assert B.Dag.from_problem(wide).sweep_lanes == 64
    # explicit workgroup size implies the workgroup walk
    assert B.Dag.from_problem(strip, sweep_threads=128).sweep_lanes == 64
    for bad in ({"sweep_lanes": 3}, {"sweep_lanes": 128},
                {"sweep_lanes": 8, "sweep_threads": 128}):
        with pytest.raises(B.BGKError) as e:
            B.Dag.from_problem(strip, **bad)
        assert e.value.code == B.BGK_E_INVALID


def test_packed_walk_with_lagged_facets_matches_workgroup_walk():
    """Lagged facets read the previous iterate in both walks."""
    pr = P.small_problem(dim=2, order=1, n_side=4, n_1d=6, state="riemann")
    geo, q, nu, prim = _inputs(pr, 81)
    V = pr.vgrid.v
    rng = np.random.default_rng(82)
    lag = np.zeros((V.shape[0], geo.n_cells), dtype=np.uint8)
    for j in range(V.shape[0]):
        s = odag.facet_speeds(geo, V[j])
        cand = (s < 0) & (geo.nbr >= 0)
        pick = cand & (rng.uniform(size=cand.shape) < 0.3)
        lag[j] = (pick * (1 << np.arange(geo.dim + 1))[None, :]).sum(axis=1)
    outs = []
    for L in (64, 1, 8):
        d = B.Dag.from_problem(pr, lagged=lag, sweep_lanes=L)
        qg = d.pack(B._dev(q))
        fprev = d.pack(B._dev(np.random.default_rng(83).uniform(0, 1, q.shape)))
        mcoef = B.maxwellian_coef_from_primitive(B._dev(prim.reshape(-1, 4)), 2)
        fo = torch.empty_like(qg)
        B.tgs_sweep(d, q=qg, nu=B._dev(nu.reshape(-1)), mcoef=mcoef, f_out=fo, sigma_shift=9.0,
                    q_scale=1.0, bc_coef=B.state_coefficients(d, pr.state, "boundary"),
                    f_prev=fprev)
        outs.append(d.unpack(fo).cpu().numpy())
    assert d.n_lagged > 0
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("L", [1, 4])
def test_steps_with_walls_on_packed_walk_match_oracle(L):
    """The Sod strip's set-up (reflecting walls, Q2 velocities, projected
    Maxwellian) on a shortened strip, whole steps against the oracle."""
    base = P.sod_strip_problem(3, 1000.0)
    mesh = P.rectangle_mesh(16, 2, -1.0, 1.0, -P.SOD_STRIP_HALF_HEIGHT, P.SOD_STRIP_HALF_HEIGHT)
    pr = P.Problem(mesh, 1, base.vgrid, base.state, nu_const=1000.0)
    d, f, bc, _ = B.problem_setup(pr, sweep_lanes=L)
    assert d.sweep_lanes == L
    kinds = P.sod_strip_wall_kinds(B.boundary_facet_midpoints(d))
    s = B.Solver(d, dt=P.SOD_STRIP_DT, bc_coef=bc, walls=B.Walls(d, kinds), fixed_iters=3,
                 mode="PROJECTED", nu_const=1000.0)
    for _ in range(2):
        s.step(f)
    geo = geometry.build(mesh.vert, mesh.cells, 1)
    okinds = owalls.boundary_kinds(geo, lambda x, n: owalls.REFLECT if abs(n[1]) > 0.5 else
                                   owalls.INFLOW)
    np.testing.assert_array_equal(okinds, kinds)
    V, w = pr.vgrid.v, pr.vgrid.w
    gens, lags = odag.build_all(geo, V)
    fr = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    for _ in range(2):
        fr, _ = solver.bgk_step(geo, V, w, fr, g, P.SOD_STRIP_DT, gens, lags, mode="PROJECTED",
                                nu_const=1000.0, fixed_iters=3, L=7.0, vcells=3, walls=okinds)
    assert rel(d.unpack(f).cpu().numpy(), fr) <= TOL64


def test_fp32_and_batched_sweeps_on_packed_walk_dags():
    """A DAG whose FP64 sweeps take the packed walk: its FP32-correction
    sweeps and its batched steps use the workgroup walk, with the same
    results as on a workgroup-walk DAG (bit for bit)."""
    pr = P.small_problem(dim=2, order=1, n_side=4, n_1d=6, state="fourier")
    geo, q, nu, prim = _inputs(pr, 91)
    outs = {}
    for L in (64, 4):
        d = B.Dag.from_problem(pr, sweep_lanes=L)
        qg = d.pack(B._dev(q))
        fprev = d.pack(B._dev(np.random.default_rng(92).uniform(0, 1, q.shape)))
        mcoef = B.maxwellian_coef_from_primitive(B._dev(prim.reshape(-1, 4)), 2)
        fo = torch.empty_like(qg)
        B.tgs_sweep(d, q=qg, nu=B._dev(nu.reshape(-1)), mcoef=mcoef, f_out=fo, sigma_shift=5.0,
                    q_scale=1.0, bc_coef=B.state_coefficients(d, pr.state, "boundary"),
                    f_prev=fprev, precision=1)
        outs[("fp32", L)] = d.unpack(fo).cpu().numpy()
        # one DIRK2 step single and batched
        d2, f, bc, dt = B.problem_setup(pr, sweep_lanes=L)
        s = B.Solver(d2, dt=dt, bc_coef=bc, tableau="DIRK2", fixed_iters=2, mode="MATCHED")
        f_b = f.clone()
        s.step(f)
        s2 = B.Solver(d2, dt=dt, bc_coef=bc, tableau="DIRK2", fixed_iters=2, mode="MATCHED")
        B.Batch([s2], graph=False).step([f_b])
        assert torch.equal(f, f_b), L
        outs[("step", L)] = d2.unpack(f).cpu().numpy()
    assert np.array_equal(outs[("fp32", 64)], outs[("fp32", 4)])
    assert np.array_equal(outs[("step", 64)], outs[("step", 4)])


def test_sweep_walk_autotuner_sets_the_fastest_walk_and_results_do_not_change(tmp_path):
    """The single-instance walk autotuner times every candidate walk
    (workgroup walk of 64-256 threads, packed walk of 2-32 lanes per
    velocity) on real sweeps, sets the fastest on the DAG and caches it by
    the DAG's shape; a second call takes it from the cache.  The sweep
    results are the same bit for bit under every walk."""
    from paper_2608_19150_amd import autotune
    pr = P.sod_strip_problem(8, 1.0)          # narrow generations: packing can win
    d = B.Dag.from_problem(pr)
    geo_inputs = _walk_inputs(d, pr)
    ref = None
    for kind, val in autotune.WALK_CANDIDATES:
        autotune._apply(d, kind, val)
        out = torch.empty_like(geo_inputs["q"])
        B.tgs_sweep(d, **dict(geo_inputs, f_out=out))
        if ref is None:
            ref = out.clone()
        assert torch.equal(out, ref), (kind, val)
    cache = str(tmp_path / "tune.json")
    best, ms = autotune.tune_sweep_walk(d, dict(geo_inputs, f_out=torch.empty_like(ref)),
                                        cache_path=cache, reps=2)
    print("walk timings (ms):", ms, "best", best, flush=True)
    assert best == min(ms, key=ms.get)
    expect_lanes = 64 if best[0] == "wg" else best[1]
    assert d.sweep_lanes == expect_lanes
    d.set_walk(0, 0)
    best2, _ = autotune.tune_sweep_walk(d, dict(geo_inputs, f_out=torch.empty_like(ref)),
                                        cache_path=cache)
    assert best2 == best and d.sweep_lanes == expect_lanes


def _walk_inputs(d, pr):
    nn = d.n_nodes
    prim = torch.zeros((nn, d.dim + 2), dtype=torch.float64, device="cuda")
    prim[:, 0] = 1.0
    prim[:, -1] = 1.0
    prim[:, 1] = 0.2
    mcoef = B.maxwellian_coef_from_primitive(prim, d.dim)
    q = d.eval_maxwellian(mcoef)
    return {"q": q, "nu": torch.full((nn,), 5.0, dtype=torch.float64, device="cuda"),
            "mcoef": mcoef, "sigma_shift": 20.0,
            "bc_coef": B.state_coefficients(d, pr.state, "boundary")}
