"""Batched stepping of uneven instances: batched = single-instance steps bit
for bit, hipGraph replay = eager launches on every step, per-instance error
reporting, and the sweep autotuner's probe."""
import math
import os

import numpy as np
import pytest

import problems as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2608_19150_amd as B
    from paper_2608_19150_amd import autotune


def _instances(dim, seed0=4100, count=5):
    """Uneven seeded instances: mesh size, element order, velocity grid and
    Kn vary (a small-size version of the batched workload)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        kn = math.exp(rng.uniform(math.log(1e-2), 0.0))
        if dim == 2:
            n_side = int(rng.integers(4, 13))
            order = int(rng.integers(1, 3))
            n1 = int(rng.integers(8, 17))
            mesh = P.jittered_square_mesh(n_side, 0.2, seed=seed0 + 1000 + i)
            vg = P.tensor_velocity_grid(n1, 8.0, 2)
        else:
            n_side = int(rng.integers(3, 5))
            order = 1
            n1 = int(rng.integers(8, 11))
            mesh = P.jittered_cube_mesh(n_side, 0.2, seed=seed0 + 1000 + i)
            vg = P.tensor_velocity_grid(n1, 6.0, 3)
        state = P.fourier_state(dim, seed0 + 2000 + i)
        out.append(P.Problem(mesh, order, vg, state, nu_model="kn", kn=kn,
                             tableau="DIRK2" if dim == 2 else "BE", name=f"inst{i}"))
    return out


def _setup(pr, tau=1e-10):
    d, f0, bc, dt = B.problem_setup(pr)
    s = B.Solver(d, dt=dt, bc_coef=bc, tableau=pr.tableau, tau=tau, mode="MATCHED",
                 nu_model=pr.nu_model, nu_const=pr.nu_const, kn=pr.kn)
    return s, f0


@pytest.mark.parametrize("dim", [2, 3])
def test_batched_steps_equal_single_instance_steps(dim):
    probs = _instances(dim)
    ref, ref_iters = [], []
    for pr in probs:
        s, f = _setup(pr)
        its = []
        for _ in range(2):
            its.append(s.step(f)["iters"])
        ref.append(f.clone())
        ref_iters.append(its)
        del s
    for graph in (False, True):
        pairs = [_setup(pr) for pr in probs]
        solvers, fs = [p[0] for p in pairs], [p[1] for p in pairs]
        batch = B.Batch(solvers, graph=graph, chunk_iters=3, sweep_threads=128)
        got_iters = [[] for _ in probs]
        for _ in range(2):
            st = batch.step(fs)
            for i, x in enumerate(st):
                assert x["status"] == 0
                got_iters[i].append(x["iters"])
        assert got_iters == ref_iters
        for i in range(len(probs)):
            assert torch.equal(fs[i], ref[i]), (graph, i)


def test_graph_replays_equal_eager_steps():
    """Several steps, each replaying every stage's captured chunk several
    times with host polls and eager stage work in between; every step's
    result is compared with the eager batch."""
    probs = _instances(2, seed0=4200, count=4)
    eager = [_setup(pr) for pr in probs]
    graph = [_setup(pr) for pr in probs]
    be = B.Batch([p[0] for p in eager], graph=False, chunk_iters=2)
    bg = B.Batch([p[0] for p in graph], graph=True, chunk_iters=2)
    fe, fg = [p[1] for p in eager], [p[1] for p in graph]
    for step in range(3):
        se = be.step(fe)
        sg = bg.step(fg)
        assert [x["iters"] for x in se] == [x["iters"] for x in sg]
        assert max(sum(x["iters"]) for x in sg) > 2    # more than one replay per stage
        for i in range(len(probs)):
            assert torch.equal(fe[i], fg[i]), (step, i)


def test_failing_instance_is_reported_and_others_finish():
    """A sharp 3D Riemann state on a 6^3 grid goes non-physical (as the
    single-instance solver reports); in a batch that instance is reported
    at the same step and the others' results are unaffected."""
    good = _instances(3, seed0=4300, count=2)
    bad = P.small_problem(dim=3, order=1, n_side=3, n_1d=6, state="riemann", nu_model="kn",
                          kn=0.1)

    def setup_bad():
        d, f0, bc, dt = B.problem_setup(bad)
        return B.Solver(d, dt=dt, bc_coef=bc, tableau="BE", fixed_iters=3, mode="MATCHED",
                        nu_model="kn", kn=0.1), f0

    s, f = setup_bad()
    fail_step = None
    for k in range(3):
        try:
            s.step(f)
        except B.BGKError as e:
            assert e.code == B.BGK_E_NONPHYSICAL
            fail_step = k
            break
    assert fail_step is not None
    refs = []
    for pr in good:
        s, f = _setup(pr)
        for _ in range(fail_step + 1):
            s.step(f)
        refs.append(f.clone())
    pairs = [_setup(good[0]), setup_bad(), _setup(good[1])]
    batch = B.Batch([p[0] for p in pairs], graph=True)
    fs = [p[1] for p in pairs]
    for k in range(fail_step):
        assert all(x["status"] == 0 for x in batch.step(fs))
    st = batch.step(fs, check=False)
    assert [x["status"] for x in st] == [0, B.BGK_E_NONPHYSICAL, 0]
    assert torch.equal(fs[0], refs[0]) and torch.equal(fs[2], refs[1])


def test_time_sweep_and_autotuner(tmp_path):
    probs = _instances(2, seed0=4400, count=3)
    pairs = [_setup(pr) for pr in probs]
    solvers, fs = [p[0] for p in pairs], [p[1] for p in pairs]
    before = [f.clone() for f in fs]
    cache = str(tmp_path / "tune.json")
    best, ms = autotune.tune_sweep_threads(solvers, fs, cache_path=cache)
    assert best in autotune.CANDIDATES and all(v > 0 for v in ms.values())
    assert ms[best] == min(ms.values())
    assert all(torch.equal(a, b) for a, b in zip(fs, before))
    assert os.path.exists(cache)
    best2, _ = autotune.tune_sweep_threads(solvers, fs, cache_path=cache)
    assert best2 == best
    walk, wms = autotune.tune_batch_walk(solvers, fs, cache_path=cache)
    assert walk in autotune.BATCH_WALK_CANDIDATES and wms[walk] == min(wms.values())
    assert all(torch.equal(a, b) for a, b in zip(fs, before))
    batch, t, _ = autotune.autotuned_batch(solvers, fs, cache_path=cache)
    assert t == walk
    st = batch.step(fs)
    assert all(x["status"] == 0 for x in st)


@pytest.mark.parametrize("dim", [2, 3])
def test_batched_packed_walk_equals_single_instance_steps(dim):
    """The batch's packed walk (64/L velocities of one instance per 64-lane
    workgroup) gives the single-instance steps bit for bit, for every L,
    eager and replayed from graphs."""
    probs = _instances(dim, seed0=4500, count=4)
    ref, ref_iters = [], []
    for pr in probs:
        s, f = _setup(pr)
        ref_iters.append([s.step(f)["iters"] for _ in range(2)])
        ref.append(f.clone())
        del s
    for lanes, graph in [(1, False), (2, True), (4, False), (8, True), (16, True), (32, False)]:
        pairs = [_setup(pr) for pr in probs]
        fs = [p[1] for p in pairs]
        batch = B.Batch([p[0] for p in pairs], graph=graph, chunk_iters=3, sweep_lanes=lanes)
        got = [[] for _ in probs]
        for _ in range(2):
            for i, x in enumerate(batch.step(fs)):
                assert x["status"] == 0
                got[i].append(x["iters"])
        assert got == ref_iters, lanes
        for i in range(len(probs)):
            assert torch.equal(fs[i], ref[i]), (lanes, graph, i)


def test_batch_walk_options_validated():
    pairs = [_setup(pr) for pr in _instances(2, seed0=4600, count=2)]
    solvers, fs = [p[0] for p in pairs], [p[1] for p in pairs]
    for bad in (3, 48, 128, -1):
        with pytest.raises(B.BGKError) as e:
            B.Batch(solvers, sweep_lanes=bad)
        assert e.value.code == B.BGK_E_INVALID
    probe = B.Batch(solvers, graph=False)
    with pytest.raises(B.BGKError) as e:
        probe.time_sweep(fs, 128, lanes=12)
    assert e.value.code == B.BGK_E_INVALID


def _oracle_instance(pr):
    from oracle import dag as odag
    from oracle import geometry, solver
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    V, w = pr.vgrid.v, pr.vgrid.w
    gens, lags = odag.build_all(geo, V)
    f0 = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    dt = solver.explicit_dt(geo, V, pr.cfl)
    return geo, V, w, gens, lags, f0, g, dt


@pytest.mark.parametrize("fixed", [0, 3])
def test_batched_steps_match_oracle(fixed):
    """Four uneven instances (P1 and P2, 8^2 to 12^2 velocities, Kn from 1e-3
    to 1: non-stiff and stiff; smooth seeded Fourier states) stepped together as one batch (hipGraph
    replay) for two DIRK2 steps; every instance's f after each step matches
    oracle.solver.bgk_step within 1e-12 of its max norm, with the same Picard
    iteration count per stage (converged to tau = 1e-10, or a fixed count)."""
    from oracle import solver
    specs = [(3, 1, 8, 1.0), (4, 2, 10, 1e-1), (3, 2, 12, 1e-3), (5, 1, 9, 1e-2)]
    probs = []
    for i, (n_side, order, n1, kn) in enumerate(specs):
        mesh = P.jittered_square_mesh(n_side, 0.2, seed=4200 + i)
        st = P.fourier_state(2, seed=4300 + i)
        probs.append(P.Problem(mesh, order, P.tensor_velocity_grid(n1, 8.0, 2), st,
                               nu_model="kn", kn=kn, tableau="DIRK2", name=f"b{i}"))
    pairs = []
    for pr in probs:
        d, f0, bc, dt = B.problem_setup(pr)
        s = B.Solver(d, dt=dt, bc_coef=bc, tableau="DIRK2", tau=1e-10, mode="MATCHED",
                     nu_model="kn", kn=pr.kn, fixed_iters=fixed)
        pairs.append((s, f0, d))
    batch = B.Batch([p[0] for p in pairs], graph=True, chunk_iters=3)
    fs = [p[1] for p in pairs]
    refs = [_oracle_instance(pr) for pr in probs]
    f_ref = [r[5] for r in refs]
    for step in range(2):
        st = batch.step(fs)
        for i, pr in enumerate(probs):
            geo, V, w, gens, lags, _, g, dt = refs[i]
            f_ref[i], sref = solver.bgk_step(geo, V, w, f_ref[i], g, dt, gens, lags,
                                             scheme="DIRK2", mode="MATCHED", nu_model="kn",
                                             kn=pr.kn, tau=1e-10, L=8.0,
                                             fixed_iters=fixed if fixed else None)
            got = pairs[i][2].unpack(fs[i]).cpu().numpy()
            err = float(np.abs(got - f_ref[i]).max() / np.abs(f_ref[i]).max())
            print(f"step {step} instance {i}: iters {st[i]['iters']} oracle {sref['iters']} "
                  f"err {err:.2e}", flush=True)
            assert st[i]["status"] == 0
            assert st[i]["iters"] == sref["iters"]
            assert err <= 1e-12
