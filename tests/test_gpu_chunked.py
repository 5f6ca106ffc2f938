"""Chunked Picard iteration: the stopping test of eq. convergence-criteria
evaluated on the device after every sweep, K iterations enqueued per host
poll (the rest of a chunk doing nothing once the test has fired), and
optionally each chunk replayed from a captured hipGraph.

Against the iteration that polls the host after every sweep (chunk_iters
0): equal iteration counts, MATCHED fallback counts and final ratios, and
bitwise-equal distributions, on every path the loop has (one and several
stages, fixed iteration counts that are not multiples of K, the FP32 form
and lagged facets, which alternate two iterate buffers, walls, a stage that
reaches l_max, a non-physical state); graph replays across steps and after
the distribution's buffer changes; and the small 2D workload against the
oracle.
"""
import os
import sys

import numpy as np
import pytest

import problems as P
from oracle import dag as odag
from oracle import geometry, solver
from oracle import walls as owalls

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
import paper_2608_19150_amd as B  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
VARIANTS = [(2, False), (3, True), (4, True)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(pr, nsteps, chunk, graph, *, fresh=False, setup_kw=None, walls=None, **kw):
    d, f, bc, dt = B.problem_setup(pr, **(setup_kw or {}))
    w = B.Walls(d, walls) if walls is not None else None
    s = B.Solver(d, dt=dt, bc_coef=bc, tableau=pr.tableau, nu_model=pr.nu_model,
                 nu_const=kw.pop("nu_const", pr.nu_const), kn=pr.kn, walls=w, chunk_iters=chunk,
                 graph=graph, **kw)
    stats = []
    for _ in range(nsteps):
        if fresh:
            f = f.clone()  # a new buffer: captured chunks are keyed on it
        st = s.step(f)
        stats.append((st["iters"], st["total_iters"], st["fallbacks"], st["last_ratio"],
                      st["sweeps"]))
    return d.unpack(f).cpu().numpy(), stats, dt


def _same(pr, nsteps, variants=VARIANTS, **kw):
    f0, st0, dt = _run(pr, nsteps, 0, False, **kw)
    for chunk, graph in variants:
        say("chunk", chunk, "graph", graph)
        f1, st1, _ = _run(pr, nsteps, chunk, graph, **kw)
        assert st1 == st0, (chunk, graph)
        assert np.array_equal(f1, f0), (chunk, graph)
    return f0, st0, dt


def test_chunked_c1_equals_per_iteration_and_oracle():
    """The small 2D workload (512 P1 triangles, 16^2 velocities, BE, MATCHED,
    tau 1e-10): five converged steps; the chunked runs equal the
    per-iteration run bitwise, and it matches the oracle (iteration counts
    equal, f within 1e-12)."""
    pr = P.config_c1()
    f, st, dt = _same(pr, 5)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    V, w = pr.vgrid.v, pr.vgrid.w
    gens, lags = odag.build_all(geo, V)
    fr = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    oit = []
    for _ in range(5):
        fr, o = solver.bgk_step(geo, V, w, fr, g, dt, gens, lags, scheme=pr.tableau,
                                mode="MATCHED", nu_model=pr.nu_model, nu_const=pr.nu_const,
                                kn=pr.kn, tau=1e-10, L=pr.vgrid.L)
        oit.append(o["iters"])
    assert [s[0] for s in st] == oit
    assert float(np.abs(f - fr).max() / np.abs(fr).max()) <= 1e-12


@pytest.mark.parametrize("tableau", ["DIRK2", "DIRK3"])
def test_chunked_multistage_converged(tableau):
    pr = P.small_problem(order=2, n_side=4, n_1d=6, state="fourier", nu_model="kn", kn=0.05,
                         tableau=tableau)
    _same(pr, 3, tau=1e-11)


def test_chunked_fixed_iterations_not_a_multiple_of_the_chunk():
    pr = P.small_problem(order=1, n_side=5, n_1d=6, state="sod", tableau="BDIRK2")
    _, st, _ = _same(pr, 2, fixed_iters=5)
    assert all(s[0] == [5, 5] for s in st)


def test_chunked_fp32_form_alternates_buffers_like_the_host_loop():
    pr = P.small_problem(order=2, n_side=4, n_1d=6, state="fourier")
    _same(pr, 2, precision=B.TGS_FP32_CORRECTION, tau=1e-10)


def test_chunked_lagged_facets_and_walls():
    """Lagged facets read the previous iterate (two buffers alternate) and
    the walls take their data from it before every sweep."""
    mesh = P.rectangle_mesh(10, 3, 0.0, 1.0, 0.0, 0.15)
    pr = P.Problem(mesh, 1, P.tensor_velocity_grid(8, 5.0, 2), P.sod_state(2))
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 1)
    V = pr.vgrid.v
    kinds = owalls.boundary_kinds(geo, lambda x, n: owalls.REFLECT if abs(n[1]) > 0.5 else
                                  owalls.INFLOW)
    rng = np.random.default_rng(31)
    lag = np.zeros((V.shape[0], geo.n_cells), dtype=np.uint8)
    for j in range(V.shape[0]):
        sp = odag.facet_speeds(geo, V[j])
        pick = (sp < 0) & (geo.nbr >= 0) & (rng.uniform(size=sp.shape) < 0.3)
        lag[j] = (pick * (1 << np.arange(3))[None, :]).sum(axis=1)
    _same(pr, 2, setup_kw={"lagged": lag}, walls=kinds, nu_const=2.0, tau=1e-10)


def test_chunked_cyclic_mesh_with_gpu_lagging():
    m = P.load_mesh_text(os.path.join(GOLDEN, "cyclic_tet_mesh.txt"))
    pr = P.Problem(mesh=m, order=1, vgrid=P.tensor_velocity_grid(6, 6.0, 3),
                   state=P.planar_riemann_state(3, seed=5, width=0.15), name="cyclic")
    _same(pr, 2, variants=[(3, True)], tau=1e-11)


def test_graph_replays_across_steps_and_new_buffers():
    """Eight steps from one solver, each on a new copy of f (so every chunk
    is captured again for the new buffer) and on one buffer (replays)."""
    pr = P.small_problem(order=1, n_side=6, n_1d=8, state="fourier", tableau="DIRK2")
    f0, st0, _ = _run(pr, 8, 0, False)
    for fresh in (True, False):
        f1, st1, _ = _run(pr, 8, 4, True, fresh=fresh)
        assert st1 == st0
        assert np.array_equal(f1, f0)


def test_chunked_not_converged_and_nonphysical_errors():
    pr = P.small_problem(order=1, n_side=5, n_1d=6, state="sod")
    outs = []
    for chunk, graph in [(0, False), (3, False), (3, True)]:
        d, f, bc, dt = B.problem_setup(pr)
        s = B.Solver(d, dt=dt, bc_coef=bc, tau=1e-30, l_max=4, chunk_iters=chunk, graph=graph)
        with pytest.raises(B.BGKError) as e:
            s.step(f)
        assert e.value.code == B.BGK_E_NOT_CONVERGED
        outs.append(d.unpack(f).cpu().numpy())
    assert all(np.array_equal(o, outs[0]) for o in outs[1:])
    bad = P.small_problem(dim=3, order=1, n_side=3, n_1d=6, state="riemann", nu_model="kn",
                          kn=0.1)
    for chunk, graph in [(0, False), (2, False), (4, True)]:
        d, f, bc, dt = B.problem_setup(bad)
        s = B.Solver(d, dt=dt, bc_coef=bc, fixed_iters=3, nu_model="kn", kn=0.1,
                     chunk_iters=chunk, graph=graph)
        with pytest.raises(B.BGKError) as e:
            for _ in range(2):
                s.step(f)
        assert e.value.code == B.BGK_E_NONPHYSICAL


def test_chunked_options_validated():
    pr = P.small_problem(order=1, n_side=3, n_1d=4)
    d, f, bc, dt = B.problem_setup(pr)
    with pytest.raises(B.BGKError) as e:
        B.Solver(d, dt=dt, bc_coef=bc, chunk_iters=2, timing=True)
    assert e.value.code == B.BGK_E_INVALID
    with pytest.raises(B.BGKError) as e:
        B.Solver(d, dt=dt, bc_coef=bc, chunk_iters=-1)
    assert e.value.code == B.BGK_E_INVALID


def test_split_moment_pass_in_steps_equals_host_loop():
    """4232 triangles with 91^2 = 8281 velocities: every moment pass is the
    velocity-split reduction (chunk sums, then their ordered sum, both
    skipped once the stopping test has fired; its values are checked against
    the oracle in the moment parity test).  Chunked and graph-replayed steps
    equal the host loop bit for bit, converged and with a fixed count."""
    pr = P.small_problem(order=1, n_side=46, n_1d=91, state="sod")
    _same(pr, 1, tau=1e-10)
    _same(pr, 1, variants=[(3, True)], fixed_iters=4)
