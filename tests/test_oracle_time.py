"""Oracle pins: Picard iteration, DIRK stages, conservation and stability.

* Tableaus: row sums equal c; the paper's printed 6-digit DIRK-3 constants
  (tests/golden/dirk3_tableau.txt, App. A) agree with the exact-gamma ones;
  B-stability matrix is PSD for backward Euler and the B-stable DIRK-2.
* A uniform Maxwellian with matching inflow stays unchanged; Picard stops
  after one iteration.
* nu = 0: Picard stops after two iterations at the pure transport solve.
* Relaxation ODE: a spatially uniform non-equilibrium state with
  stage-consistent inflow stays uniform and converges to
  M + (f0 - M) exp(-nu t) at order 1 (BE), 2 (DIRK-2), 3 (DIRK-3).
* Conservation (Prop. conservation laws): the change of the total mass,
  momentum and energy equals minus dt times the net boundary flux.
* L2 stability (Prop. linear stability): with nu = 0 or the linear
  Maxwellian, zero inflow, the phase-space L2 norm does not increase.
"""
import math

import numpy as np
import pytest

import problems as P
from oracle import dag, geometry, kinetic, solver, transport
from tests.conftest import read_golden


def test_tableaus():
    g = read_golden("dirk3_tableau.txt")
    A, b, c = solver.tableau("DIRK3")
    printed = np.array([[float(x) for x in g[f"A{i}"]] for i in (1, 2, 3)])
    assert np.abs(A - printed).max() < 1e-6
    assert np.abs(b - np.array([float(x) for x in g["b"]])).max() < 1e-6
    assert np.abs(c - np.array([float(x) for x in g["c"]])).max() < 1e-6
    for name in ("BE", "DIRK2", "DIRK3", "BDIRK2"):
        A, b, c = solver.tableau(name)
        assert np.allclose(A.sum(1), c)
        assert abs(b.sum() - 1.0) < 1e-14
    for name in ("BE", "BDIRK2"):
        A, b, _ = solver.tableau(name)
        B = np.diag(b)
        M = B @ A + A.T @ B - np.outer(b, b)
        assert np.linalg.eigvalsh(M).min() > -1e-14


def _setup(pr):
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    gens, lags = dag.build_all(geo, pr.vgrid.v)
    return geo, gens, lags


@pytest.mark.parametrize("mode", ["MATCHED", "DIRECT"])
def test_uniform_maxwellian_preserved(mode):
    L = 6.0 if mode == "MATCHED" else 10.0
    n1 = 8 if mode == "MATCHED" else 40
    pr = P.small_problem(n_side=3, n_1d=n1, L=L, state="uniform")
    geo, gens, lags = _setup(pr)
    V, w = pr.vgrid.v, pr.vgrid.w
    f0 = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    dt = solver.explicit_dt(geo, V, 10.0)
    f = f0
    for _ in range(5):
        f, st = solver.bgk_step(geo, V, w, f, g, dt, gens, lags, mode=mode, L=L)
        assert st["iters"] == [1]
    assert np.abs(f - f0).max() <= 1e-13 * f0.max()


def test_nu_zero_two_iterations_equal_transport():
    pr = P.small_problem(n_side=3, n_1d=6)
    geo, gens, lags = _setup(pr)
    V, w = pr.vgrid.v, pr.vgrid.w
    f0 = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    dt = solver.explicit_dt(geo, V, 10.0)
    f1, st = solver.bgk_step(geo, V, w, f0, g, dt, gens, lags, nu_const=0.0)
    assert st["iters"] == [2]
    sig = np.full((geo.n_cells, geo.n_p), 1.0 / dt)
    for j in range(0, V.shape[0], 7):
        fd = transport.dense_solve(geo, V[j], sig, 0 * sig, 0 * f0[:, :, j], f0[:, :, j] / dt,
                                   g[:, :, j])
        assert np.abs(fd - f1[:, :, j]).max() <= 1e-13 * np.abs(fd).max()


@pytest.mark.parametrize("scheme,order", [("BE", 1), ("DIRK2", 2), ("DIRK3", 3)])
def test_relaxation_order(scheme, order):
    pr = P.small_problem(n_side=2, n_1d=8)
    geo, gens, lags = _setup(pr)
    V, w = pr.vgrid.v, pr.vgrid.w
    nu, T = 2.0, 0.4
    f0v = (kinetic.maxwellian_values(np.array([1.0]), np.array([[0.5, 0.0]]), np.array([0.8]), V)[0]
           + kinetic.maxwellian_values(np.array([0.5]), np.array([[-1.0, 0.3]]), np.array([1.2]), V)[0])
    coef, _ = kinetic.matched_coefficients(kinetic.moments(f0v, V, w)[None], V, w)
    Mv = kinetic.coef_values(coef, V)[0]
    A, b, c = solver.tableau(scheme)
    errs = []
    for nsteps in (4, 8, 16):
        dt = T / nsteps
        f = np.broadcast_to(f0v, (geo.n_cells, geo.n_p, V.shape[0])).copy()
        y = f0v.copy()
        for _ in range(nsteps):
            # stage values of y' = nu (M - y) under this tableau, written with
            # the right-hand side evaluated directly (not the recursion)
            ys = []
            for s in range(A.shape[0]):
                rhs = y + dt * sum(A[s, r] * nu * (Mv - ys[r]) for r in range(s))
                ys.append((rhs + dt * A[s, s] * nu * Mv) / (1.0 + dt * A[s, s] * nu))
            nbf = geo.bnode_x.shape[0]
            gb = lambda s, ys=ys: np.broadcast_to(ys[s], (nbf, geo.n_fp, V.shape[0])).copy()  # noqa: E731
            f, _ = solver.bgk_step(geo, V, w, f, gb, dt, gens, lags, scheme=scheme,
                                   nu_const=nu, tau=1e-13)
            y = y + dt * sum(b[s] * nu * (Mv - ys[s]) for s in range(A.shape[0]))
        assert np.abs(f - y).max() <= 1e-11 * f.max()          # uniform, equals the ODE
        exact = Mv + (f0v - Mv) * math.exp(-nu * T)
        errs.append(np.abs(f[0, 0] - exact).max())
    slopes = [math.log(errs[i] / errs[i + 1], 2) for i in range(2)]
    assert abs(slopes[-1] - order) < 0.15, (errs, slopes)


def _boundary_flux(geo, V, w, f, g):
    """Net outward flux sum_j w_j e_j sum_{boundary facets} (v.n) int_e fhat."""
    E = kinetic.collision_invariants(V) * w[:, None]
    tot = np.zeros(E.shape[1])
    for c in range(geo.n_cells):
        for k in range(geo.dim + 1):
            if geo.nbr[c, k] >= 0:
                continue
            fn = geo.ref["face_nodes"][k]
            Mf = geo.area[c, k] * geo.ref["face_mass"][k][np.ix_(fn, fn)]
            s = V @ geo.normal[c, k]
            vals = np.where(s[None, :] > 0, f[c, fn, :], g[geo.bface[c, k]])
            tot += (Mf.sum(0) @ vals * s) @ E
    return tot


@pytest.mark.parametrize("scheme", ["BE", "DIRK2"])
def test_discrete_conservation(scheme):
    pr = P.small_problem(n_side=4, n_1d=10, order=1)
    geo, gens, lags = _setup(pr)
    V, w = pr.vgrid.v, pr.vgrid.w
    f0 = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    dt = solver.explicit_dt(geo, V, 10.0)
    f1, st = solver.bgk_step(geo, V, w, f0, g, dt, gens, lags, scheme=scheme, nu_const=5.0,
                             tau=1e-13)
    E = kinetic.collision_invariants(V) * w[:, None]
    tot = lambda f: np.einsum("c,cp,pq,cqj,jm->m", geo.vol, np.ones((geo.n_cells, geo.n_p)),  # noqa: E731
                              geo.ref["mass"], f, E)
    change = tot(f1) - tot(f0)
    if scheme == "BE":
        flux = _boundary_flux(geo, V, w, f1, g)
    else:
        A, b, _ = solver.tableau(scheme)
        # stiffly accurate two-stage scheme: recompute stage 1 for its flux
        q = f0 / (dt * A[0, 0])
        fs1, _, _, _, _ = solver.picard_stage(geo, V, w, q, g, 1.0 / (dt * A[0, 0]), f0, gens, lags,
                                              dt=dt, nu_const=5.0, tau=1e-13)
        flux = b[0] * _boundary_flux(geo, V, w, fs1, g) + b[1] * _boundary_flux(geo, V, w, f1, g)
    scale = np.abs(tot(f0)).max()
    assert np.abs(change + dt * flux).max() <= 1e-10 * scale, (change, -dt * flux)


@pytest.mark.parametrize("mode,nu", [("MATCHED", 0.0), ("LINEAR", 3.0)])
def test_l2_stability(mode, nu):
    pr = P.small_problem(n_side=3, n_1d=8, state="riemann")
    geo, gens, lags = _setup(pr)
    V, w = pr.vgrid.v, pr.vgrid.w
    f = solver.initial_condition(geo, V, pr.state)
    g = np.zeros((geo.bnode_x.shape[0], geo.n_fp, V.shape[0]))
    dt = solver.explicit_dt(geo, V, 10.0)
    norm = lambda f: np.einsum("c,cpj,pq,cqj,j->", geo.vol, f, geo.ref["mass"], f, w)  # noqa: E731
    prev = norm(f)
    for _ in range(4):
        f, _ = solver.bgk_step(geo, V, w, f, g, dt, gens, lags, mode=mode, nu_const=nu,
                               L=pr.vgrid.L)
        cur = norm(f)
        assert cur <= prev * (1 + 1e-13)
        prev = cur


def test_explicit_dt_hand_built_meshes():
    """eq. explicit-dt, dt = C (1/d) (1/(2k+1)) h_min / max_j |v_j| with
    h_min = (min cell measure)^(1/d), on meshes whose numbers are known by
    hand:
    * two triangles (0,0),(1,0),(0,1) [area 1/2] and (1,0),(3,0),(0,1)
      [area 1]: h_min = sqrt(1/2); velocities (3,4) and (-1,0): max |v| = 5;
      P1, C = 10: dt = 10 (1/2)(1/3) sqrt(1/2) / 5 = 0.23570226039551584;
      P2 (1/(2k+1) = 1/5): 0.6 of that;
    * the unit corner tetrahedron (volume 1/6), velocity (1, 2, 2) (|v| = 3),
      P1, C = 10: 10 (1/3)(1/3) (1/6)^(1/3) / 3 = 0.2038226696848535."""
    vert = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [3.0, 0.0]])
    cells = np.array([[0, 1, 2], [1, 3, 2]])
    V = np.array([[3.0, 4.0], [-1.0, 0.0]])
    geo = geometry.build(vert, cells, 1)
    assert abs(solver.explicit_dt(geo, V, 10.0) - 0.23570226039551584) < 1e-15
    geo2 = geometry.build(vert, cells, 2)
    assert abs(solver.explicit_dt(geo2, V, 10.0) - 0.6 * 0.23570226039551584) < 1e-15
    tet = geometry.build(np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]),
                         np.array([[0, 1, 2, 3]]), 1)
    assert abs(solver.explicit_dt(tet, np.array([[1.0, 2.0, 2.0], [0.5, 0, 0]]), 10.0)
               - 0.2038226696848535) < 1e-15


def test_relative_changes_hand_computed():
    """eq. convergence-criteria with the A13 guard on two 2D nodes
    (U = (n, n u_1, n u_2, E) per node).
    * A gas at rest: U_old = [(1,0,0,1), (2,0,0,3)], U_new = [(1.1,0.3,-0.4,1),
      (2,0,0,2.5)].  Density: |(0.1, 0)| / |(1, 2)| = 0.1/sqrt5.  Momentum:
      the old momentum is 0, so the denominator is |n_old| = sqrt5 and the
      change |((0.3,-0.4),(0,0))| = 0.5 gives 0.5/sqrt5.  Energy: |(0,-0.5)| /
      |(1,3)| = 0.5/sqrt10.
    * A moving gas whose momentum norm (5) exceeds its density norm (2 sqrt2):
      no guard.  Energy is never guarded: |E_old| = 0.5 sqrt2 < |n_old| and
      the ratio is 0.1 sqrt2 / (0.5 sqrt2) = 0.2."""
    Uo = np.array([[1.0, 0, 0, 1], [2, 0, 0, 3]])
    Un = np.array([[1.1, 0.3, -0.4, 1], [2, 0, 0, 2.5]])
    r = solver.relative_changes(Un, Uo, 2)
    np.testing.assert_allclose(r, [0.044721359549995794, 0.22360679774997896,
                                   0.15811388300841897], rtol=1e-15)
    Uo = np.array([[2.0, 3, 4, 0.5], [2, 0, 0, 0.5]])
    Un = np.array([[2.0, 3, 4.5, 0.6], [2, 0, 0, 0.6]])
    r = solver.relative_changes(Un, Uo, 2)
    np.testing.assert_allclose(r, [0.0, 0.1, 0.2], rtol=1e-15, atol=0)


def test_converged_step_does_not_depend_on_lagged_facets():
    """Lagging inflow facets (Sec. 4: the lagged part of the inflow boundary
    takes the previous iterate) changes every sweep but not the fixed point:
    a converged step with a random lagged set equals the unlagged one to the
    stopping tolerance."""
    pr = P.small_problem(dim=2, order=1, n_side=4, n_1d=6, state="sod")
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, pr.order)
    V, w = pr.vgrid.v, pr.vgrid.w
    rng = np.random.default_rng(11)
    lags = np.zeros((V.shape[0], geo.n_cells, geo.dim + 1), dtype=bool)
    for j in range(V.shape[0]):
        s = dag.facet_speeds(geo, V[j])
        cand = (s < 0) & (geo.nbr >= 0)
        lags[j] = cand & (rng.uniform(size=cand.shape) < 0.3)
    assert lags.sum() > 10
    f0 = solver.initial_condition(geo, V, pr.state)
    g = solver.boundary_values(geo, V, pr.state)
    dt = solver.explicit_dt(geo, V, pr.cfl)
    gens0, lag0 = dag.build_all(geo, V)
    gens1, lag1 = dag.build_all(geo, V, lagged=lags)
    f_a, st_a = solver.bgk_step(geo, V, w, f0, g, dt, gens0, lag0, tau=1e-13)
    f_b, st_b = solver.bgk_step(geo, V, w, f0, g, dt, gens1, lag1, tau=1e-13)
    assert st_b["iters"][0] > st_a["iters"][0]          # lagging slows the iteration
    assert np.abs(f_b - f_a).max() <= 1e-10 * np.abs(f_a).max()
