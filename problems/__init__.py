"""Seeded synthetic problem generators.

This module defines *problems*, not the method: meshes (vertex coordinates and
simplex connectivity), discrete velocity sets (nodes and quadrature weights as
stated by each workload), and the macroscopic states (n, u, theta) that define
initial and inflow data as functions of position.  It is the only code shared
by the CPU oracle and the GPU path; it contains none of the method's
arithmetic (no element matrices, sweeps, moments or Maxwellians).

Workloads follow the paper's Sod-type test problems (Sec. 5.1: left state
(1, 0, 1), right state (0.125, 0, 0.8), inflow data equal to the initial
equilibrium) on synthetic seeded Delaunay meshes that stand in for the
paper's meshes, which are not public.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import Delaunay

__all__ = [
    "Mesh", "VelocityGrid", "State", "Problem",
    "jittered_square_mesh", "graded_square_mesh", "jittered_cube_mesh", "flipped_cube_mesh",
    "structured_square_mesh",
    "tensor_velocity_grid",
    "sod_state", "planar_riemann_state", "fourier_state", "uniform_state",
    "config_c1", "config_c2", "config_c3", "config_c4_instances", "small_problem",
]


@dataclass
class Mesh:
    """Simplicial mesh: ``vert`` f64[n_vert][dim], ``cells`` i32[n_cells][dim+1]."""
    vert: np.ndarray
    cells: np.ndarray

    @property
    def dim(self) -> int:
        return int(self.vert.shape[1])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])


@dataclass
class VelocityGrid:
    """Discrete velocities ``v`` f64[n_v][dim] with weights ``w`` f64[n_v].

    Ordering is the row-major tensor index with the first axis slowest.
    ``nodes_1d``/``weights_1d`` hold the per-axis factors for tensor grids.
    """
    v: np.ndarray
    w: np.ndarray
    nodes_1d: np.ndarray | None = None
    weights_1d: np.ndarray | None = None
    L: float = 0.0
    dg_cells: int = 0      # > 0: Q2 DG velocity space, this many uniform cells per axis

    @property
    def n_v(self) -> int:
        return int(self.v.shape[0])

    @property
    def dim(self) -> int:
        return int(self.v.shape[1])


@dataclass
class State:
    """A macroscopic state field: ``params(x)`` -> (n, u[dim], theta) arrays."""
    kind: str
    data: dict = field(default_factory=dict)

    def params(self, x: np.ndarray):
        x = np.asarray(x, dtype=np.float64)
        npts, dim = x.shape
        if self.kind == "uniform":
            n = np.full(npts, self.data["n"])
            u = np.tile(np.asarray(self.data["u"], dtype=np.float64), (npts, 1))
            th = np.full(npts, self.data["theta"])
            return n, u, th
        if self.kind == "plane":
            nrm = np.asarray(self.data["normal"], dtype=np.float64)
            c = np.asarray(self.data["center"], dtype=np.float64)
            nl, ul, tl = self.data["left"]
            nr, ur, tr = self.data["right"]
            ul = np.asarray(ul, dtype=np.float64)[:dim]
            ur = np.asarray(ur, dtype=np.float64)[:dim]
            width = float(self.data.get("width", 0.0))
            if width > 0.0:
                # jump spread over a tanh layer of the given width
                s = 0.5 * (1.0 + np.tanh(((x - c) @ nrm) / width))
                n = nl + (nr - nl) * s
                u = ul[None, :] + (ur - ul)[None, :] * s[:, None]
                th = tl + (tr - tl) * s
                return n.astype(np.float64), u, th.astype(np.float64)
            left = (x - c) @ nrm < 0.0
            n = np.where(left, nl, nr).astype(np.float64)
            u = np.where(left[:, None], ul[None, :], ur[None, :])
            th = np.where(left, tl, tr).astype(np.float64)
            return n, u, th
        if self.kind == "fourier":
            out = []
            for name in ["n"] + [f"u{a}" for a in range(dim)] + ["theta"]:
                k, amp, phase, base, rel = (self.data[name][key] for key in
                                            ("k", "amp", "phase", "base", "relative"))
                s = np.zeros(npts)
                for m in range(len(amp)):
                    s += amp[m] * np.sin(2.0 * math.pi * (x @ k[m]) + phase[m])
                out.append(base * (1.0 + s) if rel else base + s)
            n = out[0]
            u = np.stack(out[1:1 + dim], axis=1)
            th = out[1 + dim]
            return n, u, th
        raise ValueError(f"unknown state kind {self.kind}")


@dataclass
class Problem:
    """One workload instance: mesh, polynomial order, velocities, state, physics."""
    mesh: Mesh
    order: int
    vgrid: VelocityGrid
    state: State
    nu_model: str = "const"         # "const" or "kn"
    nu_const: float = 1.0
    kn: float = 1.0
    tableau: str = "BE"             # "BE" or "DIRK2"
    cfl: float = 10.0
    n_steps: int = 1
    tau: float = 1e-10
    name: str = ""


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def _delaunay(points: np.ndarray) -> np.ndarray:
    tri = Delaunay(points, qhull_options="Qbb Qc Qz Q12")
    return np.ascontiguousarray(tri.simplices.astype(np.int32))


def _simplex_measures(vert: np.ndarray, cells: np.ndarray) -> np.ndarray:
    x0 = vert[cells[:, 0]]
    J = np.stack([vert[cells[:, k + 1]] - x0 for k in range(vert.shape[1])], axis=2)
    return np.abs(np.linalg.det(J)) / math.factorial(vert.shape[1])


def _drop_degenerate(vert, cells, rel=1e-9):
    vol = _simplex_measures(vert, cells)
    keep = vol > rel * vol.mean()
    if not np.all(keep):
        raise RuntimeError(f"Delaunay produced {np.count_nonzero(~keep)} degenerate simplices")
    return cells


def jittered_square_mesh(n_side: int, jitter: float, seed: int) -> Mesh:
    """(n_side+1)^2 lattice on [0,1]^2, interior points jittered by U(-jitter*h, jitter*h)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n_side
    g = np.linspace(0.0, 1.0, n_side + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    interior = (pts[:, 0] > 0) & (pts[:, 0] < 1) & (pts[:, 1] > 0) & (pts[:, 1] < 1)
    pts[interior] += rng.uniform(-jitter * h, jitter * h, size=(np.count_nonzero(interior), 2))
    cells = _drop_degenerate(pts, _delaunay(pts))
    expected = 2 * n_side * n_side
    if cells.shape[0] != expected:
        raise RuntimeError(f"expected {expected} triangles, got {cells.shape[0]}")
    return Mesh(pts, cells)


def structured_square_mesh(n_side: int) -> Mesh:
    """Right-triangle mesh of [0,1]^2: each lattice square split along its (0,0)-(1,1) diagonal."""
    g = np.linspace(0.0, 1.0, n_side + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    idx = lambda i, j: i * (n_side + 1) + j  # noqa: E731
    cells = []
    for i in range(n_side):
        for j in range(n_side):
            a, b, c, d = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
            cells.append((a, b, c))
            cells.append((a, c, d))
    return Mesh(pts, np.asarray(cells, dtype=np.int32))


def rectangle_mesh(nx: int, ny: int, x0: float, x1: float, y0: float, y1: float) -> Mesh:
    """Right-triangle mesh of [x0,x1] x [y0,y1]: an nx x ny lattice of
    rectangles, each split along its lower-left to upper-right diagonal."""
    gx = np.linspace(x0, x1, nx + 1)
    gy = np.linspace(y0, y1, ny + 1)
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    idx = lambda i, j: i * (ny + 1) + j  # noqa: E731
    cells = []
    for i in range(nx):
        for j in range(ny):
            a, b, c, d = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
            cells.append((a, b, c))
            cells.append((a, c, d))
    return Mesh(pts, np.asarray(cells, dtype=np.int32))


def graded_square_mesh(n_side: int, jitter: float, seed: int, ratio: float = 4.0) -> Mesh:
    """Jittered lattice warped per axis by g(s) = s + a sin(2 pi s)/(2 pi).

    With a = (ratio-1)/(ratio+1) the spacing at the centre is ``ratio`` times
    finer than at the boundary.  2*n_side^2 triangles.
    """
    rng = np.random.default_rng(seed)
    a = (ratio - 1.0) / (ratio + 1.0)
    h = 1.0 / n_side
    g = np.linspace(0.0, 1.0, n_side + 1)
    S, T = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([S.ravel(), T.ravel()], axis=1)
    interior = (pts[:, 0] > 0) & (pts[:, 0] < 1) & (pts[:, 1] > 0) & (pts[:, 1] < 1)
    pts[interior] += rng.uniform(-jitter * h, jitter * h, size=(np.count_nonzero(interior), 2))
    pts = pts + a * np.sin(2.0 * math.pi * pts) / (2.0 * math.pi)
    pts[np.isclose(pts, 0.0, atol=1e-15)] = 0.0
    pts[np.isclose(pts, 1.0, atol=1e-15)] = 1.0
    cells = _drop_degenerate(pts, _delaunay(pts))
    return Mesh(pts, cells)


def jittered_cube_mesh(n_side: int, jitter: float, seed: int) -> Mesh:
    """(n_side+1)^3 lattice on [0,1]^3.  Interior points are jittered in all
    directions; boundary points only tangentially (edges along the edge,
    corners fixed), so the cube stays exact and no boundary square is
    cocircular."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n_side
    g = np.linspace(0.0, 1.0, n_side + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    free = (pts > 0) & (pts < 1)
    pts = pts + np.where(free, rng.uniform(-jitter * h, jitter * h, size=pts.shape), 0.0)
    cells = _drop_degenerate(pts, _delaunay(pts))
    return Mesh(pts, cells)


def flipped_cube_mesh(n_interior: int = 30, n_flips: int = 40, seed: int = 3) -> Mesh:
    """A valid tetrahedral mesh of [0,1]^3 that is not Delaunay: the Delaunay
    mesh of the cube's corners and ``n_interior`` seeded random points, then
    ``n_flips`` random 2-3 flips (two tetrahedra abcd, abce whose union is
    convex across abc become abde, bcde, cade).  Such meshes have upwind
    cycles for some directions (Delaunay meshes never do).  Cells are
    positively oriented; flips that would leave a tetrahedron thinner than
    1e-3 of its neighbours' volume are skipped."""
    rng = np.random.default_rng(seed)
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], float)
    pts = np.vstack([corners, rng.uniform(0.1, 0.9, size=(n_interior, 3))])

    def det(c):
        x = pts[list(c)]
        return float(np.linalg.det(np.stack([x[1] - x[0], x[2] - x[0], x[3] - x[0]])))

    cells = [list(c) for c in Delaunay(pts).simplices.astype(np.int64)]
    for c in cells:
        if det(c) < 0:
            c[0], c[1] = c[1], c[0]
    done = 0
    for _ in range(200000):
        if done >= n_flips:
            break
        fmap = {}
        for t, c in enumerate(cells):
            for k in range(4):
                key = tuple(sorted(c[i] for i in range(4) if i != k))
                fmap.setdefault(key, []).append((t, c[k]))
        faces = [(f, w) for f, w in fmap.items() if len(w) == 2]
        (a, b, c), ((t1, d), (t2, e)) = faces[rng.integers(len(faces))]
        # does segment d-e pass through the inside of triangle abc?
        M = np.stack([pts[e] - pts[d], pts[a] - pts[b], pts[a] - pts[c]], 1)
        try:
            s_, u_, w_ = np.linalg.solve(M, pts[a] - pts[d])
        except np.linalg.LinAlgError:
            continue
        if not (0 < s_ < 1 and u_ > 0.05 and w_ > 0.05 and 1 - u_ - w_ > 0.05):
            continue
        new = [[a, b, d, e], [b, c, d, e], [c, a, d, e]]
        ref = 0.5 * (abs(det(cells[t1])) + abs(det(cells[t2])))
        if min(abs(det(q)) for q in new) < 1e-3 * ref:
            continue
        for q in new:
            if det(q) < 0:
                q[0], q[1] = q[1], q[0]
        for t in sorted([t1, t2], reverse=True):
            cells.pop(t)
        cells.extend(new)
        done += 1
    out = np.array(cells, dtype=np.int32)
    if abs(_simplex_measures(pts, out).sum() - 1.0) > 1e-12:
        raise RuntimeError("flipped mesh does not tile the cube")
    return Mesh(pts, out)


def load_mesh_text(path: str) -> Mesh:
    """Reads a mesh written as text: '#' comment lines, "vert N" then N lines
    of coordinates, "cells M" then M lines of vertex indices."""
    with open(path) as fh:
        lines = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    nv = int(lines[0][1])
    vert = np.array([[float(x) for x in ln] for ln in lines[1:1 + nv]], dtype=np.float64)
    assert lines[1 + nv][0] == "cells"
    nc = int(lines[1 + nv][1])
    cells = np.array([[int(x) for x in ln] for ln in lines[2 + nv:2 + nv + nc]], dtype=np.int32)
    return Mesh(vert, cells)


def jittered_box_mesh(nx: int, ny: int, nz: int, lx: float, ly: float, lz: float,
                      jitter: float, seed: int) -> Mesh:
    """(nx+1) x (ny+1) x (nz+1) lattice on [0,lx] x [0,ly] x [0,lz] with
    spacings lx/nx, ly/ny, lz/nz; interior points jittered in all directions,
    boundary points only tangentially (the faces stay exact), then
    Delaunay."""
    rng = np.random.default_rng(seed)
    L = np.array([lx, ly, lz])
    n = np.array([nx, ny, nz])
    h = L / n
    axes = [np.linspace(0.0, L[a], n[a] + 1) for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    free = (pts > 0) & (pts < L[None, :])
    pts = pts + np.where(free, rng.uniform(-1.0, 1.0, size=pts.shape) * jitter * h[None, :], 0.0)
    cells = _drop_degenerate(pts, _delaunay(pts))
    return Mesh(pts, cells)


# ----------------------------------------------------------------------------
# velocity grids
# ----------------------------------------------------------------------------

def tensor_velocity_grid(n_1d: int, L: float, dim: int) -> VelocityGrid:
    """n_1d equispaced nodes v_k = -L + 2Lk/(n_1d-1) per axis with trapezoid
    weights h*(1/2, 1, ..., 1, 1/2), h = 2L/(n_1d-1); tensor product with the
    first axis slowest and product weights, as the workloads state."""
    x = np.linspace(-L, L, n_1d)
    hv = 2.0 * L / (n_1d - 1)
    w1 = np.full(n_1d, hv)
    w1[0] *= 0.5
    w1[-1] *= 0.5
    grids = np.meshgrid(*([x] * dim), indexing="ij")
    v = np.stack([gg.ravel() for gg in grids], axis=1)
    wg = np.meshgrid(*([w1] * dim), indexing="ij")
    w = np.ones(v.shape[0])
    for gg in wg:
        w = w * gg.ravel()
    return VelocityGrid(np.ascontiguousarray(v), w, x, w1, L)


def gl_velocity_grid(n_cells: int, L: float, dim: int) -> VelocityGrid:
    """The velocity space of the paper's Sec. 3.2: n_cells uniform cells per
    axis on [-L, L], in each the 3 Gauss-Legendre nodes and weights of Q2
    (k_v = 2); tensor product with the first axis slowest."""
    h = 2.0 * L / n_cells
    ref = np.array([-math.sqrt(0.6), 0.0, math.sqrt(0.6)])
    wref = np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])
    centres = -L + h * (np.arange(n_cells) + 0.5)
    x = (centres[:, None] + 0.5 * h * ref[None, :]).ravel()
    w1 = np.tile(0.5 * h * wref, n_cells)
    grids = np.meshgrid(*([x] * dim), indexing="ij")
    v = np.stack([gg.ravel() for gg in grids], axis=1)
    wg = np.meshgrid(*([w1] * dim), indexing="ij")
    w = np.ones(v.shape[0])
    for gg in wg:
        w = w * gg.ravel()
    return VelocityGrid(np.ascontiguousarray(v), w, x, w1, L, n_cells)


# ----------------------------------------------------------------------------
# states
# ----------------------------------------------------------------------------

SOD_LEFT = (1.0, (0.0, 0.0, 0.0), 1.0)
SOD_RIGHT = (0.125, (0.0, 0.0, 0.0), 0.8)


def uniform_state(n=1.0, u=(0.0, 0.0, 0.0), theta=1.0, dim=2) -> State:
    return State("uniform", {"n": n, "u": list(u)[:dim], "theta": theta})


def sod_state(dim: int) -> State:
    """Sod split at x_1 = 0.5: left (x_1 < 0.5) = (1,0,1), right = (0.125,0,0.8)."""
    nrm = np.zeros(dim)
    nrm[0] = 1.0
    return State("plane", {"normal": nrm, "center": np.full(dim, 0.5),
                           "left": SOD_LEFT, "right": SOD_RIGHT})


def planar_riemann_state(dim: int, seed: int, width: float = 0.0) -> State:
    """Sod states split by the plane through the domain centre with a seeded
    random normal; width > 0 spreads the jump over a tanh layer."""
    rng = np.random.default_rng(seed)
    nrm = rng.normal(size=dim)
    nrm /= np.linalg.norm(nrm)
    return State("plane", {"normal": nrm, "center": np.full(dim, 0.5),
                           "left": SOD_LEFT, "right": SOD_RIGHT, "width": width})


def random_riemann_state(dim: int, seed: int, width: float = 0.0) -> State:
    """Sod-like planar Riemann problem with seeded states and normal: left
    (n, theta) in [0.5, 1.5] x [0.7, 1.3], right n in [0.1, 0.5], theta in
    [0.6, 1.0], both at rest; the plane passes through a seeded point of the
    central half of the domain."""
    rng = np.random.default_rng(seed)
    nrm = rng.normal(size=dim)
    nrm /= np.linalg.norm(nrm)
    left = (float(rng.uniform(0.5, 1.5)), (0.0, 0.0, 0.0), float(rng.uniform(0.7, 1.3)))
    right = (float(rng.uniform(0.1, 0.5)), (0.0, 0.0, 0.0), float(rng.uniform(0.6, 1.0)))
    return State("plane", {"normal": nrm, "center": rng.uniform(0.25, 0.75, size=dim),
                           "left": left, "right": right, "width": width})


def fourier_state(dim: int, seed: int, modes: int = 8, amplitude: float = 0.1) -> State:
    """Smooth seeded perturbation of (1, 0, 1): each field gets a sum of
    ``modes`` sines with integer wave vectors in [1,4]^dim, scaled so the
    worst-case amplitude is ``amplitude`` (relative for n and theta,
    absolute for u)."""
    rng = np.random.default_rng(seed)
    data = {}
    names = ["n"] + [f"u{a}" for a in range(dim)] + ["theta"]
    for name in names:
        k = rng.integers(1, 5, size=(modes, dim)).astype(np.float64)
        amp = rng.uniform(0.2, 1.0, size=modes)
        amp *= amplitude / amp.sum()
        phase = rng.uniform(0.0, 2.0 * math.pi, size=modes)
        rel = name in ("n", "theta")
        data[name] = {"k": k, "amp": amp, "phase": phase, "base": 1.0 if rel else 0.0,
                      "relative": rel}
    return State("fourier", data)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def config_c1() -> Problem:
    """512-triangle jittered Delaunay square, P1, 16x16 velocities on [-6,6]^2,
    nu = 1, Sod, backward Euler at CFL 10, 5 steps, tau = 1e-10."""
    mesh = jittered_square_mesh(16, 0.25, seed=1000)
    return Problem(mesh, 1, tensor_velocity_grid(16, 6.0, 2), sod_state(2),
                   nu_model="const", nu_const=1.0, tableau="BE", cfl=10.0,
                   n_steps=5, tau=1e-10, name="c1_sod_p1_512tri_16x16")


def config_c2(n_side: int = 316) -> Problem:
    """~200k-triangle graded Delaunay square (4x finer at the centre), P2,
    32x32 velocities on [-8,8]^2, nu = n theta^{-1/2}/Kn with Kn = 1e-2,
    seeded 8-mode Fourier perturbation of (1,0,1), 2-stage L-stable DIRK,
    CFL 10, 20 steps."""
    mesh = graded_square_mesh(n_side, 0.2, seed=2000)
    return Problem(mesh, 2, tensor_velocity_grid(32, 8.0, 2), fourier_state(2, seed=2001),
                   nu_model="kn", kn=1e-2, tableau="DIRK2", cfl=10.0, n_steps=20,
                   tau=1e-10, name=f"c2_fourier_p2_{2 * n_side * n_side}tri_32x32")


def config_c2_q2(n_side: int = 316, vcells: int = 10) -> Problem:
    """The 2D workload's mesh, state and physics on the Q2 velocity space of
    Sec. 3.2: vcells uniform cells per axis on [-8, 8] with 3 Gauss-Legendre
    nodes each (10 cells: 30^2 = 900 velocities)."""
    base = config_c2(n_side)
    return Problem(base.mesh, 2, gl_velocity_grid(vcells, 8.0, 2), base.state,
                   nu_model=base.nu_model, kn=base.kn, tableau=base.tableau, cfl=base.cfl,
                   n_steps=base.n_steps, tau=base.tau,
                   name=f"c2_fourier_p2_{2 * n_side * n_side}tri_q2_{3 * vcells}x{3 * vcells}")


DUCT = (0.3, 0.1, 0.1)


def duct_problem(vcells: int = 16, nu: float = 1.0, lattice=(24, 8, 8)) -> Problem:
    """The paper's duct (Sec. 5.3) at one GPU's scale: [0, 0.3] x [0, 0.1] x
    [0, 0.1] as a jittered lattice (24 x 8 x 8 cells of 0.0125, Delaunay
    tetrahedra, P1; the paper's meshes are graded, clustered at the walls
    and far larger), initial Maxwellian (1, 0, 1) except near the inlet
    (below), Q2 velocity space on [-12, 12]^3 with vcells cells per axis
    (16: 110,592 velocities, the paper's count for its collisional case),
    constant nu = 1 (its transition regime), backward Euler with DUCT_DT.
    On this mesh the layers at the inlet and the walls have the width
    |v| / (1/dt + nu), far below a cell at the paper's dt = 1e-3 or
    nu = 1000, and the method (no limiter) then produces non-physical nodal
    moments; dt = 5e-3 with nu = 1 stays physical.  Boundary data:
    duct_boundary."""
    mesh = jittered_box_mesh(*lattice, *DUCT, 0.2, 8000)
    # the inflow (1, (2, 0, 0), 1) ramps down to the gas at rest over a tanh
    # layer 1.5 lattice cells wide centred 3 such widths from the inlet, so
    # the data at the inlet agree with the inflow: a jump there is a boundary
    # layer far thinner than a cell (|v|/(1/dt + nu) << h), which P1 cannot
    # resolve without non-physical nodal moments
    w = 1.5 * DUCT[0] / lattice[0]
    st = State("plane", {"normal": np.array([1.0, 0.0, 0.0]), "center": np.array([3 * w, 0, 0]),
                         "left": (1.0, (2.0, 0.0, 0.0), 1.0), "right": (1.0, (0.0, 0.0, 0.0), 1.0),
                         "width": w})
    return Problem(mesh, 1, gl_velocity_grid(vcells, 12.0, 3), st, nu_model="const",
                   nu_const=nu, tableau="BE", name=f"duct_q2_{vcells}")


DUCT_DT = 5e-3


def duct_boundary(facet_midpoints: np.ndarray):
    """Per boundary facet: kind (0 inflow, 1 bounce-back on the x_2 walls,
    2 reflection on the x_3 walls) and the inflow state's (n, u, theta) with
    n = 0 meaning zero inflow: Maxwellian (1, (2, 0, 0), 1) at x_1 = 0, zero
    at x_1 = 0.3."""
    x = facet_midpoints
    tol = 1e-12
    kinds = np.zeros(x.shape[0], dtype=np.int8)
    kinds[(np.abs(x[:, 1]) < tol) | (np.abs(x[:, 1] - DUCT[1]) < tol)] = 1
    kinds[(np.abs(x[:, 2]) < tol) | (np.abs(x[:, 2] - DUCT[2]) < tol)] = 2
    left = np.abs(x[:, 0]) < tol
    prim = np.tile(np.array([0.0, 0.0, 0.0, 0.0, 1.0]), (x.shape[0], 1))
    prim[left] = [1.0, 2.0, 0.0, 0.0, 1.0]
    return kinds, prim


SOD_STRIP_HALF_HEIGHT = 3.0 / 128.0


def sod_strip_problem(vcells: int, nu: float, tableau: str = "BE") -> Problem:
    """The 1D Sod problem embedded in 2D (the paper's Sec. 5.1.1): [-1, 1] x
    [-3/128, 3/128], left (x_1 < 0) = (1, 0, 1), right = (0.125, 0, 0.8),
    velocity space [-7, 7]^2 with vcells Q2 cells per axis, constant nu, the
    paper's dt = 1.76e-3 for 85 steps.  Here the 256 x 6 lattice is split
    into 3072 right triangles (P1) instead of quadrilaterals, and the jump
    is spread over a tanh layer 1.5 lattice cells wide (with a sharp jump the
    two-stage DIRK drives a nodal density non-positive at nu = 1000 on these
    elements); the top and bottom walls reflect (sod_strip_wall_kinds) and
    the ends take the initial state as inflow."""
    mesh = rectangle_mesh(256, 6, -1.0, 1.0, -SOD_STRIP_HALF_HEIGHT, SOD_STRIP_HALF_HEIGHT)
    st = State("plane", {"normal": np.array([1.0, 0.0]), "center": np.zeros(2),
                         "left": SOD_LEFT, "right": SOD_RIGHT, "width": 1.5 * 2.0 / 256})
    return Problem(mesh, 1, gl_velocity_grid(vcells, 7.0, 2), st, nu_model="const",
                   nu_const=nu, tableau=tableau, n_steps=85, name=f"sod_strip_q2_{vcells}")


SOD_STRIP_DT = 1.76e-3


def sod_strip_wall_kinds(facet_midpoints: np.ndarray) -> np.ndarray:
    """2 (reflection) on the top and bottom walls, 0 (inflow) at the ends."""
    top = np.abs(np.abs(facet_midpoints[:, 1]) - SOD_STRIP_HALF_HEIGHT) < 1e-12
    return np.where(top, 2, 0).astype(np.int8)


# Riemann-type workloads spread the jump over a tanh layer about this many
# lattice cells wide: a sharp jump drives some P1 nodal moments non-physical
# (the method has no limiter; both the oracle and the library reject it).
RIEMANN_WIDTH_CELLS = 1.5


def config_c3(kn: float = 1e-2, n_side: int = 20) -> Problem:
    """~5e4-tet jittered Delaunay cube, P1, 16^3 velocities on [-6,6]^3,
    planar Riemann problem with a seeded normal, backward Euler, CFL 10."""
    mesh = jittered_cube_mesh(n_side, 0.2, seed=3000)
    return Problem(mesh, 1, tensor_velocity_grid(16, 6.0, 3),
                   planar_riemann_state(3, seed=3001, width=RIEMANN_WIDTH_CELLS / n_side),
                   nu_model="kn", kn=kn, tableau="BE", cfl=10.0, n_steps=10, tau=1e-10,
                   name=f"c3_riemann_p1_{mesh.n_cells}tet_16^3_kn{kn:g}")


def config_c4_instances(count: int = 64, seed0: int = 4000, max_tri: int = 50000):
    """Uneven batch: meshes of 1e3..max_tri triangles (log-uniform), P1/P2,
    n_1d in [8, 32] on [-8,8]^2, Kn log-uniform in [1e-4, 1], planar Riemann."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        ntri = math.exp(rng.uniform(math.log(1000.0), math.log(max_tri)))
        n_side = max(4, int(round(math.sqrt(ntri / 2.0))))
        order = int(rng.integers(1, 3))
        n1 = int(rng.integers(8, 33))
        kn = math.exp(rng.uniform(math.log(1e-4), 0.0))
        mesh = jittered_square_mesh(n_side, 0.2, seed=seed0 + 1000 + i)
        out.append(Problem(mesh, order, tensor_velocity_grid(n1, 8.0, 2),
                           planar_riemann_state(2, seed=seed0 + 2000 + i,
                                                width=RIEMANN_WIDTH_CELLS / n_side),
                           nu_model="kn", kn=kn,
                           tableau="DIRK2", cfl=10.0, n_steps=5, tau=1e-10,
                           name=f"c4_{i}"))
    return out


def learned_guess_problem(dim: int, seed: int, n_side: int, n_1d: int, L: float = 6.0,
                          kn_range=(1e-2, 1.0)) -> Problem:
    """A seeded backward-Euler Riemann run for the learned initial guess:
    jittered mesh, P1, tensor velocity grid, random Sod-like states and
    normal, Kn log-uniform in kn_range, CFL 10."""
    rng = np.random.default_rng(seed)
    kn = math.exp(rng.uniform(math.log(kn_range[0]), math.log(kn_range[1])))
    if dim == 2:
        mesh = jittered_square_mesh(n_side, 0.2, seed=seed + 100000)
    else:
        mesh = jittered_cube_mesh(n_side, 0.2, seed=seed + 100000)
    return Problem(mesh, 1, tensor_velocity_grid(n_1d, L, dim),
                   random_riemann_state(dim, seed + 200000, width=RIEMANN_WIDTH_CELLS / n_side),
                   nu_model="kn", kn=kn,
                   tableau="BE", cfl=10.0, n_steps=10, tau=1e-9,
                   name=f"learned_{dim}d_{seed}_kn{kn:.3g}")


def small_problem(dim=2, order=1, n_side=4, n_1d=6, L=6.0, seed=7, state="sod",
                  nu_model="const", nu_const=1.0, kn=1.0, tableau="BE", jitter=0.25) -> Problem:
    """A tiny instance for oracle pins and parity tests."""
    if dim == 2:
        mesh = jittered_square_mesh(n_side, jitter, seed)
    else:
        mesh = jittered_cube_mesh(n_side, min(jitter, 0.2), seed)
    st = {"sod": lambda: sod_state(dim), "riemann": lambda: planar_riemann_state(dim, seed + 1),
          "fourier": lambda: fourier_state(dim, seed + 2),
          "uniform": lambda: uniform_state(dim=dim)}[state]()
    return Problem(mesh, order, tensor_velocity_grid(n_1d, L, dim), st, nu_model=nu_model,
                   nu_const=nu_const, kn=kn, tableau=tableau, name="small")


# ----------------------------------------------------------------------------
# learned initial guess: seeded initial weights (random numbers only)
# ----------------------------------------------------------------------------
MLP_ARCH = (11, 64, 64, 64, 5)


def mlp_init_params(seed: int, arch=MLP_ARCH):
    """Glorot-uniform weights and zero biases for the fully connected network
    ``arch``; W_l has shape [fan_in][fan_out]."""
    rng = np.random.default_rng(seed)
    out = {}
    for l in range(len(arch) - 1):
        fi, fo = arch[l], arch[l + 1]
        lim = math.sqrt(6.0 / (fi + fo))
        out[f"W{l + 1}"] = rng.uniform(-lim, lim, size=(fi, fo))
        out[f"b{l + 1}"] = np.zeros(fo)
    return out
