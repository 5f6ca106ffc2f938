"""Python binding of libbgktgs.so, the MI355X topological-generation sweep library.

Argument marshalling only: every computation runs in the library's HIP
kernels; PyTorch provides device memory and streams.  Entry points carry the
C names (build_mesh_dag, tgs_sweep, moments, maxwellian, bgk_step, ...).
The library must have been built (``python -m paper_2608_19150_amd.build``);
importing this package without it raises immediately.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# BGK_LIBRARY may name another build of the same library (e.g. a variant
# built for comparison); the default is the in-tree build
LIB_PATH = os.environ.get("BGK_LIBRARY") or os.path.join(_HERE, "libbgktgs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2608_19150_amd.build`")
_lib = C.CDLL(LIB_PATH)

BGK_OK, BGK_E_INVALID, BGK_E_HIP, BGK_E_NOMEM = 0, -1, -2, -3
BGK_E_NOT_CONVERGED, BGK_E_NONPHYSICAL, BGK_E_UNSUPPORTED = -4, -5, -6
TGS_FP64, TGS_FP32_CORRECTION = 0, 1
MAXW = {"DIRECT": 0, "MATCHED": 1, "LINEAR": 2, "PROJECTED": 3}
NU = {"const": 0, "kn": 1}
TABLEAU = {"BE": 0, "DIRK2": 1, "DIRK3": 2, "BDIRK2": 3}

EXPORTED = [
    "bgk_last_error", "build_mesh_dag", "tgs_dag_destroy", "tgs_dag_sizes",
    "tgs_dag_generations", "tgs_dag_lagged", "tgs_dag_geometry", "tgs_dag_explicit_dt",
    "tgs_pack", "tgs_unpack",
    "tgs_sweep", "moments", "moments_noalloc", "maxwellian", "maxwellian_coef_from_primitive",
    "tgs_eval_maxwellian", "bgk_solver_create", "bgk_solver_destroy", "bgk_step",
    "bgk_mlp_create", "bgk_mlp_destroy", "bgk_mlp_set_params", "bgk_mlp_get_params",
    "bgk_mlp_set_normalization", "bgk_mlp_forward", "bgk_mlp_loss_grad", "bgk_mlp_adam_step",
    "bgk_mlp_features", "bgk_mlp_targets", "bgk_mlp_guess",
    "bgk_batch_create", "bgk_batch_destroy", "bgk_batch_step", "bgk_batch_time_sweep",
    "tgs_walls_create", "tgs_walls_destroy", "tgs_walls_count", "tgs_wall_values",
    "tgs_dag_sweep_lanes", "tgs_dag_set_walk",
]


class BGKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib.bgk_last_error.restype = C.c_char_p


def _check(rc):
    if rc != BGK_OK:
        raise BGKError(rc, _lib.bgk_last_error().decode())


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("order", C.c_int), ("n_vert", C.c_int64),
                ("vert", C.c_void_p), ("n_cells", C.c_int64), ("cells", C.c_void_p)]


class VGridDesc(C.Structure):
    _fields_ = [("n_v", C.c_int), ("v", C.c_void_p), ("w", C.c_void_p), ("n_1d", C.c_int),
                ("nodes_1d", C.c_void_p), ("weights_1d", C.c_void_p), ("L", C.c_double),
                ("dg_cells", C.c_int)]


class DagOpts(C.Structure):
    _fields_ = [("lagged", C.c_void_p), ("sweep_threads", C.c_int), ("ring_slots", C.c_int),
                ("sweep_lanes", C.c_int)]


class SweepIO(C.Structure):
    _fields_ = [("precision", C.c_int), ("sigma_shift", C.c_double), ("q_scale", C.c_double),
                ("nu", C.c_void_p), ("mcoef", C.c_void_p), ("q", C.c_void_p),
                ("bc_coef", C.c_void_p), ("bc_dense", C.c_void_p), ("f_prev", C.c_void_p),
                ("f_out", C.c_void_p)]


class NuModel(C.Structure):
    _fields_ = [("kind", C.c_int), ("nu_const", C.c_double), ("kn", C.c_double)]


class SolverOpts(C.Structure):
    _fields_ = [("tableau", C.c_int), ("dt", C.c_double), ("tau", C.c_double),
                ("l_max", C.c_int), ("fixed_iters", C.c_int), ("precision", C.c_int),
                ("maxw_mode", C.c_int), ("nu_model", NuModel), ("bc_coef", C.c_void_p),
                ("timing", C.c_int), ("walls", C.c_void_p), ("chunk_iters", C.c_int),
                ("graph", C.c_int)]


class StepStats(C.Structure):
    _fields_ = [("stages", C.c_int), ("iters", C.c_int * 4), ("total_iters", C.c_int),
                ("last_ratio", C.c_double * 4), ("maxw_fallbacks", C.c_int),
                ("seconds", C.c_double), ("sweep_ms", C.c_double), ("moments_ms", C.c_double),
                ("maxwellian_ms", C.c_double), ("other_ms", C.c_double), ("sweeps", C.c_int)]


def _p(t):
    """Device or host pointer of a tensor/array (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return C.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    raise TypeError(type(t))


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev(x, dtype=torch.float64):
    t = torch.as_tensor(x, dtype=dtype)
    return t.to("cuda").contiguous()


_lib.build_mesh_dag.argtypes = [C.POINTER(MeshDesc), C.POINTER(VGridDesc), C.POINTER(DagOpts),
                                C.c_void_p, C.POINTER(C.c_void_p)]
_lib.tgs_dag_destroy.argtypes = [C.c_void_p]
_lib.tgs_dag_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
_lib.tgs_dag_sweep_lanes.argtypes = [C.c_void_p]
_lib.tgs_dag_generations.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
_lib.tgs_dag_lagged.argtypes = [C.c_void_p, C.c_void_p]
_lib.tgs_dag_geometry.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.tgs_dag_explicit_dt.argtypes = [C.c_void_p, C.c_double, C.POINTER(C.c_double)]
_lib.tgs_dag_set_walk.argtypes = [C.c_void_p, C.c_int, C.c_int]
_lib.tgs_pack.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.tgs_unpack.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.tgs_sweep.argtypes = [C.c_void_p, C.POINTER(SweepIO), C.c_void_p]
_lib.moments.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.moments_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p]
_lib.maxwellian.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(NuModel), C.c_void_p,
                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.maxwellian_coef_from_primitive.argtypes = [C.c_int, C.c_int64, C.c_void_p, C.c_void_p,
                                                C.c_void_p]
_lib.tgs_eval_maxwellian.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.bgk_solver_create.argtypes = [C.c_void_p, C.POINTER(SolverOpts), C.POINTER(C.c_void_p)]
_lib.bgk_solver_destroy.argtypes = [C.c_void_p]
_lib.bgk_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(StepStats),
                          C.c_void_p]


class Dag:
    """Handle returned by build_mesh_dag (mesh geometry + per-velocity DAGs)."""

    def __init__(self, vert, cells, order, v, w, *, n_1d=0, nodes_1d=None, weights_1d=None,
                 L=0.0, dg_cells=0, lagged=None, sweep_threads=0, ring_slots=0, sweep_lanes=0,
                 stream=None):
        vert = np.ascontiguousarray(vert, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        v = np.ascontiguousarray(v, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        self._keep = [vert, cells, v, w]
        md = MeshDesc(vert.shape[1], order, vert.shape[0], vert.ctypes.data, cells.shape[0],
                      cells.ctypes.data)
        n1 = np.ascontiguousarray(nodes_1d, dtype=np.float64) if n_1d else None
        w1 = np.ascontiguousarray(weights_1d, dtype=np.float64) if n_1d else None
        self._keep += [n1, w1]
        vd = VGridDesc(v.shape[0], v.ctypes.data, w.ctypes.data, int(n_1d),
                       n1.ctypes.data if n_1d else None, w1.ctypes.data if n_1d else None,
                       float(L), int(dg_cells))
        lag = None
        if lagged is not None:
            lag = np.ascontiguousarray(lagged, dtype=np.uint8)
            self._keep.append(lag)
        opts = DagOpts(lag.ctypes.data if lag is not None else None, int(sweep_threads),
                       int(ring_slots), int(sweep_lanes))
        h = C.c_void_p()
        _check(_lib.build_mesh_dag(C.byref(md), C.byref(vd), C.byref(opts), _stream(stream),
                                   C.byref(h)))
        self.h = h
        s = (C.c_int64 * 9)()
        _check(_lib.tgs_dag_sizes(h, s))
        (self.dim, self.order, self.n_p, self.n_fp, self.n_cells, self.n_v, self.n_bfaces,
         self.max_G, self.n_lagged) = [int(x) for x in s]
        self.n_nodes = self.n_cells * self.n_p
        self.v = torch.as_tensor(v)
        self.w = torch.as_tensor(w)
        self.L = float(L)
        self.dg_cells = int(dg_cells)
        self.sweep_lanes = int(_lib.tgs_dag_sweep_lanes(h))

    @classmethod
    def from_problem(cls, pr, **kw):
        vg = pr.vgrid
        tensor = vg.nodes_1d is not None
        return cls(pr.mesh.vert, pr.mesh.cells, pr.order, vg.v, vg.w,
                   n_1d=len(vg.nodes_1d) if tensor else 0, nodes_1d=vg.nodes_1d,
                   weights_1d=vg.weights_1d, L=vg.L, dg_cells=vg.dg_cells, **kw)

    def __del__(self, _destroy=_lib.tgs_dag_destroy):
        # the library function is bound at definition time: module globals
        # may already be gone when this runs at interpreter exit
        h = getattr(self, "h", None)
        if h is not None and h.value:
            _destroy(h)
            self.h = None

    @property
    def f_shape(self):
        return (self.n_cells, self.n_p, self.n_v)

    def f_numel(self):
        return self.n_cells * self.n_p * self.n_v

    def generations(self):
        gen = np.zeros((self.n_v, self.n_cells), dtype=np.int32)
        G = np.zeros(self.n_v, dtype=np.int32)
        _check(_lib.tgs_dag_generations(self.h, gen.ctypes.data, G.ctypes.data))
        return gen, G

    def lagged(self):
        out = np.zeros((self.n_v, self.n_cells), dtype=np.uint8)
        _check(_lib.tgs_dag_lagged(self.h, out.ctypes.data))
        return out

    def geometry(self):
        nx = np.zeros((self.n_cells, self.n_p, self.dim))
        bx = np.zeros((self.n_bfaces, self.n_fp, self.dim))
        vol = np.zeros(self.n_cells)
        _check(_lib.tgs_dag_geometry(self.h, nx.ctypes.data, bx.ctypes.data, vol.ctypes.data))
        return nx, bx, vol

    def pack(self, f_canonical, out=None, stream=None):
        out = torch.empty(self.f_numel(), dtype=torch.float64, device="cuda") if out is None else out
        _check(_lib.tgs_pack(self.h, _p(f_canonical), _p(out), _stream(stream)))
        return out

    def unpack(self, f_sweep, out=None, stream=None):
        out = torch.empty(self.f_shape, dtype=torch.float64, device="cuda") if out is None else out
        _check(_lib.tgs_unpack(self.h, _p(f_sweep), _p(out), _stream(stream)))
        return out

    def eval_maxwellian(self, coef, out=None, stream=None):
        out = torch.empty(self.f_numel(), dtype=torch.float64, device="cuda") if out is None else out
        _check(_lib.tgs_eval_maxwellian(self.h, _p(coef), _p(out), _stream(stream)))
        return out

    def set_walk(self, threads=0, lanes=0):
        """Sweep walk: workgroup walk of `threads` per workgroup, or packed
        walk of `lanes` per velocity (0, 0: the library's automatic rule)."""
        _check(_lib.tgs_dag_set_walk(self.h, int(threads), int(lanes)))
        self.sweep_lanes = int(_lib.tgs_dag_sweep_lanes(self.h))

    def explicit_dt(self, cfl):
        """dt = C dt_e of eq. explicit-dt, computed by the library."""
        dt = C.c_double()
        _check(_lib.tgs_dag_explicit_dt(self.h, C.c_double(cfl), C.byref(dt)))
        return dt.value


def tgs_sweep(dag, *, q, nu, mcoef, f_out, sigma_shift, q_scale=1.0, bc_coef=None,
              bc_dense=None, f_prev=None, precision=TGS_FP64, stream=None):
    io = SweepIO(precision, float(sigma_shift), float(q_scale), _p(nu), _p(mcoef), _p(q),
                 _p(bc_coef), _p(bc_dense), _p(f_prev), _p(f_out))
    _check(_lib.tgs_sweep(dag.h, C.byref(io), _stream(stream)))
    return f_out


def moments(dag, f, U=None, U_prev=None, stream=None):
    """Returns U (and the three convergence ratios when U_prev is given)."""
    U = torch.empty((dag.n_nodes, dag.dim + 2), dtype=torch.float64, device="cuda") if U is None else U
    rel = torch.empty(3, dtype=torch.float64, device="cuda") if U_prev is not None else None
    _check(_lib.moments(dag.h, _p(f), _p(U), _p(U_prev), _p(rel), _stream(stream)))
    return (U, rel) if U_prev is not None else U


def moments_noalloc(dag, f, U, U_prev=None, rel3=None, stream=None):
    """moments() into caller-provided buffers (U [n_nodes][d+2], and rel3 [3]
    when U_prev is given); the library allocates nothing."""
    _check(_lib.moments_noalloc(dag.h, _p(f), _p(U), _p(U_prev), _p(rel3), _stream(stream)))
    return (U, rel3) if U_prev is not None else U


def maxwellian(dag, U, mode="MATCHED", nu_model="const", nu_const=1.0, kn=1.0, dense=False,
               stream=None):
    """Returns (coef [n_nodes][d+2], nu [n_nodes], M_dense or None, status[2])."""
    coef = torch.empty((dag.n_nodes, dag.dim + 2), dtype=torch.float64, device="cuda")
    nu = torch.empty(dag.n_nodes, dtype=torch.float64, device="cuda")
    Md = torch.empty((dag.n_nodes, dag.n_v), dtype=torch.float64, device="cuda") if dense else None
    status = torch.zeros(2, dtype=torch.int32, device="cuda")
    nm = NuModel(NU[nu_model], float(nu_const), float(kn))
    _check(_lib.maxwellian(dag.h, MAXW[mode], _p(U), C.byref(nm), _p(coef), _p(nu), _p(Md),
                           _p(status), _stream(stream)))
    return coef, nu, Md, status


def maxwellian_coef_from_primitive(prim, dim, stream=None):
    prim = prim.contiguous()
    coef = torch.empty_like(prim)
    _check(_lib.maxwellian_coef_from_primitive(int(dim), int(prim.shape[0]), _p(prim), _p(coef),
                                               _stream(stream)))
    return coef


def state_coefficients(dag, state, where="nodes"):
    """Maxwellian coefficients of a problems.State at the DG nodes or at the
    boundary facet nodes (the state's (n, u, theta) is sampled on the host,
    the conversion runs on the GPU)."""
    nx, bx, _ = dag.geometry()
    pts = nx.reshape(-1, dag.dim) if where == "nodes" else bx.reshape(-1, dag.dim)
    n, u, th = state.params(pts)
    prim = _dev(np.concatenate([n[:, None], u, th[:, None]], axis=1))
    return maxwellian_coef_from_primitive(prim, dag.dim)


class Solver:
    """bgk_solver: DIRK stages with sweep-based Picard iteration."""

    def __init__(self, dag, *, dt, bc_coef, tableau="BE", tau=1e-10, l_max=2000, fixed_iters=0,
                 precision=TGS_FP64, mode="MATCHED", nu_model="const", nu_const=1.0, kn=1.0,
                 timing=False, walls=None, chunk_iters=0, graph=False):
        self.dag = dag
        self.bc_coef = bc_coef
        self.walls = walls            # keep the wall handle alive with the solver
        o = SolverOpts(TABLEAU[tableau], float(dt), float(tau), int(l_max), int(fixed_iters),
                       int(precision), MAXW[mode], NuModel(NU[nu_model], float(nu_const), float(kn)),
                       _p(bc_coef), int(bool(timing)), walls.h if walls is not None else None,
                       int(chunk_iters), int(bool(graph)))
        h = C.c_void_p()
        _check(_lib.bgk_solver_create(dag.h, C.byref(o), C.byref(h)))
        self.h = h

    def __del__(self, _destroy=_lib.bgk_solver_destroy):
        # the library function is bound at definition time: module globals
        # may already be gone when this runs at interpreter exit
        h = getattr(self, "h", None)
        if h is not None and h.value:
            _destroy(h)
            self.h = None

    def step(self, f, U_guess=None, U_out=None, stream=None):
        st = StepStats()
        _check(_lib.bgk_step(self.h, _p(f), _p(U_guess), _p(U_out), C.byref(st), _stream(stream)))
        return {"iters": list(st.iters[:st.stages]), "total_iters": st.total_iters,
                "last_ratio": list(st.last_ratio[:st.stages]), "fallbacks": st.maxw_fallbacks,
                "seconds": st.seconds, "sweep_ms": st.sweep_ms, "moments_ms": st.moments_ms,
                "maxwellian_ms": st.maxwellian_ms, "sweeps": st.sweeps}


BC = {"INFLOW": 0, "BOUNCE_BACK": 1, "REFLECT": 2}

_lib.tgs_walls_create.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]
_lib.tgs_walls_destroy.argtypes = [C.c_void_p]
_lib.tgs_walls_count.argtypes = [C.c_void_p]
_lib.tgs_walls_count.restype = C.c_int64
_lib.tgs_wall_values.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]


class Walls:
    """tgs_walls: the bounce-back and reflecting facets of a DAG's boundary.

    ``kinds`` int8 [n_bfaces] of BC values (or their names), boundary facets
    in the order of Dag.geometry()'s boundary nodes."""

    def __init__(self, dag, kinds):
        k = np.asarray([BC[x] if isinstance(x, str) else int(x) for x in kinds], dtype=np.int8)
        if k.shape != (dag.n_bfaces,):
            raise ValueError(f"need {dag.n_bfaces} boundary kinds, got {k.shape}")
        self.dag = dag
        self.kinds = k
        h = C.c_void_p()
        _check(_lib.tgs_walls_create(dag.h, k.ctypes.data, C.byref(h)))
        self.h = h

    @property
    def n_walls(self):
        return int(_lib.tgs_walls_count(self.h))

    def __del__(self, _destroy=_lib.tgs_walls_destroy):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            _destroy(h)
            self.h = None


def wall_values(walls, f, bc_dense, stream=None):
    """Fills the wall rows of bc_dense [n_bfaces][n_fp][n_v] from f (sweep layout)."""
    _check(_lib.tgs_wall_values(walls.h, _p(f), _p(bc_dense), _stream(stream)))


def boundary_facet_midpoints(dag):
    """Mean of each boundary facet's nodes, [n_bfaces][dim] (host)."""
    _, bx, _ = dag.geometry()
    return bx.reshape(dag.n_bfaces, -1, dag.dim).mean(axis=1)


def exported_symbols():
    """Names of the C entry points the binding uses (all must resolve)."""
    return [n for n in EXPORTED if hasattr(_lib, n)]


def problem_setup(pr, dag=None, **dag_kw):
    """Device-side setup of a problems.Problem: DAG, initial f (sweep layout),
    boundary coefficients and dt = C dt_e."""
    dag = Dag.from_problem(pr, **dag_kw) if dag is None else dag
    f0 = dag.eval_maxwellian(state_coefficients(dag, pr.state, "nodes"))
    bc = state_coefficients(dag, pr.state, "boundary")
    return dag, f0, bc, dag.explicit_dt(pr.cfl)


# ---------------------------------------------------------------------------
# batched instances
# ---------------------------------------------------------------------------
class BatchOpts(C.Structure):
    _fields_ = [("graph", C.c_int), ("chunk_iters", C.c_int), ("sweep_threads", C.c_int),
                ("sweep_lanes", C.c_int)]


class BatchStats(C.Structure):
    _fields_ = [("status", C.c_int), ("stages", C.c_int), ("iters", C.c_int * 4),
                ("total_iters", C.c_int), ("last_ratio", C.c_double * 4),
                ("maxw_fallbacks", C.c_int), ("finish_ms", C.c_double)]


_lib.bgk_batch_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.POINTER(BatchOpts),
                                  C.POINTER(C.c_void_p)]
_lib.bgk_batch_destroy.argtypes = [C.c_void_p]
_lib.bgk_batch_step.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(BatchStats),
                                C.c_void_p]
_lib.bgk_batch_time_sweep.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.c_int, C.c_int,
                                      C.c_int, C.POINTER(C.c_float), C.c_void_p]


class Batch:
    """bgk_batch: many solvers stepped together (one launch per kernel per
    Picard iteration, optional hipGraph replay of iteration chunks)."""

    def __init__(self, solvers, *, graph=True, chunk_iters=4, sweep_threads=0, sweep_lanes=0):
        self.solvers = list(solvers)          # keep them (and their DAGs) alive
        arr = (C.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        o = BatchOpts(int(bool(graph)), int(chunk_iters), int(sweep_threads), int(sweep_lanes))
        h = C.c_void_p()
        _check(_lib.bgk_batch_create(arr, len(self.solvers), C.byref(o), C.byref(h)))
        self.h = h

    def __del__(self, _destroy=_lib.bgk_batch_destroy):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            _destroy(h)
            self.h = None

    def _fptrs(self, fs):
        assert len(fs) == len(self.solvers)
        return (C.c_void_p * len(fs))(*[f.data_ptr() for f in fs])

    def step(self, fs, stream=None, check=True):
        """One DIRK step of every instance; returns per-instance stats."""
        st = (BatchStats * len(fs))()
        rc = _lib.bgk_batch_step(self.h, self._fptrs(fs), st, _stream(stream))
        if check:
            _check(rc)
        return [{"status": s.status, "iters": list(s.iters[:s.stages]),
                 "total_iters": s.total_iters, "last_ratio": list(s.last_ratio[:s.stages]),
                 "fallbacks": s.maxw_fallbacks, "finish_ms": s.finish_ms} for s in st]

    def time_sweep(self, fs, threads, reps=3, stream=None, lanes=0):
        """Milliseconds per batched sweep with the workgroup walk of `threads`
        (lanes 0) or the packed walk of `lanes` per velocity."""
        ms = C.c_float()
        _check(_lib.bgk_batch_time_sweep(self.h, self._fptrs(fs), int(threads), int(lanes),
                                         int(reps), C.byref(ms), _stream(stream)))
        return ms.value


# ---------------------------------------------------------------------------
# learned Picard initial guess
# ---------------------------------------------------------------------------
MLP_ARCH = (11, 64, 64, 64, 5)
MLP_PARAMS = 9413

_vp = C.c_void_p
_lib.bgk_mlp_create.argtypes = [_vp, C.POINTER(_vp)]
_lib.bgk_mlp_destroy.argtypes = [_vp]
_lib.bgk_mlp_set_params.argtypes = [_vp, _vp]
_lib.bgk_mlp_get_params.argtypes = [_vp, _vp]
_lib.bgk_mlp_set_normalization.argtypes = [_vp, _vp]
_lib.bgk_mlp_forward.argtypes = [_vp, _vp, C.c_int64, _vp, _vp]
_lib.bgk_mlp_loss_grad.argtypes = [_vp, _vp, _vp, C.c_int64, _vp, _vp, _vp]
_lib.bgk_mlp_adam_step.argtypes = [_vp, _vp, _vp, C.c_int64, C.c_float, _vp, _vp]
_lib.bgk_mlp_features.argtypes = [_vp, _vp, _vp, C.POINTER(NuModel), C.c_double, _vp, _vp]
_lib.bgk_mlp_targets.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
_lib.bgk_mlp_guess.argtypes = [_vp, _vp, _vp, _vp, C.POINTER(NuModel), C.c_double, _vp, _vp, _vp]


def mlp_flatten(params):
    """{W1, b1, ..., W4, b4} (W_l [fan_in][fan_out]) -> float32 [9413] in the
    library's logical order."""
    parts = []
    for l in range(1, len(MLP_ARCH)):
        parts += [np.asarray(params[f"W{l}"], dtype=np.float32).ravel(),
                  np.asarray(params[f"b{l}"], dtype=np.float32).ravel()]
    flat = np.ascontiguousarray(np.concatenate(parts))
    assert flat.size == MLP_PARAMS
    return flat


def mlp_unflatten(flat):
    out, o = {}, 0
    for l in range(1, len(MLP_ARCH)):
        fi, fo = MLP_ARCH[l - 1], MLP_ARCH[l]
        out[f"W{l}"] = np.asarray(flat[o:o + fi * fo]).reshape(fi, fo)
        o += fi * fo
        out[f"b{l}"] = np.asarray(flat[o:o + fo])
        o += fo
    return out


class Mlp:
    """bgk_mlp: per-node network on BF16 MFMA with FP32 master weights."""

    def __init__(self, params=None):
        flat = None if params is None else mlp_flatten(params)
        h = C.c_void_p()
        _check(_lib.bgk_mlp_create(_p(flat), C.byref(h)))
        self.h = h

    def __del__(self, _destroy=_lib.bgk_mlp_destroy):
        # the library function is bound at definition time: module globals
        # may already be gone when this runs at interpreter exit
        h = getattr(self, "h", None)
        if h is not None and h.value:
            _destroy(h)
            self.h = None

    def set_params(self, params):
        _check(_lib.bgk_mlp_set_params(self.h, _p(mlp_flatten(params))))

    def get_params(self):
        flat = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(_lib.bgk_mlp_get_params(self.h, _p(flat)))
        return mlp_unflatten(flat)

    def set_normalization(self, mean_in, std_in, mean_out, std_out):
        st = np.ascontiguousarray(np.concatenate(
            [np.asarray(a, dtype=np.float32).ravel() for a in (mean_in, std_in, mean_out, std_out)]))
        assert st.size == 32
        _check(_lib.bgk_mlp_set_normalization(self.h, _p(st)))

    def forward(self, X, stream=None):
        X = X.contiguous()
        Y = torch.empty((X.shape[0], 5), dtype=torch.float32, device="cuda")
        _check(_lib.bgk_mlp_forward(self.h, _p(X), int(X.shape[0]), _p(Y), _stream(stream)))
        return Y

    def loss_grad(self, X, T, stream=None):
        """(loss tensor [1], gradient [9413] in logical order)."""
        X, T = X.contiguous(), T.contiguous()
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(_lib.bgk_mlp_loss_grad(self.h, _p(X), _p(T), int(X.shape[0]), _p(g), _p(loss),
                                      _stream(stream)))
        return loss, g

    def adam_step(self, X, T, lr, loss=None, stream=None):
        _check(_lib.bgk_mlp_adam_step(self.h, _p(X), _p(T), int(X.shape[0]), float(lr), _p(loss),
                                      _stream(stream)))

    def guess(self, dag, U_tm1, U_tm2, dt, nu_model="const", nu_const=1.0, kn=1.0, n_fallback=None,
              stream=None):
        Ug = torch.empty_like(U_tm1)
        nm = NuModel(NU[nu_model], float(nu_const), float(kn))
        _check(_lib.bgk_mlp_guess(self.h, dag.h, _p(U_tm1), _p(U_tm2), C.byref(nm), float(dt),
                                  _p(Ug), _p(n_fallback), _stream(stream)))
        return Ug


def mlp_features(dag, U_tm1, U_tm2, dt, nu_model="const", nu_const=1.0, kn=1.0, stream=None):
    X = torch.empty((dag.n_nodes, 11), dtype=torch.float32, device="cuda")
    nm = NuModel(NU[nu_model], float(nu_const), float(kn))
    _check(_lib.bgk_mlp_features(dag.h, _p(U_tm1), _p(U_tm2), C.byref(nm), float(dt), _p(X),
                                 _stream(stream)))
    return X


def mlp_targets(dag, U_t, U_tm1, U_tm2, stream=None):
    T = torch.empty((dag.n_nodes, 5), dtype=torch.float32, device="cuda")
    _check(_lib.bgk_mlp_targets(dag.h, _p(U_t), _p(U_tm1), _p(U_tm2), _p(T), _stream(stream)))
    return T


__all__ = ["Dag", "Solver", "tgs_sweep", "moments", "maxwellian", "maxwellian_coef_from_primitive",
           "state_coefficients", "problem_setup", "BGKError", "exported_symbols", "Mlp",
           "mlp_features", "mlp_targets", "mlp_flatten", "mlp_unflatten", "Batch", "math"]
