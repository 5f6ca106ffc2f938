/*
 * bgktgs.h -- C ABI of the MI355X (gfx950) topological-generation sweep
 * library for the implicit BGK equation.
 *
 * The library implements the hot path of the sweep-based implicit BGK
 * method: per-velocity upwind DAGs grouped into generations (Sec. 4.1), the
 * upwind DG transport-plus-relaxation solve of every (velocity, cell) pair in
 * generation order (eq. bgk-ss-picard), the velocity-moment reduction
 * (eq. moments) and the discrete Maxwellian rebuild it alternates with
 * (eq. Maxwellian-projection), DIRK stages (Sec. 3.5, App. A) and the Picard
 * stopping rule (eq. convergence-criteria).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns BGK_OK (0) or a negative BGK_E_* code; the text
 *    of the last error on the calling thread is bgk_last_error().  No C++
 *    exception crosses this boundary.
 *  - Device pointers are hipMalloc'ed (or torch-owned) memory on the device
 *    that was current when the DAG was built; host pointers are ordinary
 *    host memory.  Each argument says which.
 *  - Kernels run asynchronously on the caller's hipStream_t (0 = the null
 *    stream).  Only build_mesh_dag, bgk_step and the host-output query
 *    functions synchronise.
 *  - The caller owns every data buffer.  The library owns the opaque handles
 *    (tgs_dag, bgk_solver, bgk_mlp) and the device workspaces inside them;
 *    they are freed by the matching *_destroy call.
 *  - Precision: FP64 unless a field says otherwise.
 *
 * Layouts
 * -------
 *  - Cells are the caller's simplices, numbered 0..n_cells-1 ("user order").
 *  - DG nodes per cell: P1 = the d+1 vertices in the order of the cell's
 *    vertex list; P2 (triangles) = vertices 0,1,2 then the midpoints of
 *    edges (0,1), (1,2), (2,0).  Node i of cell c has nodal index c*n_p + i.
 *  - Facet k of a cell is the facet opposite its vertex k; facet nodes are
 *    the cell's nodes on it in ascending local index.
 *  - Boundary facets are numbered in ascending (cell, facet) order; boundary
 *    data is indexed [boundary facet][facet node].
 *  - Velocities: the order of tgs_vgrid_desc.v (for tensor grids the
 *    row-major tensor index, first axis slowest).
 *  - "Canonical" phase-space layout: f[cell][node][velocity], velocity
 *    fastest, user cell order.
 *  - "Sweep" phase-space layout: the library's internal velocity-major
 *    layout in which every velocity's cells are stored in its generation
 *    order.  tgs_sweep, moments and bgk_step take phase-space arrays in
 *    sweep layout; tgs_pack / tgs_unpack convert.  Its size is
 *    n_v * n_cells * n_p doubles, like the canonical layout.
 *  - Nodal arrays (U, Maxwellian coefficients, nu) are [node][...] in user
 *    order with node = cell*n_p + local node.
 *  - Maxwellians are carried as exponential-family coefficients
 *    (a, b_1..b_d, c): M(v) = exp(a + b.v + c|v|^2).
 */
#ifndef BGKTGS_H
#define BGKTGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* bgk_stream_t; /* same object as hipStream_t */

enum {
  BGK_OK = 0,
  BGK_E_INVALID = -1,       /* bad argument, degenerate or non-conforming mesh */
  BGK_E_HIP = -2,           /* a HIP runtime call failed */
  BGK_E_NOMEM = -3,         /* device allocation failed */
  BGK_E_NOT_CONVERGED = -4, /* Picard iteration reached l_max */
  BGK_E_NONPHYSICAL = -5,   /* n <= 0 or theta <= 0 (or non-finite) at a node */
  BGK_E_UNSUPPORTED = -6    /* element type or option not implemented */
};

/* Text of the last error raised on this thread ("" if none). */
const char* bgk_last_error(void);

/* ------------------------------------------------------------------------ */
/* Mesh, velocity grid and the per-velocity sweep DAGs (Sec. 3.1, Sec. 4.1)   */
/* ------------------------------------------------------------------------ */

typedef struct {
  int dim;                /* 2 (triangles) or 3 (tetrahedra) */
  int order;              /* DG degree: 1 (d = 2, 3) or 2 (d = 2) */
  int64_t n_vert;
  const double* vert;     /* host [n_vert][dim], copied */
  int64_t n_cells;
  const int32_t* cells;   /* host [n_cells][dim+1] vertex ids, copied */
} tgs_mesh_desc;

typedef struct {
  int n_v;
  const double* v;        /* host [n_v][dim], copied */
  const double* w;        /* host [n_v] quadrature weights, copied */
  int n_1d;               /* > 0 declares a tensor grid: v and w are the tensor
                             product of nodes_1d / weights_1d (checked) */
  const double* nodes_1d; /* host [n_1d] or NULL */
  const double* weights_1d;
  double L;               /* half-width of the velocity box (LINEAR and
                             PROJECTED modes) */
  int dg_cells;           /* > 0: the Q2 discontinuous-Galerkin velocity space
                             of Sec. 3.2: [-L, L] cut into dg_cells uniform
                             cells per axis, nodes_1d the 3
                             Gauss-Legendre points of each cell in order and
                             weights_1d their weights (n_1d = 3*dg_cells;
                             checked).  Enables BGK_MAXW_PROJECTED.  0 = a
                             point set. */
} tgs_vgrid_desc;

typedef struct {
  /* Optional host bitmask [n_v][n_cells] (user cell order): bit k set forces
     facet k of that cell to take its inflow from the previous Picard iterate
     (the lagged part of the inflow boundary, Sec. 4).  NULL = lag only what
     cycle breaking requires. */
  const uint8_t* lagged;
  /* Threads per workgroup of the sweep kernel (64..256, multiple of 64);
     0 = the library's choice (256 for P1 triangles, else 128). */
  int sweep_threads;
  /* Slots of the sweep's LDS ring of recent cell outputs (a power of two in
     16..1024, capped at what the element type's ring holds: 1024, or 512 for
     P2 triangles); 0 = that maximum.  Upwind values older than the ring are
     read from HBM after a workgroup fence: a small ring exercises that path
     on small meshes (tests); it never changes results. */
  int ring_slots;
  /* Walk of the FP64 single-instance sweep (Sec. 4.1 names two: a thread per
     velocity walking its whole graph, TS, and generation-parallel TGS).
     1, 2, 4, 8, 16 or 32: the packed walk, a wavefront serving 64/L
     velocities with L lanes each, every lane group stepping through its
     velocity's generations L cells at a time (L = 1 is TS); 64: the
     workgroup walk (a workgroup per velocity, sweep_threads wide); 0 = chosen
     from the DAG: the packed walk with L the power of two nearest the mean
     generation width when that is below 32, raised (up to 32) until the
     launch has 1024 wavefronts, else the workgroup walk.  The
     cell arithmetic is the same in both walks: results are bitwise equal.
     The FP32 form and batched sweeps use the workgroup walk. */
  int sweep_lanes;
} tgs_dag_opts;

typedef struct tgs_dag tgs_dag;

/* Builds cell geometry and facet connectivity on the host, then every
 * velocity's upwind DAG and its longest-path generations on the GPU
 * (Sec. 4.1).  An edge a->b exists when b's facet shared with a has
 * v.n < 0 from b's side; tangential facets (|v.n| <= 1e-12 |v| |n|, with n
 * the area-weighted normal stored once per facet) carry no edge.  When a
 * velocity's graph has a cycle (never the case on Delaunay meshes) the
 * builder releases the lowest-numbered unreleased cell into the next
 * generation and lags its unreleased in-edges (exported by
 * tgs_dag_lagged).  Synchronises `stream`.
 * Errors: BGK_E_INVALID (degenerate cell, facet shared by more than two
 * cells, malformed tensor grid), BGK_E_UNSUPPORTED (element type),
 * BGK_E_NOMEM, BGK_E_HIP. */
int build_mesh_dag(const tgs_mesh_desc* mesh, const tgs_vgrid_desc* vgrid,
                   const tgs_dag_opts* opts, bgk_stream_t stream, tgs_dag** out);

int tgs_dag_destroy(tgs_dag* dag);

/* sizes[0..8] = dim, order, n_p, n_fp, n_cells, n_v, n_bfaces, max_G, n_lagged. */
int tgs_dag_sizes(const tgs_dag* dag, int64_t sizes[9]);

/* Host outputs (any may be NULL): gen [n_v][n_cells] in user cell order,
 * G [n_v] generation counts.  Synchronises. */
int tgs_dag_generations(const tgs_dag* dag, int32_t* gen, int32_t* G);

/* Host output [n_v][n_cells] (user order) lagged-facet bitmasks. */
int tgs_dag_lagged(const tgs_dag* dag, uint8_t* lagged);
/* Lanes per velocity of the FP64 single-instance sweep (sweep_lanes as
 * chosen at build: 1..32 = the packed walk, 64 = the workgroup walk). */
int tgs_dag_sweep_lanes(const tgs_dag* dag);

/* Sets the sweep walk of an existing DAG, as tgs_dag_opts.sweep_threads and
 * sweep_lanes do at build time: threads = workgroup size of the workgroup
 * walk (a multiple of 64 in [64, 256]; 0 = the element type's default),
 * lanes = lanes per velocity of the packed walk (a power of two up to 32;
 * 64 = the workgroup walk; 0 = the library's automatic rule); threads and
 * packed lanes exclude each other.  Every walk gives the same results bit
 * for bit; this is the sweep autotuner's knob (tile shape: velocities per
 * workgroup and cells per wave).  Solvers on the DAG take the new walk from
 * their next sweep.  Synchronises the device.  Errors: BGK_E_INVALID. */
int tgs_dag_set_walk(tgs_dag* dag, int threads, int lanes);

/* Host outputs (any may be NULL): node_x [n_cells][n_p][dim] node
 * coordinates, bnode_x [n_bfaces][n_fp][dim] boundary facet node
 * coordinates, vol [n_cells] cell measures. */
int tgs_dag_geometry(const tgs_dag* dag, double* node_x, double* bnode_x, double* vol);

/* The time step of eq. explicit-dt (Sec. 5) scaled by a CFL factor:
 * dt = cfl * (1/d) * (1/(2k+1)) * h_min / max_j |v_j|, with
 * h_min = (min_K |K|)^(1/d) over the DAG's cells and the maximum over its
 * velocity set (k the DG order).  Host computation on data the DAG keeps;
 * no device work.  BGK_E_INVALID for a null argument, cfl <= 0 or a velocity
 * set of zero speed. */
int tgs_dag_explicit_dt(const tgs_dag* dag, double cfl, double* dt);

/* Canonical -> sweep layout and back (device pointers, no aliasing). */
int tgs_pack(const tgs_dag* dag, const double* f_canonical, double* f_sweep, bgk_stream_t stream);
int tgs_unpack(const tgs_dag* dag, const double* f_sweep, double* f_canonical, bgk_stream_t stream);

/* ------------------------------------------------------------------------ */
/* One transport sweep (eq. bgk-ss-picard)                                   */
/* ------------------------------------------------------------------------ */

enum { TGS_FP64 = 0, TGS_FP32_CORRECTION = 1 };

typedef struct {
  int precision;          /* TGS_FP64: solve for f in FP64.
                             TGS_FP32_CORRECTION: form the FP64 residual of
                             f_prev per cell, solve for the correction in FP32
                             with upwind correction traces, add it in FP64. */
  double sigma_shift;     /* 1/(dt A_ss): sigma_i = nu_i + sigma_shift */
  double q_scale;         /* the stage source enters as q_scale * q */
  const double* nu;       /* device [n_nodes] collision frequency */
  const double* mcoef;    /* device [n_nodes][dim+2] Maxwellian coefficients */
  const double* q;        /* device, sweep layout */
  const double* bc_coef;  /* device [n_bfaces][n_fp][dim+2] inflow Maxwellians, or NULL */
  const double* bc_dense; /* device canonical [n_bfaces][n_fp][n_v] inflow values, or NULL */
  const double* f_prev;   /* device, sweep layout: previous iterate; required when
                             lagged facets exist or for TGS_FP32_CORRECTION */
  double* f_out;          /* device, sweep layout; must not alias f_prev */
} tgs_sweep_io;

/* Solves, for every velocity j and every cell K in generation order,
 *   A f_K = b,
 *   A = M_K diag(sigma) - |det J| sum_b (J^-1 v_j)_b S_b + sum_{v.n>0} (v.n) M_e
 *   b = M_K (nu*M_j + q_scale*q) + sum_{v.n<0} |v.n| M_e fhat
 * with fhat the upwind neighbour's new value, the lagged f_prev, or the
 * boundary value (exactly one of bc_coef / bc_dense non-NULL).  Exactly one
 * sweep; no convergence logic.  Asynchronous on `stream`; allocates stream-
 * ordered scratch (nu and the coefficients in the library's internal cell
 * order, n_nodes*(dim+3) doubles; on a tensor velocity grid the factorised
 * Maxwellian tables, (dim+1)*n_1d*n_nodes doubles before padding; the FP32
 * corrections in that form) and frees it on the same stream.  The sweep
 * runs the same kernels as bgk_step's.
 * Errors: BGK_E_INVALID (missing or aliased buffers), BGK_E_NOMEM, BGK_E_HIP. */
int tgs_sweep(const tgs_dag* dag, const tgs_sweep_io* io, bgk_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Moments and Maxwellians (eq. moments, eq. convergence-criteria)           */
/* ------------------------------------------------------------------------ */

/* U[node][m] = sum_j w_j e_m(v_j) f_j(node), e = (1, v, |v|^2/2); f in sweep
 * layout, U device [n_nodes][dim+2].  When U_prev is non-NULL, rel3 (device
 * double[3]) receives the three ratios of eq. convergence-criteria,
 * |U^m - U_prev^m| / max(|U_prev^m|, s_m |U_prev^0|), s = (0, 1, 0).
 * Reductions run in a fixed order (bitwise reproducible). */
int moments(const tgs_dag* dag, const double* f, double* U, const double* U_prev,
            double* rel3, bgk_stream_t stream);

/* moments() for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, bit for bit, with no hipMalloc/hipFree or
 * allocating call.  The scratch (the chunk sums of a velocity-split moment
 * pass, at most 2^21 doubles, used on meshes of 4096 to 16,383 cells with
 * 8192 velocities or more; with U_prev, 6 doubles per moment block, 64
 * cells per block on meshes of 16,384 cells or more and in split passes
 * (256 on such tetrahedral meshes), at most 1024 blocks otherwise) lives
 * in a fixed 32 MiB device array per GPU, held until the process ends and
 * shared by every call on that GPU: calls that overlap on one GPU race on
 * it and must be ordered by the caller (one stream, or events).  Nothing
 * in it needs clearing between calls.  BGK_E_INVALID when the mesh needs
 * more scratch than that (with U_prev, about 44 million cells). */
int moments_noalloc(const tgs_dag* dag, const double* f, double* U, const double* U_prev,
                    double* rel3, bgk_stream_t stream);

/* DIRECT: the Maxwellian of (n, u, theta) at the nodes; MATCHED: the nodal
 * Gaussian whose discrete moments equal U (Newton from DIRECT); LINEAR:
 * n/|V|; PROJECTED (Q2 velocity space only, App. B): the projection of
 * M_{n,u,theta} onto the velocity space with the first and last cells
 * extended to infinity, whose discrete moments equal U exactly. */
enum { BGK_MAXW_DIRECT = 0, BGK_MAXW_MATCHED = 1, BGK_MAXW_LINEAR = 2, BGK_MAXW_PROJECTED = 3 };
enum { BGK_NU_CONST = 0, BGK_NU_KN = 1 };

typedef struct {
  int kind;               /* BGK_NU_CONST: nu = nu_const; BGK_NU_KN: nu = n theta^-1/2 / kn */
  double nu_const;
  double kn;
} tgs_nu_model;

/* From nodal moments U (device [n_nodes][dim+2]) computes the Maxwellian
 * coefficients mcoef (device [n_nodes][dim+2]) and nu (device [n_nodes]):
 * DIRECT = the Maxwellian of (n, u, theta); MATCHED = the nodal Gaussian
 * whose discrete moments equal U (Newton from DIRECT, residual <= 1e-14|U|,
 * at most 30 steps, else that node falls back to DIRECT and is counted);
 * LINEAR = n/|V| (the simplified linear Maxwellian); PROJECTED (needs
 * dg_cells > 0) = the conservative projection of App. B, for which mcoef
 * holds the primitive (n, u_1..u_d, theta) instead of log-coefficients and
 * the values are n (2 pi theta)^(-d/2) times the product over the axes of
 * the projected 1-D Gaussians (erf/erfc closed forms).  Optional outputs:
 * M_dense (device canonical [n_nodes][n_v]) and status (device int32[2]:
 * fallback count, non-physical count; accumulated, caller zeroes). */
int maxwellian(const tgs_dag* dag, int mode, const double* U, const tgs_nu_model* nu_model,
               double* mcoef, double* nu, double* M_dense, int32_t* status, bgk_stream_t stream);

/* Coefficients of M_{n,u,theta} for n_pts primitive states prim (device
 * [n_pts][dim+2] = (n, u, theta)) into coef (device [n_pts][dim+2]). */
int maxwellian_coef_from_primitive(int dim, int64_t n_pts, const double* prim, double* coef,
                                   bgk_stream_t stream);

/* f = exp(coef . (1, v, |v|^2)) at every node and velocity: coef device
 * [n_nodes][dim+2]; f device, sweep layout (initial conditions). */
int tgs_eval_maxwellian(const tgs_dag* dag, const double* coef, double* f_sweep,
                        bgk_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Wall boundaries (Sec. "Boundary conditions")                             */
/* ------------------------------------------------------------------------ */

/* Kind of a boundary facet: given inflow data; bounce-back,
 * f_bc(x, v) = f(x, -v); specular reflection, f_bc(x, v) = f(x, R_n v) with
 * R_n v = v - 2 (v.n) n.  The velocity set must be closed under the map of
 * every wall facet (as the paper assumes: walls normal to a coordinate axis
 * and a grid symmetric about 0). */
enum { BGK_BC_INFLOW = 0, BGK_BC_BOUNCE_BACK = 1, BGK_BC_REFLECT = 2 };

typedef struct tgs_walls tgs_walls;

/* Prepares the wall facets of a DAG.  bface_kind: host int8 [n_bfaces]
 * (BGK_BC_*), boundary facets in ascending (user cell, local facet) order,
 * the order of tgs_dag_geometry's bnode_x and of bc_coef / bc_dense.  For
 * every distinct (kind, normal) the velocity map is found by matching the
 * mapped velocity against the set (tolerance 1e-9 max(1, max|v|));
 * BGK_E_INVALID if a kind is unknown or an image is not a velocity of the
 * set.  The DAG must outlive the handle.  Synchronises the device. */
int tgs_walls_create(const tgs_dag* dag, const int8_t* bface_kind, tgs_walls** out);
int tgs_walls_destroy(tgs_walls* walls);
/* number of wall (non-inflow) facets */
int64_t tgs_walls_count(const tgs_walls* walls);

/* For every wall facet bf, facet node p and every velocity j that can enter
 * through it (v_j.n <= 1e-9 |v_j| for the facet's outward unit normal n, a
 * superset of the velocities whose boundary data a sweep reads):
 *   bc_dense[bf][p][j] = f(cell of bf, its local node at p, T_bf(j)),
 * f device in the sweep layout, bc_dense device [n_bfaces][n_fp][n_v]
 * (rows of inflow facets and entries of outgoing velocities are left
 * untouched).  This is the boundary update of a Picard iteration: the
 * solver calls it with the previous iterate before each sweep. */
int tgs_wall_values(const tgs_walls* walls, const double* f, double* bc_dense,
                    bgk_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Implicit time step: DIRK stages with Picard iteration (Sec. 3.5, Sec. 4)  */
/* ------------------------------------------------------------------------ */

enum { BGK_TAB_BE = 0, BGK_TAB_DIRK2 = 1, BGK_TAB_DIRK3 = 2, BGK_TAB_BDIRK2 = 3 };
enum { BGK_GUESS_PREVIOUS = 0, BGK_GUESS_USER = 1 };

typedef struct {
  int tableau;            /* BGK_TAB_* (App. A) */
  double dt;
  double tau;             /* Picard tolerance of eq. convergence-criteria */
  int l_max;              /* iteration cap per stage (BGK_E_NOT_CONVERGED) */
  int fixed_iters;        /* > 0: run exactly this many Picard iterations per stage */
  int precision;          /* TGS_FP64 or TGS_FP32_CORRECTION */
  int maxw_mode;          /* BGK_MAXW_* */
  tgs_nu_model nu_model;
  const double* bc_coef;  /* device [n_bfaces][n_fp][dim+2] time-independent inflow */
  int timing;             /* 1: time every kernel with HIP events on the step's
                             stream (bgk_step_stats.*_ms); 0: no events */
  const tgs_walls* walls; /* NULL, or wall facets of the same DAG: before each
                             sweep their boundary data are taken from the
                             previous Picard iterate (the first iteration of a
                             stage: the stage's initial iterate); bc_coef
                             gives the data of the inflow facets */
  int chunk_iters;        /* 0 or 1: the host tests convergence after every
                             Picard iteration; K >= 2: K iterations are
                             enqueued at a time, the stopping test runs on the
                             device after each, and once it has fired the
                             rest of the chunk does nothing; the host reads a
                             small control block once per chunk.  Iteration
                             counts and results equal K = 1's.  Needs
                             timing = 0. */
  int graph;              /* with chunk_iters >= 2: each chunk is captured once
                             in a hipGraph (per stage, moment-buffer parity and
                             the f passed to bgk_step; at most 16 kept) and
                             replayed on the step's stream */
} bgk_solver_opts;

typedef struct {
  int stages;
  int iters[4];           /* Picard iterations per stage */
  int total_iters;
  double last_ratio[4];   /* final max_m ratio per stage */
  int maxw_fallbacks;
  double seconds;         /* host wall time of the step */
  double sweep_ms;        /* summed device time of the sweep kernels (timing = 1) */
  double moments_ms;      /* summed device time of the moment kernels */
  double maxwellian_ms;   /* summed device time of the Maxwellian kernels */
  double other_ms;        /* DIRK combinations and copies */
  int sweeps;             /* number of sweep launches */
} bgk_step_stats;

typedef struct bgk_solver bgk_solver;

int bgk_solver_create(const tgs_dag* dag, const bgk_solver_opts* opts, bgk_solver** out);
int bgk_solver_destroy(bgk_solver* solver);

/* One DIRK step.  f (device, sweep layout) holds f^k on entry and f^{k+1}
 * on exit.  U_guess (device [n_nodes][dim+2] or NULL) replaces the moments
 * of f^k as the first stage's initial Picard iterate (learned guess); U_out
 * (device or NULL) receives the converged moments of f^{k+1}.
 * With MATCHED Maxwellians a node whose Newton solve fails keeps the DIRECT
 * coefficients for the rest of the stage (maxw_fallbacks counts such nodes
 * in every iteration).
 * Synchronises `stream` once per Picard iteration to test convergence, or
 * once per chunk of opts.chunk_iters iterations.
 * Errors: BGK_E_NOT_CONVERGED, BGK_E_NONPHYSICAL, BGK_E_HIP.  After an error
 * f still holds f^k unless the failure came where f is written: in the last
 * stage of a stiffly accurate tableau (backward Euler's only stage), which
 * iterates in f, or in the final combination of the other tableaux. */
int bgk_step(bgk_solver* solver, double* f, const double* U_guess, double* U_out,
             bgk_step_stats* stats, bgk_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Batched instances (an addition to the paper's method: many independent    */
/* problems stepped together, for uneven workloads that each fill only part  */
/* of the GPU)                                                               */
/* ------------------------------------------------------------------------ */

/* A batch steps n solvers together: every stage's Picard iteration (Sec. 4)
 * is one launch each of the Maxwellian, the Maxwellian tables, the sweep
 * (a persistent launch over all instances' velocities, longest generation
 * counts first), the moments and the stopping test of eq.
 * convergence-criteria, the last evaluated per instance on the device.  A
 * converged or failed instance is skipped by the rest of its stage.  With
 * `graph` set, each stage's chunk of `chunk_iters` iterations is captured
 * once in a hipGraph and replayed until every instance has stopped; the
 * host polls a small control block once per chunk.  Per instance the
 * arithmetic is bgk_step's, so results equal single-instance steps bit for
 * bit, except for an instance of 4096 to 16,383 cells with 8192 velocities
 * or more: bgk_step splits its moment sums over velocity chunks, the batch
 * does not, and the two agree to rounding.  (On tetrahedral instances of
 * 16,384 cells or more bgk_step sums the convergence norms over wider
 * blocks: equal moments, ratios equal to rounding.)  Requirements: all solvers share the dimension and the tableau, use
 * the FP64 sweep and have acyclic sweep graphs (else BGK_E_UNSUPPORTED).
 * The batch borrows the solvers (and their DAGs): destroy it first. */
typedef struct bgk_batch bgk_batch;

typedef struct {
  int graph;          /* 1: replay captured hipGraphs; 0: launch the same kernels eagerly */
  int chunk_iters;    /* Picard iterations between convergence polls (0: 4) */
  int sweep_threads;  /* workgroup size of the batched sweep, a multiple of 64 up to 256
                         (0: 128) */
  int sweep_lanes;    /* 0 or 64: the workgroup walk (one velocity per workgroup
                         of sweep_threads); 1, 2, 4, 8, 16 or 32: the packed walk,
                         64/sweep_lanes velocities of one instance per 64-lane
                         workgroup, sweep_lanes lanes each (as tgs_dag_set_walk;
                         results are the same bit for bit) */
} bgk_batch_opts;

typedef struct {
  int status;             /* BGK_OK or this instance's error code */
  int stages;
  int iters[4];           /* Picard iterations per stage */
  int total_iters;
  double last_ratio[4];
  int maxw_fallbacks;
  double finish_ms;       /* host milliseconds from the step's start to the poll
                             that saw this instance's last stage stop */
} bgk_batch_stats;

int bgk_batch_create(bgk_solver* const* solvers, int n, const bgk_batch_opts* opts,
                     bgk_batch** out);
int bgk_batch_destroy(bgk_batch* batch);

/* One DIRK step of every instance.  f: host array of n device pointers
 * (sweep layout), f^k on entry and f^{k+1} on exit; an instance that fails
 * leaves its f unspecified and reports its code in stats[i].status (stats:
 * host array of n, or NULL).  Returns BGK_OK when every instance succeeded,
 * else the first failing instance's code.  Ordered after prior work on
 * `stream` and before later work on it; runs on an internal stream of
 * default priority and synchronises once per chunk. */
int bgk_batch_step(bgk_batch* batch, double* const* f, bgk_batch_stats* stats,
                   bgk_stream_t stream);

/* Autotuning probe: from f's moments builds the Maxwellians, then times
 * `reps` batched sweeps of the first stage with the workgroup walk of
 * `threads` per workgroup (lanes 0 or 64) or the packed walk of `lanes` per
 * velocity (1, 2, 4, 8, 16 or 32; threads is then ignored but must be
 * valid), reading f and writing the solvers' f^k scratch; *ms = milliseconds
 * per sweep (host float).  Leaves f unchanged. */
int bgk_batch_time_sweep(bgk_batch* batch, double* const* f, int threads, int lanes, int reps,
                         float* ms, bgk_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Learned Picard initial guess (an addition to the paper's method: the       */
/* paper initialises Picard from the previous stage, Sec. 4)                  */
/* ------------------------------------------------------------------------ */

/* Network: 11 inputs -> 64 -> 64 -> 64 (GELU, exact erf) -> 5 outputs, per
 * DG node.  Inputs (raw): the primitive state (n, u1, u2, u3, theta) at
 * step t-1, its change from t-2 to t-1 (state and difference rather than two
 * states, so the small change survives BF16 rounding), and dt*nu at t-1
 * (u3 = 0 in 2D).  Outputs: the difference between (n, u1, u2, u3, theta)
 * at t and its linear extrapolation from t-2 and t-1 (a zero output gives
 * the extrapolated guess).  Inputs and outputs are z-scored inside the
 * library with the statistics given to bgk_mlp_set_normalization.  Matrix products run on
 * BF16 MFMA with FP32 accumulation; the master weights and the optimiser
 * state are FP32.  Gradients are reduced in a fixed order (reproducible).
 * Logical parameter layout (host arrays, 9413 floats): W1[11][64], b1[64],
 * W2[64][64], b2[64], W3[64][64], b3[64], W4[64][5], b4[5]; W_l[fan_in][fan_out]. */
typedef struct bgk_mlp bgk_mlp;
enum { BGK_MLP_PARAMS = 9413, BGK_MLP_IN = 11, BGK_MLP_OUT = 5 };

int bgk_mlp_create(const float* params /* host [9413] or NULL = zeros */, bgk_mlp** out);
int bgk_mlp_destroy(bgk_mlp* mlp);
int bgk_mlp_set_params(bgk_mlp* mlp, const float* params /* host [9413] */);  /* resets Adam */
int bgk_mlp_get_params(const bgk_mlp* mlp, float* params /* host [9413] */);
/* stats (host): mean_in[11], std_in[11], mean_out[5], std_out[5] */
int bgk_mlp_set_normalization(bgk_mlp* mlp, const float* stats);

/* Y (device [n][5]) = network output, de-normalised, for raw features X
 * (device [n][11]). */
int bgk_mlp_forward(bgk_mlp* mlp, const float* X, int64_t n, float* Y, bgk_stream_t stream);

/* Mean squared error between the normalised outputs and the normalised
 * targets T (device [n][5], raw changes); writes grad (device [9413],
 * logical layout, may be NULL) and loss (device float[1], may be NULL). */
int bgk_mlp_loss_grad(bgk_mlp* mlp, const float* X, const float* T, int64_t n, float* grad,
                      float* loss, bgk_stream_t stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the batch (X, T). */
int bgk_mlp_adam_step(bgk_mlp* mlp, const float* X, const float* T, int64_t n, float lr,
                      float* loss, bgk_stream_t stream);

/* Raw features (device float [n_nodes][11]) from nodal moments at t-1 and
 * t-2 (device [n_nodes][dim+2], user order) and the collision model. */
int bgk_mlp_features(const tgs_dag* dag, const double* U_tm1, const double* U_tm2,
                     const tgs_nu_model* nu_model, double dt, float* X, bgk_stream_t stream);

/* Raw targets (device float [n_nodes][5]): the primitive state at t minus its
 * linear extrapolation 2 p(t-1) - p(t-2). */
int bgk_mlp_targets(const tgs_dag* dag, const double* U_t, const double* U_tm1,
                    const double* U_tm2, float* T, bgk_stream_t stream);

/* Initial Picard moments for the next step:
 * U_guess = U(2 prim(U_tm1) - prim(U_tm2) + net),
 * per node; a node whose prediction has n <= 0, theta <= 0 or is not finite
 * falls back to U_tm1 (the plain previous-step guess) and is counted in
 * n_fallback (device int32, accumulated).  All nodal arrays in user order. */
int bgk_mlp_guess(bgk_mlp* mlp, const tgs_dag* dag, const double* U_tm1, const double* U_tm2,
                  const tgs_nu_model* nu_model, double dt, double* U_guess, int32_t* n_fallback,
                  bgk_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* BGKTGS_H */
