"""FP64 CPU oracle for the sweep-based implicit BGK method.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of what the paper's method computes.  It exists to
judge the GPU path: only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the GPU library or
its Python binding; the only common dependency is the seeded problem
generator in ``problems``.

Modules and the passages they follow:

* ``refel``     reference-element matrices, exact rational integration
                (Sec. 3.1: nodal Lagrange basis by affine map, quadrature exact
                to degree 2k, Table of reference elements).
* ``geometry``  physical cells, outward unit normals, face matching
                (Sec. 3.1 and eq. cell-inflow-outflow-boundaries).
* ``dag``       upwind graphs, DFS with back-edge lagging, longest-path
                generations (Sec. 4.1).
* ``transport`` the per-cell upwind DG solve, the sweep and a dense global
                solve of the same system (eq. bgk-ss-inflow-outflow,
                eq. bgk-ss-picard).
* ``kinetic``   velocity moments, primitive variables, Maxwellians
                (eq. primitive_g, eq. moments, eq. Maxwellian-projection,
                eq. linear-Maxwellian) and the collision frequency.
* ``solver``    Picard iteration with its stopping rule, DIRK stages and the
                explicit time-step bound (Sec. 3.5, Sec. 4, eq. explicit-dt,
                App. A).
* ``mlp``       the learned initial-guess network (not in the paper: an
                FP64 and a BF16-emulating reference for the GPU kernels).

Readings where the paper is silent or garbled are listed in the design
notes of the repository; each function states the reading it takes.
"""
