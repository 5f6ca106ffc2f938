"""Writes cyclic_tet_mesh.txt: the seeded non-Delaunay tetrahedral mesh of
the unit cube (problems.flipped_cube_mesh(30, 40, seed=3)) whose upwind
graphs have cycles for 62 of the 216 velocities of the 6^3 grid on [-6, 6]^3.
It is an input fixture (no expected values): the cycle tests read it so that
they do not depend on Qhull's output.

Usage: python tests/golden/make_cyclic_tet_mesh.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import problems as P  # noqa: E402


def main():
    m = P.flipped_cube_mesh(30, 40, seed=3)
    with open(os.path.join(HERE, "cyclic_tet_mesh.txt"), "w") as fh:
        fh.write("# problems.flipped_cube_mesh(n_interior=30, n_flips=40, seed=3)\n")
        fh.write("# written by tests/golden/make_cyclic_tet_mesh.py\n")
        fh.write(f"vert {m.vert.shape[0]}\n")
        for x in m.vert:
            fh.write(" ".join(repr(float(c)) for c in x) + "\n")
        fh.write(f"cells {m.cells.shape[0]}\n")
        for c in m.cells:
            fh.write(" ".join(str(int(i)) for i in c) + "\n")


if __name__ == "__main__":
    main()
