"""Oracle pins: reference-element matrices and cell geometry.

Pinned against textbook element matrices (tests/golden/reference_matrices.txt)
and against the divergence theorem, which ties the stiffness matrices to the
facet normals and facet mass matrices independently of how either is built.
"""
import numpy as np
import pytest

import problems as P
from oracle import geometry, refel
from tests.conftest import read_golden


def _mat(tokens):
    rows = " ".join(tokens).split("/")
    return np.array([[float(x) for x in r.split()] for r in rows])


def test_textbook_mass_matrices():
    g = read_golden("reference_matrices.txt")
    np.testing.assert_array_equal(refel.reference(2, 1)["mass"] * 12, _mat(g["P1TRI_MASS_TIMES_12"]))
    np.testing.assert_allclose(refel.reference(3, 1)["mass"] * 20, _mat(g["P1TET_MASS_TIMES_20"]),
                               rtol=0, atol=1e-13)
    np.testing.assert_allclose(refel.reference(2, 2)["mass"] * 180,
                               _mat(g["P2TRI_MASS_TIMES_180"]), rtol=0, atol=1e-12)


def test_textbook_facet_mass_matrices():
    g = read_golden("reference_matrices.txt")
    r1 = refel.reference(2, 1)
    for k in range(3):
        fn = r1["face_nodes"][k]
        np.testing.assert_allclose(r1["face_mass"][k][np.ix_(fn, fn)] * 6,
                                   _mat(g["P1EDGE_MASS_TIMES_6"]), atol=1e-14)
    r2 = refel.reference(2, 2)
    for k in range(3):
        fn = r2["face_nodes"][k]           # two vertices (ascending) then the midpoint
        np.testing.assert_allclose(r2["face_mass"][k][np.ix_(fn, fn)] * 30,
                                   _mat(g["P2EDGE_MASS_TIMES_30"]), atol=1e-13)
    r3 = refel.reference(3, 1)
    for k in range(4):
        fn = r3["face_nodes"][k]
        np.testing.assert_allclose(r3["face_mass"][k][np.ix_(fn, fn)] * 12,
                                   np.ones((3, 3)) + np.eye(3), atol=1e-14)


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1)])
def test_partition_of_unity_and_reproduction(dim, order):
    r = refel.reference(dim, order)
    # sum of all mass entries = integral of 1 = |K| (normalised to 1)
    assert abs(r["mass"].sum() - 1.0) < 1e-14
    # basis sums to one: sum_a d(phi_a) = 0, so every column sum of stiff is 0
    assert np.abs(r["stiff"].sum(axis=1)).max() < 1e-14


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1)])
def test_integration_by_parts(dim, order):
    """int_K phi_b v.grad phi_a + int_K phi_a v.grad phi_b = sum_e (v.n_e) int_e phi_a phi_b.

    G[a][b] = |det J| sum_beta (J^{-1} v)_beta stiff_beta[a][b] is the first
    integral, so G + G^T must equal the sum of facet terms built from the
    geometric normals and facet measures.
    """
    pr = P.small_problem(dim=dim, order=order, n_side=3)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, order)
    rng = np.random.default_rng(5)
    r = geo.ref
    for c in range(geo.n_cells):
        v = rng.normal(size=dim)
        vt = geo.jinv[c] @ v
        G = geo.det[c] * np.einsum("b,bxy->xy", vt, r["stiff"])
        rhs = sum((v @ geo.normal[c, k]) * geo.area[c, k] * r["face_mass"][k] for k in range(dim + 1))
        np.testing.assert_allclose(G + G.T, rhs, atol=1e-14 * max(1.0, np.abs(rhs).max()))


@pytest.mark.parametrize("dim", [2, 3])
def test_geometry_closure(dim):
    """Facet normals are unit, area-weighted normals of a closed cell sum to zero,
    interior facets are shared with opposite normals, and volumes tile the box."""
    pr = P.small_problem(dim=dim, order=1, n_side=3)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, 1)
    assert np.allclose(np.linalg.norm(geo.normal, axis=2), 1.0)
    closure = np.einsum("ck,ckd->cd", geo.area, geo.normal)
    assert np.abs(closure).max() < 1e-14
    assert abs(geo.vol.sum() - 1.0) < 1e-13
    for c in range(geo.n_cells):
        for k in range(dim + 1):
            b = geo.nbr[c, k]
            if b >= 0:
                kb = geo.nbr_face[c, k]
                assert geo.nbr[b, kb] == c
                np.testing.assert_array_equal(geo.normal[b, kb], -geo.normal[c, k])
    # boundary facets lie on the box and point outward along an axis
    for c in range(geo.n_cells):
        for k in range(dim + 1):
            if geo.nbr[c, k] < 0:
                n = geo.normal[c, k]
                assert np.isclose(np.abs(n).max(), 1.0)


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1)])
def test_local_matrix_symmetric_part_is_the_energy_form(dim, order):
    """For a cell-constant sigma the local DG matrix has symmetric part
    sigma|K| M + (1/2) sum_k |v.n_k| |e_k| M_k (integration by parts turns the
    transport term into half the facet fluxes; eq. l2-estimate), which is
    positive definite."""
    from oracle import transport
    pr = P.small_problem(dim=dim, order=order, n_side=3, n_1d=4)
    geo = geometry.build(pr.mesh.vert, pr.mesh.cells, order)
    rng = np.random.default_rng(3)
    cells = rng.integers(0, geo.n_cells, 40)
    V = rng.normal(size=(40, dim)) * 3.0
    sig = rng.uniform(0.1, 5.0, 40)
    A, s = transport.cell_matrices(geo, cells, V, np.repeat(sig[:, None], geo.n_p, axis=1))
    ref = geo.ref
    for i in range(40):
        sym = 0.5 * (A[i] + A[i].T)
        expect = sig[i] * geo.vol[cells[i]] * ref["mass"]
        for k in range(dim + 1):
            expect = expect + 0.5 * abs(s[i, k]) * geo.area[cells[i], k] * ref["face_mass"][k]
        assert np.abs(sym - expect).max() <= 1e-13 * np.abs(expect).max()
        assert np.linalg.eigvalsh(sym).min() > 0.0
