"""Pins of the oracle's quadrature and geometry against closed forms.

The oracle integrates with the paper's own rules (Sec. 2.1 three-point face
rule; Sec. 4.1 five-point volume rule with the centre weight read as -2/15).
These tests check those rules and the resulting geometry against exact
integrals of monomials and closed-form tetrahedron formulas that the oracle
does not use.
"""
from math import factorial

import numpy as np
import pytest

from paper_2102_01366_amd import inputs as I


def _simplex3_monomial(a, b, c):
    # exact integral of xi^a eta^b zeta^c over the unit tetrahedron
    return factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)


def _simplex2_monomial(a, b):
    return factorial(a) * factorial(b) / factorial(a + b + 2)


def test_volume_rule_exact_to_degree_3(oracle_lib):
    pts, w = oracle_lib.volume_rule()
    assert abs(w.sum() - 1.0 / 6.0) < 1e-15
    for a in range(4):
        for b in range(4 - a):
            for c in range(4 - a - b):
                q = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
                assert abs(q - _simplex3_monomial(a, b, c)) < 1e-15, (a, b, c)
    # not exact at degree 4: the rule is what the paper prints, no better
    q4 = np.sum(w * pts[:, 0] ** 4)
    assert abs(q4 - _simplex3_monomial(4, 0, 0)) > 1e-6


def test_face_rule_exact_to_degree_2(oracle_lib):
    pts, w = oracle_lib.face_rule()
    for a in range(3):
        for b in range(3 - a):
            q = 0.5 * np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b)
            assert abs(q - _simplex2_monomial(a, b)) < 1e-15, (a, b)


@pytest.fixture(scope="module")
def jittered(oracle_lib):
    m = I.kuhn_cube_mesh(4, 1.3, 0.1, 7, True)
    orc = oracle_lib.Oracle(m, oracle_lib.make_config())
    return m, orc


def test_cell_geometry_closed_form(jittered):
    m, orc = jittered
    vol, cen, m2, dr = orc.geometry()
    v = m.xyz[m.tet]
    e = v[:, 1:] - v[:, :1]
    vol_cf = np.abs(np.linalg.det(e)) / 6.0
    np.testing.assert_allclose(vol, vol_cf, rtol=1e-13, atol=0)
    assert abs(vol.sum() - 1.3 ** 3) < 1e-13
    np.testing.assert_allclose(cen.T, v.mean(axis=1), rtol=0, atol=1e-14)
    # second moment about the centroid: (1/20)(sum v v^T + S S^T) - c c^T, S = sum v
    S = v.sum(axis=1)
    full = (np.einsum("cai,caj->cij", v, v) + np.einsum("ci,cj->cij", S, S)) / 20.0
    cc = np.einsum("ci,cj->cij", cen.T, cen.T)
    M = full - cc
    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for k, (i, j) in enumerate(idx):
        np.testing.assert_allclose(m2[k], M[:, i, j], rtol=1e-9, atol=1e-15)


def test_face_geometry_and_closed_surfaces(jittered):
    m, orc = jittered
    vol, cen, m2, dr = orc.geometry()
    area, nrm, gp = orc.face_geometry()
    x = m.xyz[m.face_vert]  # [nf,3,3]
    cr = np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0])
    np.testing.assert_allclose(area, 0.5 * np.linalg.norm(cr, axis=1), rtol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(nrm, axis=0), 1.0, atol=1e-15)
    # Gauss points at barycentric (2/3,1/6,1/6) and its permutations
    bary = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])
    for q in range(3):
        np.testing.assert_allclose(gp[q].T, np.einsum("k,fkd->fd", bary[q], x), atol=1e-14)
    # owner-outward: the normal points away from the owner's centroid
    L = m.face_cell[:, 0]
    out = np.einsum("df,fd->f", nrm, gp[0].T - cen[:, L].T)
    assert np.all(out > 0)
    # every cell surface is closed: sum of n |Gamma| over its faces vanishes
    s = np.zeros((m.n_cell, 3))
    np.add.at(s, L, (nrm * area).T)
    np.add.at(s, m.face_cell[:, 1], -(nrm * area).T)
    assert np.abs(s).max() < 1e-15
    # inscribed-sphere estimate 3 |Omega| / sum |Gamma|
    sa = np.zeros(m.n_cell)
    np.add.at(sa, L, area)
    np.add.at(sa, m.face_cell[:, 1], area)
    np.testing.assert_allclose(dr, 3 * vol / sa, rtol=1e-14)
