"""The oracle with slip walls (Sec. 4.4), pinned by what the mathematics fixes.

Cells next to a wall reconstruct one-sidedly: with at least three
neighbours the same least-squares fits as inside (fewer rows); with fewer
than three, the cell's own averaged gradient in step 1 and a linear
least-squares fit of the step-2 data.  The flux at a wall sees the mirror
image of the interior state.  Pins: exactness of the one-sided fits on
linear and quadratic data; a gas at rest in a closed box stays at rest;
the interface distribution at a slip wall is even in the normal velocity,
so the wall carries no mass, tangential momentum or energy flux and no
normal momentum at the interface; mass and energy are conserved exactly.
Meshes: the unit cube, N^3 hexahedra x 6 Kuhn tetrahedra, interior vertices
jittered (boundary vertices slide along the walls), seeded.
"""
import numpy as np
import pytest

import oracle
from paper_2102_01366_amd import inputs as I


def _box(n=4, seed=2, jitter=0.1):
    return I.kuhn_cube_mesh(n, 1.0, jitter, seed, False)


def _volumes(m):
    v = m.xyz[m.tet]
    return np.abs(np.linalg.det(v[:, 1:] - v[:, :1])) / 6.0


def _neighbour_counts(m):
    cnt = np.zeros(m.n_cell, int)
    for L, R in m.face_cell:
        if R >= 0:
            cnt[L] += 1
            cnt[R] += 1
    return cnt


def _polynomial_field(deg, seed=1):
    """W_q = a_q + b_q . x (+ x^T C_q x); exact gradients."""
    rng = np.random.default_rng(seed)
    a = np.array([1.3, 0.1, -0.2, 0.15, 4.0])
    b = 0.3 * rng.standard_normal((5, 3))
    C = 0.2 * rng.standard_normal((5, 3, 3)) if deg == 2 else np.zeros((5, 3, 3))
    C = 0.5 * (C + C.transpose(0, 2, 1))

    def f(X):
        Q = a[:, None, None] + np.einsum("qd,cpd->qcp", b, X) + np.einsum("cpd,qde,cpe->qcp", X, C, X)
        dQ = b[:, :, None, None] + 2.0 * np.einsum("qde,cpe->qdcp", C, X)
        return Q, dQ
    return f


def test_wall_mesh_has_cells_with_two_and_three_neighbours():
    cnt = _neighbour_counts(_box())
    assert cnt.min() == 2 and (cnt == 3).any() and cnt.max() == 4


def test_one_sided_slopes_reproduce_linear_data():
    m = _box()
    orc = oracle.Oracle(m, oracle.make_config())
    W, gW = I.cell_averages(m, _polynomial_field(1))
    b = orc.slopes(W, gW)
    # every cell: >= 3 neighbours (least squares) or its own exact gradient
    assert np.abs(b - gW).max() <= 1e-12 * np.abs(gW).max()


def test_boundary_step2_fits_reproduce_polynomials():
    m = _box()
    cnt = _neighbour_counts(m)
    orc = oracle.Oracle(m, oracle.make_config(nonlinear=False))
    # linear data: both the constrained fit and the linear fallback are exact
    W, gW = I.cell_averages(m, _polynomial_field(1))
    coef, flag, p2 = orc.reconstruct(W, gW, with_p2=True)
    G = p2[[1, 2, 3, 11, 12, 13, 21, 22, 23, 31, 32, 33, 41, 42, 43]]
    assert np.abs(G - gW).max() <= 1e-11 * np.abs(gW).max()
    H = p2[[r for q in range(5) for r in range(10 * q + 4, 10 * q + 10)]]
    assert np.abs(H).max() <= 1e-10
    # quadratic data: the constrained fit of cells with >= 3 neighbours is exact
    W, gW = I.cell_averages(m, _polynomial_field(2))
    coef, flag, p2 = orc.reconstruct(W, gW, with_p2=True)
    cen = m.xyz[m.tet].mean(axis=1)
    f = _polynomial_field(2)
    Q, dQ = f(cen[:, None, :])
    inner = cnt >= 3
    for q in range(5):
        assert np.abs(p2[10 * q + 1:10 * q + 4][:, inner] - dQ[q, :, inner, 0].T).max() <= 1e-10
    # the linear fallback (two neighbours) keeps the mean and has no curvature
    two = cnt == 2
    assert two.any()
    assert np.abs(p2[[10 * q for q in range(5)]][:, two] - W[:, two]).max() <= 1e-13 * np.abs(W).max()
    assert np.abs(p2[[r for q in range(5) for r in range(10 * q + 4, 10 * q + 10)]][:, two]).max() == 0.0


def test_gas_at_rest_stays_at_rest():
    m = _box(n=3)
    orc = oracle.Oracle(m, oracle.make_config(viscous=True, mu=0.01, prandtl=0.72))
    W = np.zeros((5, m.n_cell))
    W[0], W[4] = 1.2, 3.0
    gW = np.zeros((15, m.n_cell))
    dt = orc.compute_dt(W, 0.5)
    W1, g1 = W, gW
    for _ in range(3):
        W1, g1 = orc.step(dt, W1, g1)
    assert np.abs(W1 - W).max() <= 1e-14 * np.abs(W).max()
    dr = orc.geometry()[3]
    assert np.abs(g1).max() <= 1e-13 * np.abs(W).max() / dr.min()


def test_wall_faces_carry_no_mass_energy_or_tangential_flux():
    m = _box(n=3)
    orc = oracle.Oracle(m, oracle.make_config(viscous=True, mu=0.01, prandtl=0.72))
    W, gW = I.cell_averages(m, I.box_vortex_field())
    dt = orc.compute_dt(W, 0.5)
    ft = orc.face_terms(W, gW, dt)  # [20, nf]: F, dF/dt, W(0), W(dt) per component
    wall = m.face_cell[:, 1] < 0
    area, nrm, _ = orc.face_geometry()
    scale = np.abs(ft[1:4, wall]).max()  # momentum flux (pressure) scale
    for blk in (0, 5):
        assert np.abs(ft[blk + 0, wall]).max() <= 1e-13 * scale  # mass
        assert np.abs(ft[blk + 4, wall]).max() <= 1e-13 * scale * 10  # energy
        # the momentum flux is normal to the wall
        Fm = ft[blk + 1:blk + 4, wall]
        tang = Fm - nrm[:, wall] * np.einsum("dk,dk->k", Fm, nrm[:, wall])
        assert np.abs(tang).max() <= 1e-12 * np.abs(Fm).max()
    for blk in (10, 15):  # no normal momentum at the wall's interface
        mn = np.einsum("dk,dk->k", ft[blk + 1:blk + 4, wall], nrm[:, wall])
        assert np.abs(mn).max() <= 1e-13 * np.abs(ft[blk + 1:blk + 4, wall]).max()


@pytest.mark.parametrize("visc", [False, True])
def test_mass_and_energy_conserved_in_a_closed_box(visc):
    m = _box(n=3, seed=7)
    kw = dict(viscous=True, mu=0.01, prandtl=0.72) if visc else {}
    orc = oracle.Oracle(m, oracle.make_config(**kw))
    W, gW = I.cell_averages(m, I.box_vortex_field())
    s0 = orc.conservation_sums(W)
    dt = orc.compute_dt(W, 0.5)
    for _ in range(4):
        W, gW = orc.step(dt, W, gW)
    s1 = orc.conservation_sums(W)
    for q in (0, 4):
        assert abs(s1[q] - s0[q]) <= 1e-14 * abs(s0[q]) * 10
