"""Pins of the oracle's quadratic elements (Sec. 2.1 quadratic triangles with
a normal and a weight per Gauss point, eq. flux-para-coord-gauss; Sec. 4.1
quadratic tetrahedra integrated by the five-point rule on the isoparametric
map, eq. base-int-change):

* with every control point at its edge midpoint the quadratic element is the
  linear one (the paper's remark closing Sec. 2.1): the same volumes,
  centroids, moments, face areas, normals and Gauss points;
* a tetrahedron with one edge bent has det J = 1 - 4 delta xi, so its
  volume, centroid and the area of its flat bent face have closed forms that
  the rules integrate exactly;
* the cells of a periodic mesh with bent edges still tile the box: their
  volumes add up to the box's;
* on such a mesh a uniform flow stays uniform and mass, momentum and energy
  are conserved (the per-point normals and weights close every cell);
* on the sphere the quadratic wall converges at fourth order: the wall area
  to 4 pi and the volume it encloses to 4 pi / 3, where straight faces give
  second order; its Gauss-point normals converge to the radial direction at
  second order, where straight faces give first;
* the scheme keeps its third order on bent cells;
* on a no-slip sphere the constrained fits (Sec. 4.4) meet the wall values at
  the quadratic wall's own points: step 1 at the mean of a face's Gauss
  points, step 2 at its three Gauss points on the curved surface, where the
  fits of the straight-faced sphere miss them by O(h^2).
"""
import math

import numpy as np
import pytest

from paper_2102_01366_amd import inputs as I


def _ref_monomial(a, b, c, d):
    """integral over the reference tetrahedron of xi^a eta^b zeta^c L^d,
    L = 1 - xi - eta - zeta: a! b! c! d! / (a + b + c + d + 3)!"""
    f = math.factorial
    return f(a) * f(b) * f(c) * f(d) / f(a + b + c + d + 3)


def _single_tet(delta):
    """the reference tetrahedron, the control point of edge (0,1) moved to
    (1/2, delta, 0): X = xi + 4 delta xi L e_y"""
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    tet = np.array([[0, 1, 2, 3]], np.int64)
    fv = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]], np.int64)
    fc = np.array([[0, -1]] * 4, np.int64)
    m = I.TetMesh(xyz=xyz, tet=tet, face_vert=fv, face_cell=fc,
                  face_tag=np.full(4, I.FACE_SLIP, np.int32), face_shift=np.zeros((4, 3)),
                  length=1.0, n=1, periodic=False)
    m.tet_mid = I.straight_edge_points(m)
    m.tet_mid[0, 0] = (0.5, delta, 0.0)
    return m


def test_straight_control_points_are_the_linear_element(oracle_lib):
    cfg = oracle_lib.make_config()
    m = I.kuhn_cube_mesh(3, 1.0, 0.1, 3, True)
    lin = oracle_lib.Oracle(m, cfg)
    m.tet_mid = I.straight_edge_points(m)
    quad = oracle_lib.Oracle(m, cfg)
    for a, b in zip(lin.geometry() + lin.face_geometry() + lin.face_points(),
                    quad.geometry() + quad.face_geometry() + quad.face_points()):
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-14 * np.abs(a).max())


@pytest.mark.parametrize("delta", [0.05, -0.1, 0.2])
def test_bent_edge_closed_forms(oracle_lib, delta):
    orc = oracle_lib.Oracle(_single_tet(delta), oracle_lib.make_config())
    vol, cen, m2, dr = orc.geometry()
    # det J = 1 - 4 delta xi
    V = _ref_monomial(0, 0, 0, 0) - 4 * delta * _ref_monomial(1, 0, 0, 0)
    assert vol[0] == pytest.approx(V, rel=1e-14)
    mx = _ref_monomial(1, 0, 0, 0) - 4 * delta * _ref_monomial(2, 0, 0, 0)
    my = (_ref_monomial(0, 1, 0, 0) - 4 * delta * _ref_monomial(1, 1, 0, 0)
          + 4 * delta * (_ref_monomial(1, 0, 0, 1) - 4 * delta * _ref_monomial(2, 0, 0, 1)))
    mz = _ref_monomial(0, 0, 1, 0) - 4 * delta * _ref_monomial(1, 0, 1, 0)
    np.testing.assert_allclose(cen[:, 0], np.array([mx, my, mz]) / V, rtol=1e-13)
    area, nrm, gp = orc.face_geometry()
    pn, pw = orc.face_points()
    # face 3 (z = 0) stays in its plane: normal -e_z at every point, area
    # integral of (1 - 4 delta xi) over the reference triangle
    np.testing.assert_allclose(pn[:, :, 3], np.tile([0.0, 0.0, -1.0], (3, 1)), atol=1e-15)
    assert area[3] == pytest.approx(0.5 - 4 * delta / 6.0, rel=1e-14)
    # the faces that do not hold the bent edge are unchanged
    assert area[0] == pytest.approx(math.sqrt(3) / 2, rel=1e-14)
    assert area[1] == pytest.approx(0.5, rel=1e-14)


def test_bent_cells_tile_the_box(oracle_lib):
    m = I.kuhn_cube_mesh(4, 1.0, 0.1, 1, True, curve=0.1)
    straight = I.straight_edge_points(m)
    assert np.abs(m.tet_mid - straight).max() > 0.01
    vol = oracle_lib.Oracle(m, oracle_lib.make_config()).geometry()[0]
    lin = oracle_lib.Oracle(I.kuhn_cube_mesh(4, 1.0, 0.1, 1, True), oracle_lib.make_config()).geometry()[0]
    assert np.abs(vol - lin).max() > 1e-5          # the cells did change
    assert vol.sum() == pytest.approx(1.0, rel=1e-14)


def test_free_stream_and_conservation_on_quadratic_cells(oracle_lib):
    m = I.kuhn_cube_mesh(4, 1.0, 0.1, 2, True, curve=0.08)
    orc = oracle_lib.Oracle(m, oracle_lib.make_config())
    W, gW = I.uniform_state(m, 1.0, (0.4, -0.3, 0.2), 1.0)
    dt = orc.compute_dt(W, 0.5)
    W1, g1 = orc.step(dt, W, gW)
    assert np.abs(W1 - W).max() < 1e-13
    assert np.abs(g1).max() < 1e-10
    W, gW = I.cell_averages(m, I.sine_wave_field())
    vol = orc.geometry()[0]
    s0 = W @ vol
    for _ in range(3):
        W, gW = orc.step(orc.compute_dt(W, 0.5), W, gW)
    np.testing.assert_allclose(W @ vol, s0, rtol=1e-13, atol=1e-13)


def _sphere_wall(oracle_lib, n, curved):
    s = I.cubed_sphere_shell(n, 2, r_out=2.0, ratio=1.0, curved=curved)
    orc = oracle_lib.Oracle(s, oracle_lib.make_config())
    wall = s.face_tag == I.FACE_SLIP
    pn, pw = orc.face_points()
    gp = orc.face_geometry()[2]
    area = pw[:, wall].sum()
    vol = orc.geometry()[0].sum()
    # angle between the Gauss-point normals and the inward radial direction
    x = gp[:, :, wall]
    r = -x / np.linalg.norm(x, axis=1, keepdims=True)
    ang = np.arccos(np.clip((pn[:, :, wall] * r).sum(axis=1), -1.0, 1.0)).max()
    return area, vol, ang


def test_quadratic_sphere_wall_converges_at_fourth_order(oracle_lib):
    res = {(n, c): _sphere_wall(oracle_lib, n, c) for n in (4, 8) for c in (False, True)}
    # wall area
    e = {k: abs(v[0] - 4 * math.pi) for k, v in res.items()}
    assert e[(4, True)] < 0.01 * e[(4, False)]
    assert e[(4, True)] / e[(8, True)] > 12.0        # fourth order: 16
    assert 3.0 < e[(4, False)] / e[(8, False)] < 5.0  # second order: 4
    # the volume the wall encloses: the shell's volume falls by what the
    # bent wall adds to the ball; the straight wall's inscribed polyhedron
    # misses 4 pi / 3 - V_poly, the quadratic wall much less
    for n in (4, 8):
        added = res[(n, False)][1] - res[(n, True)][1]
        s = I.cubed_sphere_shell(n, 2, r_out=2.0, ratio=1.0)
        tri = s.xyz[s.face_vert[s.face_tag == I.FACE_SLIP]]
        v_poly = abs(np.einsum("ij,ij->i", tri[:, 0], np.cross(tri[:, 1], tri[:, 2]))).sum() / 6.0
        res[(n, "ball")] = abs(v_poly + added - 4 * math.pi / 3), abs(v_poly - 4 * math.pi / 3)
    assert res[(4, "ball")][0] < 0.01 * res[(4, "ball")][1]
    assert res[(4, "ball")][0] / res[(8, "ball")][0] > 12.0
    # normals at the wall Gauss points
    assert res[(4, True)][2] / res[(8, True)][2] > 3.0   # second order
    assert res[(4, False)][2] / res[(8, False)][2] < 2.5  # first order
    assert res[(8, True)][2] < 0.1 * res[(8, False)][2]


def test_third_order_on_bent_cells(oracle_lib):
    """The sine wave (Sec. 5.1 set-up, linear weights) on periodic meshes whose
    every edge is bent by up to 5% of h converges like the straight mesh:
    the density L1 error against exact cell averages over the quadratic
    cells converges at order 2.8 from 8 to 16 cells per side (straight
    cells: 2.9)."""
    cfg = oracle_lib.make_config(nonlinear=False)
    T = 0.02
    errs = []
    for N in (4, 8, 16):
        m = I.kuhn_cube_mesh(N, 1.0, 0.1, 0, True, curve=0.05)
        orc = oracle_lib.Oracle(m, cfg)
        W, gW = I.cell_averages(m, I.sine_wave_field())
        vol = orc.geometry()[0]
        ns = int(np.ceil(T / orc.compute_dt(W, 0.5)))
        dt = T / ns
        for _ in range(ns):
            W, gW = orc.step(dt, W, gW)
        We, _ = I.cell_averages(m, I.sine_wave_field(t=T))
        errs.append(np.sum(vol * np.abs(W[0] - We[0])) / vol.sum())
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert order[-1] > 2.6, (errs, order)
    assert order[0] > 2.0, (errs, order)


def _quad_value(c, x):
    """R(x) = c0 + G.x + x^T H x / 2 with c = (c0, G, Hxx, Hyy, Hzz, Hxy, Hxz, Hyz)"""
    H = np.array([[c[4], c[7], c[8]], [c[7], c[5], c[9]], [c[8], c[9], c[6]]])
    return c[0] + c[1:4] @ x + 0.5 * x @ H @ x


@pytest.mark.parametrize("tag", [I.FACE_NOSLIP_ADIABATIC, I.FACE_NOSLIP_ISOTHERMAL],
                         ids=["adiabatic", "isothermal"])
def test_constraints_met_at_the_curved_wall_points(oracle_lib, tag):
    gamma, Tw = 1.4, 0.9
    cfg = oracle_lib.make_config(viscous=True, mu=0.01, wall_T=Tw)
    curved = I.cubed_sphere_shell(4, 2, r_out=2.0, ratio=1.0, curved=True, wall_tag=tag)
    gp = oracle_lib.Oracle(curved, cfg).face_geometry()[2]
    wall = np.nonzero(curved.face_tag == tag)[0]
    own = curved.face_cell[wall, 0]
    one = np.bincount(own, minlength=curved.n_cell)[own] == 1    # cells with a single wall face
    wall, own = wall[one], own[one]
    assert wall.size > 100
    worst = {}
    for name, m in (("curved", curved),
                    ("straight", I.cubed_sphere_shell(4, 2, r_out=2.0, ratio=1.0, wall_tag=tag))):
        orc = oracle_lib.Oracle(m, cfg)
        W, gW = I.cell_averages(m, I.bump_stream_field(gamma))
        b = orc.slopes(W, gW)
        coef, flag, p2 = orc.reconstruct(W, gW, with_p2=True)
        assert not flag.any()
        cen = orc.geometry()[1]
        e1 = e2 = 0.0
        for f, i in zip(wall, own):
            # step 1: P^1 of each constrained component at the mean of the
            # face's Gauss points against the wall value from P^1 of density
            x = gp[:, :, f].mean(axis=0) - cen[:, i]
            rho1 = W[0, i] + b[0:3, i] @ x
            for q in range(1, 5 if tag == I.FACE_NOSLIP_ISOTHERMAL else 4):
                target = rho1 * Tw / (gamma - 1) if q == 4 else 0.0
                e1 = max(e1, abs(W[q, i] + b[3 * q:3 * q + 3, i] @ x - target))
            # step 2: the constrained P^2 at each Gauss point against the wall
            # value from the final density polynomial
            for k in range(3):
                x = gp[k, :, f] - cen[:, i]
                rho2 = _quad_value(coef[0:10, i], x)
                for q in range(1, 5 if tag == I.FACE_NOSLIP_ISOTHERMAL else 4):
                    target = rho2 * Tw / (gamma - 1) if q == 4 else 0.0
                    e2 = max(e2, abs(_quad_value(p2[10 * q:10 * q + 10, i], x) - target))
        worst[name] = e1, e2
    assert max(worst["curved"]) < 1e-13, worst
    assert min(worst["straight"]) > 1e-3, worst


@pytest.mark.parametrize("tag", [I.FACE_NOSLIP_ADIABATIC, I.FACE_NOSLIP_ISOTHERMAL],
                         ids=["adiabatic", "isothermal"])
def test_gas_at_rest_stays_at_rest_around_the_curved_no_slip_sphere(oracle_lib, tag):
    """A gas at rest at the wall temperature around the quadratic no-slip
    sphere, with the same gas as free stream: the constrained fits at the
    curved wall points, the reflected ghost and the far field leave it at
    rest (the quadratic faces close every cell)."""
    gamma, Tw = 1.4, 1.0 / 1.4
    m = I.cubed_sphere_shell(4, 2, r_out=2.0, ratio=1.0, curved=True, wall_tag=tag)
    W, gW = I.uniform_state(m, 1.0, (0.0, 0.0, 0.0), Tw, gamma)
    orc = oracle_lib.Oracle(m, oracle_lib.make_config(viscous=True, mu=0.01, prandtl=0.72, wall_T=Tw,
                                                      farfield=tuple(W[:, 0])))
    dt = orc.compute_dt(W, 0.5)
    Wo, gWo = W, gW
    for _ in range(3):
        Wo, gWo = orc.step(dt, Wo, gWo)
    assert np.abs(Wo - W).max() < 1e-13
    dr = orc.geometry()[3]
    assert np.abs(gWo).max() < 1e-13 * 3 * np.abs(W).max() / dr.min()
