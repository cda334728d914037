"""Pins of the oracle's no-slip walls (Sec. 4.4), against what the paper and
the mathematics fix.

* Ghost state, adiabatic wall at rest: the paper's printed rules, (rho,
  -rho U, rho E), unchanged momentum derivatives, reversed density and
  energy derivatives.
* Ghost state in general (moving walls, isothermal walls): the point
  reflection through the wall point of the primitive fields, velocity odd
  about U_wall, pressure even, temperature even (adiabatic) or odd about
  T_wall (isothermal) -- composed as functions of position and
  differentiated by complex step, independently of the chain rule the
  oracle uses.
* Reconstruction step 1: a linear field that meets the wall constraints
  (rho U = rho U_wall, and rho E = rho (|U_wall|^2/2 + T_wall/(gamma-1)) on
  isothermal walls) is reproduced exactly by the constrained fit.
* Reconstruction step 2: a quadratic field that meets them is reproduced
  exactly by the constrained P^2 (linear weights, so R = P^2).
* A gas at rest at the wall temperature in an isothermal box, and any gas at
  rest in an adiabatic box, stays at rest.
"""
import numpy as np
import pytest

from paper_2102_01366_amd import inputs as I

GAMMA = 1.4
ADIA, ISO = I.FACE_NOSLIP_ADIABATIC, I.FACE_NOSLIP_ISOTHERMAL


def _state(rng):
    rho = rng.uniform(0.8, 1.3)
    U = rng.uniform(-0.5, 0.5, 3)
    p = rng.uniform(0.7, 1.4)
    return np.array([rho, *(rho * U), p / (GAMMA - 1) + 0.5 * rho * U @ U])


def _prim(W):
    rho = W[0]
    U = W[1:4] / rho
    p = (GAMMA - 1) * (W[4] - 0.5 * rho * (U @ U))
    return rho, U, p


def _cons(U, p, T):
    rho = p / T
    return np.concatenate([[rho], rho * U, [p / (GAMMA - 1) + 0.5 * rho * (U @ U)]])


def test_adiabatic_ghost_at_rest_is_the_papers_rule(oracle_lib):
    rng = np.random.default_rng(1)
    cfg = oracle_lib.make_config()
    for _ in range(5):
        W, gW = _state(rng), 0.3 * rng.standard_normal(15)
        n = rng.standard_normal(3)
        Wg, gWg = oracle_lib.wall_ghost(cfg, ADIA, n / np.linalg.norm(n), np.zeros(3), W, gW)
        np.testing.assert_allclose(Wg, W * np.array([1, -1, -1, -1, 1]), rtol=1e-14, atol=1e-15)
        G, Gg = gW.reshape(5, 3), gWg.reshape(5, 3)
        np.testing.assert_allclose(Gg[1:4], G[1:4], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(Gg[[0, 4]], -G[[0, 4]], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("tag", [ADIA, ISO], ids=["adiabatic", "isothermal"])
def test_ghost_is_the_point_reflection_of_the_primitive_fields(oracle_lib, tag):
    rng = np.random.default_rng(2)
    Tw = 0.9
    cfg = oracle_lib.make_config(wall_T=Tw)
    for _ in range(5):
        W0, G = _state(rng), 0.3 * rng.standard_normal((5, 3))
        uw = rng.uniform(-0.3, 0.3, 3)

        def ghost_field(x):
            # interior field at the reflected point, to primitives, reflected, back
            rho, U, p = _prim(W0 + G @ (-x))
            T = p / rho
            return _cons(2 * uw - U, p, (2 * Tw - T) if tag == ISO else T)

        h = 1e-30
        ref_g = np.stack([ghost_field(1j * h * np.eye(3)[j]).imag / h for j in range(3)], axis=1)
        Wg, gWg = oracle_lib.wall_ghost(cfg, tag, np.array([0.0, 0.0, 1.0]), uw, W0, G.reshape(15))
        np.testing.assert_allclose(Wg, ghost_field(np.zeros(3)).real, rtol=1e-14)
        np.testing.assert_allclose(gWg.reshape(5, 3), ref_g, rtol=1e-12, atol=1e-13)


def _wall_mesh(n, tag, uw=(0.0, 0.0, 0.0), seed=3):
    m = I.kuhn_cube_mesh(n, 1.0, 0.1, seed, False)
    return I.with_walls(m, {"x0": tag}, {"x0": uw})


def _fields_meeting_constraints(tag, uw, Tw, quadratic):
    """Component functions of x (3, npts): rho; rho U = rho U_wall + x (.);
    rho E = rho (|U_wall|^2/2 + T_wall/(gamma-1)) + x (.) -- all meeting the
    wall values on the plane x = 0."""
    uw = np.asarray(uw)
    ew = 0.5 * uw @ uw + Tw / (GAMMA - 1)

    def f(X):
        x, y, z = X[..., 0], X[..., 1], X[..., 2]
        rho = 1.0 + 0.1 * x + 0.05 * y - 0.04 * z + (0.03 * x * y - 0.02 * z * z if quadratic else 0)
        q = [0.2 + (0.1 * x - 0.05 * z if quadratic else 0), -0.1 + (0.07 * y if quadratic else 0),
             0.15 + (0.04 * x + 0.06 * y if quadratic else 0)]
        W = [rho] + [rho * uw[d] + x * q[d] for d in range(3)]
        W.append(rho * ew + x * (0.3 + (0.05 * y if quadratic else 0)) if tag == ISO else 2.5 + 0.1 * y)
        return np.stack(W)
    return f


def _averages(mesh, f):
    """Exact cell averages and averaged gradients of a polynomial field of
    degree <= 2 (a rule exact for quadratics; gradients by central
    differences, exact for polynomials of degree <= 2)."""
    def field(X):
        h = 1e-4
        G = np.stack([(f(X + h * np.eye(3)[d]) - f(X - h * np.eye(3)[d])) / (2 * h) for d in range(3)], axis=1)
        return f(X), G
    return I.cell_averages(mesh, field)


@pytest.mark.parametrize("tag,uw", [(ADIA, (0, 0, 0)), (ISO, (0, 0, 0)), (ISO, (0.0, 0.3, -0.1))],
                         ids=["adiabatic", "isothermal", "isothermal_moving"])
def test_step1_constrained_fit_reproduces_linear_fields(oracle_lib, tag, uw):
    Tw = 0.8
    m = _wall_mesh(3, tag, uw)
    cfg = oracle_lib.make_config(wall_T=Tw)
    orc = oracle_lib.Oracle(m, cfg)
    f = _fields_meeting_constraints(tag, uw, Tw, quadratic=False)
    W, gW = _averages(m, f)
    b = orc.slopes(W, gW)
    np.testing.assert_allclose(b, gW, rtol=0, atol=1e-11)
    # a field that violates the constraint is not reproduced at the wall cells
    W2 = W.copy()
    W2[1] += 0.05
    assert np.abs(orc.slopes(W2, gW)[3:6] - gW[3:6]).max() > 1e-3


@pytest.mark.parametrize("tag,uw", [(ADIA, (0, 0, 0)), (ISO, (0, 0, 0)), (ISO, (0.0, 0.3, -0.1))],
                         ids=["adiabatic", "isothermal", "isothermal_moving"])
def test_step2_constrained_fit_reproduces_quadratic_fields(oracle_lib, tag, uw):
    Tw = 0.8
    m = _wall_mesh(4, tag, uw)
    cfg = oracle_lib.make_config(wall_T=Tw, nonlinear=False)
    orc = oracle_lib.Oracle(m, cfg)
    f = _fields_meeting_constraints(tag, uw, Tw, quadratic=True)
    W, gW = _averages(m, f)
    coef, flag = orc.reconstruct(W, gW)
    assert not flag.any()
    # cells with one wall face (three neighbours) on the constrained side:
    # every component exact there (the density unconstrained, the rest
    # constrained); interior cells exact as well
    nwall = np.zeros(m.n_cell, int)
    np.add.at(nwall, m.face_cell[m.face_cell[:, 1] < 0, 0], 1)
    cells = np.nonzero(nwall <= 1)[0]
    cen = orc.geometry()[1]
    h = 1e-4
    for i in cells[::3]:
        X = cen[:, i]
        for q in range(5):
            c = coef[10 * q:10 * q + 10, i]
            val = f(X)[q]
            grad = [(f(X + h * np.eye(3)[d]) - f(X - h * np.eye(3)[d]))[q] / (2 * h) for d in range(3)]
            assert abs(c[0] - val) <= 1e-10 and np.abs(c[1:4] - grad).max() <= 1e-8, (i, q, c[:4], val, grad)
    on_wall = np.unique(m.face_cell[(m.face_cell[:, 1] < 0) & (m.face_tag == tag), 0])
    checked = np.intersect1d(on_wall, cells)
    assert checked.size > 10  # constrained cells are covered
    # the constraint is active: a shift of the constrained components (which
    # an unconstrained fit would follow exactly) changes the wall cells' fits
    W2 = W.copy()
    W2[1] += 0.05
    if tag == ISO:
        W2[4] += 0.05
    coef2, _ = orc.reconstruct(W2, gW)
    for q in ([1, 4] if tag == ISO else [1]):
        assert np.abs(coef2[10 * q + 1:10 * q + 4, checked] - coef[10 * q + 1:10 * q + 4, checked]).max() > 1e-2


@pytest.mark.parametrize("tag", [ADIA, ISO], ids=["adiabatic", "isothermal"])
def test_gas_at_rest_stays_at_rest(oracle_lib, tag):
    Tw = 1.0 / GAMMA
    m = I.with_walls(I.kuhn_cube_mesh(3, 1.0, 0.1, 5, False),
                     {s: tag for s in ("x0", "x1", "y0", "y1", "z0", "z1")})
    orc = oracle_lib.Oracle(m, oracle_lib.make_config(viscous=True, mu=0.01, prandtl=0.72, wall_T=Tw))
    W = np.zeros((5, m.n_cell))
    W[0] = 1.0
    W[4] = 1.0 * Tw / (GAMMA - 1)  # p = rho T_wall
    gW = np.zeros((15, m.n_cell))
    dt = orc.compute_dt(W, 0.5)
    Wo, gWo = W, gW
    for _ in range(3):
        Wo, gWo = orc.step(dt, Wo, gWo)
    assert np.abs(Wo - W).max() < 1e-13
    dr = orc.geometry()[3]
    assert np.abs(gWo).max() < 1e-13 * 3 * np.abs(W).max() / dr.min()
