"""Pins of the oracle's cell update and time stepping (Secs. 2.1, 2.3, 3, 5).

* Free-stream preservation on a jittered periodic mesh: a uniform state stays
  uniform and its averaged gradient stays zero (closed cell surfaces).
* Exact discrete conservation of mass, momentum and energy on a periodic
  mesh (each face flux enters its two cells with opposite signs).
* The time step of eq. time-step against closed-form tetrahedron geometry.
* Stage sequencing of the two-stage fourth-order step.
* The same with the smooth-flow flux of eq. 2nd-smooth-flux where it applies
  (free stream, conservation, convergence).
* Third-order convergence of the density on the smooth sine-wave advection
  against exact cell averages of the translated profile (the paper's Tables
  1-2 show order ~3; magnitudes depend on the mesh and are not compared).
"""
import numpy as np
import pytest

from paper_2102_01366_amd import inputs as I


def _uniform(mesh, rho=1.2, u=(0.3, -0.2, 0.5), p=0.9, gamma=1.4):
    u = np.asarray(u)
    W = np.empty((5, mesh.n_cell))
    W[0] = rho
    W[1:4] = rho * u[:, None]
    W[4] = p / (gamma - 1) + 0.5 * rho * u @ u
    return W, np.zeros((15, mesh.n_cell))


@pytest.mark.parametrize("viscous,flux", [(False, 0), (True, 0), (True, 1)])
def test_free_stream_preservation(oracle_lib, viscous, flux):
    m = I.kuhn_cube_mesh(4, 1.0, 0.15, 21, True)
    orc = oracle_lib.Oracle(m, oracle_lib.make_config(viscous=viscous, mu=0.01, flux=flux,
                                                      prandtl=0.72 if viscous else 1))
    W0, gW0 = _uniform(m)
    W, gW = W0, gW0
    dt = orc.compute_dt(W, 0.5)
    for _ in range(4):
        W, gW = orc.step(dt, W, gW)
    assert np.abs(W - W0).max() < 1e-13
    # the Gauss sums cancel terms of size |W| sum|Gamma| / |Omega| = 3 |W| / dr
    dr = orc.geometry()[3]
    scale = np.abs(W0).max() * 3.0 / dr.min()
    assert np.abs(gW).max() < 1e-13 * scale


@pytest.mark.parametrize("flux", [0, 1])
def test_exact_conservation(oracle_lib, flux):
    m = I.kuhn_cube_mesh(4, 2 * np.pi, 0.1, 22, True)
    orc = oracle_lib.Oracle(m, oracle_lib.make_config(viscous=True, mu=0.05, prandtl=0.72, flux=flux))
    W, gW = I.cell_averages(m, I.taylor_green_field(mach=0.3))
    rng = np.random.default_rng(0)
    W = W * (1 + 0.02 * rng.standard_normal(W.shape))
    s0 = orc.conservation_sums(W)
    dt = orc.compute_dt(W, 0.5)
    for _ in range(3):
        W, gW = orc.step(dt, W, gW)
    s1 = orc.conservation_sums(W)
    scale = np.abs(s0).max()
    assert np.abs(s1 - s0).max() < 1e-13 * scale


def test_time_step_formula(oracle_lib):
    m = I.kuhn_cube_mesh(3, 1.0, 0.1, 23, True)
    mu = 0.3
    W, gW = I.cell_averages(m, I.taylor_green_field(mach=0.5))
    v = m.xyz[m.tet]
    vol = np.abs(np.linalg.det(v[:, 1:] - v[:, :1])) / 6
    faces = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    area = 0.5 * np.linalg.norm(np.cross(v[:, faces[:, 1]] - v[:, faces[:, 0]],
                                         v[:, faces[:, 2]] - v[:, faces[:, 0]]), axis=-1).sum(1)
    dr = 3 * vol / area
    rho, u, p = I.conservative_to_primitive(W, 1.4)
    a = np.sqrt(1.4 * p / rho)
    conv = dr / (np.linalg.norm(u, axis=0) + a)
    for viscous in (False, True):
        orc = oracle_lib.Oracle(m, oracle_lib.make_config(viscous=viscous, mu=mu))
        ref = conv.min() if not viscous else min(conv.min(), (dr ** 2 / (3 * mu / rho)).min())
        assert abs(orc.compute_dt(W, 0.7) - 0.7 * ref) < 1e-15 * ref
    # the viscous bound must have been the active one for mu = 0.3
    assert (dr ** 2 / (3 * mu / rho)).min() < conv.min()


def test_stage_sequence(oracle_lib):
    m = I.kuhn_cube_mesh(3, 1.0, 0.1, 24, True)
    orc = oracle_lib.Oracle(m, oracle_lib.make_config())
    W, gW = I.cell_averages(m, I.sine_wave_field())
    dt = orc.compute_dt(W, 0.5)
    with pytest.raises(RuntimeError):
        orc.stage(2, dt, W, gW)
    Ws, gWs = orc.stage(1, dt, W, gW)
    W2, gW2 = orc.stage(2, dt, Ws, gWs)
    W3, gW3 = orc.step(dt, W, gW)
    np.testing.assert_array_equal(W2, W3)
    np.testing.assert_array_equal(gW2, gW3)


@pytest.mark.parametrize("nonlinear,flux", [(False, 0), (True, 0), (True, 1)],
                         ids=["linear", "weno", "weno_smooth_flux"])
def test_third_order_convergence(oracle_lib, nonlinear, flux):
    cfg = oracle_lib.make_config(nonlinear=nonlinear, flux=flux)
    T = 0.02
    errs, gerrs = [], []
    for N in (4, 8, 16):
        m = I.kuhn_cube_mesh(N, 1.0, 0.1, 0, True)
        orc = oracle_lib.Oracle(m, cfg)
        W, gW = I.cell_averages(m, I.sine_wave_field())
        vol = orc.geometry()[0]
        ns = int(np.ceil(T / orc.compute_dt(W, 0.5)))
        dt = T / ns
        for _ in range(ns):
            W, gW = orc.step(dt, W, gW)
        We, gWe = I.cell_averages(m, I.sine_wave_field(t=T))
        errs.append(np.sum(vol * np.abs(W[0] - We[0])) / vol.sum())
        gerrs.append(np.sum(vol * np.abs(gW[:3] - gWe[:3])) / vol.sum())
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert order[-1] > 2.6, (errs, order)
    assert order[0] > 2.0, (errs, order)
    # the Gauss-theorem gradients of O(h^3) interface values converge at order ~2
    gorder = np.log2(np.array(gerrs[:-1]) / np.array(gerrs[1:]))
    assert gorder[-1] > 1.7, (gerrs, gorder)
