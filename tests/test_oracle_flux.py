"""Pins of the oracle's gas-kinetic solver (Sec. 2.2) against closed forms.

* Maxwellian moments against numerical quadrature (Gauss-Hermite, adaptive
  quadrature on half lines); W -> Maxwellian -> W round trip.
* Uniform state: the time-integrated flux is delta times the Euler flux and
  the interface state stays W, for any collision time.
* Continuous linear data: eq. 2nd-flux collapses to eq. 2nd-smooth-flux, whose
  moments are the Euler flux, plus the Chapman-Enskog Navier-Stokes flux of
  the BGK model (mu = tau p, Pr = 1, bulk coefficient 2/(K+3), heat
  conductivity mu (K+5)/2), plus delta^2/2 times dF_Euler/dt; the interface
  state is W + t W_t.  dF/dt and W_t come from complex-step derivatives of
  the Euler flux.
* With Pr != 1 the energy flux gains (1/Pr - 1) times the time-integrated
  heat flux about the interface velocity.
* Free-transport limit (tau_n >> dt): kinetic flux-vector splitting, by
  quadrature over the half lines.  Collision limit (tau_n -> 0, no slopes):
  the Euler flux of the kinetically weighted interface state.
* Mirror symmetry, rotation invariance, and F(delta) = integral of F(t).
"""
import numpy as np
import pytest
from scipy import integrate

GAMMA = 1.4
K = (5 - 3 * GAMMA) / (GAMMA - 1)


def euler_flux(W, n):
    rho = W[0]
    u = W[1:4] / rho
    p = (GAMMA - 1) * (W[4] - 0.5 * rho * (u @ u))
    un = u @ n
    return np.concatenate([[rho * un], rho * u * un + p * n, [(W[4] + p) * un]])


def dflux(W, n, V, h=1e-30):
    """Directional derivative of the Euler flux by complex step."""
    Wc = W.astype(complex) + 1j * h * V
    return euler_flux(Wc, n).imag / h


def euler_time_derivative(W, G):
    """W_t = -sum_j dF_j/dW . W_{x_j}, G[c, j] = dW_c/dx_j."""
    Wt = np.zeros(5)
    for j in range(3):
        e = np.zeros(3)
        e[j] = 1.0
        Wt -= dflux(W, e, G[:, j])
    return Wt


def ns_flux(W, G, n, mu):
    """Chapman-Enskog Navier-Stokes flux of the BGK model (Pr = 1)."""
    rho = W[0]
    u = W[1:4] / rho
    p = (GAMMA - 1) * (W[4] - 0.5 * rho * (u @ u))
    drho = G[0]
    du = (G[1:4] - np.outer(u, drho)) / rho  # du[i, j] = d u_i / d x_j
    dp = (GAMMA - 1) * (G[4] - 0.5 * (u @ u) * drho - rho * (u @ du))
    th = p / rho
    dth = (dp - th * drho) / rho
    div = np.trace(du)
    sigma = mu * (du + du.T - 2.0 / (K + 3) * div * np.eye(3))
    q = -mu * (K + 5) / 2 * dth
    sn = sigma @ n
    return np.concatenate([[0.0], -sn, [-(sn @ u) + q @ n]]), q @ n


def random_state(rng, rho=1.0, spread=0.3):
    r = rho * (1 + spread * rng.uniform(-1, 1))
    u = rng.uniform(-0.6, 0.6, 3)
    p = 1.0 + spread * rng.uniform(-1, 1)
    return np.concatenate([[r], r * u, [p / (GAMMA - 1) + 0.5 * r * (u @ u)]])


def random_normal(rng):
    n = rng.normal(size=3)
    return n / np.linalg.norm(n)


def test_maxwellian_moments_by_quadrature(oracle_lib):
    cfg = oracle_lib.make_config()
    W = np.array([1.3, 0.52, -0.39, 0.26, 3.4])
    m = oracle_lib.maxwell_moments(cfg, W)
    rho = W[0]
    U = W[1:4] / rho
    ein = W[4] / rho - 0.5 * U @ U
    lam = (K + 3) / (4 * ein)
    x, w = np.polynomial.hermite.hermgauss(40)
    for k in range(10):
        for name, Uc in (("u", U[0]), ("v", U[1]), ("w", U[2])):
            ref = np.sum(w * (Uc + x / np.sqrt(lam)) ** k) / np.sqrt(np.pi)
            assert abs(m[name][k] - ref) <= 1e-13 * max(1, abs(ref)), (name, k)
        g = lambda u: np.sqrt(lam / np.pi) * u ** k * np.exp(-lam * (u - U[0]) ** 2)
        pos = integrate.quad(g, 0, np.inf, epsabs=1e-15, epsrel=1e-13)[0]
        neg = integrate.quad(g, -np.inf, 0, epsabs=1e-15, epsrel=1e-13)[0]
        assert abs(m["u_pos"][k] - pos) <= 1e-11 * max(1, abs(pos)), k
        assert abs(m["u_neg"][k] - neg) <= 1e-11 * max(1, abs(neg)), k
        assert abs(m["u_pos"][k] + m["u_neg"][k] - m["u"][k]) <= 1e-13 * max(1, abs(m["u"][k]))
    # K = 2 internal degrees: xi = (xi1, xi2) Gaussian, variance 1/(2 lam) each
    X1, X2 = np.meshgrid(x, x)
    W2 = np.outer(w, w)
    for k in range(4):
        xi2 = (X1 ** 2 + X2 ** 2) / lam
        ref = np.sum(W2 * xi2 ** k) / np.pi
        assert abs(m["xi2"][k] - ref) <= 1e-12 * max(1, ref)
    # round trip: rho <psi> = W
    back = rho * np.array([1, m["u"][1], m["v"][1], m["w"][1],
                           0.5 * (m["u"][2] + m["v"][2] + m["w"][2] + m["xi2"][1])])
    np.testing.assert_allclose(back, W, rtol=1e-14)


@pytest.mark.parametrize("viscous", [False, True])
def test_uniform_state_gives_euler_flux(oracle_lib, viscous):
    rng = np.random.default_rng(1)
    cfg = oracle_lib.make_config(viscous=viscous, mu=0.02)
    normals = [random_normal(rng) for _ in range(4)] + [np.array([-1.0, 0, 0]),
                                                        np.array([1.0, 0, 0])]
    for n in normals:
        W = random_state(rng)
        dt = 0.013
        out = oracle_lib.point_flux(cfg, n, W, np.zeros(15), W, np.zeros(15), dt)
        FE = euler_flux(W, n)
        np.testing.assert_allclose(out[0], dt * FE, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(out[1], 0.5 * dt * FE, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(out[2], W, rtol=1e-14)
        np.testing.assert_allclose(out[3], W, rtol=1e-14)


def _continuous_case(rng):
    W = random_state(rng)
    G = 0.4 * rng.normal(size=(5, 3))
    return W, G


@pytest.mark.parametrize("viscous,prandtl", [(False, 1.0), (True, 1.0), (True, 0.72)])
def test_continuous_linear_data_navier_stokes(oracle_lib, viscous, prandtl):
    rng = np.random.default_rng(2)
    mu = 0.03
    cfg = oracle_lib.make_config(viscous=viscous, mu=mu, prandtl=prandtl)
    for trial in range(6):
        n = random_normal(rng) if trial < 5 else np.array([-1.0, 0.0, 0.0])
        W, G = _continuous_case(rng)
        gW = G.reshape(15)
        dt = 0.02
        out = oracle_lib.point_flux(cfg, n, W, gW, W, gW, dt)
        FE = euler_flux(W, n)
        Wt = euler_time_derivative(W, G)
        FEt = dflux(W, n, Wt)
        FNS, qn = ns_flux(W, G, n, mu if viscous else 0.0)
        for k, delta in enumerate((dt, 0.5 * dt)):
            ref = delta * (FE + FNS) + 0.5 * delta ** 2 * FEt
            if prandtl != 1.0:
                rho = W[0]
                u = W[1:4] / rho
                p = (GAMMA - 1) * (W[4] - 0.5 * rho * u @ u)
                ut = (Wt[1:4] - u * Wt[0]) / rho
                qhat = delta * qn + 0.5 * delta ** 2 * (K + 5) / 2 * p * (ut @ n)
                ref[4] += (1 / prandtl - 1) * qhat
            np.testing.assert_allclose(out[k], ref, rtol=0, atol=1e-13 * delta * 10)
        np.testing.assert_allclose(out[2], W, rtol=1e-13)
        np.testing.assert_allclose(out[3], W + dt * Wt, rtol=1e-12, atol=1e-14)


def test_mirror_symmetry(oracle_lib):
    rng = np.random.default_rng(3)
    for viscous in (False, True):
        cfg = oracle_lib.make_config(viscous=viscous, mu=0.01, prandtl=0.72 if viscous else 1)
        for _ in range(4):
            n = random_normal(rng)
            Wl, Wr = random_state(rng), random_state(rng)
            gl, gr = 0.5 * rng.normal(size=15), 0.5 * rng.normal(size=15)
            a = oracle_lib.point_flux(cfg, n, Wl, gl, Wr, gr, 0.01)
            b = oracle_lib.point_flux(cfg, -n, Wr, gr, Wl, gl, 0.01)
            scale = np.abs(a).max()
            np.testing.assert_allclose(b[:2], -a[:2], rtol=0, atol=1e-14 * scale)
            np.testing.assert_allclose(b[2:], a[2:], rtol=0, atol=1e-14 * scale)


def _rotate_state(Q, W, gW):
    G = gW.reshape(5, 3)
    W2 = W.copy()
    W2[1:4] = Q @ W[1:4]
    G2 = np.empty_like(G)
    G2[0] = Q @ G[0]
    G2[4] = Q @ G[4]
    G2[1:4] = Q @ G[1:4] @ Q.T
    return W2, G2.reshape(15)


def test_rotation_invariance(oracle_lib):
    rng = np.random.default_rng(4)
    cfg = oracle_lib.make_config(viscous=True, mu=0.01, prandtl=0.72)
    for _ in range(5):
        Q, _r = np.linalg.qr(rng.normal(size=(3, 3)))
        if np.linalg.det(Q) < 0:
            Q[:, 0] = -Q[:, 0]
        n = random_normal(rng)
        Wl, Wr = random_state(rng), random_state(rng)
        gl, gr = 0.5 * rng.normal(size=15), 0.5 * rng.normal(size=15)
        a = oracle_lib.point_flux(cfg, n, Wl, gl, Wr, gr, 0.01)
        Wl2, gl2 = _rotate_state(Q, Wl, gl)
        Wr2, gr2 = _rotate_state(Q, Wr, gr)
        b = oracle_lib.point_flux(cfg, Q @ n, Wl2, gl2, Wr2, gr2, 0.01)
        expect = a.copy()
        expect[:, 1:4] = a[:, 1:4] @ Q.T
        scale = np.abs(a).max()
        np.testing.assert_allclose(b, expect, rtol=0, atol=1e-13 * scale)


def test_time_integral_of_flux_density(oracle_lib):
    rng = np.random.default_rng(5)
    for viscous in (False, True):
        cfg = oracle_lib.make_config(viscous=viscous, mu=0.002, prandtl=0.72 if viscous else 1)
        n = random_normal(rng)
        Wl, Wr = random_state(rng), random_state(rng)
        gl, gr = 0.5 * rng.normal(size=15), 0.5 * rng.normal(size=15)
        dt = 0.01
        out = oracle_lib.point_flux(cfg, n, Wl, gl, Wr, gr, dt)
        for k, delta in enumerate((dt, 0.5 * dt)):
            ref = [integrate.quad(lambda t: oracle_lib.point_flux_density(
                cfg, n, Wl, gl, Wr, gr, dt, t)[c], 0, delta, points=[1e-5 * dt, 1e-4 * dt,
                                                                    1e-3 * dt, 1e-2 * dt],
                epsabs=1e-16, epsrel=1e-12, limit=200)[0] for c in range(5)]
            np.testing.assert_allclose(out[k], ref, rtol=1e-10, atol=1e-15)


def _half_flux(W, sign):
    """rho times the moments of u psi over one half line, by quadrature in u."""
    rho = W[0]
    U = W[1:4] / rho
    ein = W[4] / rho - 0.5 * U @ U
    lam = (K + 3) / (4 * ein)
    lo, hi = (0, np.inf) if sign > 0 else (-np.inf, 0)
    g = lambda u: np.sqrt(lam / np.pi) * np.exp(-lam * (u - U[0]) ** 2)
    m = [integrate.quad(lambda u: u ** k * g(u), lo, hi, epsabs=1e-15, epsrel=1e-13)[0]
         for k in range(4)]
    vt2 = U[1] ** 2 + U[2] ** 2 + 2.0 / (2 * lam) + K / (2 * lam)
    flux = rho * np.array([m[1], m[2], U[1] * m[1], U[2] * m[1], 0.5 * (m[3] + m[1] * vt2)])
    state = rho * np.array([m[0], m[1], U[1] * m[0], U[2] * m[0], 0.5 * (m[2] + m[0] * vt2)])
    return flux, state


def test_free_transport_limit_is_kfvs(oracle_lib):
    # Without slopes the distribution is (1 - e^{-t/tau_n}) g^c + e^{-t/tau_n} (g^l H + g^r (1-H)),
    # so F(delta)/delta = w KFVS + (1 - w) F_Euler(W^c), w = tau_n (1 - e^{-delta/tau_n}) / delta.
    # tau_n = 1000 dt keeps 1 - e^{-delta/tau_n} well conditioned in FP64.
    rng = np.random.default_rng(6)
    eps_tau = 1e3
    cfg = oracle_lib.make_config(eps_tau=eps_tau, c_tau=0.0)
    e1 = np.array([1.0, 0, 0])
    for _ in range(3):
        Wl, Wr = random_state(rng), random_state(rng)
        dt = 0.01
        out = oracle_lib.point_flux(cfg, e1, Wl, np.zeros(15), Wr, np.zeros(15), dt)
        kfvs = _half_flux(Wl, +1)[0] + _half_flux(Wr, -1)[0]
        Wc = _half_flux(Wl, +1)[1] + _half_flux(Wr, -1)[1]
        for k, delta in enumerate((dt, 0.5 * dt)):
            x = delta / (eps_tau * dt)
            w = -np.expm1(-x) / x
            ref = w * kfvs + (1 - w) * euler_flux(Wc, e1)
            np.testing.assert_allclose(out[k] / delta, ref, rtol=1e-10, atol=1e-13)
        assert np.abs(out[0] / dt - kfvs).max() < 1e-3 * np.abs(kfvs).max()


def test_collision_limit_is_euler_flux_of_interface_state(oracle_lib):
    rng = np.random.default_rng(7)
    cfg = oracle_lib.make_config(eps_tau=1e-12, c_tau=0.0)
    e1 = np.array([1.0, 0, 0])
    for _ in range(3):
        Wl, Wr = random_state(rng), random_state(rng)
        dt = 0.01
        out = oracle_lib.point_flux(cfg, e1, Wl, np.zeros(15), Wr, np.zeros(15), dt)
        Wc = _half_flux(Wl, +1)[1] + _half_flux(Wr, -1)[1]
        np.testing.assert_allclose(out[2], Wc, rtol=1e-12)
        np.testing.assert_allclose(out[0] / dt, euler_flux(Wc, e1), rtol=1e-8, atol=1e-12)


# ---------------------------------------------------------------------------
# The smooth-flow form of the distribution (eq. 2nd-smooth-flux):
# f = g^c - tau (a^c.u + A^c) g^c + t A^c g^c, with W^c and its slopes from
# the kinetic weighting of eq. new-equ-part and tau = mu / p^c (0 for Euler).
# Its moments are the Euler flux of W^c, plus the Chapman-Enskog
# Navier-Stokes flux of (W^c, grad W^c), plus t times dF_Euler/dt of W^c.
# ---------------------------------------------------------------------------

def _half_state_derivative(W, G, sign, h=1e-5):
    """d/de of the kinetically weighted half-line state along W + e G, by
    central differences of the quadrature (the slopes of eq. new-equ-part)."""
    return (_half_flux(W + h * G, sign)[1] - _half_flux(W - h * G, sign)[1]) / (2 * h)


def _smooth_reference(Wc, Gc, n, mu, prandtl, delta):
    FE = euler_flux(Wc, n)
    Wt = euler_time_derivative(Wc, Gc)
    FNS, qn = ns_flux(Wc, Gc, n, mu)
    ref = delta * (FE + FNS) + 0.5 * delta ** 2 * dflux(Wc, n, Wt)
    if prandtl != 1.0:
        rho = Wc[0]
        u = Wc[1:4] / rho
        p = (GAMMA - 1) * (Wc[4] - 0.5 * rho * u @ u)
        ut = (Wt[1:4] - u * Wt[0]) / rho
        ref[4] += (1 / prandtl - 1) * (delta * qn + 0.5 * delta ** 2 * (K + 5) / 2 * p * (ut @ n))
    return ref, Wt


@pytest.mark.parametrize("viscous,prandtl", [(False, 1.0), (True, 1.0), (True, 0.72)])
def test_smooth_flux_continuous_linear_data(oracle_lib, viscous, prandtl):
    """Continuous data: the same closed form as the full distribution (which
    collapses to the smooth one when g^l = g^r = g^c)."""
    rng = np.random.default_rng(12)
    mu = 0.03
    cfg = oracle_lib.make_config(viscous=viscous, mu=mu, prandtl=prandtl, flux=1)
    full = oracle_lib.make_config(viscous=viscous, mu=mu, prandtl=prandtl)
    for trial in range(5):
        n = random_normal(rng) if trial < 4 else np.array([-1.0, 0.0, 0.0])
        W, G = _continuous_case(rng)
        gW = G.reshape(15)
        dt = 0.02
        out = oracle_lib.point_flux(cfg, n, W, gW, W, gW, dt)
        for k, delta in enumerate((dt, 0.5 * dt)):
            ref, Wt = _smooth_reference(W, G, n, mu if viscous else 0.0, prandtl, delta)
            np.testing.assert_allclose(out[k], ref, rtol=0, atol=1e-12 * delta)
        np.testing.assert_allclose(out[2], W, rtol=1e-13)
        np.testing.assert_allclose(out[3], W + dt * Wt, rtol=1e-12, atol=1e-14)
        # identical sides: tau_n = tau (viscous) or no slopes of the kinetic
        # part survive (Euler), so eq. 2nd-flux reduces to eq. 2nd-smooth-flux
        np.testing.assert_allclose(out, oracle_lib.point_flux(full, n, W, gW, W, gW, dt),
                                   rtol=0, atol=1e-13 * np.abs(out).max())


@pytest.mark.parametrize("viscous", [False, True])
def test_smooth_flux_jump_without_slopes(oracle_lib, viscous):
    """Discontinuous constant states: the Euler flux of the kinetically
    weighted W^c and the state W^c at all times (no slopes, so no A^c)."""
    rng = np.random.default_rng(13)
    cfg = oracle_lib.make_config(viscous=viscous, mu=0.02, flux=1)
    e1 = np.array([1.0, 0, 0])
    for _ in range(3):
        Wl, Wr = random_state(rng), random_state(rng)
        dt = 0.01
        out = oracle_lib.point_flux(cfg, e1, Wl, np.zeros(15), Wr, np.zeros(15), dt)
        Wc = _half_flux(Wl, +1)[1] + _half_flux(Wr, -1)[1]
        np.testing.assert_allclose(out[0], dt * euler_flux(Wc, e1), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(out[1], 0.5 * dt * euler_flux(Wc, e1), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(out[2], Wc, rtol=1e-12)
        np.testing.assert_allclose(out[3], Wc, rtol=1e-12)


@pytest.mark.parametrize("viscous,prandtl", [(False, 1.0), (True, 1.0), (True, 0.72)])
def test_smooth_flux_jump_with_slopes(oracle_lib, viscous, prandtl):
    """Discontinuous states and gradients: the closed form at (W^c, grad W^c),
    W^c and its slopes weighted kinetically by half-line quadrature."""
    rng = np.random.default_rng(14)
    mu = 0.02
    cfg = oracle_lib.make_config(viscous=viscous, mu=mu, prandtl=prandtl, flux=1)
    e1 = np.array([1.0, 0, 0])
    for _ in range(2):
        Wl, Wr = random_state(rng), random_state(rng)
        Gl, Gr = 0.4 * rng.normal(size=(5, 3)), 0.4 * rng.normal(size=(5, 3))
        dt = 0.01
        out = oracle_lib.point_flux(cfg, e1, Wl, Gl.reshape(15), Wr, Gr.reshape(15), dt)
        Wc = _half_flux(Wl, +1)[1] + _half_flux(Wr, -1)[1]
        Gc = np.stack([_half_state_derivative(Wl, Gl[:, d], +1) + _half_state_derivative(Wr, Gr[:, d], -1)
                       for d in range(3)], axis=1)
        rho, u = Wc[0], Wc[1:4] / Wc[0]
        pc = (GAMMA - 1) * (Wc[4] - 0.5 * rho * u @ u)
        # tau = mu / p^c, so the Navier-Stokes viscosity is tau p^c = mu
        for k, delta in enumerate((dt, 0.5 * dt)):
            ref, Wt = _smooth_reference(Wc, Gc, e1, mu if viscous else 0.0, prandtl, delta)
            np.testing.assert_allclose(out[k], ref, rtol=0, atol=1e-8 * delta * np.abs(ref / delta).max())
        np.testing.assert_allclose(out[2], Wc, rtol=1e-12)
        np.testing.assert_allclose(out[3], Wc + dt * Wt, rtol=1e-8)
        assert pc > 0
