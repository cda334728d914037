"""The oracle's second-order scheme (eq. final_weno_expression-2nd).

R = w11 p1 + w01 p0 with the step-1 polynomial P^1, P^0 and the two-step
indicator; sigma = |beta1 - beta0|^(4/3); linear weights 10:1.  Pins:
linear data are reproduced exactly (all indicators agree, sigma = 0, the
weights are linear, R = P^1); second-order convergence on the smooth sine
wave.  The magnitudes of the paper's Table 3 are not reproduced: like the
third-order WENO results of Table 2, the paper's errors are larger than ours
(at N = 5: 2.7e-2 printed, 2.0e-2 here) while the linear scheme's Table 1 is
reproduced; the paper does not state its weights fully, so the WENO
magnitudes are parity unpinned and only the order is pinned.
"""
import numpy as np

import oracle
from paper_2102_01366_amd import inputs as I


def test_order2_reproduces_linear_data():
    """On a box with walls (a periodic mesh cannot carry a linear field)."""
    rng = np.random.default_rng(2)
    a = np.array([1.3, 0.1, -0.2, 0.15, 4.0])
    b = 0.3 * rng.standard_normal((5, 3))
    m = I.kuhn_cube_mesh(4, 1.0, 0.1, 3, False)

    def f(X):
        Q = a[:, None, None] + np.einsum("qd,cpd->qcp", b, X)
        dQ = np.broadcast_to(b[:, :, None, None], (5, 3) + X.shape[:2]).copy()
        return Q, dQ
    W, gW = I.cell_averages(m, f)
    orc = oracle.Oracle(m, oracle.make_config(order=2))
    coef, flag = orc.reconstruct(W, gW)
    assert not flag.any()
    for q in range(5):
        assert np.abs(coef[10 * q] - W[q]).max() <= 1e-13 * np.abs(W).max()
        assert np.abs(coef[10 * q + 1:10 * q + 4] - b[q][:, None]).max() <= 1e-11
        assert np.abs(coef[10 * q + 4:10 * q + 10]).max() == 0.0


def _sine_error(n, order, t_end=0.1):
    m = I.kuhn_cube_mesh(n, 1.0, 0.1, 5, True)
    orc = oracle.Oracle(m, oracle.make_config(order=order))
    W, gW = I.cell_averages(m, I.sine_wave_field())
    t = 0.0
    while t < t_end - 1e-14:
        dt = min(orc.compute_dt(W, 0.5), t_end - t)
        W, gW = orc.step(dt, W, gW)
        t += dt
    We, _ = I.cell_averages(m, I.sine_wave_field(t=t_end))
    vol = orc.geometry()[0]
    return np.sum(vol * np.abs(W[0] - We[0])) / vol.sum()


def test_order2_converges_at_second_order():
    """On the coarse pair N = 4, 8 (jittered, t = 0.1) the rate is still
    pre-asymptotic: 1.75 with WENO or linear weights, while the third-order
    scheme reaches 2.1 on the same pair (the paper's Table 3 shows 1.55-1.96
    between its finer meshes).  Pinned: a rate above 1.6, and the third-order
    scheme more accurate on the finer mesh."""
    e4, e8 = _sine_error(4, 2), _sine_error(8, 2)
    order = np.log2(e4 / e8)
    assert order > 1.6, (e4, e8, order)
    assert _sine_error(8, 3) < 0.8 * e8
