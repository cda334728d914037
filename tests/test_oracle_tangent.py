"""The oracle's tangent build (oracle/or_dual.hpp: gks_oracle.c compiled as
C++ over forward-mode dual numbers), the FP64 reference for the discrete
adjoint, pinned to the plain oracle:

* its values are bitwise those of the plain build (same source, same
  operation order), on periodic meshes, slip and no-slip walls and the far
  field, and with quadratic (curved) wall faces;
* its derivatives are the limit of central differences of the plain build:
  along seeded directions (f(h) - f(-h)) / (2h) approaches them as h^2, in
  configurations where the step map is smooth (no collision-time jump,
  smooth WENO weights eps = 1, no far-field point on a branch switch);
* the kink counter counts nothing at distance zero.
"""
import math

import numpy as np
import pytest

from paper_2102_01366_amd import inputs as I


def _cases():
    ell = 1.0 / (2.0 * math.pi)
    m = I.kuhn_cube_mesh(3, 1.0, 0.1, 0, True)
    W, gW = I.cell_averages(m, I.taylor_green_field(mach=0.3, ell=ell))
    yield "tgv_ns", m, dict(viscous=True, mu=0.01, prandtl=0.72), W, gW
    mw = I.kuhn_cube_mesh(3, 1.0, 0.1, 5, False)
    Ww, gWw = I.cell_averages(mw, I.box_vortex_field())
    yield "slip_walls", mw, dict(), Ww, gWw
    mn = I.with_walls(I.kuhn_cube_mesh(3, 1.0, 0.1, 1, False),
                      {"x0": I.FACE_NOSLIP_ADIABATIC, "y1": I.FACE_NOSLIP_ISOTHERMAL}, {"y1": (0.1, 0.0, 0.0)})
    Wn, gWn = I.cell_averages(mn, I.box_vortex_field())
    yield "noslip", mn, dict(viscous=True, mu=0.01, wall_T=1.0), Wn, gWn
    ms = I.cubed_sphere_shell(2, 2, r_out=3.0, ratio=1.3)
    Ws, gWs = I.cell_averages(ms, I.bump_stream_field(1.4))
    free = I.uniform_state(ms, 1.0, (0.3, 0.0, 0.0), 1.0 / 1.4, 1.4)[0][:, 0]
    yield "farfield", ms, dict(farfield=tuple(free)), Ws, gWs
    mq = I.cubed_sphere_shell(2, 2, r_out=3.0, ratio=1.3, curved=True)
    yield "quadratic_wall", mq, dict(farfield=tuple(free)), Ws, gWs


CASES = list(_cases())


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_tangent_values_are_the_oracle(oracle_lib, case):
    name, m, kw, W, gW = case
    orc = oracle_lib.Oracle(m, oracle_lib.make_config(**kw))
    tor = oracle_lib.TangentOracle(m, oracle_lib.make_config(**kw))
    dW, dG = I.rms_directions(W, gW, tor.ndir, 1)
    dt = orc.compute_dt(W, 0.5)
    Wd, Gd = tor.step(dt, tor.pack(W, dW), tor.pack(gW, dG))
    Wo, gWo = orc.step(dt, W, gW)
    np.testing.assert_array_equal(tor.unpack(Wd)[0], Wo)
    np.testing.assert_array_equal(tor.unpack(Gd)[0], gWo)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_tangent_is_the_limit_of_central_differences(oracle_lib, case):
    name, m, kw, W, gW = case
    kw = dict(kw, c_tau=0.0, eps_weno=1.0)
    if name in ("farfield", "quadratic_wall"):
        # an oblique free stream: no far-field point sits exactly on the
        # switch between the upwind sides of the characteristic state
        U = (0.3, 0.1, 0.05)
        kw["farfield"] = (1.0, *U, 1.0 / 1.4 / 0.4 + 0.5 * sum(u * u for u in U))
    orc = oracle_lib.Oracle(m, oracle_lib.make_config(**kw))
    tor = oracle_lib.TangentOracle(m, oracle_lib.make_config(**kw))
    dW, dG = I.rms_directions(W, gW, tor.ndir, 2)
    dt = orc.compute_dt(W, 0.5)
    Wd, Gd = tor.step(dt, tor.pack(W, dW), tor.pack(gW, dG))
    tW, tG = tor.unpack(Wd)[1], tor.unpack(Gd)[1]

    def fd2(k, h):
        def f(s):
            Wx, Gx = orc.step(dt, W + s * h * dW[k], gW + s * h * dG[k])
            return np.concatenate([Wx.ravel(), Gx.ravel()])
        return (f(1) - f(-1)) / (2.0 * h)

    for k in (0, 7):
        t = np.concatenate([tW[k].ravel(), tG[k].ravel()])
        e = [np.abs(fd2(k, h) - t).max() / np.abs(t).max() for h in (3e-5, 1e-5, 3e-6)]
        # second order: a step three times smaller divides the error by about
        # 9, until rounding (~1e-8 here) takes over
        for a, b in zip(e, e[1:]):
            assert b < 5e-8 or b < a / 5, (name, k, e)
        assert e[-1] < 2e-5, (name, k, e)


def test_kink_counter(oracle_lib):
    name, m, kw, W, gW = CASES[0]
    tor = oracle_lib.TangentOracle(m, oracle_lib.make_config(**kw))
    dW, dG = I.rms_directions(W, gW, tor.ndir, 3)
    tor.set_kink_eps(0.0)
    tor.kinks(reset=True)
    tor.step(1e-3, tor.pack(W, dW), tor.pack(gW, dG))
    assert tor.kinks().sum() == 0
    tor.set_kink_eps(1e300)  # every evaluation with a non-zero derivative is "near" its kink
    tor.step(1e-3, tor.pack(W, dW), tor.pack(gW, dG))
    k = tor.kinks()
    assert (k[0] > 0).all() and (k[1] > 0).all()
    tor.set_kink_eps(0.0)
