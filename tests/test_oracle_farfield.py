"""Pins of the oracle's far-field boundary (the Riemann invariants the paper
applies at the outer boundary of its external-flow cases; the locally
one-dimensional characteristic reading):

* an interior state equal to the free stream gives the free stream;
* supersonic outflow gives the interior state, supersonic inflow the free
  stream;
* subsonic: the ghost carries the interior's outgoing invariant
  u_n + 2a/(gamma-1) and the free stream's incoming u_n - 2a/(gamma-1), and
  the entropy p/rho^gamma and tangential velocity of the upwind side;
* a uniform free stream in a box bounded by far-field faces stays uniform.
"""
import numpy as np
import pytest

from paper_2102_01366_amd import inputs as I

GAMMA = 1.4
FAR = I.FACE_FARFIELD


def _cons(rho, U, p):
    U = np.asarray(U, float)
    return np.concatenate([[rho], rho * U, [p / (GAMMA - 1) + 0.5 * rho * U @ U]])


def _prim(W):
    rho = W[0]
    U = W[1:4] / rho
    return rho, U, (GAMMA - 1) * (W[4] - 0.5 * rho * U @ U)


FREE = _cons(1.0, (0.3, 0.0, 0.0), 1.0 / GAMMA)


def _ghost(oracle_lib, n, W):
    cfg = oracle_lib.make_config(farfield=FREE)
    Wg, gWg = oracle_lib.wall_ghost(cfg, FAR, n, np.zeros(3), W, np.ones(15))
    assert np.all(gWg == 0.0)
    return Wg


def _normal(rng):
    n = rng.standard_normal(3)
    return n / np.linalg.norm(n)


def test_free_stream_is_a_fixed_point(oracle_lib):
    rng = np.random.default_rng(1)
    for _ in range(10):
        np.testing.assert_allclose(_ghost(oracle_lib, _normal(rng), FREE), FREE, rtol=1e-14, atol=1e-15)


def test_supersonic_outflow_and_inflow(oracle_lib):
    n = np.array([0.0, 1.0, 0.0])
    W = _cons(0.8, (0.1, 1.6, -0.2), 0.6)  # a = 1.08, u_n = 1.6
    np.testing.assert_array_equal(_ghost(oracle_lib, n, W), W)
    W = _cons(0.8, (0.1, -1.6, -0.2), 0.6)
    np.testing.assert_array_equal(_ghost(oracle_lib, n, W), FREE)


@pytest.mark.parametrize("sign", [1.0, -1.0], ids=["outflow", "inflow"])
def test_subsonic_invariants_entropy_and_tangential_velocity(oracle_lib, sign):
    rng = np.random.default_rng(2)
    for _ in range(6):
        n = _normal(rng)
        rho, p = rng.uniform(0.8, 1.2), rng.uniform(0.6, 0.8)
        U = 0.2 * rng.standard_normal(3)
        U = U - (U @ n) * n + sign * 0.4 * n  # |u_n| = 0.4 < a
        W = _cons(rho, U, p)
        rb, Ub, pb = _prim(_ghost(oracle_lib, n, W))
        ab, ai = np.sqrt(GAMMA * pb / rb), np.sqrt(GAMMA * p / rho)
        rf, Uf, pf = _prim(FREE)
        af = np.sqrt(GAMMA * pf / rf)
        assert abs((Ub @ n + 2 * ab / (GAMMA - 1)) - (U @ n + 2 * ai / (GAMMA - 1))) < 1e-13
        assert abs((Ub @ n - 2 * ab / (GAMMA - 1)) - (Uf @ n - 2 * af / (GAMMA - 1))) < 1e-13
        up = (rho, U, p) if Ub @ n > 0 else (rf, Uf, pf)
        assert abs(pb / rb ** GAMMA - up[2] / up[0] ** GAMMA) < 1e-13
        np.testing.assert_allclose(Ub - (Ub @ n) * n, up[1] - (up[1] @ n) * n, atol=1e-14)


def test_uniform_free_stream_in_a_far_field_box_stays_uniform(oracle_lib):
    m = I.with_walls(I.kuhn_cube_mesh(3, 1.0, 0.1, 7, False),
                     {s: FAR for s in ("x0", "x1", "y0", "y1", "z0", "z1")})
    orc = oracle_lib.Oracle(m, oracle_lib.make_config(farfield=FREE))
    W = np.tile(FREE[:, None], (1, m.n_cell))
    gW = np.zeros((15, m.n_cell))
    dt = orc.compute_dt(W, 0.5)
    Wo, gWo = W, gW
    for _ in range(3):
        Wo, gWo = orc.step(dt, Wo, gWo)
    assert np.abs(Wo - W).max() < 1e-13
