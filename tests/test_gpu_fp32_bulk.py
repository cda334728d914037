"""The FP32-bulk precision form against the FP64 oracle.

Reconstruction and flux arithmetic, the per-stage bulk arrays and the
least-squares operators (formed in FP64 and rounded once) are FP32; the
state, its accumulation, the Gauss-sum normals, the time step and the
conservation sums stay FP64.  The differences Q_m - Q_0 are formed in FP64
before rounding, and the face frame avoids the cancellation in 1 + n1.

Tolerances follow from the FP32 unit roundoff u = 6e-8: reconstruction and
face values within ~30-80 u of their group scale; the time derivative of
the flux, 4 (F(dt) - 2 F(dt/2)) / dt^2, cancels O(|F| / (dt |dF/dt|)) and
is held to 5e-3; the state after 10 steps within 2e-5 (groupwise) and the
density L1 difference within 1e-6 of the mean density; conservation stays
exact because every FP32 face term enters its two cells, widened to FP64,
with opposite signs.
"""
import numpy as np
import pytest

import oracle
import paper_2102_01366_amd as G
from paper_2102_01366_amd import inputs as I

pytestmark = pytest.mark.gpu

MU = 1.0 / 1600.0
W_GROUPS = [[0], [1, 2, 3], [4]]
GW_GROUPS = [[0, 1, 2], list(range(3, 12)), [12, 13, 14]]
C0_GROUPS = [[0], [10, 20, 30], [40]]
CD_GROUPS = [list(range(1, 10)), [r for q in (1, 2, 3) for r in range(10 * q + 1, 10 * q + 10)],
             list(range(41, 50))]


def groups_err(a, b, groups, floors=None):
    out = []
    for i, g in enumerate(groups):
        scale = np.abs(b[g]).max()
        if floors is not None:
            scale = max(scale, floors[i])
        out.append(np.abs(a[g] - b[g]).max() / scale)
    return max(out)


@pytest.fixture(scope="module", params=[(5, 0.3), (8, 0.1)], ids=["n5_ma0.3", "n8_ma0.1"])
def case(request):
    n, mach = request.param
    m = I.kuhn_cube_mesh(n, 2 * np.pi, 0.05, 1, True)
    W, gW = I.cell_averages(m, I.taylor_green_field(mach=mach))
    kw = dict(viscous=True, mu=MU, prandtl=0.72)
    s32 = G.Solver(m, G.default_config(precision=G.GKS_FP32_BULK, **kw))
    orc = oracle.Oracle(m, oracle.make_config(**kw))
    return m, s32, orc, W, gW


def test_fp32_reconstruction(case):
    m, s, orc, W, gW = case
    s.init(W, gW)
    b, coef, flag = s.debug_reconstruct()
    co, fo = orc.reconstruct(W, gW)
    np.testing.assert_array_equal(flag, fo)
    assert groups_err(b, orc.slopes(W), GW_GROUPS) < 2e-6
    assert groups_err(coef, co, C0_GROUPS) < 2e-6
    assert groups_err(coef, co, CD_GROUPS) < 2e-6


def test_fp32_face_terms(case):
    m, s, orc, W, gW = case
    s.init(W, gW)
    dt = orc.compute_dt(W, 0.5)
    ft = s.debug_face_terms(dt)
    fo = orc.face_terms(W, gW, dt)
    for blk in (0, 2, 3):  # F, W(0), W(dt)
        assert groups_err(ft[5 * blk:5 * blk + 5], fo[5 * blk:5 * blk + 5], W_GROUPS) < 5e-6, blk
    assert groups_err(ft[5:10], fo[5:10], W_GROUPS) < 5e-3


def test_fp32_steps(case):
    m, s, orc, W, gW = case
    s.init(W, gW)
    s0 = s.conservation_sums()
    Wo, gWo = W, gW
    for _ in range(10):
        dt = orc.compute_dt(Wo, 0.5)
        s.step(dt)
        Wo, gWo = orc.step(dt, Wo, gWo)
    Wg, gWg = s.read_state()
    vol, _, _, dr = orc.geometry()
    l1 = np.sum(vol * np.abs(Wg[0] - Wo[0])) / np.sum(vol * Wo[0])
    assert l1 < 1e-6, l1
    assert groups_err(Wg, Wo, W_GROUPS) < 2e-5
    floors = [np.abs(Wo[g]).max() / dr.min() for g in W_GROUPS]
    assert groups_err(gWg, gWo, GW_GROUPS, floors) < 1e-5
    s1 = s.conservation_sums()
    assert np.abs(s1 - s0).max() <= 1e-14 * np.abs(s0).max()


def test_fp32_free_stream():
    m = I.kuhn_cube_mesh(5, 1.0, 0.15, 3, True)
    s = G.Solver(m, G.default_config(precision=G.GKS_FP32_BULK))
    W = np.empty((5, m.n_cell))
    W[0], W[1], W[2], W[3] = 1.1, 0.3, -0.2, 0.4
    W[4] = 1.0 / 0.4 + 0.5 * (0.3 ** 2 + 0.2 ** 2 + 0.4 ** 2) / 1.1
    s.init(W, np.zeros((15, m.n_cell)))
    dt = s.compute_dt(0.5)
    for _ in range(5):
        s.step(dt)
    Wg, gWg = s.read_state()
    assert np.abs(Wg - W).max() < 1e-5 * np.abs(W).max()
