"""Flow past a sphere on a cubed-sphere shell (slip wall on r = 1, far field
by Riemann invariants on the outer sphere), GPU against the oracle to the
normwise 1e-12 bar of test_gpu_parity.py.

Mesh: 6 panels of 4 x 4 cells, 4 radial layers out to r = 3 (ratio 1.3),
each hexahedron split into 6 tetrahedra by the minimum-vertex-id rule (2,304
cells, straight faces).  Field: the free stream rho = 1, U = (0.3, 0, 0),
p = 1/gamma with a smooth density and pressure bump near (2, 0, 0), so that
reconstruction, wall ghost and far-field state are all exercised.  The
discrete adjoint of a step is checked against central differences.
"""
import numpy as np
import pytest

import oracle
import paper_2102_01366_amd as G
from paper_2102_01366_amd import inputs as I

from test_gpu_parity import COEF_GROUPS, GW_GROUPS, W_GROUPS, assert_parity, check_face_terms, check_steps

pytestmark = pytest.mark.gpu

GAMMA = 1.4
FREE = np.array([1.0, 0.3, 0.0, 0.0, (1.0 / GAMMA) / (GAMMA - 1) + 0.5 * 0.09])


def _bump_field():
    return I.bump_stream_field(GAMMA)


def _case(viscous=False):
    m = I.cubed_sphere_shell(4, 4, r_out=3.0, ratio=1.3)
    W, gW = I.cell_averages(m, _bump_field())
    kw = dict(farfield=tuple(FREE))
    if viscous:
        kw.update(viscous=True, mu=0.01, prandtl=0.72)
    return m, kw, W, gW


@pytest.fixture(params=[False, True], ids=["euler", "navier_stokes"])
def pair(request):
    m, kw, W, gW = _case(request.param)
    return m, G.Solver(m, G.default_config(**kw)), oracle.Oracle(m, oracle.make_config(**kw)), W, gW


def test_sphere_reconstruction(pair):
    m, s, orc, W, gW = pair
    s.init(W, gW)
    b, coef, flag = s.debug_reconstruct()
    co, fo = orc.reconstruct(W, gW)
    assert_parity(b, orc.slopes(W, gW), GW_GROUPS, "slopes")
    assert_parity(coef, co, COEF_GROUPS, "coef")
    np.testing.assert_array_equal(flag, fo)


def test_sphere_face_terms(pair):
    m, s, orc, W, gW = pair
    s.init(W, gW)
    check_face_terms(s, orc, W, gW, orc.compute_dt(W, 0.5))


def test_sphere_steps(pair):
    m, s, orc, W, gW = pair
    check_steps(m, s, orc, W, gW, check_dt=False)


def test_sphere_fp32_bulk_close_to_fp64():
    m, kw, W, gW = _case()
    res = []
    for prec in (G.GKS_FP64, G.GKS_FP32_BULK):
        s = G.Solver(m, G.default_config(precision=prec, **kw))
        s.init(W, gW)
        for _ in range(3):
            s.step(0.02)
        res.append(s.read_state()[0])
    for g in W_GROUPS:
        assert np.abs(res[1][g] - res[0][g]).max() <= 1e-5 * np.abs(res[0][g]).max()


@pytest.mark.parametrize("viscous,extra,eps,tol", [
    (False, dict(c_tau=0.0, eps_weno=1.0), 1e-6, 1e-6),
    (True, dict(c_tau=0.0, nonlinear=False), 1e-6, 1e-6),
    (False, dict(c_tau=0.0), 1e-8, 1e-4),
], ids=["euler_smooth_weights", "ns_linear", "euler_weno"])
def test_sphere_adjoint_matches_finite_differences(viscous, extra, eps, tol):
    """<J v, w> by central differences of one step against <v, J^T w> by the
    adjoint, through the slip wall and the far-field state (subsonic here)."""
    torch = pytest.importorskip("torch")
    m, kw, W, gW = _case(viscous)
    s = G.Solver(m, G.default_config(**dict(kw, **extra)))
    Wt, Gt = torch.from_numpy(W).cuda(), torch.from_numpy(gW).cuda()
    s.init(Wt, Gt)
    dt = s.compute_dt(0.5)

    def F(Wx, Gx):
        s.init(Wx, Gx)
        s.step(dt)
        return s.read_state(device=True)

    gen = torch.Generator().manual_seed(41)
    sW = torch.from_numpy(np.sqrt((W ** 2).mean(axis=1, keepdims=True))).cuda()
    sG = torch.from_numpy(np.sqrt((gW ** 2).mean(axis=1, keepdims=True)) + 1e-3).cuda()
    for _ in range(3):
        vW = torch.randn(W.shape, generator=gen, dtype=torch.float64).cuda() * sW
        vG = torch.randn(gW.shape, generator=gen, dtype=torch.float64).cuda() * sG
        bW = torch.randn(W.shape, generator=gen, dtype=torch.float64).cuda()
        bG = torch.randn(gW.shape, generator=gen, dtype=torch.float64).cuda()
        Wp, Gp = F(Wt + eps * vW, Gt + eps * vG)
        Wm, Gm = F(Wt - eps * vW, Gt - eps * vG)
        lhs = (((Wp - Wm) * bW).sum() + ((Gp - Gm) * bG).sum()).item() / (2 * eps)
        aW, aG = s.step_adjoint(dt, Wt, Gt, bW, bG)
        rhs = ((aW * vW).sum() + (aG * vG).sum()).item()
        assert abs(lhs - rhs) <= tol * abs(rhs), (lhs, rhs)
