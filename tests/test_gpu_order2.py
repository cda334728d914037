"""The second-order scheme (eq. final_weno_expression-2nd) on the GPU against
the oracle, to the normwise 1e-12 bar of test_gpu_parity.py, periodic and
with slip walls, and its adjoint against finite differences."""
import numpy as np
import pytest

import oracle
import paper_2102_01366_amd as G
from paper_2102_01366_amd import inputs as I

from test_gpu_parity import COEF_GROUPS, MU_TGV, assert_parity, check_face_terms, check_steps

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "sine_periodic":
        m = I.kuhn_cube_mesh(5, 1.0, 0.1, 3, True)
        W, gW = I.cell_averages(m, I.sine_wave_field())
        return m, dict(order=2), W, gW
    if name == "tgv_viscous":
        m = I.kuhn_cube_mesh(4, 2 * np.pi, 0.05, 1, True)
        W, gW = I.cell_averages(m, I.taylor_green_field(mach=0.3))
        return m, dict(order=2, viscous=True, mu=MU_TGV, prandtl=0.72), W, gW
    if name == "blast_walls":
        m = I.kuhn_cube_mesh(6, 1.0, 0.1, 4, False)
        W, gW = I.blast_cell_averages(m, radius=0.2)
        return m, dict(order=2), W, gW
    raise KeyError(name)


CASES = ["sine_periodic", "tgv_viscous", "blast_walls"]


@pytest.mark.parametrize("name", CASES)
def test_order2_parity(name):
    m, kw, W, gW = _case(name)
    s = G.Solver(m, G.default_config(**kw))
    orc = oracle.Oracle(m, oracle.make_config(**kw))
    s.init(W, gW)
    b, coef, flag = s.debug_reconstruct()
    co, fo = orc.reconstruct(W, gW)
    assert_parity(coef, co, COEF_GROUPS, "coef")
    np.testing.assert_array_equal(flag, fo)
    check_face_terms(s, orc, W, gW, orc.compute_dt(W, 0.5))
    check_steps(m, s, orc, W, gW, by_stage=False, check_dt=False)


def test_order2_adjoint_matches_finite_differences():
    import torch
    m = I.kuhn_cube_mesh(4, 2 * np.pi, 0.1, 3, True)
    W, gW = I.cell_averages(m, I.taylor_green_field(mach=0.3))
    s = G.Solver(m, G.default_config(order=2, viscous=True, mu=0.01, prandtl=0.72, c_tau=0.0, eps_weno=1.0))
    dev = "cuda:0"
    Wt, Gt = torch.from_numpy(W).to(dev), torch.from_numpy(gW).to(dev)
    s.init(Wt, Gt)
    dt = s.compute_dt(0.5)

    def F(Wx, Gx):
        s.init(Wx, Gx)
        s.step(dt)
        return s.read_state(device=True)

    gen = torch.Generator().manual_seed(11)
    sW = torch.from_numpy(np.sqrt((W ** 2).mean(axis=1, keepdims=True))).to(dev)
    sG = torch.from_numpy(np.sqrt((gW ** 2).mean(axis=1, keepdims=True)) + 1e-3).to(dev)
    for _ in range(3):
        vW = torch.randn(W.shape, generator=gen, dtype=torch.float64).to(dev) * sW
        vG = torch.randn(gW.shape, generator=gen, dtype=torch.float64).to(dev) * sG
        bW = torch.randn(W.shape, generator=gen, dtype=torch.float64).to(dev)
        bG = torch.randn(gW.shape, generator=gen, dtype=torch.float64).to(dev)
        eps = 1e-6
        Wp, Gp = F(Wt + eps * vW, Gt + eps * vG)
        Wm, Gm = F(Wt - eps * vW, Gt - eps * vG)
        lhs = (((Wp - Wm) * bW).sum() + ((Gp - Gm) * bG).sum()).item() / (2 * eps)
        aW, aG = s.step_adjoint(dt, Wt, Gt, bW, bG)
        rhs = ((aW * vW).sum() + (aG * vG).sum()).item()
        assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)
