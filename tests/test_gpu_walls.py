"""Slip walls on the GPU (Sec. 4.4) against the oracle, to the same normwise
1e-12 bar as the periodic cases (see test_gpu_parity.py for the metric).

Meshes: the unit cube with six slip walls, N^3 hexahedra x 6 Kuhn
tetrahedra, interior vertices jittered (wall vertices slide along the
walls), seeded; so cells with two, three and four neighbours all occur.
Fields: a smooth swirl with a pressure bump (no normal velocity on the
walls) and the spherical blast (rho 1, p 10 inside r < 0.1 -- here r < 0.2
on the coarse meshes -- p 0.1 outside, gas at rest), whose jump triggers
the positivity fallback in some cells.
"""
import numpy as np
import pytest

import oracle
import paper_2102_01366_amd as G
from paper_2102_01366_amd import inputs as I

from test_gpu_parity import COEF_GROUPS, GW_GROUPS, assert_parity, check_face_terms, check_steps

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "vortex_euler":
        m = I.kuhn_cube_mesh(4, 1.0, 0.1, 2, False)
        W, gW = I.cell_averages(m, I.box_vortex_field())
        return m, dict(), W, gW
    if name == "vortex_ns_ragged":
        m = I.kuhn_cube_mesh(5, 1.0, 0.1, 3, False)  # 750 cells
        W, gW = I.cell_averages(m, I.box_vortex_field(amp=0.3))
        return m, dict(viscous=True, mu=0.005, prandtl=0.72), W, gW
    if name == "blast":
        m = I.kuhn_cube_mesh(6, 1.0, 0.1, 4, False)
        W, gW = I.blast_cell_averages(m, radius=0.2)
        return m, dict(), W, gW
    raise KeyError(name)


CASES = ["vortex_euler", "vortex_ns_ragged", "blast"]


def _pair(name):
    m, kw, W, gW = _case(name)
    return m, G.Solver(m, G.default_config(**kw)), oracle.Oracle(m, oracle.make_config(**kw)), W, gW


@pytest.mark.parametrize("name", CASES)
def test_wall_reconstruction(name):
    m, s, orc, W, gW = _pair(name)
    s.init(W, gW)
    b, coef, flag = s.debug_reconstruct()
    co, fo = orc.reconstruct(W, gW)
    assert_parity(b, orc.slopes(W, gW), GW_GROUPS, "slopes")
    assert_parity(coef, co, COEF_GROUPS, "coef")
    np.testing.assert_array_equal(flag, fo)
    if name == "blast":
        assert fo.sum() > 0  # the fallback is exercised


@pytest.mark.parametrize("name", CASES)
def test_wall_face_terms(name):
    m, s, orc, W, gW = _pair(name)
    s.init(W, gW)
    check_face_terms(s, orc, W, gW, orc.compute_dt(W, 0.5))


@pytest.mark.parametrize("name", CASES)
def test_wall_steps(name):
    m, s, orc, W, gW = _pair(name)
    check_steps(m, s, orc, W, gW, by_stage=False)


def test_wall_conservation_on_gpu():
    """Mass and energy are conserved with slip walls; momentum is not (the
    walls push back)."""
    m = I.kuhn_cube_mesh(8, 1.0, 0.1, 5, False)
    W, gW = I.cell_averages(m, I.box_vortex_field())
    s = G.Solver(m, G.default_config(viscous=True, mu=0.002, prandtl=0.72))
    s.init(W, gW)
    s0 = s.conservation_sums()
    for _ in range(10):
        s.step_cfl(0.5)
    s1 = s.conservation_sums()
    for q in (0, 4):
        assert abs(s1[q] - s0[q]) <= 1e-13 * abs(s0[q])


def test_wall_fp32_bulk_close_to_fp64():
    m = I.kuhn_cube_mesh(6, 1.0, 0.1, 6, False)
    W, gW = I.cell_averages(m, I.box_vortex_field())
    out = []
    for prec in (G.GKS_FP64, G.GKS_FP32_BULK):
        s = G.Solver(m, G.default_config(precision=prec))
        s.init(W, gW)
        for _ in range(5):
            s.step(2e-3)
        out.append(s.read_state()[0])
    v = np.abs(np.linalg.det(m.xyz[m.tet][:, 1:] - m.xyz[m.tet][:, :1])) / 6
    l1 = np.sum(v * np.abs(out[1][0] - out[0][0])) / np.sum(v * out[0][0])
    assert l1 <= 1e-6


def test_wall_adjoint_matches_finite_differences():
    """gks_step_adjoint through wall faces (the ghost's adjoint returns to the
    owner) and own-gradient cells; smooth configuration (see
    test_gpu_adjoint.py)."""
    import torch
    m = I.kuhn_cube_mesh(4, 1.0, 0.1, 2, False)
    W, gW = I.cell_averages(m, I.box_vortex_field())
    s = G.Solver(m, G.default_config(viscous=True, mu=0.01, prandtl=0.72, c_tau=0.0, eps_weno=1.0))
    dev = "cuda:0"
    Wt, Gt = torch.from_numpy(W).to(dev), torch.from_numpy(gW).to(dev)
    s.init(Wt, Gt)
    dt = s.compute_dt(0.5)

    def F(Wx, Gx):
        s.init(Wx, Gx)
        s.step(dt)
        return s.read_state(device=True)

    gen = torch.Generator().manual_seed(8)
    sW = torch.from_numpy(np.sqrt((W ** 2).mean(axis=1, keepdims=True)) + 1e-3).to(dev)
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
