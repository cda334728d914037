"""Full-size parity of the two large workloads, in the launch configuration
the benchmark times: one whole step (CFL 0.5 time step, both stages) on the
GPU against the oracle, element by element, to the normwise 1e-12 bar of
test_gpu_parity.py.

* walled blast: unit cube, 64^3 hexahedra x 6 Kuhn tetrahedra (1,572,864
  cells), 10% jitter (seed 2), slip walls, Euler, (rho, p) = (1, 10) inside
  r < 0.1 and (1, 0.1) outside, WENO weights and the positivity fallback
  active;
* sphere: cubed-sphere shell 6 x 32^2 x 48 layers x 6 tetrahedra (1,769,472
  cells) out to r = 20, slip wall, Riemann-invariant far field, free stream
  rho = 1, U = (0.3, 0, 0), p = 1/gamma, after one step from the free stream
  (so that the wall has disturbed the flow).
The oracle takes about half a minute per step here.
"""
import numpy as np
import pytest

import oracle
import paper_2102_01366_amd as G
from paper_2102_01366_amd import inputs as I

from test_gpu_parity import GW_GROUPS, W_GROUPS, assert_parity, gradient_floors

pytestmark = pytest.mark.gpu


def _one_step(mesh, kw, W, gW):
    s = G.Solver(mesh, G.default_config(**kw))
    orc = oracle.Oracle(mesh, oracle.make_config(**kw))
    s.init(W, gW)
    dt = s.compute_dt(0.5)
    assert abs(orc.compute_dt(W, 0.5) - dt) <= 1e-15 * dt
    s.step(dt)
    Wo, gWo = orc.step(dt, W, gW)
    Wg, gWg = s.read_state()
    assert_parity(Wg, Wo, W_GROUPS, "W")
    assert_parity(gWg, gWo, GW_GROUPS, "gW", floors=gradient_floors(Wo, orc))
    return Wo, gWo


def test_blast_full_size_one_step():
    mesh = I.kuhn_cube_mesh(64, 1.0, 0.1, 2, False)
    W, gW = I.blast_cell_averages(mesh)
    _one_step(mesh, dict(), W, gW)


def test_sphere_full_size_one_step():
    gamma = 1.4
    mesh = I.cubed_sphere_shell(32, 48, r_out=20.0, ratio=1.08)
    W, gW = I.uniform_state(mesh, 1.0, (0.3, 0.0, 0.0), 1.0 / gamma, gamma)
    kw = dict(farfield=tuple(W[:, 0]))
    # one step from the free stream on the GPU, then the compared step
    s = G.Solver(mesh, G.default_config(**kw))
    s.init(W, gW)
    s.step(s.compute_dt(0.5))
    W1, gW1 = s.read_state()
    _one_step(mesh, kw, W1, gW1)
