"""Full-size parity of the large workloads, in the launch configuration the
benchmark times (gks_step_cfl: the CFL time step computed and used on the
device, then both stages): two whole steps on the GPU against the oracle,
element by element, to the bars of test_gpu_parity.py (the state normwise at
1e-12, the averaged gradients against the magnitude of their Gauss sums).

* walled blast: unit cube, 64^3 hexahedra x 6 Kuhn tetrahedra (1,572,864
  cells), 10% jitter (seed 2), slip walls, Euler, (rho, p) = (1, 10) inside
  r < 0.1 and (1, 0.1) outside, WENO weights and the positivity fallback
  active;
* sphere: cubed-sphere shell 6 x 32^2 x 48 layers x 6 tetrahedra (1,769,472
  cells) out to r = 20, slip wall, Riemann-invariant far field, the free
  stream rho = 1, U = (0.3, 0, 0), p = 1/gamma disturbed by a smooth density
  and pressure bump next to the wall (inputs.bump_stream_field, centre
  (1.5, 0, 0));
* the Taylor-Green workload (196,608 cells) is in test_gpu_parity.py.
The oracle takes about half a minute per step on the large meshes.
"""
import pytest

import oracle
import paper_2102_01366_amd as G
from paper_2102_01366_amd import inputs as I

from test_gpu_parity import check_steps

pytestmark = pytest.mark.gpu


def two_steps(mesh, kw, W, gW):
    s = G.Solver(mesh, G.default_config(**kw))
    orc = oracle.Oracle(mesh, oracle.make_config(**kw))
    return check_steps(mesh, s, orc, W, gW, nsteps=2, by_stage=False, on_device_dt=True)


@pytest.mark.timeout(900)
def test_blast_full_size_two_steps():
    mesh = I.kuhn_cube_mesh(64, 1.0, 0.1, 2, False)
    W, gW = I.blast_cell_averages(mesh)
    two_steps(mesh, dict(), W, gW)


@pytest.mark.timeout(900)
def test_sphere_full_size_two_steps():
    gamma = 1.4
    mesh = I.cubed_sphere_shell(32, 48, r_out=20.0, ratio=1.08)
    W, gW = I.cell_averages(mesh, I.bump_stream_field(gamma, center=(1.5, 0.0, 0.0)))
    free = I.uniform_state(mesh, 1.0, (0.3, 0.0, 0.0), 1.0 / gamma, gamma)[0][:, 0]
    two_steps(mesh, dict(farfield=tuple(free)), W, gW)
