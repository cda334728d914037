"""The benchmark's flow measures on synthetic fields whose answers are set
by construction (CPU): the wake length and separation angle of the flow past
the sphere (bench.sphere_wake)."""
import numpy as np

import bench
from paper_2102_01366_amd import inputs as I


def _shell_field(sep_deg, reattach_x):
    m = I.cubed_sphere_shell(16, 24, r_out=20.0, ratio=1.16, curved=True, wall_tag=I.FACE_NOSLIP_ADIABATIC)
    c = m.xyz[m.tet].mean(axis=1)
    r = np.linalg.norm(c, axis=1)
    phi = np.arccos(np.clip(-c[:, 0] / r, -1, 1))
    psi = np.arctan2(c[:, 2], c[:, 1])
    e_phi = np.stack([np.sin(phi), np.cos(phi) * np.cos(psi), np.cos(phi) * np.sin(psi)])
    # meridional velocity that turns against the flow at sep_deg; axial
    # velocity behind the sphere negative up to x = reattach_x
    U = e_phi * np.cos(np.pi / 2 * np.degrees(phi) / sep_deg)
    axis = (c[:, 0] > 1) & (np.hypot(c[:, 1], c[:, 2]) < 0.3)
    U[0, axis] = c[axis, 0] - reattach_x
    W = np.zeros((5, m.n_cell))
    W[0] = 1.0
    W[1:4] = U
    W[4] = 2.5
    wall = np.nonzero((m.face_cell[:, 1] < 0) & (m.face_tag != I.FACE_FARFIELD))[0]
    return m, W, np.unique(m.face_cell[wall, 0])


def test_sphere_wake_measures():
    for sep, xr in ((125.0, 2.4), (140.0, 3.0)):
        m, W, wall_cells = _shell_field(sep, xr)
        out = bench.sphere_wake(m, W, wall_cells)
        assert abs(out["separation_angle_degrees"] - sep) < 1.0, out
        assert abs(out["wake_length_diameters"] - (xr - 1.0) / 2.0) < 0.03, out


def test_sphere_wake_without_recirculation():
    m, W, wall_cells = _shell_field(200.0, 0.5)   # attached flow, no reverse flow on the axis
    out = bench.sphere_wake(m, W, wall_cells)
    assert "separation_angle_degrees" not in out and "wake_length_diameters" not in out, out
