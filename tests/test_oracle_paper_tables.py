"""The oracle against the paper's printed accuracy results (Sec. 5.1, Table 1).

The paper runs rho = 1 + 0.2 sin(pi (x+y+z)), U = (1,1,1), p = 1 on [0,2]^3
with 6 N^3 tetrahedra, tau = 0, CFL 1, to t = 2, and prints L1/L2/Linf
density errors (tests/golden/paper_sine_wave_tables.json).  The split of
each hexahedron is not stated.  On a Kuhn split whose six tetrahedra share
the (1,1,1) diagonal the wave runs along every cell's longest edge and the
errors are ~10x the printed ones; on the mirrored split (shared diagonal
(1,1,-1)) the linear third-order scheme reproduces Table 1.  The mirrored
split is used here as the (1,1,-1) direction of the wave on the unmirrored
mesh, which is the same problem up to the reflection z -> -z.
"""
import json
import os

import numpy as np

from paper_2102_01366_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_sine_wave_tables.json")


def run_sine_wave(oracle_lib, N, nonlinear, T=2.0, cfl=1.0):
    d = (1.0, 1.0, -1.0)
    m = I.kuhn_cube_mesh(N, 2.0, 0.0, 0, True)
    orc = oracle_lib.Oracle(m, oracle_lib.make_config(nonlinear=nonlinear))
    W, gW = I.cell_averages(m, I.sine_wave_field(length=2.0, direction=d, vel=d))
    t = 0.0
    while t < T - 1e-14:
        dt = min(orc.compute_dt(W, cfl), T - t)
        W, gW = orc.step(dt, W, gW)
        t += dt
    We, _ = I.cell_averages(m, I.sine_wave_field(length=2.0, direction=d, vel=d, t=T))
    vol = orc.geometry()[0]
    e = W[0] - We[0]
    return (np.sum(vol * np.abs(e)) / vol.sum(), np.sqrt(np.sum(vol * e * e) / vol.sum()),
            np.abs(e).max())


def test_table1_linear_n5(oracle_lib):
    gold = json.load(open(GOLDEN))["table1_linear_third_order"]
    l1, l2, linf = run_sine_wave(oracle_lib, 5, nonlinear=False)
    assert abs(l1 / gold["L1"][0] - 1) < 0.05, (l1, gold["L1"][0])
    assert abs(l2 / gold["L2"][0] - 1) < 0.05, (l2, gold["L2"][0])
    assert abs(linf / gold["Linf"][0] - 1) < 0.08, (linf, gold["Linf"][0])
