"""Writes weno_readings.json: the oracle's sine-wave errors (the set-up of the
paper's Sec. 5.1, Tables 2 and 3) under each reading of the nonlinear
weights that the paper leaves open.

Set-up: [0,2]^3 periodic, 6 N^3 tetrahedra (Kuhn split, mirrored so that the
wave does not run along the shared diagonal: the split on which the linear
scheme reproduces Table 1), rho = 1 + 0.2 sin(pi (x+y-z)), U = (1,1,-1),
p = 1, tau = 0, CFL 1, t = 2; density L1, L2, Linf against the exact cell
averages.  Readings (oracle.READ_* and the linear weights):
  text        the readings the library follows (gamma_{2,2} = 100/111 on P^2)
  caption     the Table 2 caption's d0:d1:d2 = 100:10:1 taken with d0 on P^0
              (Table 3: d0:d1 = 10:1 with d0 on P^0)
  pow1        power 1 in omega_{m,n}
  pow1st2     power 2 in omega^{1st}_j
  b0vol       |Delta_0| = |Omega_0| in beta_{0,j}
  mixed2      mixed second derivatives twice in beta_2
  beta_lower  indicators of the hierarchical p_1, p_2
  sigma1      sigma without the power 4/3
  linear      linear weights (Table 1 for the third-order scheme)
Run: python tests/golden/weno_readings.py [N ...]   (calls only oracle/)
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2102_01366_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weno_readings.json")


def readings(order):
    base = {"order": order}
    cap = {"lw2": (1.0, 10.0, 100.0)} if order == 3 else {"lw1": (1.0, 10.0)}
    r = {"text": {}, "caption": cap, "pow1": {"weno_reading": oracle.READ_POW1},
         "pow1st2": {"weno_reading": oracle.READ_POW1ST2}, "b0vol": {"weno_reading": oracle.READ_B0VOL},
         "beta_lower": {"weno_reading": oracle.READ_BETA_LOWER},
         "sigma1": {"weno_reading": oracle.READ_SIGMA1}, "linear": {"nonlinear": False}}
    if order == 3:
        r["mixed2"] = {"weno_reading": oracle.READ_MIXED2}
    return {k: dict(base, **v) for k, v in r.items()}


def sine_wave_errors(N, cfg_kw, T=2.0, cfl=1.0):
    d = (1.0, 1.0, -1.0)
    m = I.kuhn_cube_mesh(N, 2.0, 0.0, 0, True)
    orc = oracle.Oracle(m, oracle.make_config(**cfg_kw))
    W, gW = I.cell_averages(m, I.sine_wave_field(length=2.0, direction=d, vel=d))
    t = 0.0
    while t < T - 1e-14:
        dt = min(orc.compute_dt(W, cfl), T - t)
        W, gW = orc.step(dt, W, gW)
        t += dt
    We, _ = I.cell_averages(m, I.sine_wave_field(length=2.0, direction=d, vel=d, t=T))
    vol = orc.geometry()[0]
    e = W[0] - We[0]
    return [float(np.sum(vol * np.abs(e)) / vol.sum()), float(np.sqrt(np.sum(vol * e * e) / vol.sum())),
            float(np.abs(e).max())]


def main():
    Ns = [int(a) for a in sys.argv[1:]] or [5, 10]
    oracle.build(force=False)
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for order in (3, 2):
        for name, kw in readings(order).items():
            for N in Ns:
                key = f"order{order}/{name}/N{N}"
                res[key] = sine_wave_errors(N, kw)
                print(key, res[key], flush=True)
                with open(OUT, "w") as fh:
                    json.dump(res, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
