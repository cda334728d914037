#!/usr/bin/env python3
"""Throughput of the compact third-order gas-kinetic scheme on one MI355X.

Workload: the viscous Taylor-Green vortex on the periodic cube [0, 2 pi]^3,
32^3 hexahedra each split into 6 Kuhn tetrahedra (196,608 cells), vertices
jittered by 5% of h (seed 1), gamma 1.4, Ma 0.1, Re 1600 (mu = 1/1600),
Pr 0.72, CFL 0.5, third-order MR-WENO.  One "step" is the whole hot path:
the CFL time step, then both stages (slopes, MR-WENO reconstruction,
gas-kinetic face fluxes, cell update).  The state lives in HBM before the
timed region starts.

Prints one JSON line: cell-stage-updates/s over an uninstrumented timed
region, the roofline of the dominant kernel (per-kernel durations from HIP
events that the library records on its stream around each kernel, over the
same number of steps right after the timed region), the device's measured copy bandwidth (each
memory-bound kernel's rate is also given as a fraction of it), the FP32-bulk form's throughput and error, the
differentiation form (adjoint / forward time and its finite-difference
check), the walled blast workload (1.57M cells, slip walls), the lid-driven
cavity (no-slip isothermal walls, smooth-flow flux), flow past a sphere on a
cubed-sphere shell (1.77M cells, slip wall and far field) and the FP64 CPU
oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP64_VECTOR_TFLOPS = 78.6    # MI355X FP64 vector peak, TFLOP/s

# Algorithmic HBM bytes per unit of each FP64 kernel: every array element the
# kernel needs is counted once (neighbour gathers assumed served by caches).
#   slopes   per cell: W 5, M1 12, slopes out 15 doubles; 4 neighbour ids
#   recon    per cell: W 5, gW 15, slopes 15, M2 144, geometry 20 doubles,
#            4 neighbour ids; coefficients out 50 doubles, 1 flag
#   flux     per face: 2 cell ids, 16 geometry doubles, the coefficients (50 per
#            cell, read by its 4 faces; 2 faces per cell, so 25 per face), out
#            20 (stage 1) / 10 (stage 2) doubles
#   update   per cell: 4 face codes, 2 faces x (15 face terms + 3 normal),
#            W 5 / W^n, L, L_t 15, 1/|Omega|; out 20 + 15 (stage 1) / 20 (stage 2)
#   dt       per cell: W 5 + dr 1 doubles
BYTES_PER_UNIT = {
    "slopes": 8 * (5 + 12 + 15) + 4 * 4,
    "reconstruct": 8 * (5 + 15 + 15 + 144 + 20 + 50) + 4 * 4 + 4,
    "flux_stage1": 4 * 2 + 8 * (16 + 25 + 20),
    "flux_stage2": 4 * 2 + 8 * (16 + 25 + 10),
    "update_stage1": 4 * 4 + 8 * (2 * 18 + 5 + 1 + 35),
    "update_stage2": 4 * 4 + 8 * (2 * 18 + 15 + 1 + 20),
    "dt": 8 * 6,
}
UNIT = {"slopes": "cell", "reconstruct": "cell", "flux_stage1": "face", "flux_stage2": "face",
        "update_stage1": "cell", "update_stage2": "cell", "dt": "cell"}

# rocprofv3 names of each timed kernel (FP64, FP32-bulk) of this workload
# (viscous, Pr != 1)
PROFILE_NAMES = {
    "slopes": ("gks::slopes_kernel<double>", "gks::slopes_kernel<float>"),
    "reconstruct": ("gks::reconstruct_kernel<double>", "gks::reconstruct_kernel<float>"),
    "flux_stage1": ("gks::flux_kernel<double, 0, true, true, false, false>",
                    "gks::flux_kernel<float, 0, true, true, false, false>"),
    "flux_stage2": ("gks::flux_kernel<double, 1, true, true, false, false>",
                    "gks::flux_kernel<float, 1, true, true, false, false>"),
    "update_stage1": ("gks::update_kernel<double, 1>", "gks::update_kernel<float, 1>"),
    "update_stage2": ("gks::update_kernel<double, 2>", "gks::update_kernel<float, 2>"),
    "dt": ("gks::dt_pass1", None),  # one kernel serves both forms
}
# the kernel sources whose digest the committed counter summary records
KERNEL_SOURCES = ("paper_2102_01366_amd/csrc/gks_kernels.hip", "paper_2102_01366_amd/csrc/gks_flux.h",
                  "paper_2102_01366_amd/csrc/gks_flux_kernel.h", "paper_2102_01366_amd/csrc/gks_device.h",
                  "paper_2102_01366_amd/csrc/gks_internal.h", "paper_2102_01366_amd/csrc/gks_m2stage.h",
                  "paper_2102_01366_amd/csrc/gks_recon_adj.h")
COUNTERS = os.path.join(ROOT, "profiles", "taylor_green_196608_counters.md")


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key):
    """HBM bytes per launch of the FP64 kernel `key` on the 196,608-cell mesh,
    from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by
    the copy-kernel calibration it states); None when that summary was taken
    on other kernel sources."""
    try:
        with open(COUNTERS) as fh:
            text = fh.read()
    except OSError:
        return None
    if f"`{kernel_digest()}`" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 6 and cells[1] == f"{key} (fp64)":
            return float(cells[5].replace(",", ""))
    return None


def I_cell_volumes(mesh):
    import numpy as np
    v = mesh.xyz[mesh.tet]
    return np.abs(np.linalg.det(v[:, 1:] - v[:, :1])) / 6.0


def cpu_baseline(mesh, W, gW, cfg_kw, steps):
    """The FP64 oracle, as it stands, on `steps` steps of the same mesh."""
    import oracle
    oracle.build(force=False)
    threads = oracle.set_threads(0)
    orc = oracle.Oracle(mesh, oracle.make_config(**cfg_kw))
    dt = orc.compute_dt(W, 0.5)
    t0 = time.perf_counter()
    Wo, gWo = W, gW
    for _ in range(steps):
        Wo, gWo = orc.step(dt, Wo, gWo)
    el = time.perf_counter() - t0
    return {"value": mesh.n_cell * 2 * steps / el, "unit": "cell-stage-updates/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{steps} step(s) = {2 * steps} stages of the full {mesh.n_cell}-cell mesh, "
                      f"{el:.1f} s on {threads} OpenMP threads"}


def adjoint_leg(G, I, mesh, W, gW, cfg_kw, nsteps, ndir, precision):
    """Differentiation form on the same mesh: J = kinetic energy after
    `nsteps` CFL steps (time steps of an undifferentiated run, then fixed);
    dJ/d(W0, grad W0) by the discrete adjoint through the autograd rollout.
    Times one forward pass of plain steps and the adjoint pass, and checks
    the gradient against central differences along `ndir` seeded directions
    (rows scaled by their RMS, step 1e-6)."""
    import numpy as np
    import torch
    from paper_2102_01366_amd.autograd import rollout, time_steps
    dev = "cuda:0"
    s = G.Solver(mesh, G.default_config(precision=precision, **cfg_kw), device=dev)
    vol = torch.from_numpy(I_cell_volumes(mesh)).to(dev)
    W0, G0 = torch.from_numpy(W).to(dev), torch.from_numpy(gW).to(dev)
    dts = time_steps(s, W0, G0, 0.5, nsteps)

    def ke(Wx):
        return (vol * 0.5 * (Wx[1] ** 2 + Wx[2] ** 2 + Wx[3] ** 2) / Wx[0]).sum()

    s.init(W0, G0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for dt in dts:
        s.step(dt)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    # one step forward and back first, so that loading the reverse kernels and
    # allocating the adjoint workspace fall outside the timed pass
    Ww, Gw = W0.clone().requires_grad_(True), G0.clone().requires_grad_(True)
    ke(rollout(s, Ww, Gw, dts[:1])[0]).backward()
    del Ww, Gw
    Wr, Gr = W0.clone().requires_grad_(True), G0.clone().requires_grad_(True)
    J = ke(rollout(s, Wr, Gr, dts)[0])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t1
    out = {"steps": nsteps, "objective": "kinetic energy sum |Omega| |rho U|^2 / (2 rho) at the final time",
           "forward_ms_per_step": t_fwd / nsteps * 1e3, "adjoint_ms_per_step": t_adj / nsteps * 1e3,
           "adjoint_over_forward": t_adj / t_fwd,
           "checkpoint_bytes": nsteps * 20 * 8 * mesh.n_cell}
    if ndir:
        gen = torch.Generator().manual_seed(4)
        sW = torch.from_numpy(np.sqrt((W ** 2).mean(axis=1, keepdims=True))).to(dev)
        sG = torch.from_numpy(np.sqrt((gW ** 2).mean(axis=1, keepdims=True)) + 1e-3).to(dev)
        # the jump term |p_l - p_r| and the WENO indicators' |.| are kinks: a
        # difference whose step straddles one measures a secant, so the check
        # is reported at two steps
        errs = {1e-6: [], 1e-7: []}
        for _ in range(ndir):
            vW = torch.randn(W.shape, generator=gen, dtype=torch.float64).to(dev) * sW
            vG = torch.randn(gW.shape, generator=gen, dtype=torch.float64).to(dev) * sG
            ad = ((Wr.grad * vW).sum() + (Gr.grad * vG).sum()).item()
            for eps in errs:
                with torch.no_grad():
                    Jp = ke(rollout(s, W0 + eps * vW, G0 + eps * vG, dts)[0]).item()
                    Jm = ke(rollout(s, W0 - eps * vW, G0 - eps * vG, dts)[0]).item()
                errs[eps].append(abs((Jp - Jm) / (2 * eps) - ad) / abs(ad))
        out.update({"fd_directions": ndir,
                    "fd": [{"eps": eps, "max_rel_err": max(e), "median_rel_err": float(np.median(e))}
                           for eps, e in errs.items()]})
    return out, (Wr.grad.detach(), Gr.grad.detach())


def timed_kernels(solver, steps):
    """Per-kernel HIP-event durations over `steps` further steps (the events
    are recorded by the library on its stream around each kernel)."""
    import torch
    solver.timing_read(reset=True)
    solver.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        solver.step_cfl(0.5)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    solver.timing_enable(False)
    return solver.timing_read(reset=True), el


def copy_bandwidth(torch, nbytes=1 << 30, reps=20):
    """Achievable HBM bandwidth of this device: a device-to-device copy of
    `nbytes` (reads and writes `nbytes` each), median of `reps` timed copies
    after a warm-up, in GB/s.  The 1 GiB buffers exceed the 256 MB last-level
    cache, so the copy streams through HBM."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    del a, b
    ms.sort()
    return 2 * nbytes / (ms[len(ms) // 2] * 1e-3) / 1e9


def blast_leg(G, I, n, steps, warmup, copy_gbs):
    """Shock-robustness workload with reflective walls: the spherical blast
    (rho 1, p 10 inside r < 0.1, p 0.1 outside, at rest) in the unit cube,
    n^3 hexahedra x 6 Kuhn tetrahedra, 10% jitter (seed 2), six slip walls,
    Euler, third-order WENO, CFL 0.5; FP64 and FP32-bulk.  On this mesh
    (well beyond the last-level cache) the FP64 per-kernel rates are also given
    as fractions of the HBM peak and of the measured copy bandwidth, and the
    flux's as counted FP64 work against the FP64 vector peak."""
    import numpy as np
    import torch
    mesh = I.kuhn_cube_mesh(n, 1.0, 0.1, 2, False)
    W, gW = I.blast_cell_averages(mesh)
    vol = I_cell_volumes(mesh)
    out = {"workload": f"spherical blast in the unit cube, {n}^3 hexes x 6 Kuhn tets "
                       f"({mesh.n_cell} cells, {mesh.n_face} faces), 10% jitter, slip walls, Euler, CFL 0.5",
           "cells": mesh.n_cell, "faces": mesh.n_face, "steps": steps}
    res = {}
    for name, prec in (("fp64", G.GKS_FP64), ("fp32_bulk", G.GKS_FP32_BULK)):
        s = G.Solver(mesh, G.default_config(precision=prec), device="cuda:0")
        s.init(W, gW)
        sums0 = s.conservation_sums()
        for _ in range(warmup):
            s.step_cfl(0.5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step_cfl(0.5)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        Wf, _ = s.read_state()
        sums1 = s.conservation_sums()
        kt, _ = timed_kernels(s, steps)
        flag = s.debug_reconstruct()[2]
        units = {"cell": mesh.n_cell, "face": mesh.n_face}
        kern = {}
        flops_face = G.flux_op_count(G.default_config(precision=prec))["total"]
        for k, (ms, cnt) in kt.items():
            if cnt:
                kern[k] = {"avg_ms": ms / cnt}
                if prec == G.GKS_FP64:
                    gbs = BYTES_PER_UNIT[k] * units[UNIT[k]] / (ms / cnt * 1e-3) / 1e9
                    kern[k]["hbm_GBs"] = gbs
                    if k.startswith("flux"):
                        tf = flops_face * mesh.n_face / (ms / cnt * 1e-3) / 1e12
                        kern[k]["fp64_TFLOPs"] = tf
                        kern[k]["fp64_frac"] = tf / FP64_VECTOR_TFLOPS
                    else:
                        kern[k]["hbm_frac"] = gbs / HBM_PEAK_GBS
                        kern[k]["frac_of_copy"] = gbs / copy_gbs
        res[name] = (Wf, {"value": mesh.n_cell * 2 * steps / el, "unit": "cell-stage-updates/s",
                          "ms_per_step": el / steps * 1e3,
                          "mass_energy_drift": float(max(abs(sums1[q] - sums0[q]) / abs(sums0[q]) for q in (0, 4))),
                          "fallback_cells": int(flag.sum()), "kernels": kern})
    out["fp64"] = res["fp64"][1]
    out["fp32_bulk"] = res["fp32_bulk"][1]
    W64, W32 = res["fp64"][0], res["fp32_bulk"][0]
    out["fp32_bulk"]["l1_density_vs_fp64"] = float(np.sum(vol * np.abs(W32[0] - W64[0])) / np.sum(vol * W64[0]))
    out["fp32_bulk"]["speedup_vs_fp64"] = out["fp32_bulk"]["value"] / out["fp64"]["value"]
    return out


def cavity_leg(G, I, n, steps, warmup):
    """No-slip walls and the smooth-flow flux: the lid-driven cavity of the
    paper's Sec. 5 set-up -- unit cube, n^3 hexahedra x 6 Kuhn tetrahedra,
    uniform (no jitter), six isothermal no-slip walls at T = p/rho = 1/gamma,
    the lid y = 1 moving at 0.15 along x (Ma 0.15), gamma 5/3, Re 1000 on
    the lid speed and side, gas initially at rest (rho 1, p 1/gamma), linear
    reconstruction weights, eq. 2nd-smooth-flux, CFL 0.5; FP64 and
    FP32-bulk."""
    import numpy as np
    import torch
    gamma, ulid = 5.0 / 3.0, 0.15
    sides = ("x0", "x1", "y0", "y1", "z0", "z1")
    mesh = I.with_walls(I.kuhn_cube_mesh(n, 1.0, 0.0, 0, False), {s: I.FACE_NOSLIP_ISOTHERMAL for s in sides},
                        {"y1": (ulid, 0.0, 0.0)})
    W = np.zeros((5, mesh.n_cell))
    W[0] = 1.0
    W[4] = (1.0 / gamma) / (gamma - 1.0)
    gW = np.zeros((15, mesh.n_cell))
    kw = dict(gamma=gamma, viscous=True, mu=ulid / 1000.0, prandtl=1.0, nonlinear=False, flux=G.GKS_FLUX_SMOOTH,
              wall_T=1.0 / gamma)
    nwall_cells = int(np.unique(mesh.face_cell[mesh.face_cell[:, 1] < 0, 0]).size)
    out = {"workload": f"lid-driven cavity, {n}^3 hexes x 6 Kuhn tets ({mesh.n_cell} cells, {mesh.n_face} faces, "
                       f"{nwall_cells} wall cells), uniform, isothermal no-slip walls, lid Ma 0.15, gamma 5/3, "
                       f"Re 1000, linear weights, smooth-flow flux, CFL 0.5",
           "cells": mesh.n_cell, "faces": mesh.n_face, "wall_cells": nwall_cells, "steps": steps}
    for name, prec in (("fp64", G.GKS_FP64), ("fp32_bulk", G.GKS_FP32_BULK)):
        s = G.Solver(mesh, G.default_config(precision=prec, **kw), device="cuda:0")
        s.init(W, gW)
        for _ in range(warmup):
            s.step_cfl(0.5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step_cfl(0.5)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        Wf, _ = s.read_state()
        kt, _ = timed_kernels(s, steps)
        out[name] = {"value": mesh.n_cell * 2 * steps / el, "unit": "cell-stage-updates/s",
                     "ms_per_step": el / steps * 1e3,
                     "max_speed_over_lid": float(np.abs(Wf[1:4] / Wf[0]).max() / ulid),
                     "kernels_ms": {k: ms / cnt for k, (ms, cnt) in kt.items() if cnt}}
    return out


def sphere_leg(G, I, n, layers, steps, warmup):
    """The curved-wall workload's mesh with straight faces: inviscid Mach 0.3
    flow past the unit sphere on a cubed-sphere shell (6 panels of n x n
    cells, `layers` radial layers stretched by 1.08 out to r = 20, each
    hexahedron split into 6 tetrahedra), slip wall on the sphere, far field
    by Riemann invariants, impulsive start from the free stream rho = 1,
    U = (0.3, 0, 0), p = 1/gamma, third-order WENO, CFL 0.5; FP64 and
    FP32-bulk."""
    import numpy as np
    import torch
    gamma = 1.4
    mesh = I.cubed_sphere_shell(n, layers, r_out=20.0, ratio=1.08)
    W, gW = I.uniform_state(mesh, 1.0, (0.3, 0.0, 0.0), 1.0 / gamma, gamma)
    free = tuple(W[:, 0])
    out = {"workload": f"Mach 0.3 past the unit sphere, cubed-sphere shell 6 x {n}^2 x {layers} layers "
                       f"x 6 tets ({mesh.n_cell} cells, {mesh.n_face} faces), straight faces, slip wall, "
                       f"Riemann-invariant far field at r = 20, Euler, CFL 0.5",
           "cells": mesh.n_cell, "faces": mesh.n_face, "steps": steps}
    for name, prec in (("fp64", G.GKS_FP64), ("fp32_bulk", G.GKS_FP32_BULK)):
        s = G.Solver(mesh, G.default_config(precision=prec, farfield=free), device="cuda:0")
        s.init(W, gW)
        for _ in range(warmup):
            s.step_cfl(0.5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step_cfl(0.5)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        Wf, _ = s.read_state()
        assert np.isfinite(Wf).all()
        kt, _ = timed_kernels(s, steps)
        out[name] = {"value": mesh.n_cell * 2 * steps / el, "unit": "cell-stage-updates/s",
                     "ms_per_step": el / steps * 1e3,
                     "kernels_ms": {k: ms / cnt for k, (ms, cnt) in kt.items() if cnt}}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=32, help="hexahedra per side of the mesh")
    ap.add_argument("--cpu-baseline-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-bulk leg")
    ap.add_argument("--adjoint-steps", type=int, default=50,
                    help="steps of the differentiation leg (0 skips it)")
    ap.add_argument("--adjoint-directions", type=int, default=16)
    ap.add_argument("--cavity-n", type=int, default=32,
                    help="hexahedra per side of the lid-driven cavity leg (0 skips it)")
    ap.add_argument("--cavity-steps", type=int, default=20)
    ap.add_argument("--sphere-n", type=int, default=32,
                    help="cells per panel side of the sphere leg (0 skips it)")
    ap.add_argument("--sphere-layers", type=int, default=48)
    ap.add_argument("--sphere-steps", type=int, default=4)
    ap.add_argument("--blast-n", type=int, default=64,
                    help="hexahedra per side of the walled blast leg (0 skips it)")
    ap.add_argument("--blast-steps", type=int, default=20)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with a 256 MiB fill (writes 256 MiB) and a 256 MiB elementwise add "
                         "(reads and writes 256 MiB): known byte counts that calibrate rocprofv3 "
                         "FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the mesh would shard by cell partition with halo exchange).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2102_01366_amd as G
    from paper_2102_01366_amd import inputs as I

    mu = 1.0 / 1600.0
    cfg_kw = dict(viscous=True, mu=mu, prandtl=0.72)
    mesh = I.kuhn_cube_mesh(args.n, 2 * math.pi, 0.05, 1, True)
    W, gW = I.cell_averages(mesh, I.taylor_green_field(gamma=1.4, mach=0.1))
    config = G.default_config(**cfg_kw)
    solver = G.Solver(mesh, config, device="cuda:0")
    solver.init(W, gW)
    nc, nf = mesh.n_cell, mesh.n_face

    # each step: dt = CFL bound on the device, then both stages with that dt;
    # the timed region runs uninstrumented, then the same number of steps
    # runs with HIP events around every kernel for the per-kernel durations
    for _ in range(args.warmup):
        solver.step_cfl(0.5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.step_cfl(0.5)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    Wf, _ = solver.read_state()
    kt, el_instr = timed_kernels(solver, args.steps)
    assert np.isfinite(Wf).all()

    flops_face = G.flux_op_count(config)["total"]
    copy_gbs = copy_bandwidth(torch)
    units = {"cell": nc, "face": nf}
    kernels = {}
    for k, (ms, cnt) in kt.items():
        if cnt == 0:
            continue
        avg_s = ms / cnt * 1e-3
        nbytes = BYTES_PER_UNIT[k] * units[UNIT[k]]
        entry = {"avg_ms": ms / cnt, "launches": cnt, "total_ms": ms,
                 "bytes_per_launch": nbytes, "hbm_GBs": nbytes / avg_s / 1e9}
        if k.startswith("flux"):
            entry["flops_per_launch"] = flops_face * nf
            entry["fp64_TFLOPs"] = flops_face * nf / avg_s / 1e12
        else:
            entry["frac_of_copy"] = entry["hbm_GBs"] / copy_gbs
        kernels[k] = entry
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    d = kernels[dom]
    traffic = measured_traffic(dom) if args.n == 32 else None
    if dom.startswith("flux"):
        roof = {"kernel": dom, "bound": "alu", "achieved": d["fp64_TFLOPs"],
                "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": d["fp64_TFLOPs"] / FP64_VECTOR_TFLOPS, "traffic": traffic,
                "work_per_launch": f"{flops_face:.0f} FP64 ops/face x {nf} faces"}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": d["hbm_GBs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": d["hbm_GBs"] / HBM_PEAK_GBS, "frac_of_copy": d["frac_of_copy"],
                "traffic": traffic,
                "work_per_launch": f"{BYTES_PER_UNIT[dom]} B/{UNIT[dom]} x {units[UNIT[dom]]}"}

    value = nc * 2 * args.steps / elapsed

    fp32 = None
    if not args.no_fp32:
        # FP32-bulk leg: the same workload, steps and time-step rule; its
        # density L1 difference from the FP64 run and conservation drift
        s32 = G.Solver(mesh, G.default_config(precision=G.GKS_FP32_BULK, **cfg_kw), device="cuda:0")
        s32.init(W, gW)
        sums0 = s32.conservation_sums()
        for _ in range(args.warmup):
            s32.step_cfl(0.5)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            s32.step_cfl(0.5)
        torch.cuda.synchronize()
        el32 = time.perf_counter() - t1
        W32, _ = s32.read_state()
        sums1 = s32.conservation_sums()
        kt32, _ = timed_kernels(s32, args.steps)
        vol = I_cell_volumes(mesh)
        fp32 = {"value": nc * 2 * args.steps / el32, "unit": "cell-stage-updates/s",
                "ms_per_step": el32 / args.steps * 1e3, "speedup_vs_fp64": elapsed / el32,
                "l1_density_vs_fp64": float(np.sum(vol * np.abs(W32[0] - Wf[0])) / np.sum(vol * Wf[0])),
                "conservation_drift": float(np.max(np.abs(sums1 - sums0) / np.abs(sums0).max())),
                "dtype": "fp32 bulk / fp64 state",
                "kernels_ms": {k: ms / cnt for k, (ms, cnt) in kt32.items() if cnt}}
    out = {
        "metric": "cell-stage-updates/s",
        "value": value,
        "unit": "cell-stage-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "ms_per_step_with_kernel_events": el_instr / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"viscous Taylor-Green vortex, [0,2pi]^3 periodic, {args.n}^3 hexes "
                               f"x 6 Kuhn tets ({nc} cells, {nf} faces), 5% jitter, Ma 0.1, "
                               "Re 1600, Pr 0.72, CFL 0.5, third-order MR-WENO, FP64",
                   "cells": nc, "faces": nf, "precision": "fp64"},
        "roofline": roof,
        "hbm_copy_GBs": copy_gbs,
        "kernels": kernels,
    }
    out["fp32_bulk"] = fp32
    if args.adjoint_steps > 0:
        adj, g64 = adjoint_leg(G, I, mesh, W, gW, cfg_kw, args.adjoint_steps, args.adjoint_directions,
                               G.GKS_FP64)
        adj32, g32 = adjoint_leg(G, I, mesh, W, gW, cfg_kw, args.adjoint_steps, 0, G.GKS_FP32_BULK)
        adj["fp32_bulk"] = {k: adj32[k] for k in ("forward_ms_per_step", "adjoint_ms_per_step",
                                                  "adjoint_over_forward")}
        adj["fp32_bulk"]["gradient_rel_diff_vs_fp64"] = max(
            float((a - b).abs().max() / a.abs().max()) for a, b in zip(g64, g32))
        out["adjoint"] = adj
    else:
        out["adjoint"] = None
    out["blast_walls"] = (blast_leg(G, I, args.blast_n, args.blast_steps, 2, copy_gbs)
                          if args.blast_n > 0 else None)
    out["cavity_noslip"] = cavity_leg(G, I, args.cavity_n, args.cavity_steps, 2) if args.cavity_n > 0 else None
    out["sphere_farfield"] = (sphere_leg(G, I, args.sphere_n, args.sphere_layers, args.sphere_steps, 1)
                              if args.sphere_n > 0 else None)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh, W, gW, cfg_kw, args.cpu_baseline_steps)
    else:
        out["cpu_baseline"] = None
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        torch.add(a, 1, out=b)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
