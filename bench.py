#!/usr/bin/env python3
"""Throughput of the compact third-order gas-kinetic scheme on one MI355X.

Headline workload: the spherical blast with reflective walls in the unit
cube, 64^3 hexahedra each split into 6 Kuhn tetrahedra (1,572,864 cells,
3,170,304 faces), vertices jittered by 10% of h (seed 2), slip walls, Euler,
gamma 1.4, (rho, p) = (1, 10) inside r < 0.1 and (1, 0.1) outside, at rest,
third-order MR-WENO with its nonlinear weights and positivity fallback
active, CFL 0.5, FP64.  One "step" is the whole hot path: the CFL time step,
then both stages (slopes, MR-WENO reconstruction, gas-kinetic face fluxes,
cell update), all on the device.  The state lives in HBM before the timed
region starts.

Prints one JSON line: cell-stage-updates/s over an uninstrumented timed
region; the roofline of the dominant kernel (per-kernel durations from HIP
events that the library records on its stream around each kernel, over the
same number of steps right after the timed region; executed FP64 work and
HBM traffic from the committed rocprofv3 counter summaries of the same
kernel sources); the device's measured copy bandwidth; the FP32-bulk form on
the same workload; the blast run to t = 0.2 in both precisions (density L1
of FP32-bulk against FP64, mass and energy drift, fallback counts); the
viscous Taylor-Green vortex (196,608 cells: throughput, kinetic-energy decay,
FP32-bulk error); the differentiation form (adjoint / forward time, central
differences, and the 3,072-cell check against the oracle's tangent build);
the lid-driven cavity (no-slip isothermal walls, smooth-flow flux); flow past
a sphere on a cubed-sphere shell (1.77M cells, quadratic slip wall and far
field: throughput, and 2,000 steps with drag and entropy error beside the
same mesh with straight wall faces); and
the FP64 CPU oracle timed on a bounded sample of the headline workload.
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
# the survey's algorithmic estimate of the flux's FP64 work per face (4-5k
# FLOP per Gauss point, three Gauss points), beside the executed count
FLUX_ALGORITHMIC_FLOP_PER_FACE = 13.5e3

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

# rocprofv3 names of the FP64 kernels of the headline workload (Euler, slip
# walls: interior and wall-face launches of the flux)
PROFILE_NAMES = {
    "slopes": ("gks::slopes_kernel<double>",),
    "reconstruct": ("gks::reconstruct_kernel<double>",),
    "flux_stage1": ("gks::flux_kernel<double, 0, false, false, false, false, false>",
                    "gks::flux_kernel<double, 0, false, false, true, false, false>"),
    "flux_stage2": ("gks::flux_kernel<double, 1, false, false, false, false, false>",
                    "gks::flux_kernel<double, 1, false, false, true, false, false>"),
    "update_stage1": ("gks::update_kernel<double, 1, false>",),
    "update_stage2": ("gks::update_kernel<double, 2, false>",),
    "dt": ("gks::dt_pass1",),
}
# the kernel sources whose digest the committed counter summaries record
KERNEL_SOURCES = ("paper_2102_01366_amd/csrc/gks_kernels.hip", "paper_2102_01366_amd/csrc/gks_flux.h",
                  "paper_2102_01366_amd/csrc/gks_flux_kernel.h", "paper_2102_01366_amd/csrc/gks_device.h",
                  "paper_2102_01366_amd/csrc/gks_internal.h", "paper_2102_01366_amd/csrc/gks_m2stage.h",
                  "paper_2102_01366_amd/csrc/gks_recon_adj.h")
TRAFFIC = os.path.join(ROOT, "profiles", "blast_walls_1572864_counters.md")
VALU = os.path.join(ROOT, "profiles", "blast_walls_1572864_valu_f64.md")


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def summary_value(path, key, column):
    """A number from a committed rocprofv3 summary table under profiles/: the
    row whose first cell is `key`, the column headed `column`; None when the
    file is missing or records other kernel sources than the current ones."""
    try:
        with open(path) as fh:
            text = fh.read()
    except OSError:
        return None
    if f"`{kernel_digest()}`" not in text:
        return None
    header = None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if header is None and column in cells:
            header = cells
            continue
        if header and len(cells) == len(header) and cells[0] == key:
            return float(cells[header.index(column)].replace(",", ""))
    return None


def I_cell_volumes(mesh):
    import numpy as np
    v = mesh.xyz[mesh.tet]
    return np.abs(np.linalg.det(v[:, 1:] - v[:, :1])) / 6.0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(I, mesh, W, gW, cfg_kw, steps, serial_n):
    """The FP64 oracle, as it stands, on `steps` steps of the headline mesh
    with all of the host's OpenMP threads, and on one stage of the same
    workload at serial_n^3 x 6 cells with one thread."""
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
    out = {"value": mesh.n_cell * 2 * steps / el, "unit": "cell-stage-updates/s",
           "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{steps} step(s) = {2 * steps} stages of the full {mesh.n_cell}-cell mesh, "
                     f"{el:.1f} s on {threads} OpenMP threads"}
    if serial_n > 0:
        ms = I.kuhn_cube_mesh(serial_n, 1.0, 0.1, 2, False)
        Ws, gWs = I.blast_cell_averages(ms)
        so = oracle.Oracle(ms, oracle.make_config(**cfg_kw))
        dts = so.compute_dt(Ws, 0.5)
        oracle.set_threads(1)
        t0 = time.perf_counter()
        so.stage(1, dts, Ws, gWs)
        el1 = time.perf_counter() - t0
        oracle.set_threads(threads)
        out["serial"] = {"value": ms.n_cell / el1, "unit": "cell-stage-updates/s", "cores": 1,
                         "sample": f"stage 1 of one step of the same workload on {serial_n}^3 x 6 = "
                                   f"{ms.n_cell} cells, {el1:.1f} s on 1 thread"}
    return out


def adjoint_leg(G, I, mesh, W, gW, cfg_kw, nsteps, ndir, precision):
    """Differentiation form on the Taylor-Green mesh: J = kinetic energy after
    `nsteps` CFL steps (time steps of an undifferentiated run, then fixed);
    dJ/d(W0, grad W0) by the discrete adjoint through the autograd rollout.
    Times one forward pass of plain steps and the adjoint pass, and checks
    the gradient against central differences along `ndir` seeded directions
    (inputs.rms_directions, seed 4): in the paper's configuration (steps
    1e-6 and 1e-7), and with the step map made smooth (no collision-time
    jump, WENO eps = 1; step 1e-6)."""
    import numpy as np
    import torch
    from paper_2102_01366_amd.autograd import rollout, time_steps
    dev = "cuda:0"
    vol = torch.from_numpy(I_cell_volumes(mesh)).to(dev)
    W0, G0 = torch.from_numpy(W).to(dev), torch.from_numpy(gW).to(dev)

    def ke(Wx):
        return (vol * 0.5 * (Wx[1] ** 2 + Wx[2] ** 2 + Wx[3] ** 2) / Wx[0]).sum()

    def gradient(s, dts):
        Wr, Gr = W0.clone().requires_grad_(True), G0.clone().requires_grad_(True)
        J = ke(rollout(s, Wr, Gr, dts)[0])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        return Wr.grad.detach(), Gr.grad.detach(), time.perf_counter() - t1

    def fd_check(s, dts, gW_, gG_, steps_eps, order=2):
        """central differences (f(e) - f(-e)) / 2e, or with order 4
        (8 (f(e) - f(-e)) - (f(2e) - f(-2e))) / 12e, against the adjoint"""
        dW, dG = I.rms_directions(W, gW, ndir, 4)
        errs = {e: [] for e in steps_eps}

        def J(vW, vG, e):
            with torch.no_grad():
                return ke(rollout(s, W0 + e * vW, G0 + e * vG, dts)[0]).item()
        for k in range(ndir):
            vW, vG = torch.from_numpy(dW[k]).to(dev), torch.from_numpy(dG[k]).to(dev)
            ad = ((gW_ * vW).sum() + (gG_ * vG).sum()).item()
            for eps in steps_eps:
                if order == 2:
                    fd = (J(vW, vG, eps) - J(vW, vG, -eps)) / (2 * eps)
                else:
                    fd = (8 * (J(vW, vG, eps) - J(vW, vG, -eps)) - (J(vW, vG, 2 * eps) - J(vW, vG, -2 * eps))) / (12 * eps)
                errs[eps].append(abs(fd - ad) / abs(ad))
        return [{"eps": eps, "order": order, "max_rel_err": max(e), "median_rel_err": float(np.median(e))}
                for eps, e in errs.items()]

    s = G.Solver(mesh, G.default_config(precision=precision, **cfg_kw), device=dev)
    dts = time_steps(s, W0, G0, 0.5, nsteps)
    s.init(W0, G0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for dt in dts:
        s.step(dt)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    # one step forward and back first, so that loading the reverse kernels and
    # allocating the adjoint workspace fall outside the timed pass
    gradient(s, dts[:1])
    gWa, gGa, t_adj = gradient(s, dts)
    out = {"steps": nsteps, "objective": "kinetic energy sum |Omega| |rho U|^2 / (2 rho) at the final time",
           "forward_ms_per_step": t_fwd / nsteps * 1e3, "adjoint_ms_per_step": t_adj / nsteps * 1e3,
           "adjoint_over_forward": t_adj / t_fwd,
           "checkpoint_bytes": nsteps * 20 * 8 * mesh.n_cell}
    if ndir:
        # the jump term |p_l - p_r| and the WENO indicators' |.| are kinks: a
        # difference whose step straddles one measures a secant
        out["fd_directions"] = ndir
        out["fd"] = fd_check(s, dts, gWa, gGa, (1e-6, 1e-7))
        sm = G.Solver(mesh, G.default_config(precision=precision, **dict(cfg_kw, c_tau=0.0, eps_weno=1.0)),
                      device=dev)
        gWs, gGs, _ = gradient(sm, dts)
        out["fd_smooth_map"] = {"config": "collision-time jump off (C = 0), WENO eps = 1",
                                "checks": fd_check(sm, dts, gWs, gGs, (1e-6,)) + fd_check(sm, dts, gWs, gGs, (1e-5,), 4)}
    return out, (gWa, gGa)


def tangent_reference_leg(G, I):
    """The FP64 CPU reference gradient: the oracle's tangent build's
    directional derivatives of the 50-step kinetic energy on the 3,072-cell
    unit cube (tests/golden/adjoint_tangent_c0.json, written from the oracle
    alone), against the GPU adjoint; beside them, central differences of the
    GPU forward map along the same directions, and the oracle's count of
    kinks within 1e-6 along each direction."""
    import numpy as np
    import torch
    from paper_2102_01366_amd.autograd import rollout
    path = os.path.join(ROOT, "tests", "golden", "adjoint_tangent_c0.json")
    with open(path) as fh:
        gold = json.load(fh)
    dev = "cuda:0"
    ell = 1.0 / (2.0 * math.pi)
    m = I.kuhn_cube_mesh(8, 1.0, 0.1, 0, True)
    W, gW = I.cell_averages(m, I.taylor_green_field(mach=0.1, ell=ell))
    vol = torch.from_numpy(I_cell_volumes(m)).to(dev)

    def ke(Wx):
        return (vol * 0.5 * (Wx[1] ** 2 + Wx[2] ** 2 + Wx[3] ** 2) / Wx[0]).sum()

    s = G.Solver(m, G.default_config(**gold["config"]), device=dev)
    W0, G0 = torch.from_numpy(W).to(dev), torch.from_numpy(gW).to(dev)
    Wr, Gr = W0.clone().requires_grad_(True), G0.clone().requires_grad_(True)
    ke(rollout(s, Wr, Gr, gold["dts"])[0]).backward()
    dW, dG = I.rms_directions(W, gW, gold["ndir"], gold["direction_seed"])
    ref = np.array(gold["jvp"])
    ad, fd = [], []
    for k in range(gold["ndir"]):
        vW, vG = torch.from_numpy(dW[k]).to(dev), torch.from_numpy(dG[k]).to(dev)
        ad.append(((Wr.grad * vW).sum() + (Gr.grad * vG).sum()).item())
        with torch.no_grad():
            Jp = ke(rollout(s, W0 + 1e-6 * vW, G0 + 1e-6 * vG, gold["dts"])[0]).item()
            Jm = ke(rollout(s, W0 - 1e-6 * vW, G0 - 1e-6 * vG, gold["dts"])[0]).item()
        fd.append((Jp - Jm) / 2e-6)
    ad, fd = np.array(ad), np.array(fd)
    return {"workload": gold["workload"], "steps": gold["steps"], "directions": gold["ndir"],
            "adjoint_vs_tangent_max_rel_err": float((np.abs(ad - ref) / np.abs(ref)).max()),
            "fd_1e-6_vs_tangent_rel_err": [float(x) for x in np.abs(fd - ref) / np.abs(ref)],
            "kinks_within_1e-6_jump": gold["kinks_jump"], "kinks_within_1e-6_weno": gold["kinks_weno"]}


def timed_kernels(solver, steps, reseed=None):
    """Per-kernel HIP-event durations over `steps` further steps (the events
    are recorded by the library on its stream around each kernel)."""
    solver.timing_read(reset=True)
    solver.timing_enable(True)
    el = run_steps(solver, steps, reseed)
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


# the blast becomes non-physical after about 26 steps under the paper's
# nonlinear weights as printed, so its timed runs restart from
# the initial state (a device-to-device copy) every RESEED steps
RESEED = 20


def run_steps(solver, n, reseed=None):
    """n steps of gks_step_cfl; reseed = (W0, gW0) device tensors: restart
    from them every RESEED steps (counted from the last restart)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n):
        if reseed is not None and i % RESEED == 0:
            solver.init(*reseed)
        solver.step_cfl(0.5)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def kernel_rates(kt, units, copy_gbs, flops_face):
    """Per-kernel average durations and rates from the HIP-event timings."""
    out = {}
    for k, (ms, cnt) in kt.items():
        if cnt == 0:
            continue
        avg_s = ms / cnt * 1e-3
        nbytes = BYTES_PER_UNIT[k] * units[UNIT[k]]
        e = {"avg_ms": ms / cnt, "launches": cnt, "total_ms": ms, "bytes_per_launch": nbytes,
             "hbm_GBs": nbytes / avg_s / 1e9}
        if k.startswith("flux"):
            e["fp64_flop_per_launch"] = flops_face * units["face"]
            e["fp64_TFLOPs"] = flops_face * units["face"] / avg_s / 1e12
            e["fp64_frac"] = e["fp64_TFLOPs"] / FP64_VECTOR_TFLOPS
        else:
            e["hbm_frac"] = e["hbm_GBs"] / HBM_PEAK_GBS
            e["frac_of_copy"] = e["hbm_GBs"] / copy_gbs
        out[k] = e
    return out


def blast_to_time(G, I, mesh, W, gW, t_end, compare_step=20):
    """The blast run from rest toward t_end in FP64 and FP32-bulk (CFL 0.5,
    the last step shortened to land on t_end), stopped where a cell average
    becomes non-physical: steps, time reached, density L1 of FP32-bulk
    against FP64 and the positivity-fallback cells of both after
    `compare_step` steps; at t_end also mass and energy drift and
    positivity-fallback cells."""
    import numpy as np
    import torch
    vol = I_cell_volumes(mesh)
    res = {}
    for name, prec in (("fp64", G.GKS_FP64), ("fp32_bulk", G.GKS_FP32_BULK)):
        s = G.Solver(mesh, G.default_config(precision=prec), device="cuda:0")
        s.init(W, gW)
        s0 = s.conservation_sums()
        t, n, last_good, failed, fb, extra = 0.0, 0, None, False, None, 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while t < t_end * (1 - 1e-12):
            try:
                dt = min(s.compute_dt(0.5), t_end - t)
            except G.GksError:
                failed = True  # the state of the last step is non-physical
                break
            if n == compare_step:
                # read back outside the time of the run
                torch.cuda.synchronize()
                tx = time.perf_counter()
                last_good = s.read_state()[0]
                fb = int(s.debug_reconstruct()[2].sum())
                extra += time.perf_counter() - tx
            s.step(dt)
            t += dt
            n += 1
        torch.cuda.synchronize()
        el = time.perf_counter() - t0 - extra
        r = {"steps": n, "t_reached": t, "nonphysical": failed, "wall_s": el,
             "cell_stage_updates_per_s": mesh.n_cell * 2 * n / el, "fallback_cells_at_compare_step": fb}
        if not failed:
            s1 = s.conservation_sums()
            r["mass_energy_drift"] = float(max(abs(s1[q] - s0[q]) / abs(s0[q]) for q in (0, 4)))
            r["fallback_cells"] = int(s.debug_reconstruct()[2].sum())
        res[name] = (last_good, r)
    out = {"t_end": t_end, "fp64": res["fp64"][1], "fp32_bulk": res["fp32_bulk"][1]}
    W64, W32 = res["fp64"][0], res["fp32_bulk"][0]
    if W64 is not None and W32 is not None:
        out["fp32_bulk"]["compare_step"] = compare_step
        out["fp32_bulk"]["l1_density_vs_fp64"] = float(np.sum(vol * np.abs(W32[0] - W64[0])) / np.sum(vol * W64[0]))
        out["fp32_bulk"]["max_density_diff_vs_fp64"] = float(np.abs(W32[0] - W64[0]).max())
    return out


def taylor_green_leg(G, I, n, steps, warmup, copy_gbs, ek_steps=200, ek_every=20):
    """The viscous Taylor-Green vortex on [0, 2 pi]^3, n^3 hexahedra x 6 Kuhn
    tetrahedra (196,608 cells at n = 32), 5% jitter (seed 1), Ma 0.1, Re 1600
    (mu = 1/1600), Pr 0.72, CFL 0.5: FP64 and FP32-bulk throughput over
    `steps` steps, the FP32-bulk density L1 against FP64, and the kinetic
    energy E_k(t) = sum |Omega| |rho U|^2 / (2 rho) / (2 pi)^3 every `ek_every`
    steps of a further FP64 run of `ek_steps` steps from the initial state."""
    import numpy as np
    import torch
    cfg_kw = dict(viscous=True, mu=1.0 / 1600.0, prandtl=0.72)
    mesh = I.kuhn_cube_mesh(n, 2 * math.pi, 0.05, 1, True)
    W, gW = I.cell_averages(mesh, I.taylor_green_field(gamma=1.4, mach=0.1))
    vol = I_cell_volumes(mesh)
    out = {"workload": f"viscous Taylor-Green vortex, [0,2pi]^3 periodic, {n}^3 hexes x 6 Kuhn tets "
                       f"({mesh.n_cell} cells, {mesh.n_face} faces), 5% jitter, Ma 0.1, Re 1600, Pr 0.72, CFL 0.5",
           "cells": mesh.n_cell, "faces": mesh.n_face, "steps": steps}
    finals = {}
    for name, prec in (("fp64", G.GKS_FP64), ("fp32_bulk", G.GKS_FP32_BULK)):
        s = G.Solver(mesh, G.default_config(precision=prec, **cfg_kw), device="cuda:0")
        s.init(W, gW)
        s0 = s.conservation_sums()
        run_steps(s, warmup)
        el = run_steps(s, steps)
        kt, _ = timed_kernels(s, steps)
        s1 = s.conservation_sums()
        finals[name] = s.read_state()[0]
        units = {"cell": mesh.n_cell, "face": mesh.n_face}
        out[name] = {"value": mesh.n_cell * 2 * steps / el, "unit": "cell-stage-updates/s",
                     "ms_per_step": el / steps * 1e3,
                     "conservation_drift": float(np.max(np.abs(s1 - s0) / np.abs(s0).max())),
                     "kernels_ms": {k: ms / c for k, (ms, c) in kt.items() if c}}
        if prec == G.GKS_FP64:
            # E_k(t) from the initial state
            s.init(W, gW)
            t, ek = 0.0, []
            for k in range(ek_steps + 1):
                if k % ek_every == 0:
                    Wk, _ = s.read_state()
                    ek.append([t, float(np.sum(vol * 0.5 * (Wk[1] ** 2 + Wk[2] ** 2 + Wk[3] ** 2) / Wk[0])
                                        / (2 * math.pi) ** 3)])
                if k < ek_steps:
                    s.step_cfl(0.5)
                    t += s.last_dt()
            out["kinetic_energy"] = ek
            e = np.array(ek)
            out["dissipation_rate_last"] = float(-(e[-1, 1] - e[-2, 1]) / (e[-1, 0] - e[-2, 0]))
    out["fp32_bulk"]["speedup_vs_fp64"] = out["fp32_bulk"]["value"] / out["fp64"]["value"]
    out["fp32_bulk"]["l1_density_vs_fp64"] = float(
        np.sum(vol * np.abs(finals["fp32_bulk"][0] - finals["fp64"][0])) / np.sum(vol * finals["fp64"][0]))
    return out, (mesh, W, gW, cfg_kw)


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


def sphere_leg(G, I, n, layers, steps, warmup, long_steps, viscous_steps):
    """The curved-wall workload: inviscid Mach 0.3 flow past the unit sphere
    on a cubed-sphere shell (6 panels of n x n cells, `layers` radial layers
    stretched by 1.08 out to r = 20, each hexahedron split into 6
    tetrahedra) with quadratic elements whose wall edges are arcs of the
    sphere (Sec. 2.1), slip wall, far field by Riemann invariants, impulsive
    start from the free stream rho = 1, U = (0.3, 0, 0), p = 1/gamma,
    third-order WENO, CFL 0.5.  Throughput in FP64 and FP32-bulk over
    `steps` steps; then `long_steps` FP64 steps with the quadratic wall and
    with straight wall faces on the same vertices, reporting the drag
    coefficient (the wall faces' momentum flux, the pressure force on the
    sphere, over rho U^2 pi / 2) and the entropy error s / s_inf - 1, s =
    p / rho^gamma, over the cells next to the wall and over all cells."""
    import numpy as np
    import torch
    gamma = 1.4
    mesh = I.cubed_sphere_shell(n, layers, r_out=20.0, ratio=1.08, curved=True)
    W, gW = I.uniform_state(mesh, 1.0, (0.3, 0.0, 0.0), 1.0 / gamma, gamma)
    free = tuple(W[:, 0])
    out = {"workload": f"Mach 0.3 past the unit sphere, cubed-sphere shell 6 x {n}^2 x {layers} layers "
                       f"x 6 tets ({mesh.n_cell} cells, {mesh.n_face} faces), quadratic wall faces, slip wall, "
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
        del s
    if long_steps > 0:
        kw = dict(farfield=free)
        every = max(500, long_steps // 16)
        out["long_run"] = {"steps": long_steps,
                           "quadratic_wall": sphere_long_run(G, I, mesh, W, gW, kw, 0.3, long_steps, every=every)}
        mesh.tet_mid = None
        out["long_run"]["straight_wall"] = sphere_long_run(G, I, mesh, W, gW, kw, 0.3, long_steps, every=every)
    del mesh
    out["viscous_noslip"] = sphere_viscous_leg(G, I, n, layers, steps, warmup, viscous_steps)
    return out


def sphere_viscous_leg(G, I, n, layers, steps, warmup, long_steps):
    """The viscous sphere of Sec. 5 (Re 118 on the diameter, Mach 0.2535,
    adiabatic no-slip wall) on the same quadratic shell: free stream rho = 1,
    U = (0.2535, 0, 0), p = 1/gamma, mu = rho U D / 118 with D = 2, Pr 1 (the
    paper states none), third-order WENO, CFL 0.5, impulsive start.  The
    constrained least squares of the wall cells (Sec. 4.4) take their
    equality rows at the Gauss points of the curved wall faces.  Throughput in
    FP64 and FP32-bulk over `steps` steps, then `long_steps` FP64 steps with
    the drag coefficient (pressure and viscous force on the sphere)."""
    import numpy as np
    import torch
    gamma, u = 1.4, 0.2535
    mesh = I.cubed_sphere_shell(n, layers, r_out=20.0, ratio=1.08, curved=True, wall_tag=I.FACE_NOSLIP_ADIABATIC)
    W, gW = I.uniform_state(mesh, 1.0, (u, 0.0, 0.0), 1.0 / gamma, gamma)
    kw = dict(farfield=tuple(W[:, 0]), viscous=True, mu=u * 2.0 / 118.0, prandtl=1.0)
    out = {"workload": f"Re 118, Mach 0.2535 past the unit sphere, the same shell ({mesh.n_cell} cells), "
                       f"quadratic adiabatic no-slip wall, Navier-Stokes, Pr 1, CFL 0.5",
           "cells": mesh.n_cell, "steps": steps}
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
        assert np.isfinite(s.read_state()[0]).all()
        kt, _ = timed_kernels(s, steps)
        out[name] = {"value": mesh.n_cell * 2 * steps / el, "unit": "cell-stage-updates/s",
                     "ms_per_step": el / steps * 1e3,
                     "kernels_ms": {k: ms / cnt for k, (ms, cnt) in kt.items() if cnt}}
        del s
    if long_steps > 0:
        out["long_run"] = sphere_long_run(G, I, mesh, W, gW, kw, u, long_steps, every=max(500, long_steps // 16),
                                          entropy=False, wake=True)
    return out


def sphere_long_run(G, I, mesh, W, gW, kw, u, nsteps, every=500, entropy=True, wake=False):
    """FP64 steps of the sphere flow from the free stream (speed u): time
    reached, the drag coefficient every `every` steps, the entropy errors at
    the end (`entropy`), the wake and separation measures at the end (`wake`:
    sphere_wake); stops where a cell turns non-physical."""
    import numpy as np
    import torch
    gamma = 1.4
    wall = np.nonzero((mesh.face_cell[:, 1] < 0) & (mesh.face_tag != I.FACE_FARFIELD))[0]
    wall_cells = np.unique(mesh.face_cell[wall, 0])
    s = G.Solver(mesh, G.default_config(**kw), device="cuda:0")
    s.init(W, gW)
    t, n, cd, failed = 0.0, 0, [], False
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def drag(dt):
        ft = s.debug_face_terms(dt)
        return float(ft[1, wall].sum() / (0.5 * 1.0 * u ** 2 * np.pi))

    while n < nsteps:
        try:
            s.step_cfl(0.5)
        except G.GksError:
            failed = True
            break
        t += s.last_dt()
        n += 1
        if n % every == 0 or n == nsteps:
            cd.append([n, t, drag(s.last_dt())])
            print(f"sphere long run: step {n}, t {t:.3f}, drag coefficient {cd[-1][2]:.4f}", file=sys.stderr,
                  flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    r = {"steps": n, "t_reached": t, "nonphysical": failed, "wall_s": el, "drag_coefficient": cd}
    if entropy and not failed:
        Wf = s.read_state()[0]
        rho = Wf[0]
        p = (gamma - 1.0) * (Wf[4] - 0.5 * (Wf[1] ** 2 + Wf[2] ** 2 + Wf[3] ** 2) / rho)
        e = (p / rho ** gamma) / ((1.0 / gamma) / 1.0) - 1.0
        r["entropy_error"] = {"wall_cells_rms": float(np.sqrt((e[wall_cells] ** 2).mean())),
                              "wall_cells_max": float(np.abs(e[wall_cells]).max()),
                              "all_cells_rms": float(np.sqrt((e ** 2).mean())),
                              "all_cells_max": float(np.abs(e).max())}
    if wake and not failed:
        ft = s.debug_face_terms(s.last_dt())
        side = np.hypot(ft[2, wall].sum(), ft[3, wall].sum())
        r["final"] = dict(sphere_wake(mesh, s.read_state()[0], wall_cells),
                          side_force_coefficient=float(side / (0.5 * u ** 2 * np.pi)))
    return r


def sphere_wake(mesh, W, wall_cells):
    """Measures of the flow past the unit sphere (free stream along +x) from
    cell averages at their vertex centroids: the length of the closed wake
    behind the sphere in diameters (from the rear point x = 1 to where the
    mean axial velocity of the cells within 0.15 of the downstream axis turns
    positive) and the separation angle in degrees from the front stagnation
    point (where the mean meridional velocity of the wall cells, binned by
    their polar angle in 2-degree bins, first turns against the flow beyond
    90 degrees)."""
    import numpy as np
    c = mesh.xyz[mesh.tet].mean(axis=1)
    U = W[1:4] / W[0]
    out = {}
    on_axis = (c[:, 0] > 1.0) & (np.hypot(c[:, 1], c[:, 2]) < 0.15)
    edges = np.arange(1.0, 6.0001, 0.05)
    k = np.digitize(c[on_axis, 0], edges) - 1
    ux = np.array([U[0, on_axis][k == b].mean() if np.any(k == b) else np.nan for b in range(edges.size - 1)])
    xm = 0.5 * (edges[1:] + edges[:-1])
    ok = np.isfinite(ux)
    ux, xm = ux[ok], xm[ok]
    neg = np.nonzero(ux < 0)[0]
    if neg.size and neg[0] < 4:
        b = neg[0]
        while b + 1 < ux.size and not (ux[b + 1] > 0):
            b += 1
        if b + 1 < ux.size:
            x0 = xm[b] + (xm[b + 1] - xm[b]) * (-ux[b]) / (ux[b + 1] - ux[b])
            out["wake_length_diameters"] = float((x0 - 1.0) / 2.0)
    wc = c[wall_cells]
    r = np.linalg.norm(wc, axis=1)
    phi = np.arccos(np.clip(-wc[:, 0] / r, -1.0, 1.0))          # 0 at the front stagnation point
    psi = np.arctan2(wc[:, 2], wc[:, 1])
    e_phi = np.stack([np.sin(phi), np.cos(phi) * np.cos(psi), np.cos(phi) * np.sin(psi)])
    u_phi = (U[:, wall_cells] * e_phi).sum(axis=0)
    bins = np.arange(0.0, 180.0001, 2.0)
    kb = np.digitize(np.degrees(phi), bins) - 1
    um = np.array([u_phi[kb == b].mean() if np.any(kb == b) else np.nan for b in range(bins.size - 1)])
    pm = 0.5 * (bins[1:] + bins[:-1])
    ok = np.isfinite(um)
    um, pm = um[ok], pm[ok]
    for b in range(int(np.searchsorted(pm, 90.0)), um.size - 1):
        if um[b] > 0 and um[b + 1] <= 0:
            out["separation_angle_degrees"] = float(pm[b] + (pm[b + 1] - pm[b]) * um[b] / (um[b] - um[b + 1]))
            break
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=64, help="hexahedra per side of the headline blast mesh")
    ap.add_argument("--t-end", type=float, default=0.2, help="end time of the blast run in both precisions "
                                                                 "(0 skips it)")
    ap.add_argument("--tgv-n", type=int, default=32, help="hexahedra per side of the Taylor-Green leg (0 skips it)")
    ap.add_argument("--cpu-baseline-steps", type=int, default=1)
    ap.add_argument("--cpu-serial-n", type=int, default=32,
                    help="mesh of the one-thread oracle leg: n^3 x 6 cells of the same workload (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-bulk headline leg")
    ap.add_argument("--adjoint-steps", type=int, default=50,
                    help="steps of the differentiation leg on the Taylor-Green mesh (0 skips it)")
    ap.add_argument("--adjoint-directions", type=int, default=16)
    ap.add_argument("--cavity-n", type=int, default=32,
                    help="hexahedra per side of the lid-driven cavity leg (0 skips it)")
    ap.add_argument("--cavity-steps", type=int, default=20)
    ap.add_argument("--sphere-n", type=int, default=32,
                    help="cells per panel side of the sphere leg (0 skips it)")
    ap.add_argument("--sphere-layers", type=int, default=48)
    ap.add_argument("--sphere-steps", type=int, default=20)
    ap.add_argument("--sphere-long-steps", type=int, default=2000,
                    help="FP64 steps of the sphere flow with quadratic and with straight wall faces "
                         "(drag, entropy error; 0 skips them)")
    ap.add_argument("--sphere-viscous-steps", type=int, default=2000,
                    help="FP64 steps of the viscous sphere (Re 118) from its impulsive start, with the drag "
                         "coefficient at 16 points (0 skips them)")
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

    mesh = I.kuhn_cube_mesh(args.n, 1.0, 0.1, 2, False)
    W, gW = I.blast_cell_averages(mesh)
    nc, nf = mesh.n_cell, mesh.n_face
    config = G.default_config()
    solver = G.Solver(mesh, config, device="cuda:0")
    seed = (torch.from_numpy(W).to("cuda:0"), torch.from_numpy(gW).to("cuda:0"))
    solver.init(*seed)
    sums0 = solver.conservation_sums()
    print(f"headline: blast {nc} cells, {args.warmup} + {args.steps} steps", file=sys.stderr, flush=True)

    # each step: dt = CFL bound on the device, then both stages with that dt;
    # the timed region runs uninstrumented, then the same number of steps
    # runs with HIP events around every kernel for the per-kernel durations
    run_steps(solver, args.warmup, seed)
    elapsed = run_steps(solver, args.steps, seed)
    Wf, _ = solver.read_state()
    sums1 = solver.conservation_sums()
    kt, el_instr = timed_kernels(solver, args.steps, seed)
    assert np.isfinite(Wf).all()

    copy_gbs = copy_bandwidth(torch)
    op_count = G.flux_op_count(config)["total"]
    full = args.n == 64
    # executed FP64 work of the flux kernel per face: rocprofv3 counts of the
    # FP64 add, multiply, FMA (2 FLOP) and transcendental instructions of
    # both launches per stage, times 64 lanes, over the faces
    executed = summary_value(VALU, "flux_stage1", "executed FP64 FLOP per face") if full else None
    flops_face = executed if executed is not None else op_count
    units = {"cell": nc, "face": nf}
    kernels = kernel_rates(kt, units, copy_gbs, flops_face)
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    d = kernels[dom]
    traffic = summary_value(TRAFFIC, dom, "scaled bytes per launch") if full else None
    if dom.startswith("flux"):
        roof = {"kernel": dom, "bound": "alu", "achieved": d["fp64_TFLOPs"],
                "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": d["fp64_TFLOPs"] / FP64_VECTOR_TFLOPS, "traffic": traffic,
                "work_source": ("executed FP64 FLOP from rocprofv3 counters (profiles/"
                                "blast_walls_1572864_valu_f64.md)" if executed is not None else
                                "source operation count of the flux routine (gks_flux_op_count)"),
                "work_per_launch": f"{flops_face:.0f} FP64 FLOP/face x {nf} faces",
                "executed_fp64_flop_per_face": executed, "algorithmic_fp64_flop_per_face":
                FLUX_ALGORITHMIC_FLOP_PER_FACE, "source_op_count_per_face": op_count,
                "algorithmic_frac": FLUX_ALGORITHMIC_FLOP_PER_FACE * nf / (d["avg_ms"] * 1e-3) / 1e12
                / FP64_VECTOR_TFLOPS}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": d["hbm_GBs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": d["hbm_GBs"] / HBM_PEAK_GBS, "frac_of_copy": d["frac_of_copy"],
                "traffic": traffic, "work_per_launch": f"{BYTES_PER_UNIT[dom]} B/{UNIT[dom]} x {units[UNIT[dom]]}"}
    value = nc * 2 * args.steps / elapsed
    # the flux's own roofline (both stages' kernels), beside the dominant kernel's
    f1 = kernels.get("flux_stage1")
    flux_roof = None if f1 is None else {
        "kernel": "flux_stage1", "bound": "alu", "achieved": f1["fp64_TFLOPs"], "peak": FP64_VECTOR_TFLOPS,
        "unit": "TFLOP/s", "frac": f1["fp64_TFLOPs"] / FP64_VECTOR_TFLOPS,
        "traffic": summary_value(TRAFFIC, "flux_stage1", "scaled bytes per launch") if full else None,
        "work_per_launch": f"{flops_face:.0f} FP64 FLOP/face x {nf} faces",
        "work_source": roof.get("work_source") if dom.startswith("flux") else (
            "executed FP64 FLOP from rocprofv3 counters (profiles/blast_walls_1572864_valu_f64.md)"
            if executed is not None else "source operation count of the flux routine (gks_flux_op_count)"),
        "executed_fp64_flop_per_face": executed, "algorithmic_fp64_flop_per_face": FLUX_ALGORITHMIC_FLOP_PER_FACE,
        "source_op_count_per_face": op_count}

    fp32 = None
    if not args.no_fp32:
        s32 = G.Solver(mesh, G.default_config(precision=G.GKS_FP32_BULK), device="cuda:0")
        s32.init(*seed)
        a0 = s32.conservation_sums()
        run_steps(s32, args.warmup, seed)
        el32 = run_steps(s32, args.steps, seed)
        W32, _ = s32.read_state()
        a1 = s32.conservation_sums()
        kt32, _ = timed_kernels(s32, args.steps, seed)
        vol = I_cell_volumes(mesh)
        fp32 = {"value": nc * 2 * args.steps / el32, "unit": "cell-stage-updates/s",
                "ms_per_step": el32 / args.steps * 1e3, "speedup_vs_fp64": elapsed / el32,
                "l1_density_vs_fp64_same_steps": float(np.sum(vol * np.abs(W32[0] - Wf[0])) / np.sum(vol * Wf[0])),
                "mass_energy_drift": float(max(abs(a1[q] - a0[q]) / abs(a0[q]) for q in (0, 4))),
                "dtype": "fp32 bulk / fp64 state",
                "kernels_ms": {k: ms / c for k, (ms, c) in kt32.items() if c}}
        del s32
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
        "config": {"workload": f"spherical blast with reflective walls, unit cube, {args.n}^3 hexes x 6 Kuhn tets "
                               f"({nc} cells, {nf} faces), 10% jitter (seed 2), slip walls, Euler, "
                               "(rho, p) = (1, 10) inside r < 0.1 and (1, 0.1) outside, third-order MR-WENO "
                               "with nonlinear weights and positivity fallback, CFL 0.5, FP64; the timed "
                               f"steps restart from the initial state every {RESEED} steps",
                   "cells": nc, "faces": nf, "precision": "fp64"},
        "roofline": roof,
        "flux_roofline": flux_roof,
        "hbm_copy_GBs": copy_gbs,
        "kernels": kernels,
        "mass_energy_drift": float(max(abs(sums1[q] - sums0[q]) / abs(sums0[q]) for q in (0, 4))),
        "restart_every_steps": RESEED,
        "fp32_bulk": fp32,
    }
    del solver
    torch.cuda.empty_cache()
    print("blast to t_end", file=sys.stderr, flush=True)
    out["blast_to_t_end"] = blast_to_time(G, I, mesh, W, gW, args.t_end) if args.t_end > 0 else None
    torch.cuda.empty_cache()
    tgv = None
    if args.tgv_n > 0:
        print("taylor-green", file=sys.stderr, flush=True)
        out["taylor_green"], tgv = taylor_green_leg(G, I, args.tgv_n, args.steps, args.warmup, copy_gbs)
    if args.adjoint_steps > 0 and tgv is not None:
        print("adjoint", file=sys.stderr, flush=True)
        tm, tW, tgW, tkw = tgv
        adj, g64 = adjoint_leg(G, I, tm, tW, tgW, tkw, args.adjoint_steps, args.adjoint_directions, G.GKS_FP64)
        adj32, g32 = adjoint_leg(G, I, tm, tW, tgW, tkw, args.adjoint_steps, 0, G.GKS_FP32_BULK)
        adj["fp32_bulk"] = {k: adj32[k] for k in ("forward_ms_per_step", "adjoint_ms_per_step",
                                                  "adjoint_over_forward")}
        adj["fp32_bulk"]["gradient_rel_diff_vs_fp64"] = max(
            float((a - b).abs().max() / a.abs().max()) for a, b in zip(g64, g32))
        adj["tangent_reference"] = tangent_reference_leg(G, I)
        out["adjoint"] = adj
    else:
        out["adjoint"] = None
    torch.cuda.empty_cache()
    print("cavity, sphere", file=sys.stderr, flush=True)
    out["cavity_noslip"] = cavity_leg(G, I, args.cavity_n, args.cavity_steps, 2) if args.cavity_n > 0 else None
    out["sphere_farfield"] = (sphere_leg(G, I, args.sphere_n, args.sphere_layers, args.sphere_steps, 1,
                                         args.sphere_long_steps, args.sphere_viscous_steps)
                              if args.sphere_n > 0 else None)
    if not args.no_cpu_baseline:
        print("cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(I, mesh, W, gW, {}, args.cpu_baseline_steps, args.cpu_serial_n)
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
