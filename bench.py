#!/usr/bin/env python3
"""Throughput benchmark of the coupled level-set lattice Boltzmann step on
one MI355X.

Workload: D3Q27 512^3 stratified liquid/gas layer with the wavy interface
z = 256 + 8 sin(2 pi x/512) cos(2 pi y/512), periodic x/y, no-slip z,
density ratio 1000, viscosity ratio 50, sigma 1e-3 (synthetic, built from
the problem statement; no dataset).  One "step" is the whole hot path:
collide-stream with wall and interface bounce-back, velocity extension,
RK3 advection, reinitialisation every 10 steps, classification, geometry,
refill.  Each storage mode (FP16-deviation, FP32, FP64) runs W untimed
warm-up steps and K timed steps bracketed by device synchronisation.

Prints one JSON line: the headline value is whole-step MLUPS of the
FP16-deviation storage path (FP32 arithmetic); the FP32/FP64 paths are in
"modes".  "roofline" refers to the dominant kernel (the bulk
collide-stream kernel) timed with HIP events on its own stream.
"cpu_baseline" times the CPU oracle on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# HBM bytes per launch of the bulk collide-stream kernel from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs, scaled by a plain 4 GiB copy; recorded in
# profiles/k_lb_bulk_wavy512_d3q27_f16dev_hbm_traffic.md with the hash of the
# sources that kernel is built from.  Reported only while those sources hash
# to the same value (null once any of them has changed).
MEASURED_TRAFFIC = {"sources": "e8f6b8909ef82b58", ("f16dev", "serial", 512): 15874179019}


def kernel_sources() -> list:
    """What the D3Q27 kernels and their launches are built from: the D3Q27
    translation unit and the plan set-up with every header they include,
    and the build flags (paths relative to the repository root)."""
    import re
    d = os.path.join(ROOT, "paper_2601_05936_amd", "csrc")
    pending = [os.path.join(d, "lsb_d3q27.hip"), os.path.join(d, "api.hip")]
    seen = []
    while pending:
        f = os.path.normpath(pending.pop())
        if f in seen:
            continue
        seen.append(f)
        for inc in re.findall(r'^#include "([^"]+)"', open(f).read(), flags=re.M):
            pending.append(os.path.join(os.path.dirname(f), inc))
    seen.append(os.path.join(ROOT, "paper_2601_05936_amd", "build.py"))
    return sorted(os.path.relpath(f, ROOT) for f in seen)


def kernel_sources_hash() -> str:
    """sha256 (first 16 hex digits) of kernel_sources()."""
    import hashlib
    h = hashlib.sha256()
    for f in kernel_sources():
        h.update(f.encode())
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(key):
    if MEASURED_TRAFFIC.get("sources") != kernel_sources_hash():
        return None
    return MEASURED_TRAFFIC.get(key)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_mode(size, storage, steps, warmup, schedule, cumulant_gas=False, workload="wavy"):
    import torch

    from paper_2601_05936_amd import workloads as W
    from paper_2601_05936_amd.lsb import Sim

    t0 = time.time()
    if workload == "cluster9":
        # nine rising bubbles, one gas baseline each (32 cells per diameter)
        w = W.nine_bubble_cluster_3d(d=32, storage=storage)
        p = w["params"]
        phi0 = torch.from_numpy(w["phi0"]).to("cuda:0")
    else:
        w = W.wavy_stratified_3d(n=size, storage=storage)
        p = w["params"]
        if cumulant_gas:
            p["collision"] = [W.BGK, W.CUMULANT]
        phi0 = torch.from_numpy(W.wavy_phi(p, 8.0 * size / 512.0)).to("cuda:0")
    s = Sim(p).set_schedule(schedule).init(phi0)
    del phi0
    torch.cuda.synchronize()
    log(f"[{storage}] init {time.time() - t0:.1f}s workspace {s.workspace_bytes / 2**30:.1f} GiB")
    s.step(warmup)
    torch.cuda.synchronize()
    s.set_kernel_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    k_ms, k_n = s.kernel_timing()
    s.set_kernel_timing(False)
    k_ms_sched = k_ms / max(k_n, 1)
    if schedule:
        # the bulk kernel alone: a few more steps in the serial schedule (the
        # schedules give the same state bit for bit, so switching at a step
        # boundary changes nothing but the timing)
        from paper_2601_05936_amd.lsb import SCHED_OVERLAP, SCHED_SERIAL
        s.set_schedule(SCHED_SERIAL)
        s.step(1)
        torch.cuda.synchronize()
        s.set_kernel_timing(True)
        s.step(max(3, steps // 4))
        torch.cuda.synchronize()
        k_ms, k_n = s.kernel_timing()
        s.set_kernel_timing(False)
        s.set_schedule(SCHED_OVERLAP)
    counts = s.counts()
    I = s.integrals()
    N = s.N
    Q = s.Q
    b = {0: 8, 1: 4, 2: 2, 3: 2}[storage]
    k_avg_ms = k_ms / max(k_n, 1)
    # cells updated by the bulk collide-stream kernel: all but the interface
    # and wall cells (serial) and also all but the LS-active tiles (overlap);
    # in this workload the band (mid-height) and the z walls are disjoint
    bulk_cells = N - counts["wall_cells"] - counts["iface_cells"]  # the serial schedule's bulk kernel
    # algorithmic bytes of one bulk launch: read Q and write Q populations of
    # every bulk cell, read one tag byte per cell
    alg_bytes = bulk_cells * 2 * Q * b + N
    achieved = alg_bytes / (k_avg_ms * 1e-3) / 1e9
    res = dict(
        mlups=N * steps / (ms * 1e-3) / 1e6,
        ms_per_step=ms / steps,
        k1_ms=k_avg_ms,
        k1_mlups=N / (k_avg_ms * 1e-3) / 1e6,
        k1_gbs=achieved,
        k1_frac=achieved / HBM_PEAK_GBS,
        k1_launches=k_n,
        k1_schedule="serial",
        k1_ms_in_step_schedule=k_ms_sched,
        alg_bytes_per_launch=alg_bytes,
        bytes_per_cell=2 * Q * b + 1,
        iface_cells=counts["iface_cells"],
        wall_cells=counts["wall_cells"],
        active_tiles=counts["active_tiles"],
        mass=[float(m) for m in I["mass"]],
        umax=float(I["umax"]),
        workload=w["name"],
        cells=N,
    )
    if p["use_pb"] == 2:
        res["bubbles"] = s.bubbles()["count"]
    log(f"[{storage}] {res}")
    del s
    torch.cuda.empty_cache()
    return res


def run_adjoint(steps: int, every: int):
    """Reverse mode on the differentiation workload (256x512 D2Q9 rising
    bubble, FP32 state, FP64 adjoints): forward with checkpoints, then the
    backward pass (segment recompute with recording, reverse)."""
    import numpy as np
    import torch

    from paper_2601_05936_amd import workloads as W
    from paper_2601_05936_amd.adjoint import _run_forward, reverse_centroid
    w = W.rising_bubble_2d(storage=W.F32)
    p = w["params"]
    phi0 = torch.as_tensor(np.ascontiguousarray(w["phi0"]).reshape(-1)).to("cuda:0")
    N = p["nx"] * p["ny"]
    torch.cuda.synchronize()
    t0 = time.time()
    sim, ckpts = _run_forward(p, p["sigma"], phi0, steps, every)
    L = float(sim.integrals()["centroid"][1])
    torch.cuda.synchronize()
    t1 = time.time()
    dphi0, dsig = reverse_centroid(sim, ckpts, steps, every, 1, phi0)
    torch.cuda.synchronize()
    t2 = time.time()
    res = dict(workload=w["name"], steps=steps, checkpoint_every=every, loss_centroid_y=L, dL_dsigma=dsig,
               dL_dphi0_max=float(dphi0.abs().max()), forward_s=t1 - t0, backward_s=t2 - t1,
               adjoint_mlups=N * steps / (t2 - t1) / 1e6, forward_backward_mlups=N * steps / (t2 - t0) / 1e6)
    log(f"[adjoint] {res}")
    return res


def run_refine(steps: int, warmup: int):
    """Two-level static refinement (D2Q9, BGK, FP64, ratio 2): 2048^2 coarse
    nodes, periodic, with a fine patch over the coarse nodes [512, 1536]^2
    (2049^2 fine nodes, two fine steps per coarse step); synthetic smooth
    shear and density fields.  Node updates per second and the whole step's
    rate against 144 algorithmic bytes per node update (9 FP64 populations
    read and written)."""
    import numpy as np
    import torch

    from paper_2601_05936_amd.lsb import Refine
    n, patch, tau_c = 2048, (512, 1536, 512, 1536), 0.6
    g = Refine(n, n, patch, tau_c, max_extent=(1200, 1200, 0))
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    def fields(x, y):
        s = np.sin(2 * np.pi * y / n)
        return 1.0 + 0.005 * np.cos(2 * np.pi * x / n), np.stack([0.02 * s, 0.01 * np.sin(2 * np.pi * x / n)], 1)
    rc, uc = fields(I.reshape(-1).astype(float), J.reshape(-1).astype(float))
    ia, ib, ja, jb = patch
    jf, i_f = np.meshgrid(np.arange(g.my + 1), np.arange(g.mx + 1), indexing="ij")
    rf, uf = fields(ia + 0.5 * i_f.reshape(-1), ja + 0.5 * jf.reshape(-1))
    g.init(rc, uc, rf, uf)
    g.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    covered = (ib - ia - 1) * (jb - ja - 1)
    updates = (n * n - covered) + 2 * g.n_fine
    gbs = updates * 144 / (ms * 1e-3) / 1e9
    # the level-set sensor on a gas disk that moves by 16 coarse nodes per
    # call, and the re-meshing onto its box (the paper re-meshes every 50
    # steps): timed per call, alternating between two positions
    phis = [torch.as_tensor((400.0 - np.hypot(I - (1024.0 + dx), J - 1024.0)).reshape(-1)).to("cuda:0")
            for dx in (0.0, 16.0)]
    torch.cuda.synchronize()
    t0 = time.time()
    for r in range(6):
        box = g.sensor(phis[r % 2], 80.0, 4)
        g.remesh(box)
    torch.cuda.synchronize()
    remesh_ms = (time.time() - t0) / 6 * 1e3
    res = dict(workload="D2Q9 two-level static refinement, 2048^2 coarse, patch [512,1536]^2 (2049^2 fine)",
               steps=steps, warmup=warmup, ms_per_step=ms, node_updates_per_step=updates,
               mlups=updates / (ms * 1e-3) / 1e6, gbs=gbs, frac=gbs / HBM_PEAK_GBS, bytes_per_update=144,
               dtype="f64", sensor_remesh_ms=remesh_ms, sensor_remesh_box=list(box),
               sensor_remesh_ms_per_step_every_50=remesh_ms / 50)
    log(f"[refine] {res}")
    return res


def run_refine3d(steps: int, warmup: int):
    """The same two-level refinement in 3D: D3Q27, 192^3 coarse nodes with a
    fine patch over [48, 144]^3 (193^3 fine nodes); synthetic smooth
    fields.  Node updates per second and the whole step's rate against
    27 x 16 = 432 algorithmic bytes per node update."""
    import numpy as np
    import torch

    from paper_2601_05936_amd.lsb import D3Q27, Refine
    n, patch, tau_c = 192, (48, 144, 48, 144, 48, 144), 0.6
    g = Refine(n, n, patch, tau_c, lattice=D3Q27, nz=n)

    def fields(x, y, z):
        return (1.0 + 0.005 * np.cos(2 * np.pi * x / n),
                np.stack([0.02 * np.sin(2 * np.pi * y / n), 0.01 * np.sin(2 * np.pi * z / n),
                          0.01 * np.sin(2 * np.pi * x / n)], 1))
    K, J, I = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    rc, uc = fields(I.reshape(-1).astype(float), J.reshape(-1).astype(float), K.reshape(-1).astype(float))
    k, j, i = np.meshgrid(np.arange(g.mz + 1), np.arange(g.my + 1), np.arange(g.mx + 1), indexing="ij")
    rf, uf = fields(48 + 0.5 * i.reshape(-1), 48 + 0.5 * j.reshape(-1), 48 + 0.5 * k.reshape(-1))
    g.init(rc, uc, rf, uf)
    del K, J, I, k, j, i, rc, uc, rf, uf
    g.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    updates = (n ** 3 - 95 ** 3) + 2 * g.n_fine
    gbs = updates * 432 / (ms * 1e-3) / 1e9
    res = dict(workload="D3Q27 two-level static refinement, 192^3 coarse, patch [48,144]^3 (193^3 fine)",
               steps=steps, warmup=warmup, ms_per_step=ms, node_updates_per_step=updates,
               mlups=updates / (ms * 1e-3) / 1e6, gbs=gbs, frac=gbs / HBM_PEAK_GBS, bytes_per_update=432,
               dtype="f64")
    log(f"[refine3d] {res}")
    return res


def run_two_phase_levels(steps: int, warmup: int):
    """The two-phase step on two levels against the uniform grid.  Uniform:
    the D3Q27 rising bubble 128x128x256 (d = 32, Eo 10, Mo 1e-3, density
    ratio 1000, viscosity ratio 100, FP16-deviation storage, container
    walls), 2 steps per coarse step.  Two levels: the same physics in coarse
    units (tau_c = (tau_f + 1/2) / 2, sigma_c = sigma_f / 2, a_c = 2 a_f) on
    64x64x128 coarse nodes (periodic: the two-level path has no coarse walls)
    and the bubble (R = 16 fine cells) on the fine level of a box of coarse
    nodes [18, 46]^2 x [10, 48] (57 x 57 x 77 fine nodes, FP16-deviation),
    re-meshed every 50 coarse steps (the level-set sensor at d_ref = 6 fine
    cells moves the box; the sensor and the re-mesh are in the timed
    region); the coarse grid is FP64."""
    import torch

    from paper_2601_05936_amd import workloads as W
    from paper_2601_05936_amd.lsb import Sim, TwoPhaseRefine, SCHED_SERIAL
    wu = W.rising_bubble_3d(storage=W.F16DEV)
    pu = wu["params"]
    s = Sim(pu).set_schedule(SCHED_SERIAL).init(wu["phi0"])
    s.step(2 * warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(2 * steps)
    e1.record()
    torch.cuda.synchronize()
    ms_uniform = e0.elapsed_time(e1) / steps  # two fine steps
    n_uniform = s.N
    del s
    torch.cuda.empty_cache()
    tau_c = [(t + 0.5) / 2.0 for t in pu["tau"]]
    g_c = 2.0 * (-pu["accel"][0][2])
    w = W.two_level_bubble(lattice=W.D3Q27, n=(64, 64, 128), box=(18, 46, 18, 46, 10, 48),
                           centre=(32.0, 32.0, 24.0), radius=8.0, rho_ratio=1.0 / pu["rho_phys"][1], tau=tau_c,
                           sigma=pu["sigma"] / 2.0, g=g_c, storage=W.F16DEV)
    r = TwoPhaseRefine(w["params"], w["box"]).init(*[w[k] for k in ("phi_c", "rho_c", "u_c", "phi_f", "rho_f",
                                                                     "u_f")])
    r.step(warmup)
    torch.cuda.synchronize()
    remeshes = 0
    e0.record()
    done = 0
    while done < steps:
        k = min(50, steps - done)
        r.step(k)
        done += k
        if k == 50:
            nb = r.sensor(6.0)
            remeshes += tuple(nb) != tuple(r.current_box)
            r.remesh(nb)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nc = r.n_coarse
    nf = r.n_fine
    b = w["box"]
    covered = (b[1] - b[0] - 1) * (b[3] - b[2] - 1) * (b[5] - b[4] - 1)
    updates = (nc - covered) + 2 * nf
    I = r.fine.integrals()
    res = dict(workload="D3Q27 two-phase step on two levels: 64x64x128 coarse (periodic), bubble R = 16 fine "
                        "cells on a 57x57x77 fine box re-meshed every 50 coarse steps, FP16-deviation fine storage, "
                        "FP64 coarse; against the uniform 128x128x256 rising bubble (FP16-deviation), two fine "
                        "steps per coarse step",
               steps=steps, warmup=warmup, ms_per_coarse_step=ms, node_updates_per_step=updates,
               mlups=updates / (ms * 1e-3) / 1e6, fine_equivalent_mlups=2 * n_uniform / (ms * 1e-3) / 1e6,
               uniform_ms_per_two_steps=ms_uniform, uniform_mlups=2 * n_uniform / (ms_uniform * 1e-3) / 1e6,
               speedup_vs_uniform=ms_uniform / ms, fine_nodes=nf, coarse_nodes=nc, remesh_every=50,
               boxes_moved=remeshes, box=list(r.current_box),
               fine_volume_gas=float(I["volume_gas"]), dtype="f32 (fine, FP16-deviation storage) / f64 (coarse)")
    log(f"[two-phase levels] {res}")
    del r
    torch.cuda.empty_cache()
    return res


def run_refine_nested(steps: int, warmup: int):
    """Three nested levels (D2Q9, BGK, FP64, ratio 2 at each jump): 2048^2
    coarse nodes, periodic; level 1 over the coarse nodes [512, 1536]^2
    (2049^2 nodes); level 2 over level 1's nodes [512, 1536]^2 (2049^2
    nodes at a quarter of the coarse spacing, four steps per coarse step);
    synthetic smooth shear and density fields.  Node updates per second and
    the whole step's rate against 144 algorithmic bytes per node update
    (covered nodes are not updated)."""
    import numpy as np
    import torch

    from paper_2601_05936_amd.lsb import Refine
    n, box, tau_c = 2048, (512, 1536, 512, 1536), 0.6
    g = Refine(n, n, [box, box], tau_c)

    def fields(x, y):
        s = np.sin(2 * np.pi * y / n)
        return 1.0 + 0.005 * np.cos(2 * np.pi * x / n), np.stack([0.02 * s, 0.01 * np.sin(2 * np.pi * x / n)], 1)
    args = []
    ox, oy, h = 0.0, 0.0, 1.0
    for lv in range(3):
        if lv:
            ox, oy, h = ox + h * box[0], oy + h * box[2], 0.5 * h
        sx, sy, _ = g.shape(lv)
        J, I = np.meshgrid(np.arange(sy), np.arange(sx), indexing="ij")
        args += list(fields(ox + h * I.reshape(-1), oy + h * J.reshape(-1)))
    g.init(*args)
    del args
    g.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    cov = (box[1] - box[0] - 1) * (box[3] - box[2] - 1)
    updates = (n * n - cov) + 2 * (g.n_level(1) - cov) + 4 * g.n_level(2)
    gbs = updates * 144 / (ms * 1e-3) / 1e9
    res = dict(workload="D2Q9 three-level static refinement, 2048^2 coarse, level 1 [512,1536]^2 (2049^2), "
                        "level 2 [512,1536]^2 of level 1 (2049^2)",
               steps=steps, warmup=warmup, ms_per_step=ms, node_updates_per_step=updates,
               mlups=updates / (ms * 1e-3) / 1e6, gbs=gbs, frac=gbs / HBM_PEAK_GBS, bytes_per_update=144,
               dtype="f64")
    log(f"[refine_nested] {res}")
    return res


def run_refine_tree(steps: int, warmup: int):
    """A tree of boxes (D2Q9, BGK, FP64): 2048^2 coarse nodes, periodic, with
    nine disjoint 200^2-cell boxes on a 3 x 3 lattice (401^2 nodes each, as
    around a cluster of nine bubbles); synthetic smooth shear and density
    fields.  Node updates per second and the whole step's rate against 144
    algorithmic bytes per node update (covered nodes are not updated)."""
    import numpy as np
    import torch

    from paper_2601_05936_amd.lsb import Refine
    n, tau_c = 2048, 0.6
    boxes = [(224 + 600 * a, 424 + 600 * a, 224 + 600 * b, 424 + 600 * b) for b in range(3) for a in range(3)]
    g = Refine(n, n, boxes, tau_c, parents=[0] * 9)

    def fields(x, y):
        s = np.sin(2 * np.pi * y / n)
        return 1.0 + 0.005 * np.cos(2 * np.pi * x / n), np.stack([0.02 * s, 0.01 * np.sin(2 * np.pi * x / n)], 1)
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    args = list(fields(I.reshape(-1).astype(float), J.reshape(-1).astype(float)))
    for bx in boxes:
        sx, sy, _ = g.shape(1)
        jj, ii = np.meshgrid(np.arange(sy), np.arange(sx), indexing="ij")
        args += list(fields(bx[0] + 0.5 * ii.reshape(-1), bx[2] + 0.5 * jj.reshape(-1)))
    g.init(*args)
    del args
    g.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    updates = (n * n - 9 * 199 * 199) + 2 * 9 * g.n_level(1)
    gbs = updates * 144 / (ms * 1e-3) / 1e9
    # one adaptive cycle per call: the seeded sensor on nine gas disks (one
    # seed each, at the boxes' centres) moving by 8 coarse nodes between
    # calls, and the re-meshing of the tree onto its boxes
    seeds = [((b[0] + b[1]) // 2, (b[2] + b[3]) // 2) for b in boxes]
    phis = [torch.as_tensor(np.max([90.0 - np.hypot(I - (sx + dx), J - sy) for sx, sy in seeds], axis=0).reshape(-1))
            .to("cuda:0") for dx in (0.0, 8.0)]
    torch.cuda.synchronize()
    t0 = time.time()
    for r in range(6):
        nb = g.sensor_seeded(phis[r % 2], 4.0, 6, seeds)
        if len(nb) != len(g.boxes):
            raise RuntimeError(f"the seeded sensor merged boxes ({len(nb)} for {len(g.boxes)}): the tree needs rebuilding")
        g.remesh_levels(nb)
        # the first coarse step after a re-mesh captures the step graphs again
        g.step(1)
    torch.cuda.synchronize()
    cycle_ms = (time.time() - t0) / 6 * 1e3 - ms  # sensor + re-mesh + re-capture, beyond a plain step
    res = dict(workload="D2Q9 refinement tree, 2048^2 coarse, nine 200^2-cell boxes (401^2 nodes each)",
               steps=steps, warmup=warmup, ms_per_step=ms, node_updates_per_step=updates,
               mlups=updates / (ms * 1e-3) / 1e6, gbs=gbs, frac=gbs / HBM_PEAK_GBS, bytes_per_update=144,
               launches_per_step=1 + 9 * 3, dtype="f64", sensor_remesh_recapture_ms=cycle_ms,
               sensor_remesh_boxes=[list(b) for b in nb])
    log(f"[refine_tree] {res}")
    return res


def cpu_baseline(seconds: float):
    """The CPU oracle (as it stands) on a bounded sample of the workload:
    the same problem at 128^3 (interface amplitude scaled to 2)."""
    import oracle as O
    from paper_2601_05936_amd import workloads as W

    n = 128
    w = W.wavy_stratified_3d(n=n, storage=W.F64)
    p = w["params"]
    phi = W.wavy_phi(p, 8.0 * n / 512.0)
    threads = os.environ.get("OMP_NUM_THREADS")
    o = O.Oracle(p, phi)
    t0 = time.time()
    o.step(1)
    t1 = time.time() - t0
    extra = max(0, int(seconds / max(t1, 1e-3)) - 1)
    t0 = time.time()
    if extra:
        o.step(extra)
    t = time.time() - t0
    steps = extra if extra else 1
    if not extra:
        t = t1
    return dict(value=n ** 3 * steps / t / 1e6, unit="MLUPS", cores=int(threads) if threads else os.cpu_count(),
                kind="oracle", sample=f"D3Q27 wavy stratified 128^3 (amplitude 2), {steps} FP64 steps after 1 warm-up step")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--modes", default="f16dev,f32,f64,f16dev-cum,cluster9",
                    help="storage modes; a '-cum' suffix runs the gas phase with the cumulant collision "
                         "(the paper's 3D pairing: BGK liquid, cumulant gas); 'cluster9' is the nine-bubble "
                         "cluster (320x640x320, FP16-deviation, cumulant gas, one gas baseline per bubble)")
    ap.add_argument("--schedule", default="auto", choices=["auto", "serial", "overlap"],
                    help="step schedule: one stream, the bulk collide-stream overlapped on a second stream, or "
                         "auto (the faster on this workload, measured: serial for FP16-deviation storage, overlap "
                         "for FP32 and FP64)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--adjoint-steps", type=int, default=2000, help="reverse-mode run length (0: skip)")
    ap.add_argument("--refine-steps", type=int, default=100,
                    help="refinement run length in coarse steps: two-level 2D and 3D legs, three-level "
                         "2D leg, nine-box 2D tree (0: skip)")
    ap.add_argument("--refine-legs", default="2d,3d,nested,tree,twophase",
                    help="refinement legs to run: 2d, 3d (two levels), nested (three levels), tree (nine boxes), "
                         "twophase (the two-phase step on two levels against the uniform rising bubble)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="also run a plain device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_2601_05936_amd.lsb import SCHED_OVERLAP, SCHED_SERIAL
    from paper_2601_05936_amd.workloads import F16DEV, F32, F64
    def sched_of(mode):
        if args.schedule == "auto":
            return "serial" if mode.startswith("f16dev") else "overlap"
        return args.schedule
    names = {"f16dev": F16DEV, "f32": F32, "f64": F64}
    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    results = {}
    for m in modes:
        if m == "cluster9":
            sm = "serial" if args.schedule == "auto" else args.schedule
            results[m] = run_mode(args.size, F16DEV, args.steps, args.warmup,
                                  SCHED_OVERLAP if sm == "overlap" else SCHED_SERIAL, workload="cluster9")
            results[m]["schedule"] = sm
            results[m]["collision"] = "BGK liquid, cumulant gas"
            continue
        sm = sched_of(m)
        base, cum = (m[:-4], True) if m.endswith("-cum") else (m, False)
        results[m] = run_mode(args.size, names[base], args.steps, args.warmup,
                              SCHED_OVERLAP if sm == "overlap" else SCHED_SERIAL, cumulant_gas=cum)
        results[m]["schedule"] = sm
        results[m]["collision"] = "BGK liquid, cumulant gas" if cum else "BGK"
    if args.copy_calibration > 0:
        nbytes = int(args.copy_calibration * 2**30)
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read and written")
        del a, b
    head = modes[0]
    r = results[head]
    out = {
        "metric": "MLUPS + HBM GB/s (% peak), FP16-storage vs FP32 vs FP64 on 1 GPU; adjoint MLUPS",
        "value": r["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head.startswith("f64") else "f32",
        "data": "synthetic",
        "config": {"workload": f"D3Q27 wavy stratified {args.size}^3, periodic x/y, no-slip z, density ratio 1000, "
                               f"viscosity ratio 50, sigma 1e-3 (throughput configuration)",
                   "storage": head, "cells": args.size ** 3, "schedule": sched_of(head),
                   "collision": results[head]["collision"]},
        "modes": results,
        "roofline": {"bound": "hbm", "achieved": r["k1_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["k1_frac"], "traffic": measured_traffic((head, "serial", args.size)),
                     "kernel_sources": kernel_sources_hash(),
                     "kernel": "k_lb_bulk (collide-stream, bulk cells)",
                     "bytes_per_cell": r["bytes_per_cell"], "alg_bytes_per_launch": r["alg_bytes_per_launch"],
                     "avg_ms": r["k1_ms"]},
    }
    if args.adjoint_steps > 0:
        out["adjoint"] = run_adjoint(args.adjoint_steps, 100)
    if args.refine_steps > 0:
        legs = {"2d": ("refine", run_refine), "3d": ("refine3d", run_refine3d),
                "nested": ("refine_nested", run_refine_nested), "tree": ("refine_tree", run_refine_tree),
                "twophase": ("two_phase_levels", run_two_phase_levels)}
        for leg in [v.strip() for v in args.refine_legs.split(",") if v.strip()]:
            key, fn = legs[leg]
            out[key] = fn(args.refine_steps, 10)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
