"""Benchmark of the flux-limited convective operator on one MI355X.

Default workload: the randomly renumbered 256^3 periodic hexahedral mesh (16.8M cells, 50.3M
faces, generic face-to-cell incidence with random face orientations), solenoidal face velocity
from the discrete curl of a seeded random edge potential, Gaussian blob + tanh step, SSP-RK3 at
CFL 0.4, for each of the limiters minmod, van Leer, superbee and SMART.  The library renumbers
the mesh for gather locality at creation (FL_MESH_REORDER, outside the timed region).

One step = one SSP-RK3 step (three stages) of one limiter; the timed region runs `--steps`
steps for every limiter.  A face-update is one face's limited flux in one stage for one scalar:
value = faces * stages * steps * limiters / time.

Prints one JSON line (see the keys below).  `roofline` is for the dominant kernel (the stage of
multi-step calls, fused_stage_lds_fwd_kernel on this lattice mesh): its algorithmic bytes per
launch (every slot index, face rate and cell value it must touch, read or written once) divided
by its average launch duration measured with HIP events on the launch stream (the timed region
also holds the one rate-table build of each call).  `cpu_baseline` times the CPU oracle on the host cores on
a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
LIM_DEFAULT = ["minmod", "vanleer", "superbee", "smart"]
METRIC = "FP64 Gface-updates/s + % HBM peak at 256^3; adjoint/forward cost ratio"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_SUMMARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "fused_stage_lds_fwd_kernel_box256_traffic.txt")
KERNEL_SOURCES = ["fl_internal.h", "fl_kernels.h", "fl_device.h", "fl_kernels.hip", "mesh.cpp"]


def kernel_source_hash():
    """sha256 of the sources that define the fused stage kernel and the tables it reads (the
    mesh builder decides the tile halos, and so the traffic)."""
    import hashlib

    h = hashlib.sha256()
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2110_03044_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(here, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(n, xcd_remap, slot_velocity, lds_stage, fwd_rates=True):
    """HBM bytes per fused-stage launch (scaled FETCH_SIZE + WRITE_SIZE) from the committed
    rocprofv3 counter summary, or None if it was taken on other kernel sources, sizes or launch
    mapping."""
    try:
        kv = {}
        for line in open(TRAFFIC_SUMMARY):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if (kv.get("kernel_source_sha256") != kernel_source_hash() or int(kv.get("n", -1)) != n
                or int(kv.get("xcd_remap", -1)) != int(xcd_remap)
                or int(kv.get("slot_velocity", 0)) != int(slot_velocity)
                or int(kv.get("lds_stage", 0)) != int(lds_stage)
                or int(kv.get("fwd_rates", 0)) != int(fwd_rates)):
            return None
        return int(float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def fwd_chunk(S):
    """Scalars the forward-rate LDS stage stages at a time (the library's fwd_chunk)."""
    return 2 if S == 4 else min(S, 3)


def lds_stage_bytes(C, K, S, stage, halo_total):
    """Compulsory bytes of one LDS-staged stage launch: local slot indices (4 B per slot), the
    per-call signed face rates (8 B per slot), the tile halo lists (4 B per entry), theta_s read
    once, theta_n read once (stages 2, 3) and the output written once.  Halo values are other
    tiles' cells: counted once, with their own tile."""
    b = C * K * 12 + 4 * halo_total + C * S * 8 * 2
    if stage > 0:
        b += C * S * 8
    return b


def lds_fwd_stage_bytes(C, K, S, stage, halo_total, halo_nexts):
    """Compulsory bytes of one forward-rate LDS stage launch (lattice meshes): the neighbours'
    16-bit local indices (2 B per slot), the per-call rates of each cell's forward faces (8 B per
    face: K/2 per cell), the tile halo lists (4 B per entry: cell and pair packed) and the next
    indices of the halo entries reached as neighbours (2 B each), theta_s read once, theta_n read
    once (stages 2, 3) and the output written once.  Halo values and halo rates are other tiles'
    cells' data: counted once, with their own tile."""
    b = C * K * 2 + C * (K // 2) * 8 + 4 * halo_total + 2 * halo_nexts + C * S * 8 * 2
    if stage > 0:
        b += C * S * 8
    return b


def fused_stage_bytes(C, F, K, S, stage, slot_velocity=True):
    """Compulsory bytes of one fused stage launch: slot records (other cell, far cell and the
    signed face rate: 16 B per slot; or, gathering u through the face index, face, cell and far
    cell, 12 B per slot, plus each face velocity once), theta_s read once, theta_n read once
    (stages 2, 3) and the output written once.  On hex meshes (F = 3C, K = 6) both give
    96 B per cell for the tables and velocities."""
    b = C * K * 16 if slot_velocity else C * K * 12 + F * 8
    b += C * S * 8 * 2
    if stage > 0:
        b += C * S * 8
    return b


def batch_stage_bytes(C, F, K, S, stage, halo_total):
    """Compulsory bytes of one problem's share of a batched LDS-staged stage launch (the face
    velocities gathered through the face index): local slot indices and slot face words (4 + 4 B
    per slot), each face velocity once, the tile halo lists (4 B per entry), theta_s read once,
    theta_n read once (stages 2, 3) and the output written once."""
    b = C * K * 8 + F * 8 + 4 * halo_total + C * S * 8 * 2
    if stage > 0:
        b += C * S * 8
    return b


def adjoint_ratio(args, torch, FL, W, dev):
    """Adjoint configuration: 128^3 periodic box, van Albada, SSP-RK3 at CFL 0.4, 400 steps,
    J = |theta_N - target|^2 / 2 with a seeded smooth target; gradients w.r.t. theta_0 and u_f
    through ceil(sqrt(N))-step checkpoints.  Returns forward (with checkpoint stores) and
    backward (recompute + reverse sweep) times and their ratio."""
    n = args.adjoint_n
    wl = W.workload_box(n, renumbered=False)
    mesh = FL.Mesh.from_arrays(wl.mesh, device=0, reorder=True)
    th0 = mesh.cells_to_mesh(torch.from_numpy(wl.theta0).to(dev))
    u = mesh.faces_to_mesh(torch.from_numpy(wl.u).to(dev))
    tgt = mesh.cells_to_mesh(torch.from_numpy(
        0.5 * W.field_smooth_random(n, 3, seed=W.SEED_TARGET) + 0.5).to(dev))
    steps = args.adjoint_steps
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]

    def once(n_steps, timed, every=None):
        t0 = th0.clone().requires_grad_(True)
        uu = u.clone().requires_grad_(True)
        torch.cuda.synchronize()
        ev[0].record(stream)
        out = FL.advect(mesh, "vanalbada", "ssprk3", wl.dt, t0, uu, n_steps, checkpoint_every=every)
        ev[1].record(stream)
        loss = 0.5 * ((out - tgt) ** 2).sum()
        ev[2].record(stream)
        loss.backward()
        ev[3].record(stream)
        ev[3].synchronize()
        return ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])

    # warm-up at full length, so that the caching allocator already holds every checkpoint and
    # stage buffer when the timed run starts
    once(steps, False)
    fwd_ms, bwd_ms = once(steps, True)
    # every stage input kept in HBM (20 GB at 128^3 x 400 steps): nothing is recomputed
    full_bytes = FL.n_stages("ssprk3") * mesh.n_cells * 8 * steps
    full = None
    if full_bytes < 0.5 * torch.cuda.mem_get_info(dev)[0]:
        once(steps, False, every=steps)  # warm-up: the caching allocator keeps the stage buffer
        full = once(steps, True, every=steps)
        torch.cuda.empty_cache()
    plain = th0.clone()
    work = FL.rk_workspace(mesh, "ssprk3", 1)
    torch.cuda.synchronize()
    ev[4].record(stream)
    FL.rk_steps(mesh, "vanalbada", "ssprk3", wl.dt, plain, u, steps, work=work)
    ev[5].record(stream)
    ev[5].synchronize()
    plain_ms = ev[4].elapsed_time(ev[5])
    log(f"adjoint {n}^3 x {steps}: forward {fwd_ms:.1f} ms, backward {bwd_ms:.1f} ms, "
        f"plain forward {plain_ms:.1f} ms" + ("" if full is None else
        f"; full stage storage: forward {full[0]:.1f} ms, backward {full[1]:.1f} ms"))
    mesh.close()
    return {"workload": f"periodic hex box {n}^3, van Albada, SSP-RK3 CFL 0.4, {steps} steps, "
                        f"L2 misfit to a seeded target, checkpoints every "
                        f"{FL.checkpoint_interval(steps)} steps",
            "forward_ms": round(fwd_ms, 2), "backward_ms": round(bwd_ms, 2),
            "plain_forward_ms": round(plain_ms, 2),
            "adjoint_forward_ratio": round(bwd_ms / fwd_ms, 3),
            "forward_plus_backward_over_plain": round((fwd_ms + bwd_ms) / plain_ms, 3),
            "full_storage": None if full is None else {
                "stage_storage_gb": round(full_bytes / 1e9, 2),
                "forward_ms": round(full[0], 2), "backward_ms": round(full[1], 2),
                "adjoint_forward_ratio": round(full[1] / full[0], 3)}}


def batch_compare(args, torch, FL, W, dev):
    """Batched configuration: `count` independent periodic boxes with sides drawn uniformly from
    12 to 96, 1-8 scalars, a limiter and a CFL number per problem, SSP-RK3.  Times the batched
    path (one launch per stage for all problems, graph replay, autotuned tile) against the same
    problems advanced by per-problem launches on the same GPU."""
    import time as _t

    t0 = _t.time()
    recipe = W.batch_recipe(count=args.batch_count)
    meshes, vel = {}, {}
    problems = []
    face_updates = 0
    step_bytes = 0  # compulsory bytes of one batched SSP-RK3 step (LDS-staged kernel)
    for p in recipe:
        if p.n not in meshes:
            m = W.box_shared_cache(p.n)
            meshes[p.n] = FL.Mesh.from_arrays(m, device=0, reorder=True)
            vel[p.n] = (m, W.velocity_curl(p.n, seed=p.n))
        mesh = meshes[p.n]
        m, u = vel[p.n]
        theta = mesh.cells_to_mesh(torch.from_numpy(W.batch_fields(p)).to(dev))
        ud = mesh.faces_to_mesh(torch.from_numpy(u).to(dev))
        problems.append((mesh, p.limiter, theta, ud, W.cfl_dt(m, u, p.cfl)))
        face_updates += m.n_faces * p.n_scalars * 3
        info = mesh.info
        step_bytes += sum(batch_stage_bytes(m.n_cells, m.n_faces, 2 * int(info.pairs),
                                            p.n_scalars, s, int(info.halo_total))
                          for s in range(3))
    W._BOX_CACHE.clear()
    log(f"batch of {len(problems)} problems ({len(meshes)} distinct meshes) built in "
        f"{_t.time() - t0:.1f}s")
    t1 = _t.time()
    b = FL.Batch(problems)  # picks the tile (timing, or the tuning cache) and records the graph
    create_s = _t.time() - t1
    stream = torch.cuda.current_stream(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    b.step(1)
    b.step_unbatched(1)
    torch.cuda.synchronize()
    K = args.batch_steps
    ev0.record(stream)
    b.step(K)
    ev1.record(stream)
    ev1.synchronize()
    batched_ms = ev0.elapsed_time(ev1) / K
    ev0.record(stream)
    b.step_unbatched(K)
    ev1.record(stream)
    ev1.synchronize()
    unbatched_ms = ev0.elapsed_time(ev1) / K
    tile = b.tile_cells
    staged = b.lds_staged
    from_cache = b.tuned_from_cache
    b.close()
    # per-problem launches of the other kernel too (LDS staging off: the gather kernel), so that
    # the batch is compared with the faster per-problem form
    FL.set_option("lds_stage", 0)
    try:
        b2 = FL.Batch(problems, tile_cells=256)
        b2.step_unbatched(1)
        torch.cuda.synchronize()
        ev0.record(stream)
        b2.step_unbatched(K)
        ev1.record(stream)
        ev1.synchronize()
        gather_ms = ev0.elapsed_time(ev1) / K
        b2.close()
    finally:
        FL.set_option("lds_stage", 1)
    best_ms = min(unbatched_ms, gather_ms)
    for mesh in meshes.values():
        mesh.close()
    log(f"batch: {batched_ms:.3f} ms/step batched (tile {tile}, LDS-staged {staged}); "
        f"per-problem launches {unbatched_ms:.3f} ms/step (same kernel), {gather_ms:.3f} ms/step "
        f"(gather kernel)")
    return {"workload": f"{len(recipe)} periodic boxes, sides 12-96, 1-8 scalars, per-problem "
                        f"limiter and CFL 0.2-0.5, SSP-RK3",
            "problems": len(recipe), "face_scalar_updates_per_step": face_updates,
            "batched_ms_per_step": round(batched_ms, 3),
            "unbatched_ms_per_step": round(best_ms, 3),
            "unbatched_same_kernel_ms_per_step": round(unbatched_ms, 3),
            "unbatched_gather_kernel_ms_per_step": round(gather_ms, 3),
            "speedup": round(best_ms / batched_ms, 3),
            "batched_gface_updates_per_s": round(face_updates / (batched_ms * 1e-3) / 1e9, 2),
            # the batched step's compulsory bytes (batch_stage_bytes over problems and stages)
            # over its time: launches, gaps and the stage tails included
            "roofline": {"bound": "hbm", "bytes_per_step": int(step_bytes),
                         "achieved": round(step_bytes / (batched_ms * 1e-3) / 1e9, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(step_bytes / (batched_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "unbatched_achieved": round(step_bytes / (best_ms * 1e-3) / 1e9, 1)}
            if staged else None,
            "lds_staged": staged,
            "autotuned_tile_cells": tile,
            "create_s": round(create_s, 3), "tile_from_tuning_cache": from_cache}


def scalar_sweep(args, torch, FL, W, dev):
    """Forward stage against the scalar count S on one periodic box (library reorder, van Leer,
    SSP-RK3, one multi-step call per S): ms per step, face-scalar updates per second and the
    compulsory bytes of the forward-rate LDS stage (lds_fwd_stage_bytes) per second."""
    n = args.scalar_sweep_n
    wl = W.workload_box(n, renumbered=True)
    mesh = FL.Mesh.from_arrays(wl.mesh, device=0, reorder=True)
    info = mesh.info
    C, F = mesh.n_cells, mesh.n_faces
    u = mesh.faces_to_mesh(torch.from_numpy(wl.u).to(dev))
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = 10
    rows = []
    for S in [int(x) for x in args.scalar_sweep.split(",") if x]:
        th0 = np.stack([wl.theta0 + 0.1 * k for k in range(S)], 1) if S > 1 else wl.theta0
        th = mesh.cells_to_mesh(torch.from_numpy(np.ascontiguousarray(th0)).to(dev))
        work = FL.rk_workspace(mesh, "ssprk3", S)
        FL.rk_steps(mesh, "vanleer", "ssprk3", wl.dt, th, u, 2, work=work)
        torch.cuda.synchronize()
        e0.record(stream)
        FL.rk_steps(mesh, "vanleer", "ssprk3", wl.dt, th, u, steps, work=work)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        byts = sum(lds_fwd_stage_bytes(C, 2 * int(info.pairs), S, s, int(info.halo_total),
                                       int(info.halo_nexts)) for s in range(3))
        rows.append({"scalars": S, "ms_per_step": round(ms, 4),
                     "gface_scalar_updates_per_s": round(F * S * 3 / (ms * 1e-3) / 1e9, 1),
                     "compulsory_gbs": round(byts / (ms * 1e-3) / 1e9, 1)})
        log(f"scalars {S}: {ms:.4f} ms/step, {rows[-1]['gface_scalar_updates_per_s']} G "
            f"face-scalar updates/s, {rows[-1]['compulsory_gbs']} GB/s")
        del th, work
    mesh.close()
    return {"workload": f"periodic hex box {n}^3, library reorder, van Leer, SSP-RK3, "
                        f"{steps} steps per scalar count", "rows": rows}


def face_path_stage_bytes(C, F, S, stage, side_entries, deg_sum, areas, vols):
    """Compulsory bytes of one stage on the face path (face kernel + cell kernel): per face its
    record (16 B), velocity (8 B), side pointers (8 B), the entries of its upwind side list (12 B
    each; half of all entries on average), the flux written and read back (8 B per scalar each);
    per cell its face list (4 B pointer, 4 B per face), theta_s read by each kernel once, the
    output written, theta_n read (stages 2, 3); face areas and cell volumes where given."""
    b = F * (16 + 8 + 8 + 16 * S) + 12 * side_entries // 2 + C * 4 + 4 * deg_sum
    b += C * S * 8 * 3 + (C * S * 8 if stage > 0 else 0)
    b += (F * 8 if areas else 0) + (C * 8 if vols else 0)
    return b


def face_path(args, torch, FL, W, dev):
    """The face path (general cells, boundary faces) on two large meshes: a box cut open along x
    with inflow values (boundary faces; the general kernel) and the periodic triangles (cells
    whose faces project with several weights).  10 SSP-RK3 steps, van Leer, one multi-step call
    each; the compulsory bytes of face_path_stage_bytes over the time."""
    rows = []
    cases = []
    n_box, n_tri = args.face_path_n, 2 * args.face_path_n * 4
    cases.append(("open box %d^3 with inflow values" % n_box, lambda: W.workload_open_box(n_box)))
    def tri():
        m = W.periodic_triangles(n_tri)
        u = W.velocity_stream_triangles(n_tri, seed=4)
        xy = W.triangle_centroids(n_tri)
        th = np.exp(-((xy[:, 0] - 0.4) ** 2 + (xy[:, 1] - 0.6) ** 2) / 0.02) + (xy[:, 0] > 0.5)
        return W.Workload(m, th, u, W.cfl_dt(m, u, 0.4), 10, "ssprk3", "triangles", None)
    cases.append(("periodic triangles %d x %d x 2" % (n_tri, n_tri), tri))
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = 10
    for name, make in cases:
        wl = make()
        m = wl.mesh
        mesh = FL.Mesh.from_arrays(m, device=0, reorder=True)
        cp, fp = mesh.permutation()
        info = mesh.info
        assert mesh.path == "face"
        if wl.inflow is not None:
            inf = np.empty_like(wl.inflow)
            inf[fp] = wl.inflow
            mesh.set_inflow(torch.from_numpy(inf).to(dev))
        th = mesh.cells_to_mesh(torch.from_numpy(wl.theta0).to(dev))
        u = mesh.faces_to_mesh(torch.from_numpy(wl.u).to(dev))
        work = FL.rk_workspace(mesh, "ssprk3", 1)
        FL.rk_steps(mesh, "vanleer", "ssprk3", wl.dt, th, u, 2, work=work)
        torch.cuda.synchronize()
        e0.record(stream)
        FL.rk_steps(mesh, "vanleer", "ssprk3", wl.dt, th, u, steps, work=work)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        C, F = m.n_cells, m.n_faces
        byts = sum(face_path_stage_bytes(C, F, 1, s, int(info.side_entries), 2 * F,
                                         not bool(info.uniform_area),
                                         not bool(info.uniform_volume)) for s in range(3))
        rows.append({"workload": name, "cells": C, "faces": F,
                     "boundary_faces": int(info.n_boundary), "side_entries": int(info.side_entries),
                     "ms_per_step": round(ms, 4),
                     "gface_updates_per_s": round(F * 3 / (ms * 1e-3) / 1e9, 1),
                     "bytes_per_step": int(byts),
                     "achieved_gbs": round(byts / (ms * 1e-3) / 1e9, 1),
                     "frac": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
        log(f"face path, {name}: {ms:.4f} ms/step, {rows[-1]['gface_updates_per_s']} "
            f"Gface-updates/s, {rows[-1]['achieved_gbs']} GB/s compulsory")
        mesh.close()
        del th, u, work, wl, m
        torch.cuda.empty_cache()
    return {"scheme": "ssprk3", "limiter": "vanleer", "rows": rows}


def deformation(args, torch, FL, W, dev):
    """The paper's deformation benchmark (Section 4.1): sphere r = 0.15 at (0.35, 0.35, 0.35),
    deformation flow reversed by cos(pi t / T), T = 3, superbee, SSP-RK3 at CFL 0.4, on the
    requested periodic boxes.  Reports the return-to-initial L1 error, the mass error and the
    face-update rate of each run."""
    out = []
    for n in [int(x) for x in args.deformation.split(",") if x]:
        t0 = time.time()
        wl = W.workload_deformation(n)
        sc = W.deformation_scales(wl.steps, wl.dt, 3.0, wl.scheme)
        log(f"  deformation {n}^3: workload built in {time.time() - t0:.1f} s")
        t0 = time.time()
        mesh = FL.Mesh.from_arrays(wl.mesh, device=0, reorder=True)
        log(f"  deformation {n}^3: mesh tables built and uploaded in {time.time() - t0:.1f} s")
        th0 = mesh.cells_to_mesh(torch.from_numpy(wl.theta0).to(dev))
        u = mesh.faces_to_mesh(torch.from_numpy(wl.u).to(dev))
        th = th0.clone()
        work = FL.rk_workspace(mesh, "ssprk3", 1)
        stream = torch.cuda.current_stream(dev)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        # in chunks so progress is printed during long runs
        chunk = 500
        for s0 in range(0, wl.steps, chunk):
            s1 = min(wl.steps, s0 + chunk)
            FL.rk_steps_scaled(mesh, "superbee", "ssprk3", wl.dt, th, u, sc[3 * s0:3 * s1],
                               work=work)
            torch.cuda.synchronize()
            log(f"  deformation {n}^3: {s1}/{wl.steps} steps")
        ev1.record(stream)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1)
        V = float(wl.mesh.cell_volume[0])
        l1 = float((th - th0).abs().sum()) * V
        mass0 = float(th0.sum()) * V
        mass_err = abs(float(th.sum()) * V - mass0) / mass0
        rate = wl.mesh.n_faces * 3 * wl.steps / (ms * 1e-3) / 1e9
        out.append({"n": n, "steps": wl.steps, "l1_error": l1, "sphere_volume": mass0,
                    "relative_mass_error": mass_err, "min": float(th.min()),
                    "max": float(th.max()), "seconds": round(ms / 1e3, 3),
                    "gface_updates_per_s": round(rate, 2)})
        log(f"deformation {n}^3: {wl.steps} steps, L1 {l1:.3e}, mass error {mass_err:.1e}, "
            f"{ms / 1e3:.2f} s, {rate:.1f} Gface-updates/s")
        mesh.close()
        del th, th0, u, work
        torch.cuda.empty_cache()
    return out


def algebraic_compare(args, torch, FL, W, dev):
    """The paper's algebraic implementation (Algorithm 3: 4 ELLPACK SpMV + 4 kbin for theta_f;
    Algorithm 4: kbin U(u), SpMV M, stage combination) against the fused stage kernel on the
    same periodic box (random numbering + library reorder, curl velocity, superbee, SSP-RK3 at
    CFL 0.4).  Section 4.2 compares the two strategies on 144^3 and 288^3 meshes."""
    out = []
    stream = torch.cuda.current_stream(dev)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    for n in [int(x) for x in args.algebraic.split(",") if x]:
        t0 = time.time()
        wl = W.workload_box(n, renumbered=True)
        log(f"algebraic {n}^3: workload in {time.time() - t0:.1f}s")
        mesh = FL.Mesh.from_arrays(wl.mesh, device=0, reorder=True)
        log(f"algebraic {n}^3: mesh in {time.time() - t0:.1f}s")
        alg = FL.Algebraic(mesh)
        log(f"algebraic {n}^3: matrices ({alg.device_bytes / 1e9:.1f} GB) in {time.time() - t0:.1f}s")
        th0 = mesh.cells_to_mesh(torch.from_numpy(wl.theta0).to(dev))
        u = mesh.faces_to_mesh(torch.from_numpy(wl.u).to(dev))
        th = th0.clone()
        awork = alg.workspace()
        work = FL.rk_workspace(mesh, "ssprk3", 1)
        tf = torch.empty_like(u)
        steps = 3
        C, F = wl.mesh.n_cells, wl.mesh.n_faces
        ell = sum(alg.rows[k] * alg.width[k] * 12 for k in ("D", "UUD", "OUD", "Pi"))
        rec = {"n": n, "cells": C, "ell_bytes_per_cell_theta_f": round(ell / C, 1),
               "matrix_device_gb": round(alg.device_bytes / 1e9, 2)}
        if not args.algebraic_chain_only:
            t_alg = timed(lambda: alg.rk_steps("superbee", "ssprk3", wl.dt, th, u, steps,
                                               work=awork), 2) / steps
            t_fused = timed(lambda: FL.rk_steps(mesh, "superbee", "ssprk3", wl.dt, th, u, steps,
                                                work=work), 2) / steps
            rec.update({"ms_per_step_algebraic": round(t_alg, 4),
                        "ms_per_step_fused": round(t_fused, 4),
                        "speedup_fused_over_algebraic": round(t_alg / t_fused, 2)})
            log(f"algebraic {n}^3: {t_alg:.3f} ms/step vs fused {t_fused:.3f} ms/step "
                f"({t_alg / t_fused:.1f}x)")
        t_tf = timed(lambda: alg.face_values("superbee", th, u, out=tf, work=awork), 5)
        rec["ms_theta_f_algebraic"] = round(t_tf, 4)
        log(f"algebraic {n}^3: theta_f chain {t_tf:.3f} ms")
        out.append(rec)
        alg.close()
        mesh.close()
        del th, th0, u, awork, work, tf
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--algebraic", default="",
                    help="comma-separated box sides for the algebraic-vs-fused comparison")
    ap.add_argument("--algebraic-chain-only", action="store_true",
                    help="time only the theta_f chain of the algebraic comparison (no stepping: "
                         "its kernels are then the run's only SpMV and kbin launches)")
    ap.add_argument("--headline", type=int, default=1,
                    help="0: skip the 256^3 headline measurement, its roofline and the oracle "
                         "timing (profiling runs of the other parts; the line's value is null)")
    ap.add_argument("--deformation", default="",
                    help="comma-separated box sides for the deformation benchmark (e.g. 72,144)")
    ap.add_argument("--scalar-sweep", default="1,2,3,4,6,8",
                    help="comma-separated scalar counts: forward stage against S ('' to skip)")
    ap.add_argument("--scalar-sweep-n", type=int, default=128)
    ap.add_argument("--face-path-n", type=int, default=192,
                    help="open box side (triangles: 8x as many squares per side; 0 to skip)")
    ap.add_argument("--batch-count", type=int, default=512, help="problems in the batch (0 to skip)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--adjoint-steps", type=int, default=400,
                    help="steps of the adjoint-cost measurement (0 to skip)")
    ap.add_argument("--adjoint-n", type=int, default=128)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed SSP-RK3 steps per limiter")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="cells per side of the periodic box")
    ap.add_argument("--limiters", default=",".join(LIM_DEFAULT))
    ap.add_argument("--no-reorder", action="store_true")
    ap.add_argument("--face-path", action="store_true")
    ap.add_argument("--xcd-remap", type=int, default=32,
                    help="FL_OPT_XCD_REMAP: M >= 2 runs of M tiles per XCD (default 32), 0 launch "
                         "order, 1 each XCD a contiguous eighth of the cells")
    ap.add_argument("--lds-stage", type=int, default=1,
                    help="0: multi-step calls use the slot records instead of LDS staging")
    ap.add_argument("--slot-velocity", type=int, default=1,
                    help="0: stages gather u through the face index (FL_OPT_SLOT_VELOCITY)")
    ap.add_argument("--fwd-rates", type=int, default=1,
                    help="0: a face rate per slot instead of one per face (FL_OPT_FWD_RATES)")
    ap.add_argument("--cpu-baseline", type=int, default=1, help="0 to skip the oracle timing")
    ap.add_argument("--cpu-steps", type=int, default=10,
                    help="SSP-RK3 steps of the oracle sample (about 0.6 s each at 256^3 on 16 "
                         "cores; a fifth of them on the given numbering, half as many Euler "
                         "stages on one thread)")
    ap.add_argument("--calib-copy-mib", type=int, default=1024,
                    help="size of the untimed calibration copy (0 to skip)")
    ap.add_argument("--compare-order", type=int, default=1,
                    help="1 (default): also time the as-given random numbering (no library "
                         "reorder); 0 to skip")
    ap.add_argument("--repeats", type=int, default=5,
                    help="times the whole timed region is run (the first gives value; all "
                         "give the median reported beside it)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (the operator's multi-GPU halo "
              "exchange is a design note, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2110_03044_amd import _lib, fluxlim as FL, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    lims = [l for l in args.limiters.split(",") if l]
    _lib.call("fl_set_option", 1, int(args.xcd_remap))  # FL_OPT_XCD_REMAP
    _lib.call("fl_set_option", 2, int(args.slot_velocity))  # FL_OPT_SLOT_VELOCITY
    _lib.call("fl_set_option", 3, int(args.lds_stage))  # FL_OPT_LDS_STAGE
    _lib.call("fl_set_option", 5, int(args.fwd_rates))  # FL_OPT_FWD_RATES
    wl = m = None
    if args.headline:
        t0 = time.time()
        wl = W.workload_box(args.n, renumbered=True)
        m = wl.mesh
        log(f"workload generated in {time.time() - t0:.1f}s: C={m.n_cells} F={m.n_faces} "
            f"dt={wl.dt:.6g}")

    def run_case(reorder: bool, reps: int = 1):
        t1 = time.time()
        mesh = FL.Mesh.from_arrays(m, device=0, reorder=reorder, face_path=args.face_path)
        log(f"mesh created (reorder={reorder}, path={mesh.path}) in {time.time() - t1:.1f}s, "
            f"{mesh.info.device_bytes / 1e9:.2f} GB on device")
        th0 = mesh.cells_to_mesh(torch.from_numpy(wl.theta0).to(dev))
        u = mesh.faces_to_mesh(torch.from_numpy(wl.u).to(dev))
        work = FL.rk_workspace(mesh, "ssprk3", 1)
        th = th0.clone()
        stream = torch.cuda.current_stream(dev)
        for lim in lims:  # warm-up
            th.copy_(th0)
            FL.rk_steps(mesh, lim, "ssprk3", wl.dt, th, u, args.warmup, work=work)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)

        def timed_region():
            per_lim, total_ms = {}, 0.0
            for lim in lims:
                th.copy_(th0)
                torch.cuda.synchronize()
                ev0.record(stream)
                FL.rk_steps(mesh, lim, "ssprk3", wl.dt, th, u, args.steps, work=work)
                ev1.record(stream)
                ev1.synchronize()
                ms = ev0.elapsed_time(ev1)
                total_ms += ms
                per_lim[lim] = ms
            return total_ms, per_lim

        total_ms, per_lim = timed_region()
        for lim, ms in per_lim.items():
            log(f"  {lim}: {ms / args.steps:.3f} ms/step")
        # the same region again (not part of value): run-to-run spread and its median
        repeats = [total_ms] + [timed_region()[0] for _ in range(max(0, reps - 1))]
        torch.cuda.synchronize()
        info = mesh.info
        res = dict(mesh=mesh, total_ms=total_ms, per_lim=per_lim, path=mesh.path,
                   repeats=repeats, aligned=bool(info.aligned),
                   K=int(info.max_degree), th=th, u=u, max_halo=int(info.max_halo),
                   tile_cells=int(info.tile_cells),
                   halo_total=int(info.halo_total), compact=bool(info.compact),
                   max_rated=int(info.max_rated), max_nexts=int(info.max_nexts),
                   halo_nexts=int(info.halo_nexts))
        return res

    # A plain device copy of known size: its FETCH_SIZE / WRITE_SIZE counters calibrate the fused
    # kernel's counters in profiled runs, and five more copies, timed, give the bandwidth a plain
    # copy reaches on this GPU (read + write bytes / time): context for the roofline fraction.
    copy_gbs = None
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream(dev)
        c0.record(stream)
        for _ in range(5):
            dst.copy_(src)
        c1.record(stream)
        c1.synchronize()
        copy_gbs = 5 * 2 * src.numel() * 8 / (c0.elapsed_time(c1) * 1e-3) / 1e9
        log(f"device copy of {args.calib_copy_mib} MiB: {copy_gbs:.0f} GB/s (read + write)")
        del src, dst

    reorder = not args.no_reorder

    def headline_part():
        r = run_case(reorder, args.repeats)
        C, F, S = m.n_cells, m.n_faces, 1
        n_steps_total = args.steps * len(lims)
        updates = F * S * 3 * n_steps_total
        value = updates / (r["total_ms"] * 1e-3) / 1e9
        ms_per_step = r["total_ms"] / n_steps_total

        out = {
            "metric": METRIC,
            "value": round(value, 3),
            "unit": "Gface-updates/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f64",
            "data": "synthetic",
            "config": {
                "workload": f"periodic hex box {args.n}^3, random cell/face numbering and face "
                            f"orientation (seed 1), curl velocity (seed 0), blob + tanh step, "
                            f"SSP-RK3 CFL 0.4",
                "cells": C, "faces": F, "scalars": S, "limiters": lims, "scheme": "ssprk3",
                "library_reorder": reorder, "path": r["path"],
            },
            "per_limiter_ms_per_step": {k: round(v / args.steps, 4) for k, v in r["per_lim"].items()},
            "repeats": {"ms_per_step": [round(t / n_steps_total, 4) for t in r["repeats"]],
                        "median_ms_per_step": round(float(np.median(r["repeats"])) / n_steps_total, 4),
                        "median_value": round(updates / (float(np.median(r["repeats"])) * 1e-3) / 1e9, 3)},
        }

        # roofline of the dominant kernel
        if r["path"] == "fused":
            K = r["K"]
            launches = 3 * n_steps_total
            sv = bool(args.slot_velocity) and args.steps >= 2
            lds = sv and bool(args.lds_stage) and r["max_halo"] >= 0 and \
                (r["tile_cells"] + r["max_halo"]) * fwd_chunk(S) * 8 <= 64 * 1024
            # the library's own choice (lds_fwd_bytes): compact tables and a staged tile of at
            # most 32 KiB (fwd_chunk(S) scalars staged at a time)
            words = K // 2 * r["tile_cells"] * 4 + (r["max_nexts"] + 1) * 2
            fwd = lds and r["aligned"] and r["compact"] and bool(args.fwd_rates) and \
                ((r["tile_cells"] + r["max_halo"] + 1) * fwd_chunk(S) + K // 2 * r["tile_cells"]
                 + r["max_rated"] + 1) * 8 + (words + 7) // 8 * 8 <= 32 * 1024
            if fwd:
                kname = "fused_stage_lds_fwd_kernel"
                bytes_per_step = sum(lds_fwd_stage_bytes(C, K, S, s, r["halo_total"],
                                                         r["halo_nexts"]) for s in range(3))
            elif lds:
                kname = "fused_stage_lds_kernel"
                bytes_per_step = sum(lds_stage_bytes(C, K, S, s, r["halo_total"]) for s in range(3))
            else:
                kname = "fused_stage_rec_kernel" if sv else "fused_stage_kernel"
                bytes_per_step = sum(fused_stage_bytes(C, F, K, S, s, sv) for s in range(3))
            # The timed region also holds the per-call table build of each call (one rk_steps call
            # per limiter): its time and its compulsory bytes (slot face words and each face
            # velocity read, rates or records written) are charged to the call's stage launches.
            table_bytes = 0
            if sv and args.steps >= 2:
                if fwd:  # forward slots' face words, each face velocity once, forward rates written
                    table_bytes = C * (K // 2) * 12 + F * 8
                else:
                    table_bytes = C * K * 12 + F * 8 if lds else C * K * 28 + F * 8
            total_bytes = bytes_per_step * n_steps_total + table_bytes * len(lims)
            avg_launch_s = r["total_ms"] * 1e-3 / launches
            achieved = total_bytes / launches / avg_launch_s / 1e9
            out["roofline"] = {"kernel": kname,
                               "bound": "hbm",
                               "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(achieved / HBM_PEAK_GBS, 4),
                               "traffic": measured_traffic(args.n, args.xcd_remap, sv, lds, fwd),
                               "algorithmic_bytes_per_launch": int(total_bytes / launches),
                               "stage_bytes_per_launch": int(bytes_per_step / 3),
                               "table_bytes_per_call": int(table_bytes),
                               "avg_launch_us": round(avg_launch_s * 1e6, 2),
                               "copy_gbs": None if copy_gbs is None else round(copy_gbs, 1),
                               "frac_of_copy": None if copy_gbs is None else
                               round(achieved / copy_gbs, 4)}
        # context: the face-kernel + cell-kernel byte model (40 B/face + 60 B/cell per stage, with a
        # flux array written and gathered back); the fused stage never forms that array, so the
        # model's effective bandwidth can exceed the HBM peak
        mb = (40 * F + 60 * C) / F
        out["two_kernel_model"] = {"bytes_per_face_update": round(mb, 2),
                                   "effective_gbs": round(value * mb, 1)}

        r["mesh"].close()
        del r
        torch.cuda.empty_cache()
        if args.compare_order and reorder:
            r2 = run_case(False)
            v2 = updates / (r2["total_ms"] * 1e-3) / 1e9
            out["as_given_numbering"] = {"value": round(v2, 3), "unit": "Gface-updates/s",
                                         "ms_per_step": round(r2["total_ms"] / n_steps_total, 4),
                                         "note": "same mesh and launch sequence without the "
                                                 "library's locality renumbering"}
            log(f"as-given numbering: {v2:.2f} Gface-updates/s")
            r2["mesh"].close()
            del r2
            torch.cuda.empty_cache()

        return out

    if args.headline:
        out = headline_part()
    else:
        out = {"metric": METRIC, "value": None, "unit": "Gface-updates/s", "n_gpus": 1,
               "steps": 0, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": "headline skipped (--headline 0)"}}

    if args.adjoint_steps > 0:
        out["adjoint"] = adjoint_ratio(args, torch, FL, W, dev)

    if args.batch_count > 0:
        out["batch"] = batch_compare(args, torch, FL, W, dev)
        torch.cuda.empty_cache()

    if args.deformation:
        out["deformation"] = deformation(args, torch, FL, W, dev)

    if args.scalar_sweep:
        out["scalar_sweep"] = scalar_sweep(args, torch, FL, W, dev)

    if args.face_path_n > 0:
        out["face_path"] = face_path(args, torch, FL, W, dev)

    if args.algebraic:
        out["algebraic"] = algebraic_compare(args, torch, FL, W, dev)

    if args.cpu_baseline and args.headline:
        from oracle import oracle as O

        C, F = m.n_cells, m.n_faces

        lim = "vanleer"
        # the oracle on the numbering the GPU runs on (the library's renumbering, applied on
        # the host from fl_mesh_permutation), then on the given random numbering
        mm, th_m, u_m = m, wl.theta0, wl.u
        if reorder:
            pm = FL.Mesh.from_arrays(m, device=-1, reorder=True)
            cp, fp = pm.permutation()
            pm.close()
            fc = np.empty_like(m.face_cells)
            fc[fp] = cp[m.face_cells]
            nrm = np.empty_like(m.face_normal)
            nrm[fp] = m.face_normal
            area = np.empty_like(m.face_area)
            area[fp] = m.face_area
            vol = np.empty_like(m.cell_volume)
            vol[cp] = m.cell_volume
            th_m = np.empty_like(wl.theta0)
            th_m[cp] = wl.theta0
            u_m = np.empty_like(wl.u)
            u_m[fp] = wl.u
            mm = (fc, nrm, area, vol)
        t1 = time.time()
        om = O.OracleMesh(*mm, n_cells=C) if reorder else O.OracleMesh.from_arrays(m)
        cpu_steps = args.cpu_steps
        t2 = time.time()
        om.run(lim, "ssprk3", wl.dt, th_m, u_m, cpu_steps)
        cpu_s = time.time() - t2
        cpu_rate = F * 3 * cpu_steps / cpu_s / 1e9
        out["cpu_baseline"] = {"value": round(cpu_rate, 4), "unit": "Gface-updates/s",
                               "cores": O.num_threads(), "kind": "oracle",
                               "sample": f"{cpu_steps} SSP-RK3 steps (3 stages each, all {F} "
                                         f"faces) of the same {args.n}^3 mesh in the numbering "
                                         f"the GPU runs on ({'library renumbering' if reorder else 'as given'}), "
                                         f"van Leer, {cpu_s:.1f} s"}
        log(f"oracle setup {t2 - t1:.1f}s, step {cpu_s:.1f}s")
        if reorder:
            og = O.OracleMesh.from_arrays(m)
            given_steps = max(1, cpu_steps // 5)
            t2 = time.time()
            og.run(lim, "ssprk3", wl.dt, wl.theta0, wl.u, given_steps)
            given_s = time.time() - t2
            del og
            out["cpu_baseline"]["as_given_numbering_value"] = round(
                F * 3 * given_steps / given_s / 1e9, 4)
            out["cpu_baseline"]["as_given_numbering_sample"] = (
                f"{given_steps} SSP-RK3 steps on the given random numbering, {given_s:.1f} s")
            log(f"oracle on the given numbering: {given_steps} steps {given_s:.1f}s")
        # the same oracle on one thread, over one stage (one forward-Euler step)
        import ctypes

        gomp = ctypes.CDLL("libgomp.so.1")
        threads = O.num_threads()
        gomp.omp_set_num_threads(1)
        one_stages = max(1, cpu_steps // 2)
        try:
            t3 = time.time()
            om.run(lim, "euler", wl.dt, th_m, u_m, one_stages)
            one_s = time.time() - t3
        finally:
            gomp.omp_set_num_threads(threads)
        out["cpu_baseline"]["single_thread_value"] = round(F * one_stages / one_s / 1e9, 5)
        out["cpu_baseline"]["single_thread_sample"] = (
            f"{one_stages} forward-Euler stages (all {F} faces each) of the same mesh and "
            f"numbering on 1 thread, {one_s:.1f} s")
        log(f"oracle on 1 thread: {one_stages} stages {one_s:.1f}s")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
