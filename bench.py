#!/usr/bin/env python
"""Throughput of the CSC narrow-band SDF path on one MI355X.

One step = the whole hot path over one batch of synthetic meshes already
resident in HBM: feature build (validation, adjacency, classes, polyhedron
lists, bricks), scan conversion of every polyhedron with the packed atomicMin,
sign pass and band compaction, then the adjoint of loss = sum of SDF^2 over the
band into the vertex gradient. value = band cells / second of that
forward+backward step.

Workloads: the 64-mesh batch (default; the batched step is one captured graph
replayed, compared with 64 per-mesh plain launches) and single large meshes.
Prints one JSON line. See --help.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "narrow-band cells/sec (fwd, fwd+bwd), batched vs per-mesh, at 1e-5·h error"
WORKLOADS = {
    # name: (config number, description)
    "batch64": (4, "64 meshes (icospheres L2-6, tori 2k-200k triangles, SH-displaced spheres degree <= 8 at 5%), "
                   "each with its own N^3 grid, N in [64, 256], band 3 cells, fwd+bwd of sum SDF^2; one batched "
                   "graph replay per step"),
    "sh_sphere9_1024": (5, "displaced sphere: icosphere L9 (5,242,880 triangles), SH degree 16 at 5%, "
                           "1024^3 grid, band 3 cells, fwd+bwd of sum SDF^2, per-mesh"),
    "noisy_torus_512": (3, "noisy torus: 360,000 triangles, tube-normal noise U(+-0.01), 512^3 grid, band 3, fwd+bwd"),
    "icosphere5_jitter_256": (2, "jittered icosphere L5: 20,480 triangles, 256^3 grid, band 4, fwd+bwd"),
}
PEAK_HBM_GBS = 8000.0
# stages timed around exactly one kernel launch, and that kernel
KERNEL_SYMBOL = {"init_keys": "k_init_keys", "scan_faces": "k_scan_small<0, false>",
                 "scan_edges": "k_scan_small<1, false>", "scan_vertices": "k_scan_small<2, false>",
                 "scan_faces_big": "k_scan_big<0, false, false>", "scan_edges_big": "k_scan_big<1, false, false>",
                 "scan_vertices_big": "k_scan_big<2, false, false>", "sign": "k_sign", "backward": "k_backward"}
SINGLE_KERNEL_STAGES = list(KERNEL_SYMBOL)
# scan launches and their tags in csc_scan_record_atomics, with their index in the atomic counts
SCAN_LAUNCHES = {"scan_faces": 0, "scan_edges": 1, "scan_vertices": 2, "scan_faces_big": 3, "scan_edges_big": 4,
                 "scan_vertices_big": 5}
# the launches of the forward pass (a5 scan conversion and a6 sign + compaction)
FORWARD_STAGES = ["init_keys", "scan_faces", "scan_edges", "scan_vertices", "scan_faces_big", "scan_edges_big",
                  "scan_vertices_big", "scan_wide", "brick_count", "sign"]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for name in ("scanconv.hip", "geometry.h", "backward.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_1903_00353_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel: str):
    """Measured HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec.get(workload, {}).get(kernel)
    if not ent or ent.get("source_sha") != kernel_source_sha():
        return None
    return ent.get("bytes_per_launch")


def algorithmic_bytes(stage, info, atomics, band_cells, vert_refs, nv, kept_store=False):
    """Bytes the method itself must move per launch of each single-kernel stage.
    atomics: packed atomicMin counts [faces, edges, vertices] of the
    one-thread-per-polyhedron launches, then of the overflow launches.
    kept_store: the key store is kept empty between scans (keep_store_empty): it
    is not filled, and the sign pass writes each key it consumed back."""
    F, E = info["n_faces"], info["n_edges"]
    if stage == "init_keys":  # every key of the allocated bricks, or only the nine overflow counters
        return 72 if kept_store else 8 * info["max_band_cells"]
    if stage == "scan_faces":   # per face its corners and unit normal (36 + 12 B), one u64 per atomic
        return 48 * F + 8 * atomics[0]
    if stage == "scan_edges":   # per edge polyhedron its record, endpoints and two normals (16 + 24 + 24 B)
        return 64 * info["n_edge_polyhedra"] + 8 * atomics[1]
    if stage == "scan_vertices":  # per vertex polyhedron its position, axis and aperture (12 + 16 B)
        return 28 * info["n_vertex_polyhedra"] + 8 * atomics[2]
    if stage.endswith("_big"):  # overflow launches: their atomics (geometry counted above)
        return 8 * atomics[3 + ["scan_faces_big", "scan_edges_big", "scan_vertices_big"].index(stage)]
    if stage == "sign":         # one key read and (sdf, id, cell) written per band cell (+ the key emptied)
        return (28 if kept_store else 20) * band_cells
    if stage == "backward":     # (sdf, id, cell) read (the loss's 2*SDF formed inside), 3 floats per weighted vertex
        return 12 * band_cells + 12 * vert_refs
    raise KeyError(stage)


def popcount64(mask_np):
    import numpy as np
    return int(np.unpackbits(np.ascontiguousarray(mask_np).view(np.uint8)).sum())


def brick_cells(info):
    """Keys per brick of the band store."""
    return int(info["max_band_cells"]) // max(1, int(info["n_bricks"]))


def atomic_rates(P, feats, ws, n_keys, nv, brick, reps=10):
    """Measured atomic peaks at the scan's own locality: the packed atomicMin
    instructions of each scan launch are logged (one round per wavefront
    instruction, with its lanes) and replayed by a kernel that does nothing
    else, on a key array of the store's size; the replay of every launch
    together gives the forward pass's rate. The replay reads 4 bytes of log per
    lane; a read-only pass over the same log is timed beside it. Also the
    scattered float atomicAdd rate (x, y, z of random vertices) that the
    adjoint's flushes meet. HIP events on the stream the kernels run on."""
    import torch
    keys = torch.empty(max(1, n_keys), dtype=torch.int64, device=ws.device)
    out = {}

    def timed(fn):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    import numpy as np
    for stage, tag in list(SCAN_LAUNCHES.items()) + [("all", -1)]:
        log, mask = P.csc_scan_record_atomics(feats, ws, tag)
        m = mask.cpu().numpy()
        n = popcount64(m)
        if n == 0:
            continue
        ms = timed(lambda: P.csc_atomic_replay(log, mask, keys, 0))
        ms_read = timed(lambda: P.csc_atomic_replay(log, mask, keys, 1))
        ms_wg = timed(lambda: P.csc_atomic_replay(log, mask, keys, 2))
        ms_st = timed(lambda: P.csc_atomic_replay(log, mask, keys, 3))
        ms_batched = timed(lambda: P.csc_atomic_replay(log, mask, keys, 4))
        # locality: distinct 128-byte lines (16 keys) and bricks per instruction, and
        # the rate of the same atomics issued in address order (64 per instruction)
        bits = np.unpackbits(m.view(np.uint8).reshape(-1, 8), axis=1, bitorder="little").astype(bool)
        addr = log.cpu().numpy().view(np.uint32).reshape(-1, 64).astype(np.int64)
        rows = np.repeat(np.arange(addr.shape[0]), 64).reshape(-1, 64)[bits]
        a = addr[bits]
        lines = np.unique(rows * (1 << 32) + (a >> 4)).size / addr.shape[0]
        bricks = np.unique(rows * (1 << 32) + a // brick).size / addr.shape[0]
        srt = np.sort(a).astype(np.uint32)
        pad = (-srt.size) % 64
        slog = torch.from_numpy(np.concatenate([srt, np.zeros(pad, np.uint32)]).view(np.int32)).to(ws.device)
        smask_np = np.full(slog.numel() // 64, -1, dtype=np.int64)
        if pad:
            smask_np[-1] = (1 << (64 - pad)) - 1
        smask = torch.from_numpy(smask_np).to(ws.device)
        ms_sorted = timed(lambda: P.csc_atomic_replay(slog, smask, keys, 0))
        out[stage] = {"atomics": n, "instructions": int(mask.numel()), "lanes_per_instruction": n / mask.numel(),
                      "lines_per_instruction": lines, "bricks_per_instruction": bricks,
                      "replay_ms": ms, "log_read_ms": ms_read, "workgroup_scope_ms": ms_wg, "plain_store_ms": ms_st,
                      "rate_G_per_s": n / (ms * 1e-3) / 1e9, "sorted_replay_ms": ms_sorted,
                      "sorted_rate_G_per_s": n / (ms_sorted * 1e-3) / 1e9, "batched_replay_ms": ms_batched,
                      "batched_rate_G_per_s": n / (ms_batched * 1e-3) / 1e9}
        del log, mask, slog, smask
    g = torch.zeros(max(1, nv), 3, dtype=torch.float32, device=ws.device)
    nadd = 1 << 23
    ms = timed(lambda: P.csc_fadd_rate(g, nadd))
    out["f32_atomicAdd_scattered"] = {"adds": 3 * nadd, "vertices": nv, "ms": ms,
                                      "rate_G_per_s": 3 * nadd / (ms * 1e-3) / 1e9}
    del keys, g
    return out


def rooflines(avg, per_step, atomics, rates, alg_bytes, fwd_bytes, fwd_span_ms=None):
    """Per single-kernel stage: T_roof = max(algorithmic bytes / 8 TB/s, atomics /
    measured atomic rate of that launch) against its measured time. The bench
    line's roofline is the dominant (slowest) kernel of the forward scan, the
    part of the method the roofline target is set on, with the whole forward
    pass's fraction beside it and the slowest kernel of the step named too. The
    forward pass (scan and sign launches) gets the same bound from its total
    bytes and atomics against the replay rate of all its launches together; its
    time is the span of the scan-and-sign call as the timed step runs it
    (fwd_span_ms), the sum of its stages timed one by one reported beside it."""
    per = {}
    for st in SINGLE_KERNEL_STAGES:
        t = avg.get(st, 0.0)
        if t <= 0:
            continue
        b = alg_bytes(st)
        ent = {"ms": t, "algorithmic_bytes": b, "hbm_GBs": b / (t * 1e-3) / 1e9}
        ent["hbm_frac"] = ent["hbm_GBs"] / PEAK_HBM_GBS
        if st in SCAN_LAUNCHES and st in rates:
            a = atomics[SCAN_LAUNCHES[st]]
            ent["atomics"] = a
            ent["atomic_G_per_s"] = a / (t * 1e-3) / 1e9
            ent["atomic_peak_G_per_s"] = rates[st]["rate_G_per_s"]
            ent["atomic_frac"] = ent["atomic_G_per_s"] / ent["atomic_peak_G_per_s"]
        ent["frac"] = max(ent["hbm_frac"], ent.get("atomic_frac", 0.0))
        ent["bound"] = "atomic" if ent.get("atomic_frac", 0.0) > ent["hbm_frac"] else "hbm"
        per[st] = ent
    slowest = max(per, key=lambda k: per[k]["ms"])
    dom = max((k for k in per if k in FORWARD_STAGES), key=lambda k: per[k]["ms"])
    d = per[dom]
    if d["bound"] == "atomic":
        main = {"bound": "atomic", "achieved": d["atomic_G_per_s"], "peak": d["atomic_peak_G_per_s"],
                "unit": "G atomics/s"}
    else:
        main = {"bound": "hbm", "achieved": d["hbm_GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    main.update({"kernel": KERNEL_SYMBOL[dom], "frac": d["frac"], "avg_ms": d["ms"],
                 "algorithmic_bytes": d["algorithmic_bytes"], "hbm_frac": d["hbm_frac"],
                 "atomic_frac": d.get("atomic_frac")})
    t_stages = sum(per_step.get(st, 0.0) for st in FORWARD_STAGES)
    t_fwd = fwd_span_ms if fwd_span_ms else t_stages
    a_all = sum(atomics)
    fwd = {"ms": t_fwd, "ms_stages_one_by_one": t_stages, "algorithmic_bytes": fwd_bytes, "atomics": a_all,
           "t_hbm_ms": fwd_bytes / (PEAK_HBM_GBS * 1e9) * 1e3}
    if "all" in rates:
        fwd["atomic_peak_G_per_s"] = rates["all"]["rate_G_per_s"]
        fwd["t_atomic_ms"] = a_all / (rates["all"]["rate_G_per_s"] * 1e9) * 1e3
    fwd["t_roof_ms"] = max(fwd["t_hbm_ms"], fwd.get("t_atomic_ms", 0.0))
    fwd["frac"] = fwd["t_roof_ms"] / t_fwd if t_fwd > 0 else None
    fwd["bound"] = "atomic" if fwd.get("t_atomic_ms", 0.0) > fwd["t_hbm_ms"] else "hbm"
    main["forward_frac"] = fwd["frac"]
    main["slowest_kernel"] = {"kernel": KERNEL_SYMBOL[slowest], "ms": per[slowest]["ms"], "frac": per[slowest]["frac"],
                              "bound": per[slowest]["bound"]}
    return main, per, dom, fwd


def forward_bytes(nv, nf, ne, atomics, band_cells):
    """Algorithmic bytes of one forward pass: the mesh (12 B per vertex, 12 B per
    triangle, 16 B per edge record), 8 B per packed atomicMin, the key read by
    the sign pass and the band written (SDF and id), 8 B each per band cell."""
    return 12 * nv + 12 * nf + 16 * ne + 8 * sum(atomics) + 8 * band_cells + 8 * band_cells


def host_info():
    """The host the CPU baseline ran on: CPU model, logical CPUs, CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def oracle_single_thread(budget_s=5.0):
    """The oracle on one thread: the cube on 64^3 (12 triangles, band 3) over the
    whole grid, and the jittered icosphere L5 on 256^3 (band 4) over z-slabs
    through the middle until about budget_s seconds. Runs in a child process,
    since the oracle's OpenMP thread count is fixed when it loads."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-single-thread",
                        "--cpu-budget", str(budget_s)], env=env, capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        return {"error": r.stderr.strip()[-300:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def _oracle_single_thread_child(budget_s):
    import meshgen
    import oracle
    out = {}
    for cfg, key in ((1, "cube_64"), (2, "icosphere5_jitter_256")):
        name, meshes, grids = meshgen.make_config(cfg)
        (v, f), g = meshes[0], grids[0]
        om = oracle.OracleMesh(v, f)
        n2, step = int(g.n[2]), 16
        cells, spent, planes, threads, i = 0, 0.0, 0, 1, 0
        while planes < n2 and (cfg == 1 or spent < budget_s):
            off = ((i + 1) // 2) * step * (1 if i % 2 else -1)
            k0 = max(0, min(n2 - step, n2 // 2 + off)) if cfg != 1 else i * step
            t0 = time.perf_counter()
            b = om.band(g, k0, k0 + step)
            spent += time.perf_counter() - t0
            cells += int(((b["flags"] & oracle.FLAG_IN_BAND) > 0).sum())
            threads = b["threads"]
            planes += step
            i += 1
        out[key] = {"value": cells / spent, "unit": "cells/s", "threads": threads, "band_cells": cells,
                    "z_planes": planes, "of_z_planes": n2, "seconds": spent}
    print(json.dumps(out))


def cpu_baseline(v, f, grid, budget_s=15.0):
    """The oracle as it stands on the host cores, on z-slabs through the middle of
    the grid until about budget_s seconds of band computation have been spent."""
    import oracle
    om = oracle.OracleMesh(v, f)
    n2 = int(grid.n[2])
    step = 16
    mid = n2 // 2
    cells, spent, planes, threads, i = 0, 0.0, 0, 1, 0
    while spent < budget_s and planes < n2:
        off = ((i + 1) // 2) * step * (1 if i % 2 else -1)  # slabs outward from the middle: 0, +16, -16, ...
        k0 = max(0, min(n2 - step, mid + off))
        t0 = time.perf_counter()
        b = om.band(grid, k0, k0 + step)
        spent += time.perf_counter() - t0
        cells += int(((b["flags"] & oracle.FLAG_IN_BAND) > 0).sum())
        threads = b["threads"]
        planes += step
        i += 1
    return {"value": cells / spent, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{planes} z-planes of {n2} through the middle of the grid ({cells} band cells, "
                      f"{spent:.1f} s); FP64 exact distance with bounding-box cull, pseudonormal sign; "
                      f"one-time edge table and normals excluded"}


def timed_steps(fn, steps):
    """Run fn `steps` times between two device synchronisations. Returns the mean
    wall-clock ms per step over the bracket and the per-step ms from HIP events
    recorded between the steps on the current stream (median, minimum)."""
    import statistics

    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i].record()
        fn()
    ev[steps].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return (t1 - t0) * 1e3 / steps, statistics.median(per), min(per)


def stage_averages(fn, steps):
    """Mean ms per launch of every library stage over `steps` eager calls of fn
    (the library's own HIP events on the stream each kernel is launched on), the
    wall-clock ms per call, and each stage's ms per call of fn."""
    import torch

    import paper_1903_00353_amd as P
    torch.cuda.synchronize()
    P.csc_timing_reset()
    P.csc_timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    P.csc_timing_enable(False)
    stages = P.csc_timing_read()
    return ({k: (ms / c if c else 0.0) for k, (ms, c) in stages.items()}, (t1 - t0) * 1e3 / steps,
            {k: ms / steps for k, (ms, c) in stages.items()})


def forward_span(steps, build, scan, finish):
    """ms of the forward scan as the timed step runs it: HIP events on the
    library's stream (torch's current stream) around the scan-and-sign call of
    `steps` eager steps without stage timing, so that a batch's edge and vertex
    kinds run beside its faces on the side stream as in the captured graph
    (the call joins that stream before it returns)."""
    import statistics

    import torch
    ev = []
    for _ in range(steps):
        build()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        band = scan()
        e1.record()
        finish(band)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    return statistics.mean(a.elapsed_time(b) for a, b in ev)


def parse_rows(text):
    rows = tuple(int(x) for x in text.split(","))
    if len(rows) != 3 or min(rows) < 1:
        raise SystemExit("--small-rows takes three positive integers: faces,edges,vertices")
    return rows


def batch_algorithmic_bytes(stage, nf, nv, n_epoly, n_vpoly, atomics, band_cells, vert_refs, max_band_cells):
    info = {"n_faces": nf, "n_edges": 3 * nf // 2, "n_edge_polyhedra": n_epoly, "n_vertex_polyhedra": n_vpoly,
            "max_band_cells": max_band_cells}
    return algorithmic_bytes(stage, info, atomics, band_cells, vert_refs, nv, kept_store=True)  # Batch keeps it


def bench_batch(args):
    import torch

    import meshgen
    import paper_1903_00353_amd as P

    cfg, desc = WORKLOADS["batch64"]
    name, meshes, grids = meshgen.make_config(cfg)
    dev = torch.device("cuda:0")
    B = P.Batch(meshes, grids, device=dev, backward=True, graph_safe=True, face_order=not args.input_order)
    from paper_1903_00353_amd import autotune
    tune_ms = None
    if args.small_rows:
        schedule = (parse_rows(args.small_rows), args.scan_grid, args.absorb, args.geom_blocks)
        B.options = autotune.options_for(schedule)
        B.f = P.csc_build_features_batched(B.verts, B.tris, B.nv, B.nf, B.grids, B.options, flags=B.flags,
                                           reuse=B.f)
    else:
        schedule, tune_ms = autotune.tune_batch(B)  # (small_rows, scan_grid, absorb_cells)
    info = B.f.info()
    # untimed diagnostics: atomics per scan launch, band size, weighted vertices per band cell
    atomics = P.csc_scan_convert_count(B.f, B.workspace)
    B.step()
    torch.cuda.synchronize()
    B.check()
    off = B.band_off.cpu().numpy()
    M = int(off[-1])
    feat = B.out[1][:M].cpu().numpy()
    vert_refs = 0
    for m, (v, f) in enumerate(meshes):
        fe = feat[off[m]:off[m + 1]]
        F, E = f.shape[0], 3 * f.shape[0] // 2
        vert_refs += int(3 * (fe < F).sum() + 2 * ((fe >= F) & (fe < F + E)).sum() + (fe >= F + E).sum())

    # the timed step: one replay of the captured batched graph (build, scan, sign, gradient zeroing, adjoint)
    run = B.step
    if not args.no_graph:
        B.capture()
        run = B.replay
    for _ in range(args.warmup):
        run()
    ms_graph, med_graph, min_graph = timed_steps(run, args.steps)
    B.check()

    # the same step launched eagerly, with the library's per-stage events (roofline)
    for _ in range(max(1, args.warmup)):
        B.step()
    avg, ms_eager, per_step = stage_averages(B.step, args.steps)
    span = forward_span(
        args.steps,
        lambda: P.csc_build_features_batched(B.verts, B.tris, B.nv, B.nf, B.grids, B.options,
                                             flags=B.flags | P.CSC_BUILD_NO_SYNC, reuse=B.f),
        lambda: P.csc_scan_convert_batched(B.f, B.workspace, B.out, B.band_off),
        lambda _: (B.grad_verts.zero_(), P.csc_sdf_backward_batched(B.f, B.out, B.band_off, None, B.grad_verts)))
    rates = atomic_rates(P, B.f, B.workspace, int(info["max_band_cells"]), int(info["n_vertices"]),
                         brick_cells(info))
    NF, NV = int(info["n_faces"]), int(info["n_vertices"])
    main, per, dom, fwd = rooflines(
        avg, per_step, atomics, rates,
        lambda st: batch_algorithmic_bytes(st, NF, NV, int(info["n_edge_polyhedra"]), int(info["n_vertex_polyhedra"]),
                                           atomics, M, vert_refs, int(info["max_band_cells"])),
        forward_bytes(NV, NF, int(info["n_edges"]), atomics, M), span)
    main["traffic"] = load_traffic("batch64", dom)
    main["measured_on"] = "eager batched steps, scan kinds one after another"
    res = {
        "metric": METRIC,
        "value": M / (ms_graph * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_graph,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch64: {desc}", "meshes": len(meshes), "faces": int(info["n_faces"]),
                   "vertices": int(info["n_vertices"]), "grids": [int(g.n[0]) for g in grids], "band_cells": 3.0,
                   "band_size": M, "parallelism": "single GPU"},
        "roofline": main,
        "roofline_forward": fwd,
        "roofline_kernels": per,
        "atomic_peaks": rates,
        "step_ms": {"median": med_graph, "min": min_graph, "launch": "eager" if args.no_graph else "graph replay"},
        "batched_eager": {"value": M / (ms_eager * 1e-3), "ms_per_step": ms_eager},
        "schedule": {"small_rows": list(schedule[0]), "scan_grid": schedule[1], "absorb_cells": schedule[2],
                     "geom_blocks": schedule[3],
                     "tuning_ms": tune_ms or None},
        "stages_ms": {k: round(x, 4) for k, x in avg.items()},
        "atomics": {"faces": atomics[0], "edges": atomics[1], "vertices": atomics[2], "faces_big": atomics[3],
                    "edges_big": atomics[4], "vertices_big": atomics[5]},
        "features": info,
        "kernel_source_sha": kernel_source_sha(),
    }
    if args.timed_only:
        print(json.dumps(res))
        return

    # forward only (build, scan, sign), batched eager
    B.backward = False
    B.step()
    ms_fwd, med_fwd, min_fwd = timed_steps(B.step, args.steps)
    B.backward = True
    B.check()
    res["fwd"] = {"value": M / (ms_fwd * 1e-3), "ms_per_step": ms_fwd, "median": med_fwd, "min": min_fwd,
                  "launch": "eager"}

    # per-mesh plain launches: 64 x (build, scan, adjoint), handles and buffers reused
    per = []
    for m, (v, f) in enumerate(meshes):
        vt, tt = B.verts[sum(B.nv[:m]):sum(B.nv[:m + 1])], torch.from_numpy(f).to(dev)
        h = P.csc_build_features(vt, tt, grids[m], B.options)
        nbytes, mx = P.csc_scan_convert_workspace(h)
        o = (torch.empty(mx, dtype=torch.float32, device=dev), torch.empty(mx, dtype=torch.int32, device=dev),
             torch.empty(mx, dtype=torch.int32, device=dev), torch.zeros(1, dtype=torch.int64, device=dev))
        per.append((vt, tt, grids[m], h, torch.empty(nbytes, dtype=torch.uint8, device=dev), o,
                    torch.empty(mx, dtype=torch.float32, device=dev), torch.zeros_like(vt)))

    def per_mesh_step():
        for vt, tt, g, h, ws, o, gsd, gv in per:
            P.csc_build_features(vt, tt, g, reuse=h)
            band = P.csc_scan_convert(h, ws, o, sync_count=False)
            gv.zero_()
            P.csc_sdf_backward(h, band, None, gv, n_band_d=o[3])  # upstream of sum SDF^2, fused

    for _ in range(args.warmup):
        per_mesh_step()
    ms_per_mesh, med_pm, min_pm = timed_steps(per_mesh_step, args.steps)
    M_per = sum(int(x[5][3].item()) for x in per)
    res["per_mesh"] = {"value": M_per / (ms_per_mesh * 1e-3), "ms_per_step": ms_per_mesh, "median": med_pm,
                       "min": min_pm, "band_size": M_per}
    res["speedup_batched_vs_per_mesh"] = ms_per_mesh / ms_graph
    # ablation: forward with every box cell tested by itself (Alg. 2 as printed)
    B2 = P.Batch(meshes, grids, options=autotune.options_for(schedule, P.make_options(scan_mode=1)), device=dev,
                 backward=False, graph_safe=True)
    B2.step()
    avg2, ms2, _ = stage_averages(B2.step, max(3, args.steps // 4))
    res["ablation_per_cell_scan"] = {"fwd_ms": ms2, "fwd_ms_row_intervals": ms_fwd,
                                     "stages_ms": {k: round(v, 4) for k, v in avg2.items() if k.startswith("scan_")}}
    del B2
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_batch(meshes, grids, args.cpu_budget)
        res["cpu_baseline"]["host"] = host_info()
        res["cpu_baseline"]["single_thread"] = oracle_single_thread()
    print(json.dumps(res))


def cpu_baseline_batch(meshes, grids, budget_s=15.0):
    """The oracle on the host cores over whole meshes of the batch, in order
    (repeating the batch if it ends first), until about budget_s seconds of band
    computation have been spent."""
    import oracle
    cells, spent, done, threads = 0, 0.0, 0, 1
    oms = {}
    while spent < budget_s and done < 64 * len(meshes):
        m = done % len(meshes)
        if m not in oms:
            oms[m] = oracle.OracleMesh(*meshes[m])
        t0 = time.perf_counter()
        b = oms[m].band(grids[m])
        spent += time.perf_counter() - t0
        cells += int(((b["flags"] & oracle.FLAG_IN_BAND) > 0).sum())
        threads = b["threads"]
        done += 1
    passes = done / len(meshes)
    return {"value": cells / spent, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} whole-grid meshes = {passes:.2f} passes over the {len(meshes)}-mesh batch "
                      f"({cells} band cells, {spent:.1f} s); FP64 exact distance with bounding-box cull, "
                      f"pseudonormal sign; one-time edge tables and normals excluded"}


def summarize_counters(args):
    """Turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of this benchmark and of the
    plain-copy calibration into bytes per launch of each kernel (profiles/traffic.json)
    and a short text summary. FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are each
    divided by what the same counter reports per byte of the 1 GiB copy."""
    import csv

    def per_kernel(path):
        acc = {}
        for r in csv.DictReader(open(path)):
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    fetch, write = per_kernel(args.fetch_csv), per_kernel(args.write_csv)
    cf, cw = per_kernel(args.copy_fetch_csv), per_kernel(args.copy_write_csv)
    copy_name = max(cf, key=lambda k: cf[k] if "copyBuffer" in k else -1)
    gib_kib = float(1 << 20)  # the calibration copies 1 GiB: 1 GiB read, 1 GiB written
    fetch_scale, write_scale = cf[copy_name] / gib_kib, cw[copy_name] / gib_kib
    symbol_of = KERNEL_SYMBOL
    out_path = os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(out_path)) if os.path.exists(out_path) else {}
    entry = {}
    lines = [f"# HBM traffic per launch, workload {args.workload}",
             f"calibration ({copy_name}, 1 GiB copy): FETCH_SIZE {cf[copy_name]:.0f} KiB -> scale {fetch_scale:.4f}; "
             f"WRITE_SIZE {cw[copy_name]:.0f} KiB -> scale {write_scale:.4f}",
             "kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes/launch (scaled)"]
    for stage, sym in symbol_of.items():
        # a plain kernel name, or any instance of a template of that name (the sign
        # pass: k_sign<true> when the batch keeps its store empty, else k_sign<false>)
        names = sorted((k for k in fetch if (sym + "(") in k or (sym + "<") in k), key=lambda k: -write.get(k, 0.0))
        if not names:
            continue
        k = names[0]
        b = (fetch[k] / fetch_scale + write.get(k, 0.0) / write_scale) * 1024.0
        entry[stage] = {"kernel": k, "fetch_kib": fetch[k], "write_kib": write.get(k, 0.0),
                        "fetch_scale": fetch_scale, "write_scale": write_scale, "bytes_per_launch": b,
                        "source_sha": kernel_source_sha()}
        lines.append(f"{k} | {fetch[k]:.0f} | {write.get(k, 0.0):.0f} | {b:.4g}")
    rec[args.workload] = entry
    os.makedirs(os.path.dirname(out_path), exist_ok=True)
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("\n".join(lines))


def bench_single(args):
    import torch

    import meshgen
    import paper_1903_00353_amd as P

    cfg, desc = WORKLOADS[args.workload]
    name, meshes, grids = meshgen.make_config(cfg)
    v, f = meshes[0]
    g = grids[0]
    dev = torch.device("cuda:0")
    verts = torch.from_numpy(v).to(dev)
    tris = torch.from_numpy(f).to(dev)
    from paper_1903_00353_amd import autotune
    tune_ms = None
    if args.small_rows:
        schedule = (parse_rows(args.small_rows), args.scan_grid, args.absorb, args.geom_blocks)
    else:
        schedule, tune_ms = autotune.tune_single(verts, tris, g)  # (small_rows, scan_grid, absorb_cells)
    opts = autotune.options_for(schedule)
    feats = P.csc_build_features(verts, tris, g, opts)
    if args.face_order:
        P.csc_features_order_faces(feats)
    info = feats.info()
    nbytes, mx = P.csc_scan_convert_workspace(feats)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = (torch.empty(mx, dtype=torch.float32, device=dev), torch.empty(mx, dtype=torch.int32, device=dev),
           torch.empty(mx, dtype=torch.int32, device=dev), torch.zeros(1, dtype=torch.int64, device=dev))
    gv = torch.zeros_like(verts)

    def forward():
        P.csc_build_features(verts, tris, g, opts, reuse=feats)
        return P.csc_scan_convert(feats, ws, out, sync_count=False)

    def step():
        band = forward()
        gv.zero_()
        P.csc_sdf_backward(feats, band, None, gv, n_band_d=out[3])  # upstream of sum SDF^2, fused

    # untimed diagnostics: atomics per scan launch, band size and vertex references
    atomics = P.csc_scan_convert_count(feats, ws)
    forward()
    torch.cuda.synchronize()
    M = int(out[3].item())
    feat_ids = out[1][:M].cpu().numpy()
    F, E = info["n_faces"], info["n_edges"]
    vert_refs = int(3 * (feat_ids < F).sum() + 2 * ((feat_ids >= F) & (feat_ids < F + E)).sum()
                    + (feat_ids >= F + E).sum())

    for _ in range(args.warmup):
        step()
    ms_step, med_step, min_step = timed_steps(step, args.steps)
    avg, _, per_step = stage_averages(step, args.steps)
    span = forward_span(args.steps, lambda: P.csc_build_features(verts, tris, g, opts, reuse=feats),
                        lambda: P.csc_scan_convert(feats, ws, out, sync_count=False),
                        lambda band: (gv.zero_(), P.csc_sdf_backward(feats, band, None, gv, n_band_d=out[3])))
    rates = atomic_rates(P, feats, ws, int(info["max_band_cells"]), int(verts.shape[0]), brick_cells(info))
    main, per, dom, fwd = rooflines(avg, per_step, atomics, rates,
                                    lambda st: algorithmic_bytes(st, info, atomics, M, vert_refs, verts.shape[0]),
                                    forward_bytes(int(verts.shape[0]), F, E, atomics, M), span)
    main["traffic"] = load_traffic(args.workload, dom)
    res = {
        "metric": METRIC,
        "value": M / (ms_step * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "faces": F, "vertices": int(verts.shape[0]),
                   "grid": list(g.n), "band_cells": g.band, "band_size": M, "parallelism": "single GPU"},
        "roofline": main,
        "roofline_forward": fwd,
        "roofline_kernels": per,
        "atomic_peaks": rates,
        "step_ms": {"median": med_step, "min": min_step},
        "stages_ms": {k: round(x, 4) for k, x in avg.items()},
        "atomics": {"faces": atomics[0], "edges": atomics[1], "vertices": atomics[2], "faces_big": atomics[3],
                    "edges_big": atomics[4], "vertices_big": atomics[5]},
        "schedule": {"small_rows": list(schedule[0]), "scan_grid": schedule[1], "absorb_cells": schedule[2],
                     "geom_blocks": schedule[3],
                     "tuning_ms": tune_ms or None},
        "features": info,
        "kernel_source_sha": kernel_source_sha(),
    }
    if not args.timed_only:
        ms_fwd, med_fwd, min_fwd = timed_steps(forward, args.steps)
        res["fwd"] = {"value": M / (ms_fwd * 1e-3), "ms_per_step": ms_fwd, "median": med_fwd, "min": min_fwd}
        # the same fwd+bwd step through the batched entry points for one mesh, captured as one graph
        B1 = P.Batch([(v, f)], [g], options=opts, device=dev, backward=True, graph_safe=True, face_order=False)
        B1.capture()
        for _ in range(args.warmup):
            B1.replay()
        ms_g, med_g, min_g = timed_steps(B1.replay, args.steps)
        B1.check()
        M1 = int(B1.band_off[-1].item())
        res["one_mesh_batch_graph"] = {"value": M1 / (ms_g * 1e-3), "ms_per_step": ms_g, "median": med_g,
                                       "min": min_g, "band_size": M1}
        del B1
        res["interior_fill"] = bench_interior_fill(P, feats, ws, out, g, max(3, args.steps // 4))
        res["weld"] = bench_weld(P, verts, tris, 5)
        res["ablation_per_cell_scan"] = bench_per_cell(P, verts, tris, g, schedule, ws, out, max(3, args.steps // 4))
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = cpu_baseline(v, f, g, args.cpu_budget)
            res["cpu_baseline"]["host"] = host_info()
            res["cpu_baseline"]["single_thread"] = oracle_single_thread()
    print(json.dumps(res))


def summarize_trace(args):
    """Markdown table of a rocprofv3 --kernel-trace --stats kernel_stats.csv (top kernels)."""
    import csv
    rows = list(csv.DictReader(open(args.trace_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# Kernel time, workload {args.workload}", "",
             "| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:args.top]:
        name = r["Name"].split("(")[0].replace("void ", "")
        if name.startswith("at::native::"):
            name = "torch " + name.split("<")[0].split("::")[-1] + " (gradient zero fill)"
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / tot * 100:.1f} |")
    print("\n".join(lines))


def bench_per_cell(P, verts, tris, g, schedule, ws, out, reps):
    """Ablation: the forward pass with every box cell tested by itself (Alg. 2 as
    printed, scan_mode 1) instead of row intervals; per-stage times."""
    from paper_1903_00353_amd import autotune
    opts = autotune.options_for(schedule, P.make_options(scan_mode=1))
    f1 = P.csc_build_features(verts, tris, g, opts)
    nbytes, _ = P.csc_scan_convert_workspace(f1)
    if nbytes > ws.numel():
        return None

    def fwd():
        P.csc_build_features(verts, tris, g, opts, reuse=f1)
        P.csc_scan_convert(f1, ws, out, sync_count=False)

    fwd()
    avg, ms, _ = stage_averages(fwd, reps)
    f1.free()
    return {"fwd_ms": ms, "stages_ms": {k: round(v, 4) for k, v in avg.items() if k.startswith("scan_")}}


def bench_weld(P, verts, tris, reps):
    """Triangle-soup ingestion: the workload mesh flattened to a soup (one
    position per corner, as an STL file lists it) and welded back into an
    indexed mesh, device resident; wall clock per call (the call synchronises
    and allocates its temporaries)."""
    import torch
    soup = verts[tris.long()].contiguous()
    vw, tw = P.csc_weld_soup(soup)
    ok = vw.shape[0] == verts.shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        P.csc_weld_soup(soup)
    ms = (time.perf_counter() - t0) * 1e3 / reps
    n = 3 * int(tris.shape[0])
    return {"ms": ms, "faces": int(tris.shape[0]), "corners": n, "vertices": int(vw.shape[0]),
            "vertices_recovered": bool(ok), "corners_per_s": n / (ms * 1e-3)}


def bench_interior_fill(P, feats, ws, out, g, reps):
    """Interior fill of the dense field (a separate stage after the forward pass):
    each repetition rewrites the dense grid with a scan conversion, then fills;
    the fill launch alone is timed by the library's stage events. Algorithmic
    bytes: one 4-byte read per cell plus one 4-byte write per interior cell
    beyond the band."""
    import torch
    n = int(g.n[0]) * int(g.n[1]) * int(g.n[2])
    dense = torch.empty(n, dtype=torch.float32, device=out[0].device)

    def rep():
        P.csc_scan_convert(feats, ws, out, dense=dense, sync_count=False)
        P.csc_interior_fill(feats, dense)

    rep()
    torch.cuda.synchronize()
    interior = int((dense == float("-inf")).sum().item())
    avg, _, _ = stage_averages(rep, reps)
    ms = avg["interior_fill"]
    nbytes = 4 * n + 4 * interior
    del dense
    return {"ms": ms, "cells": n, "interior_cells": interior, "algorithmic_bytes": nbytes,
            "achieved_GBs": nbytes / (ms * 1e-3) / 1e9, "peak_GBs": PEAK_HBM_GBS}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--small-rows", help="fixed schedule faces,edges,vertices instead of the autotuned one")
    ap.add_argument("--scan-grid", type=int, default=2, help="with --small-rows: scan_grid (1, 2, 3)")
    ap.add_argument("--absorb", type=float, default=0.05, help="with --small-rows: absorb_cells (negative: off)")
    ap.add_argument("--geom-blocks", type=int, default=0, help="with --small-rows: geom_blocks (0: one thread per face)")
    ap.add_argument("--face-order", action="store_true", help="single mesh: scan the faces in spatial order")
    ap.add_argument("--input-order", action="store_true", help="batch64: scan the faces in input order")
    ap.add_argument("--timed-only", action="store_true",
                    help="only the timed fwd+bwd steps (for profiling: no forward-only, per-mesh or CPU legs)")
    ap.add_argument("--no-graph", action="store_true", help="batch64: time eager steps instead of graph replays")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration for rocprofv3)")
    ap.add_argument("--summarize-counters", action="store_true",
                    help="write profiles/traffic.json from rocprofv3 counter CSVs (see --*-csv)")
    ap.add_argument("--summarize-trace", action="store_true",
                    help="print a markdown summary of a rocprofv3 kernel_stats.csv (--trace-csv)")
    ap.add_argument("--trace-csv")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--oracle-single-thread", action="store_true",
                    help="(child process) time the oracle on one thread on the cube and icosphere configs")
    ap.add_argument("--fetch-csv")
    ap.add_argument("--write-csv")
    ap.add_argument("--copy-fetch-csv")
    ap.add_argument("--copy-write-csv")
    args = ap.parse_args()
    if args.oracle_single_thread:
        return _oracle_single_thread_child(args.cpu_budget)
    if args.summarize_counters:
        return summarize_counters(args)
    if args.summarize_trace:
        return summarize_trace(args)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this implementation runs on one GPU; multi-GPU runs are not part of it "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4,
                          "launches": 3}))
        return
    if args.workload == "batch64":
        return bench_batch(args)
    return bench_single(args)


if __name__ == "__main__":
    main()
