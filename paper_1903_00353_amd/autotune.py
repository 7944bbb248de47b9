"""Schedule autotuner.

The scan conversion has three schedule choices, none of which changes a value:
  * per polyhedron kind (faces, edges, vertices), the number of rows above which
    a polyhedron is walked in chunks by whole wavefronts instead of by one lane
    (``small_rows``);
  * how the one-lane-per-polyhedron pass hands out its polyhedra (``scan_grid``:
    a launch sized to the items, a persistent grid striding over them, or a
    persistent grid taking groups from a device counter);
  * the largest side slack a face prism takes on to absorb the extrusions of
    nearly flat edges and vertices (``absorb_cells``; negative: none absorbed);
  * for a batch, the grid of the build's face pass, which runs beside the
    corner sort (``geom_blocks``: 0 one thread per face, or a capped grid that
    leaves the sort compute units of its own).
The tuner times candidates on the caller's own workload with the library's stage
events (HIP events on the working stream): first ``small_rows`` per kind (each
kind's one-lane launch plus its overflow launch), then ``scan_grid`` and
``absorb_cells`` one after the other on the time of the whole forward pass
(scans and sign; for a batch, whose edge and vertex kinds run on a second
stream beside the faces, so that stage times do not add up, on the time of
its whole step, on which a batch's rows per kind are refined as well), then
(batches) ``geom_blocks`` on the build's time. It caches
the choice as JSON keyed by the device and the workload's shape.
"""
from __future__ import annotations

import json
import math
import os

CANDIDATES = (8, 16, 24, 32, 40, 48, 64, 96, 128, 1 << 24)
GRID_CANDIDATES = (1, 2, 3)
ABSORB_CANDIDATES = (-1.0, 0.02, 0.05, 0.1, 0.2)
GEOM_CANDIDATES = (0, 128, 256, 512)
KIND_STAGES = ("scan_faces", "scan_edges", "scan_vertices")
FORWARD_STAGES = ("init_keys", "scan_faces", "scan_edges", "scan_vertices", "scan_faces_big", "scan_edges_big",
                  "scan_vertices_big", "scan_wide", "brick_count", "sign")


def cache_path() -> str:
    return os.environ.get("CSC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1903_00353_amd", "autotune.json"))


def signature(nf_list, grids) -> str:
    """Device plus a coarse shape: total faces, cells and band (log2 buckets)."""
    import torch
    dev = torch.cuda.get_device_properties(0)
    faces = sum(int(x) for x in nf_list)
    cells = sum(int(g.n[0]) * int(g.n[1]) * int(g.n[2]) for g in grids)
    band = max(float(g.band) for g in grids)
    tri_cells = faces / max(1.0, cells ** (2.0 / 3.0))  # triangles per cell of surface area (rough)
    return (f"{getattr(dev, 'gcnArchName', dev.name)}|n={len(grids)}|F=2^{round(math.log2(max(faces, 1)))}"
            f"|cells=2^{round(math.log2(max(cells, 1)))}|band={band:g}|tpc=2^{round(math.log2(max(tri_cells, 1e-9)))}"
            f"|v6")


def load(sig: str):
    try:
        with open(cache_path()) as fh:
            rec = json.load(fh).get(sig)
        return ((tuple(rec["small_rows"]), int(rec["scan_grid"]), float(rec["absorb_cells"]), int(rec["geom_blocks"]))
                if rec else None)
    except (OSError, ValueError, KeyError, TypeError):
        return None


def save(sig: str, choice, timings):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        try:
            with open(path) as fh:
                data = json.load(fh)
        except (OSError, ValueError):
            data = {}
        data[sig] = {"small_rows": list(choice[0]), "scan_grid": choice[1], "absorb_cells": choice[2],
                     "geom_blocks": choice[3], "ms": timings}
        with open(path + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def _stage_times(run, reps):
    import torch

    import paper_1903_00353_amd as P
    run()
    torch.cuda.synchronize()
    P.csc_timing_reset()
    P.csc_timing_enable(True)
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    P.csc_timing_enable(False)
    return {k: ms / reps for k, (ms, c) in P.csc_timing_read().items()}


def _kind_times(t):
    # each kind's time = its one-lane-per-polyhedron launch + its overflow launch
    return [t[k] + t[k + "_big"] for k in KIND_STAGES]


def _forward_time(t):
    return sum(t[k] for k in FORWARD_STAGES)


def _score(t):
    # a batch's measurements carry its whole step's time (kinds overlapped)
    return t["step"] if "step" in t else _forward_time(t)


def _step_time(run, reps):
    import torch
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _search(measure, base, reps, build=False):
    """measure(options) -> per-stage ms per call; returns (choice, timings).
    build: measure also times the build (its stage), and geom_blocks is tuned."""
    timings = {}
    for c in CANDIDATES:
        timings[f"rows={c}"] = measure(_with(base, rows=(c, c, c)), reps)
    rows = tuple(min(CANDIDATES, key=lambda c: _kind_times(timings[f"rows={c}"])[k]) for k in range(3))
    if build:
        # a batch: its kinds overlap on two streams, so each kind's rows are
        # refined, one kind after the other, on the whole step
        rows = list(rows)
        for k in range(3):
            best_t = None
            for c in CANDIDATES:
                r = tuple(c if j == k else rows[j] for j in range(3))
                t = _score(measure(_with(base, rows=r), reps))
                timings[f"rows{k}={c}"] = t
                if best_t is None or t < best_t:
                    rows[k], best_t = c, t
        rows = tuple(rows)
    best_grid, best_t = base.scan_grid or 2, None
    for g in GRID_CANDIDATES:
        t = _score(measure(_with(base, rows=rows, grid=g), reps))
        timings[f"grid={g}"] = t
        if best_t is None or t < best_t:
            best_grid, best_t = g, t
    best_absorb, best_t = 0.05, None
    for a in ABSORB_CANDIDATES:
        t = _score(measure(_with(base, rows=rows, grid=best_grid, absorb=a), reps))
        timings[f"absorb={a}"] = t
        if best_t is None or t < best_t:
            best_absorb, best_t = a, t
    best_geom = base.geom_blocks
    if build:
        best_t = None
        for gb in GEOM_CANDIDATES:
            t = measure(_with(base, rows=rows, grid=best_grid, absorb=best_absorb, geom=gb), reps)["build_features"]
            timings[f"geom={gb}"] = t
            if best_t is None or t < best_t:
                best_geom, best_t = gb, t
    return (rows, best_grid, best_absorb, best_geom), timings


def tune_batch(batch, reps=3, use_cache=True):
    """Pick the schedule for a paper_1903_00353_amd.Batch; rebuilds it with the
    choice (before any graph capture). Returns ((small_rows, scan_grid,
    absorb_cells, geom_blocks), timings)."""
    import paper_1903_00353_amd as P
    sig = signature(batch.nf, batch.grids)
    base = batch.options if batch.options is not None else P.make_options()
    choice = load(sig) if use_cache else None
    timings = {}

    def rebuild(opt):
        batch.options = opt
        batch.f = P.csc_build_features_batched(batch.verts, batch.tris, batch.nv, batch.nf, batch.grids,
                                               batch.options, flags=batch.flags, reuse=batch.f)

    if choice is None:
        def measure(opt, reps):
            rebuild(opt)
            t = _stage_times(batch.step, reps)
            t["step"] = _step_time(batch.step, max(40, reps))  # stage timing off: kinds overlapped
            return t
        choice, timings = _search(measure, base, reps, build=True)
        save(sig, choice, timings)
    rebuild(options_for(choice, base))
    return choice, timings


def tune_single(verts, tris, grid, options=None, reps=3, use_cache=True):
    """The schedule for one mesh (single-mesh entry points); returns (choice, timings)."""
    import torch

    import paper_1903_00353_amd as P
    sig = signature([tris.shape[0]], [grid])
    base = options if options is not None else P.make_options()
    choice = load(sig) if use_cache else None
    timings = {}
    if choice is None:
        def measure(opt, reps):
            f = P.csc_build_features(verts, tris, grid, opt)
            nbytes, mx = P.csc_scan_convert_workspace(f)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=verts.device)
            out = (torch.empty(mx, dtype=torch.float32, device=verts.device),
                   torch.empty(mx, dtype=torch.int32, device=verts.device),
                   torch.empty(mx, dtype=torch.int32, device=verts.device),
                   torch.zeros(1, dtype=torch.int64, device=verts.device))
            t = _stage_times(lambda: P.csc_scan_convert(f, ws, out, sync_count=False), reps)
            f.free()
            return t
        choice, timings = _search(measure, base, reps)
        save(sig, choice, timings)
    return choice, timings


def options_for(choice, base=None):
    """csc_options with a tuner choice (small_rows, scan_grid, absorb_cells[,
    geom_blocks]) applied."""
    import paper_1903_00353_amd as P
    base = base if base is not None else P.make_options()
    return _with(base, rows=choice[0], grid=choice[1], absorb=choice[2], geom=choice[3] if len(choice) > 3 else None)


def _with(opt, rows=None, grid=None, absorb=None, geom=None):
    import paper_1903_00353_amd as P
    return P.make_options(opt.eps_rel, opt.ruff_mode, opt.saddle_mode, opt.force_both_sides,
                          tuple(opt.small_rows) if rows is None else rows, opt.scan_mode,
                          opt.absorb_cells if absorb is None else absorb,
                          opt.scan_grid if grid is None else grid,
                          opt.geom_blocks if geom is None else geom, opt.keep_store_empty)
