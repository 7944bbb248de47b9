"""Schedule autotuner.

The one schedule choice of the scan conversion is, per polyhedron kind (faces,
edges, vertices), the number of rows above which a polyhedron is walked by a
whole wavefront instead of a single thread. Only the speed depends on it. The
tuner times each candidate on the caller's own workload with the library's
stage events (HIP events on the working stream), keeps the fastest per kind,
and caches the choice as JSON keyed by the device and the workload's shape.
"""
from __future__ import annotations

import json
import math
import os

CANDIDATES = (8, 16, 32, 64, 128, 1 << 24)
KIND_STAGES = ("scan_faces", "scan_edges", "scan_vertices")


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
            f"|cells=2^{round(math.log2(max(cells, 1)))}|band={band:g}|tpc=2^{round(math.log2(max(tri_cells, 1e-9)))}")


def load(sig: str):
    try:
        with open(cache_path()) as fh:
            rec = json.load(fh).get(sig)
        return tuple(rec["small_rows"]) if rec else None
    except (OSError, ValueError, KeyError):
        return None


def save(sig: str, small_rows, timings):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        try:
            with open(path) as fh:
                data = json.load(fh)
        except (OSError, ValueError):
            data = {}
        data[sig] = {"small_rows": list(small_rows), "ms": timings}
        with open(path + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def _time_stages(run, reps):
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
    t = P.csc_timing_read()
    # each kind's time = its one-thread-per-polyhedron launch + its overflow launch
    return [t[k][0] / max(1, t[k][1]) + t[k + "_big"][0] / max(1, t[k + "_big"][1]) for k in KIND_STAGES]


def tune_batch(batch, candidates=CANDIDATES, reps=3, use_cache=True):
    """Pick small_rows per kind for a paper_1903_00353_amd.Batch; rebuilds it with the
    choice (before any graph capture). Returns (small_rows, {candidate: [ms per kind]})."""
    import paper_1903_00353_amd as P
    sig = signature(batch.nf, batch.grids)
    base = batch.options if batch.options is not None else P.make_options()
    best = load(sig) if use_cache else None
    timings = {}
    if best is None:
        for c in candidates:
            batch.options = _with_rows(base, (c, c, c))
            batch.f = P.csc_build_features_batched(batch.verts, batch.tris, batch.nv, batch.nf, batch.grids,
                                                   batch.options, flags=batch.flags, reuse=batch.f)
            timings[c] = _time_stages(batch.step, reps)
        best = tuple(min(candidates, key=lambda c: timings[c][k]) for k in range(3))
        save(sig, best, {str(c): v for c, v in timings.items()})
    batch.options = _with_rows(base, best)
    batch.f = P.csc_build_features_batched(batch.verts, batch.tris, batch.nv, batch.nf, batch.grids, batch.options,
                                           flags=batch.flags, reuse=batch.f)
    return best, timings


def tune_single(verts, tris, grid, options=None, candidates=CANDIDATES, reps=3, use_cache=True):
    """small_rows for one mesh (single-mesh entry points); returns (small_rows, timings)."""
    import torch

    import paper_1903_00353_amd as P
    sig = signature([tris.shape[0]], [grid])
    base = options if options is not None else P.make_options()
    best = load(sig) if use_cache else None
    timings = {}
    if best is None:
        f = None
        for c in candidates:
            opt = _with_rows(base, (c, c, c))
            f = P.csc_build_features(verts, tris, grid, opt, reuse=f)
            nbytes, mx = P.csc_scan_convert_workspace(f)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=verts.device)
            out = (torch.empty(mx, dtype=torch.float32, device=verts.device),
                   torch.empty(mx, dtype=torch.int32, device=verts.device),
                   torch.empty(mx, dtype=torch.int32, device=verts.device),
                   torch.zeros(1, dtype=torch.int64, device=verts.device))
            timings[c] = _time_stages(lambda: P.csc_scan_convert(f, ws, out, sync_count=False), reps)
        f.free()
        best = tuple(min(candidates, key=lambda c: timings[c][k]) for k in range(3))
        save(sig, best, {str(c): v for c, v in timings.items()})
    return best, timings


def _with_rows(opt, rows):
    import paper_1903_00353_amd as P
    return P.make_options(opt.eps_rel, opt.ruff_mode, opt.saddle_mode, opt.force_both_sides, rows, opt.scan_mode,
                          opt.absorb_cells)
