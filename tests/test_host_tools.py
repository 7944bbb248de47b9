"""Host logic without a GPU: the schedule autotuner's search and cache, and the
roofline arithmetic of bench.py."""
import json
import os

import pytest

import paper_1903_00353_amd as P
from paper_1903_00353_amd import autotune

import bench


def fake_stage_times(opt):
    """Per-stage ms of a made-up workload: faces fastest at 32 rows, edges at 8,
    vertices with no overflow pass; grid 2 and absorb 0.1 fastest."""
    rows = tuple(opt.small_rows)
    cost = {8: 3.0, 16: 2.0, 24: 1.5, 32: 1.0, 40: 1.2, 48: 1.3, 64: 1.5, 96: 2.0, 128: 2.5, 1 << 24: 4.0}
    t = {k: 0.0 for k in autotune.FORWARD_STAGES}
    t["scan_faces"] = cost[rows[0]]
    t["scan_edges"] = {8: 0.5}.get(rows[1], 1.0)
    t["scan_vertices"] = 0.2 if rows[2] == 1 << 24 else 0.3
    t["sign"] = {1: 0.4, 2: 0.3, 3: 0.5}.get(opt.scan_grid, 0.4)  # 0: the library default
    t["init_keys"] = abs(opt.absorb_cells - 0.1) if opt.absorb_cells > 0 else 0.5
    t["build_features"] = {0: 0.5, 128: 0.45, 256: 0.4, 512: 0.42}[opt.geom_blocks]
    for k in ("scan_faces", "scan_edges", "scan_vertices"):
        t[k + "_big"] = 0.0
    return t


def test_search_picks_each_minimum_in_turn():
    base = P.make_options()
    choice, timings = autotune._search(lambda opt, reps: fake_stage_times(opt), base, 1)
    rows, grid, absorb, geom = choice
    assert rows == (32, 8, 1 << 24)
    assert grid == 2
    assert absorb == 0.1
    assert geom == 0  # not tuned without the build's time (single meshes)
    assert set(timings) >= {f"rows={c}" for c in autotune.CANDIDATES}
    opt = autotune.options_for(choice)
    assert tuple(opt.small_rows) == rows and opt.scan_grid == 2 and abs(opt.absorb_cells - 0.1) < 1e-7
    choice, timings = autotune._search(lambda opt, reps: fake_stage_times(opt), base, 1, build=True)
    assert choice[:3] == (rows, grid, absorb) and choice[3] == 256
    assert set(timings) >= {f"geom={g}" for g in autotune.GEOM_CANDIDATES}
    assert autotune.options_for(choice).geom_blocks == 256


def test_batch_search_scores_grid_and_absorb_by_step():
    """A batch's measurements carry its whole step's time ("step"): the grid and
    the absorption cap are chosen on it, not on the sum of the stages, which
    overlap in a batch (here the stage sum favours grid 2 and cap 0.2, the step
    grid 1 and cap 0.1)."""
    def stages(opt):
        t = fake_stage_times(opt)
        t["init_keys"] = 0.0 if abs(opt.absorb_cells - 0.2) < 1e-6 else 0.05
        return t

    def with_step(opt):
        t = stages(opt)
        t["step"] = 2.0 + abs(opt.absorb_cells - 0.1) + {1: 0.0, 2: 0.1, 3: 0.2}.get(opt.scan_grid, 0.1)
        return t

    base = P.make_options()
    assert autotune._search(lambda opt, reps: stages(opt), base, 1)[0][1:3] == (2, 0.2)
    choice, timings = autotune._search(lambda opt, reps: with_step(opt), base, 1, build=True)
    assert choice[1:3] == (1, 0.1)
    assert timings["absorb=0.1"] == pytest.approx(2.0)


def test_batch_search_refines_rows_by_step():
    """For a batch the rows per kind are refined on the whole step: here the
    faces' own stage times favour 32 rows and the step 40."""
    def with_step(opt):
        t = fake_stage_times(opt)
        t["step"] = 2.0 + {40: 0.0}.get(opt.small_rows[0], 0.1) + 0.01 * (opt.small_rows[1] != 8)
        return t
    rows = autotune._search(lambda opt, reps: fake_stage_times(opt), P.make_options(), 1)[0][0]
    assert rows[0] == 32
    choice, timings = autotune._search(lambda opt, reps: with_step(opt), P.make_options(), 1, build=True)
    assert choice[0][:2] == (40, 8)
    assert timings["rows0=40"] == pytest.approx(2.0)


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("CSC_AUTOTUNE_CACHE", str(path))
    assert autotune.load("sig") is None
    autotune.save("sig", ((32, 8, 16), 3, 0.02, 256), {"grid=3": 1.0})
    assert autotune.load("sig") == ((32, 8, 16), 3, 0.02, 256)
    rec = json.loads(path.read_text())
    assert rec["sig"]["ms"] == {"grid=3": 1.0}
    path.write_text("not json")
    assert autotune.load("sig") is None  # a damaged cache means: tune again


def test_roofline_arithmetic():
    per_step = {"init_keys": 0.05, "scan_faces": 0.30, "sign": 0.15, "backward": 0.40}
    avg = dict(per_step)
    atomics = [10_000_000, 0, 0, 0, 0, 0]
    rates = {"scan_faces": {"rate_G_per_s": 40.0}, "all": {"rate_G_per_s": 50.0}}
    alg = {"init_keys": 400e6, "scan_faces": 100e6, "sign": 200e6, "backward": 800e6}
    main, per, dom, fwd = bench.rooflines(avg, per_step, atomics, rates, lambda st: alg[st], 300e6, 0.45)
    # face scan: 10M atomics in 0.30 ms = 33.3 G/s of 40 G/s
    assert per["scan_faces"]["atomic_frac"] == pytest.approx(10e6 / 0.30e-3 / 40e9)
    assert per["backward"]["hbm_frac"] == pytest.approx(800e6 / 0.40e-3 / 8e12)
    assert dom == "scan_faces"  # the slowest kernel of the forward pass
    assert main["slowest_kernel"]["kernel"] == bench.KERNEL_SYMBOL["backward"]
    # forward: T_roof = max(300 MB / 8 TB/s, 10M / 50 G/s) = 0.2 ms over the 0.45 ms span
    assert fwd["t_roof_ms"] == pytest.approx(0.2)
    assert fwd["frac"] == pytest.approx(0.2 / 0.45)
    assert fwd["ms_stages_one_by_one"] == pytest.approx(0.50)
    assert main["forward_frac"] == fwd["frac"]


def test_algorithmic_bytes_of_a_kept_empty_store():
    """With the key store kept empty (as a Batch does) the store is not filled and
    the sign pass also writes each consumed key back."""
    info = {"n_faces": 4, "n_edges": 6, "max_band_cells": 512 * 3}
    assert bench.algorithmic_bytes("init_keys", info, [0] * 6, 100, 0, 4) == 8 * 512 * 3
    assert bench.algorithmic_bytes("init_keys", info, [0] * 6, 100, 0, 4, kept_store=True) == 72
    assert bench.algorithmic_bytes("sign", info, [0] * 6, 100, 0, 4) == 20 * 100
    assert bench.algorithmic_bytes("sign", info, [0] * 6, 100, 0, 4, kept_store=True) == 28 * 100
    assert bench.batch_algorithmic_bytes("init_keys", 4, 4, 0, 0, [0] * 6, 100, 0, 512 * 3) == 72


def test_brick_cells_and_forward_bytes():
    assert bench.brick_cells({"max_band_cells": 512 * 7, "n_bricks": 7}) == 512
    assert bench.forward_bytes(10, 20, 30, [1, 2, 3, 4, 5, 6], 100) == 12 * 10 + 12 * 20 + 16 * 30 + 8 * 21 + 16 * 100


def test_cpu_host_info():
    h = bench.host_info()
    assert h["nproc"] == os.cpu_count()
