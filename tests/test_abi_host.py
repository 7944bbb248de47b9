"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, rejects bad arguments before touching a device, and its host-evaluated
classification predicates agree with hand-built configurations."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1903_00353_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "csc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(csc_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    L = P.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(P.EXPORTS)


def test_error_strings():
    for code in range(10):
        assert P.csc_error_string(code)
    assert P.csc_error_string(0) == "ok"


def _grid(n=(8, 8, 8), h=0.125, band=2.0, origin=(0.0, 0.0, 0.0)):
    g = P.csc_grid()
    for k in range(3):
        g.n[k] = n[k]
        g.origin[k] = origin[k]
    g.h = h
    g.band_cells = band
    return g


@pytest.mark.parametrize("case", ["null", "nv0", "nf0", "odd_faces", "grid_n", "grid_h", "band", "origin_nan",
                                  "too_many_cells", "long_axis", "bad_option",
                                  "bad_scan_mode", "absorb_too_wide", "absorb_nan", "bad_scan_grid",
                                  "bad_geom_blocks", "bad_keep_store_empty"])
def test_host_argument_checks(case):
    """Checked on the host before any device call: these never need a GPU."""
    L = P.lib()
    fake = C.c_void_p(0x1000)  # never dereferenced: every case fails its host check first
    g = _grid()
    opt = P.make_options()
    nv, nf, v, t = 8, 12, fake, fake
    out = C.c_void_p(None)
    if case == "null":
        v = None
    elif case == "nv0":
        nv = 0
    elif case == "nf0":
        nf = -1
    elif case == "odd_faces":
        nf = 13
    elif case == "grid_n":
        g.n[1] = 0
    elif case == "grid_h":
        g.h = 0.0
    elif case == "band":
        g.band_cells = -1.0
    elif case == "origin_nan":
        g.origin[2] = float("nan")
    elif case == "too_many_cells":
        g.n[0], g.n[1], g.n[2] = 2048, 2048, 1024
    elif case == "long_axis":  # few cells, but one axis beyond 16-bit cell offsets
        g.n[0], g.n[1], g.n[2] = 65536, 4, 4
    elif case == "bad_option":
        opt.saddle_mode = 7
    elif case == "bad_scan_mode":
        opt.scan_mode = 2
    elif case == "absorb_too_wide":  # the absorption proof needs the slack below a quarter cell
        opt.absorb_cells = 0.3
    elif case == "absorb_nan":
        opt.absorb_cells = float("nan")
    elif case == "bad_scan_grid":
        opt.scan_grid = 4
    elif case == "bad_geom_blocks":
        opt.geom_blocks = -1
    elif case == "bad_keep_store_empty":
        opt.keep_store_empty = 2
    code = L.csc_build_features(v, nv, t, nf, C.byref(g), C.byref(opt), None, C.byref(out))
    expect = {"odd_faces": 2, "too_many_cells": 5, "long_axis": 5}.get(case, 1)
    assert code == expect
    assert out.value is None


def test_null_handle_calls():
    L = P.lib()
    nbytes, mx = C.c_size_t(), C.c_int64()
    assert L.csc_scan_convert_workspace(None, C.byref(nbytes), C.byref(mx)) == 1
    assert L.csc_scan_convert(None, None, 0, None, None, None, None, None, None) == 1
    assert L.csc_sdf_backward(None, None, None, None, 0, None, None, None, None) == 1
    assert L.csc_scan_convert_count(None, None, 0, None, None) == 1
    assert L.csc_features_info(None, None) == 1
    assert L.csc_interior_fill(None, None, None) == 1
    assert L.csc_features_order_faces(None, 1, None) == 1
    assert L.csc_features_order_faces(None, 0, None) == 1
    n = C.c_int64()
    assert L.csc_weld_soup(None, 1, None, None, C.byref(n), None) == 1
    assert L.csc_weld_soup(C.c_void_p(0x1000), 0, C.c_void_p(0x1000), C.c_void_p(0x1000), C.byref(n), None) == 1
    L.csc_features_free(None)


def test_timing_api_without_device():
    P.csc_timing_reset()
    t = P.csc_timing_read()
    assert list(t) == ["build_features", "init_keys", "scan_faces", "scan_edges", "scan_vertices", "brick_count",
                       "sign", "backward", "scan_faces_big", "scan_edges_big", "scan_vertices_big",
                       "interior_fill", "scan_wide"]
    assert all(v == (0.0, 0) for v in t.values())


def test_edge_classes_on_a_fold():
    a, b, c1 = [0, 0, 0], [1, 0, 0], [0, 1, 0]          # left face, normal +z
    assert P.csc_classify_edge(a, b, c1, [0.5, -1, -0.5]) == 1  # right face bends down: convex
    assert P.csc_classify_edge(a, b, c1, [0.5, -1, 0.5]) == 2   # bends up: concave
    assert P.csc_classify_edge(a, b, c1, [0.5, -1, 0.0]) == 0   # coplanar: flat
    # Integer coordinates (exact in float32) with nearly parallel spanning vectors:
    # u x v = (1, -1, -2) while |u||v| ~ 1.8e13, so the double-precision estimate
    # cannot decide and the exact expansion must.
    a = np.array([1000, 1000, 1000], np.float32)
    u = np.array([3000001, 2999999, 1], np.float32)
    v = np.array([3000000, 2999998, 1], np.float32)
    b, c1 = a + u, a + v
    ez = np.array([0, 0, 1], np.float32)
    assert P.csc_classify_edge(a, b, c1, a + ez) == 1   # det = ez . (u x v) = -2 < 0
    assert P.csc_classify_edge(a, b, c1, a - ez) == 2   # +2
    assert P.csc_classify_edge(a, b, c1, a + 2 * u - v) == 0  # exactly coplanar
    # the double-precision cofactor sum alone is not reliable here
    w = (2 * u - v).astype(np.float64)
    det = w @ np.cross(u.astype(np.float64), v.astype(np.float64))
    perm = np.abs(w[0] * u[1] * v[2]) + np.abs(w[0] * u[2] * v[1]) + np.abs(w[1] * u[2] * v[0])
    assert abs(det) <= 1e-12 * perm


def _fan(apex, ring_pts):
    """Incident triangles (apex, r_i, r_{i+1}) of a closed fan, counter-clockwise."""
    n = len(ring_pts)
    return np.array([[ring_pts[i], ring_pts[(i + 1) % n]] for i in range(n)], np.float32)


def test_vertex_classes_hand_fans():
    th = np.linspace(0, 2 * np.pi, 7)[:-1]
    circle = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], 1)
    apex = np.zeros(3)
    # convex pyramid: apex above the ring (neighbours below the pseudonormal plane)
    bits, ax, ct = P.csc_classify_vertex(apex + [0, 0, 0.5], _fan(apex, circle))
    assert bits & 16 and bits & 1 and not bits & 2
    assert np.allclose(ax, [0, 0, 1], atol=1e-9) and 0 < ct < 1
    # concave: apex below the ring
    bits, ax, ct = P.csc_classify_vertex(apex - [0, 0, 0.5], _fan(apex, circle))
    assert bits & 32 and bits & 2 and not bits & 1
    # flat fan: no extrusion
    bits, ax, ct = P.csc_classify_vertex(apex, _fan(apex, circle))
    assert bits & 64 and not bits & 3
    # saddle (monkey-saddle ring heights +,-,+,-,+,-): both sides
    sad = circle.copy()
    sad[:, 2] = 0.3 * np.cos(3 * th)
    bits, ax, ct = P.csc_classify_vertex(apex, _fan(apex, sad))
    assert bits & 128 and bits & 1 and bits & 2
    # saddle_mode 2 (ablation) drops its extrusions
    bits2, _, _ = P.csc_classify_vertex(apex, _fan(apex, sad), P.make_options(saddle_mode=2))
    assert bits2 & 128 and not bits2 & 3


def test_cone_contains_positive_normals():
    """The cone axis is the pseudonormal and its aperture contains every positive-pointing
    face normal (Eq. 9): each such normal makes cos >= cos_t with the axis."""
    rng = np.random.default_rng(0)
    for _ in range(20):
        n = int(rng.integers(4, 9))
        th = np.sort(rng.uniform(0, 2 * np.pi, n))
        ring = np.stack([np.cos(th), np.sin(th), rng.uniform(-0.6, -0.1, n)], 1)
        tris = _fan(np.zeros(3), ring)
        bits, ax, ct = P.csc_classify_vertex(np.zeros(3), tris)
        for p1, p2 in tris.astype(np.float64):
            nn = np.cross(p1, p2)
            nn /= np.linalg.norm(nn)
            c = nn @ ax
            if c > 0:
                assert c >= ct - 1e-12


def test_ruff_vertex_gets_hemisphere():
    """A convex fan (all neighbours below the pseudonormal plane) with a face normal
    pointing below that plane (a ruff, Section 3.3) gets a hemisphere by default and
    a cone in ruff_mode 1. The axis is checked against an independent NumPy
    angle-weighted pseudonormal (Eq. 8)."""
    ring = np.array([[-0.1411, 0.171, -0.2172], [-0.6171, 0.5723, -0.906], [-1.0759, 0.9915, -0.0267],
                     [-0.5709, -0.0136, -0.3105], [-0.7389, -0.9106, -0.999], [0.0405, -0.7746, -0.2695]],
                    np.float32)
    tris = _fan(np.zeros(3), ring).astype(np.float64)
    N = np.zeros(3)
    normals = []
    for p1, p2 in tris:
        nn = np.cross(p1, p2)
        nn /= np.linalg.norm(nn)
        alpha = np.arccos(np.clip(p1 @ p2 / np.linalg.norm(p1) / np.linalg.norm(p2), -1, 1))
        N += alpha * nn
        normals.append(nn)
    N /= np.linalg.norm(N)
    assert np.all(ring.astype(np.float64) @ N < 0)           # convex
    assert min(nn @ N for nn in normals) < 0                  # a normal points away: ruff
    bits, ax, ct = P.csc_classify_vertex(np.zeros(3), _fan(np.zeros(3), ring))
    assert np.allclose(ax, N, atol=1e-12)
    assert bits & 256 and bits & 16 and bits & 1 and not bits & 2, bits
    assert bits & 4                                           # outward extrusion: hemisphere
    assert abs(ct - min(nn @ N for nn in normals if nn @ N > 0)) < 1e-12
    bits1, _, _ = P.csc_classify_vertex(np.zeros(3), _fan(np.zeros(3), ring), P.make_options(ruff_mode=1))
    assert bits1 & 256 and not bits1 & 4


@pytest.mark.parametrize("case", ["n0", "null_sizes", "odd_faces_mesh1", "bad_grid_mesh2", "zero_verts", "flags"])
def test_batched_host_argument_checks(case):
    L = P.lib()
    fake = C.c_void_p(0x1000)  # never dereferenced: every case fails its host check first
    n = 3
    grids = (P.csc_grid * n)(*[_grid() for _ in range(n)])
    nv = (C.c_int64 * n)(8, 8, 8)
    nf = (C.c_int64 * n)(12, 12, 12)
    opt = P.make_options()
    out = C.c_void_p(None)
    flags = 0
    nn = n
    nva, nfa = nv, nf
    if case == "n0":
        nn = 0
    elif case == "null_sizes":
        nva = None
    elif case == "odd_faces_mesh1":
        nf[1] = 13
    elif case == "bad_grid_mesh2":
        grids[2].h = -1.0
    elif case == "zero_verts":
        nv[0] = 0
    elif case == "flags":
        flags = 1  # NO_SYNC without an existing handle
    code = L.csc_build_features_batched(fake, fake, nva, nfa, grids, nn, C.byref(opt), flags, None, C.byref(out))
    assert code == {"odd_faces_mesh1": 2}.get(case, 1)
    assert out.value is None
