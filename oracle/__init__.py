"""TEST INFRASTRUCTURE ONLY -- the CPU oracle of the narrow-band signed distance field.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It shares no code with the device path
(``paper_1903_00353_amd``) and neither imports the other; both read the same
float32 mesh arrays from ``meshgen``.

``csc_oracle.c`` (plain C, FP64, OpenMP) computes, from the definitions:
  * the exact distance from every cell centre to the closed triangle set (Eq. 1,
    Section 2), via an exact bounding-box cull and the closest point of each
    candidate triangle;
  * the band d < band * h (Section 10) and the sign from the angle-weighted
    pseudonormal of the closest feature (Eq. 8, Section 4.1.3);
  * the canonical feature id of each band cell and, for any claimed feature, the
    distance to it (to check a device result's feature against the tie rule);
  * the gradient of sum_c up_c * SDF_c with respect to the vertices, with each
    cell's closest feature held fixed;
  * the generalised winding number (an independent inside/outside test).

``weld_soup`` (NumPy) turns a triangle soup into an indexed mesh by exact
equality of corner positions (Section 7), vertices numbered in order of first
appearance.

``allpairs_distance`` is a second, literal all-pairs implementation in NumPy
using a different formulation of the point-triangle distance (projection onto
the plane, else the nearest of the three edges), used to pin the C code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csc_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

FLAG_IN_BAND, FLAG_NEAR_SURFACE, FLAG_NEAR_BAND_EDGE = 1, 2, 4


def build() -> str:
    """Compile the oracle with gcc (no fast-math: FP64 evaluation as written)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
                    "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Band(C.Structure):
    _fields_ = [("count", C.c_int64), ("cell", C.POINTER(C.c_int32)), ("d", C.POINTER(C.c_double)),
                ("sdf", C.POINTER(C.c_double)), ("tri", C.POINTER(C.c_int32)),
                ("feat", C.POINTER(C.c_int32)), ("flags", C.POINTER(C.c_uint8)), ("threads", C.c_int32)]


def _load(path=None):
    global _lib
    if _lib is not None and path is None:
        return _lib
    if path is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        path = _LIB
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.oracle_edges.restype = C.c_int64
    lib.oracle_edges.argtypes = [P, C.c_int64, C.c_int64, P, P]
    lib.oracle_normals.restype = None
    lib.oracle_normals.argtypes = [P, C.c_int64, P, C.c_int64, P, C.c_int64, P, P, P]
    lib.oracle_band.restype = C.c_int
    lib.oracle_band.argtypes = [P, C.c_int64, P, C.c_int64, P, C.c_int64, P, P, P, P, C.c_double, P,
                                C.c_double, C.c_int32, C.c_int32, C.POINTER(_Band)]
    lib.oracle_band_free.restype = None
    lib.oracle_band_free.argtypes = [C.POINTER(_Band)]
    lib.oracle_cells_dist.restype = None
    lib.oracle_cells_dist.argtypes = [P, P, C.c_int64, P, C.c_int64, P, C.c_double, P, P, C.c_int64, P, P]
    lib.oracle_feature_dist.restype = None
    lib.oracle_feature_dist.argtypes = [P, P, P, C.c_int64, C.c_int64, P, C.c_double, P, P, P, C.c_int64, P]
    lib.oracle_grad.restype = None
    lib.oracle_grad.argtypes = [P, C.c_int64, P, P, C.c_int64, C.c_int64, P, C.c_double, P, P, P, P, P,
                                C.c_int64, P]
    lib.oracle_winding.restype = None
    lib.oracle_winding.argtypes = [P, P, C.c_int64, P, C.c_int64, P]
    lib.oracle_max_threads.restype = C.c_int
    _lib = lib
    return lib


class library:
    """Context manager: run the oracle from another compiled copy (used by the tests
    that plant a mistake in a copy of the source and check that a pin catches it)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.prev = _lib
        _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.prev
        return False


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _grid_args(grid):
    o = np.ascontiguousarray(grid.origin, dtype=np.float64)
    n = np.ascontiguousarray(grid.n, dtype=np.int32)
    return o, float(grid.h), n


class OracleMesh:
    """FP64 view of a float32 mesh with its features numbered as faces, edges, vertices."""

    def __init__(self, verts, tris, V64=None):
        lib = _load()
        self.T = np.ascontiguousarray(tris, dtype=np.int32)
        self.V = np.ascontiguousarray(np.asarray(verts, dtype=np.float32).astype(np.float64)
                                      if V64 is None else V64, dtype=np.float64)
        self.F, self.nv = self.T.shape[0], self.V.shape[0]
        self.face_edges = np.empty(3 * self.F, dtype=np.int32)
        edges = np.empty(4 * ((3 * self.F) // 2 + 1), dtype=np.int32)
        E = lib.oracle_edges(_p(self.T), self.F, self.nv, _p(self.face_edges), _p(edges))
        if E < 0:
            raise ValueError("mesh is not a closed, consistently oriented 2-manifold")
        self.E = int(E)
        self.edges = edges[: 4 * self.E].reshape(self.E, 4).copy()
        self.fn = np.empty((self.F, 3))
        self.en = np.empty((self.E, 3))
        self.vn = np.empty((self.nv, 3))
        lib.oracle_normals(_p(self.V), self.nv, _p(self.T), self.F, _p(self.edges), self.E,
                           _p(self.fn), _p(self.en), _p(self.vn))

    @property
    def n_features(self):
        return self.F + self.E + self.nv

    def band(self, grid, k0: int = 0, k1: int | None = None) -> dict:
        """Cells with d < band*h + 1e-6 h in z-planes [k0, k1), ascending cell index."""
        lib = _load()
        o, h, n = _grid_args(grid)
        k1 = int(n[2]) if k1 is None else int(k1)
        b = _Band()
        rc = lib.oracle_band(_p(self.V), self.nv, _p(self.T), self.F, _p(self.face_edges), self.E,
                             _p(self.fn), _p(self.en), _p(self.vn), _p(o), h, _p(n), float(grid.band),
                             int(k0), k1, C.byref(b))
        if rc != 0:
            raise MemoryError("oracle_band failed")
        m = int(b.count)

        def grab(ptr, dt):
            return np.ctypeslib.as_array(ptr, shape=(m,)).astype(dt, copy=True) if m else np.empty(0, dt)
        out = dict(cell=grab(b.cell, np.int64), d=grab(b.d, np.float64), sdf=grab(b.sdf, np.float64),
                   tri=grab(b.tri, np.int32), feat=grab(b.feat, np.int32), flags=grab(b.flags, np.uint8),
                   threads=int(b.threads))
        lib.oracle_band_free(C.byref(b))
        return out

    def cells_dist(self, grid, cells, sub=None, V64=None):
        """Distance from listed cells to the triangles ``sub`` (default all), every one tried."""
        lib = _load()
        o, h, n = _grid_args(grid)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        V = self.V if V64 is None else np.ascontiguousarray(V64, dtype=np.float64)
        sub = None if sub is None else np.ascontiguousarray(sub, dtype=np.int64)
        d = np.empty(cells.shape[0])
        t = np.empty(cells.shape[0], dtype=np.int32)
        lib.oracle_cells_dist(_p(V), _p(self.T), self.F, _p(sub), 0 if sub is None else sub.shape[0],
                              _p(o), h, _p(n), _p(cells), cells.shape[0], _p(d), _p(t))
        return d, t

    def feature_dist(self, grid, cells, feats):
        lib = _load()
        o, h, n = _grid_args(grid)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        feats = np.ascontiguousarray(feats, dtype=np.int32)
        out = np.empty(cells.shape[0])
        lib.oracle_feature_dist(_p(self.V), _p(self.T), _p(self.edges), self.F, self.E, _p(o), h, _p(n),
                                _p(cells), _p(feats), cells.shape[0], _p(out))
        return out

    def grad(self, grid, cells, feats, sign, up):
        lib = _load()
        o, h, n = _grid_args(grid)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        feats = np.ascontiguousarray(feats, dtype=np.int32)
        sign = np.ascontiguousarray(sign, dtype=np.float64)
        up = np.ascontiguousarray(up, dtype=np.float64)
        g = np.empty((self.nv, 3))
        lib.oracle_grad(_p(self.V), self.nv, _p(self.T), _p(self.edges), self.F, self.E, _p(o), h, _p(n),
                        _p(cells), _p(feats), _p(sign), _p(up), cells.shape[0], _p(g))
        return g

    def winding(self, pts):
        lib = _load()
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        out = np.empty(pts.shape[0])
        lib.oracle_winding(_p(self.V), _p(self.T), self.F, _p(pts), pts.shape[0], _p(out))
        return out


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def cell_centres(grid, cells):
    cells = np.asarray(cells, dtype=np.int64)
    n0, n1 = int(grid.n[0]), int(grid.n[1])
    i, j, k = cells % n0, (cells // n0) % n1, cells // (n0 * n1)
    o = np.asarray(grid.origin, dtype=np.float64)
    return o + (np.stack([i, j, k], 1) + 0.5) * float(grid.h)


def _seg_dist2(p, a, b):
    ab = b - a
    t = np.clip(np.einsum("...k,...k->...", p - a, ab) / np.einsum("...k,...k->...", ab, ab), 0.0, 1.0)
    r = p - (a + t[..., None] * ab)
    return np.einsum("...k,...k->...", r, r)


def allpairs_distance(verts, tris, points, chunk=4096):
    """Literal all-pairs unsigned distance from each point to the closed triangle
    set: for every (point, triangle) pair, the plane distance when the projection
    falls inside the triangle (all barycentric coordinates >= 0), else the least
    distance to its three edges. Independent of the C code's closest-point method."""
    V = np.asarray(verts, dtype=np.float32).astype(np.float64)
    a, b, c = V[tris[:, 0]], V[tris[:, 1]], V[tris[:, 2]]
    n = np.cross(b - a, c - a)
    nn = np.einsum("ij,ij->i", n, n)
    out = np.empty(points.shape[0])
    for s in range(0, points.shape[0], chunk):
        p = points[s:s + chunk, None, :]  # (m,1,3)
        ap = p - a[None]
        t = np.einsum("mfk,fk->mf", ap, n) / nn[None]
        proj = p - t[..., None] * n[None]
        # barycentric coordinates of the projection via signed sub-areas
        l0 = np.einsum("mfk,fk->mf", np.cross(c[None] - b[None], proj - b[None]), n) / nn[None]
        l1 = np.einsum("mfk,fk->mf", np.cross(a[None] - c[None], proj - c[None]), n) / nn[None]
        l2 = 1.0 - l0 - l1
        inside = (l0 >= 0) & (l1 >= 0) & (l2 >= 0)
        dplane2 = t * t * nn[None]
        de = np.minimum(np.minimum(_seg_dist2(p, a[None], b[None]), _seg_dist2(p, b[None], c[None])),
                        _seg_dist2(p, c[None], a[None]))
        d2 = np.where(inside, dplane2, de)
        out[s:s + chunk] = np.sqrt(d2.min(axis=1))
    return out


def weld_soup(soup):
    """Indexed mesh of a triangle soup (Section 7: every STL triangle lists its
    own corners; equal positions are one vertex). soup: [F, 3, 3] float32.
    Positions compare by float value (-0 == +0). Vertices are numbered in order
    of first appearance in corner order 3f + j; returns (verts [V, 3] float32
    holding each vertex's first corner as given, tris [F, 3] int32)."""
    c = np.asarray(soup, dtype=np.float32).reshape(-1, 3)
    key = np.where(c == 0, np.float32(0), c)                      # -0 -> +0
    _, first, inverse = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inverse = inverse.reshape(-1)
    order = np.argsort(first, kind="stable")                      # groups by first appearance
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    tris = rank[inverse].astype(np.int32).reshape(-1, 3)
    verts = c[first[order]].copy()
    return verts, tris

