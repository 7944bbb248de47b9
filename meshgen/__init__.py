"""Seeded synthetic inputs: closed, outward-oriented triangle meshes and grids.

These stand in for the paper's public STL models (Orion, the Stanford models,
DrivAer; Section 11, Tables 1-4), which are not reproduced here. They span the
same face-count range (tens of triangles to several million), are closed
orientable manifolds like the paper assumes (Section 6), and the jittered,
noisy and displaced variants produce the large saddle-vertex fractions the
paper reports for real scans (Table 2).

This module holds no part of the distance method: it only builds vertex and
index arrays and grid descriptors. Both the device path and the CPU oracle
read exactly the float32 arrays produced here (generated in float64, cast once).

Conventions (the paper does not fix them, Section 10):
  * grid cell (i, j, k) has centre origin + (i + 1/2, j + 1/2, k + 1/2) * h,
    linear index i + n0 * (j + n1 * k), x fastest;
  * the band half-width is ``band`` cells: a cell is in the band when its
    distance to the surface is strictly below band * h;
  * triangles are counter-clockwise seen from outside (outward normals);
  * every mesh is centred in the unit box, and the grids cover [0, 1]^3.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 190300353
CENTRE = np.array([0.5, 0.5, 0.5])


@dataclasses.dataclass(frozen=True)
class Grid:
    """Cartesian grid: ``n`` cells per axis of size ``h`` starting at ``origin``."""
    n: tuple
    h: float
    band: float
    origin: tuple = (0.0, 0.0, 0.0)

    @staticmethod
    def unit(N: int, band: float) -> "Grid":
        return Grid(n=(int(N), int(N), int(N)), h=1.0 / N, band=float(band))

    @property
    def ncells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


def _finish(v64: np.ndarray, tris: np.ndarray):
    """Cast once to the arrays both sides read, after checking orientation."""
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    v32 = np.ascontiguousarray(v64, dtype=np.float32)
    if signed_volume(v32, tris) < 0:
        tris = np.ascontiguousarray(tris[:, [0, 2, 1]])
    return v32, tris


def signed_volume(verts: np.ndarray, tris: np.ndarray) -> float:
    v = np.asarray(verts, dtype=np.float64)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


# --------------------------------------------------------------------------- cube
def cube(side: float = 0.5, centre=CENTRE):
    """Axis-aligned cube, each square face split into two triangles (12 F, 18 E, 8 V)."""
    s = side / 2.0
    v = np.array([[x, y, z] for z in (-s, s) for y in (-s, s) for x in (-s, s)]) + centre
    # vertex id = x + 2y + 4z with x,y,z in {0,1}
    quads = [(0, 2, 3, 1),  # z-
             (4, 5, 7, 6),  # z+
             (0, 1, 5, 4),  # y-
             (2, 6, 7, 3),  # y+
             (0, 4, 6, 2),  # x-
             (1, 3, 7, 5)]  # x+
    t = []
    for a, b, c, d in quads:
        t += [(a, b, c), (a, c, d)]
    return _finish(v, np.array(t))


# ---------------------------------------------------------------------- icosphere
def _icosahedron():
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                  [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def bipyramid(n: int = 24, radius: float = 0.3, height: float = 0.25, twist: float = 0.1, centre=CENTRE):
    """Two cones on an n-gon: the two apexes have n incident triangles each (fans of
    high degree); the ring is rotated by ``twist`` radians about z and tilted
    slightly so that no face is axis-aligned."""
    k = np.arange(n)
    a = 2.0 * np.pi * k / n + twist
    ring = np.stack([radius * np.cos(a), radius * np.sin(a), 0.02 * np.sin(3 * a)], 1)
    v = np.concatenate([ring, [[0.0, 0.0, height], [0.0, 0.0, -height]]]) + np.asarray(centre, dtype=np.float64)
    top, bot = n, n + 1
    nxt = (k + 1) % n
    tris = np.concatenate([np.stack([k, nxt, np.full(n, top)], 1), np.stack([nxt, k, np.full(n, bot)], 1)])
    return _finish(v, tris)


def unit_icosphere(level: int):
    """Unit-sphere directions and faces of an icosahedron subdivided ``level`` times."""
    v, f = _icosahedron()
    for _ in range(level):
        nv = v.shape[0]
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])  # (3F,2)
        key = np.minimum(e[:, 0], e[:, 1]) * nv + np.maximum(e[:, 0], e[:, 1])
        uk, inv = np.unique(key, return_inverse=True)
        a, b = uk // nv, uk % nv
        mid = v[a] + v[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        m = inv.reshape(3, -1).T + nv  # midpoint ids for edges (01, 12, 20)
        v = np.concatenate([v, mid])
        f0, f1, f2 = f[:, 0], f[:, 1], f[:, 2]
        m01, m12, m20 = m[:, 0], m[:, 1], m[:, 2]
        f = np.concatenate([np.stack([f0, m01, m20], 1), np.stack([f1, m12, m01], 1),
                            np.stack([f2, m20, m12], 1), np.stack([m01, m12, m20], 1)])
    return v, f


def icosphere(level: int, radius: float = 0.35, jitter_sigma: float = 0.0, seed=None, centre=CENTRE):
    """Icosphere; with ``jitter_sigma`` > 0 every vertex moves along its radial
    direction by an N(0, sigma) offset drawn from ``seed``."""
    u, f = unit_icosphere(level)
    r = np.full(u.shape[0], float(radius))
    if jitter_sigma > 0:
        rng = np.random.default_rng(seed)
        r = r + rng.normal(0.0, jitter_sigma, size=u.shape[0])
    return _finish(centre + u * r[:, None], f)


# -------------------------------------------------------------------------- torus
def torus(nu: int = 600, nv: int = 300, R: float = 0.3, r: float = 0.12, noise: float = 0.0,
          seed=None, centre=CENTRE):
    """Torus around the z axis: ``nu`` quads around the ring, ``nv`` around the
    tube, quad (i, j) split along its (i, j)-(i+1, j+1) diagonal. With
    ``noise`` > 0 each vertex moves along the tube normal (away from the tube's
    centre circle) by a U(-noise, noise) offset drawn from ``seed``."""
    th = 2.0 * np.pi * np.arange(nu) / nu
    ph = 2.0 * np.pi * np.arange(nv) / nv
    T, P = np.meshgrid(th, ph, indexing="ij")  # (nu, nv)
    rr = np.full(T.shape, float(r))
    if noise > 0:
        rng = np.random.default_rng(seed)
        rr = rr + rng.uniform(-noise, noise, size=T.shape)
    ring = np.stack([R * np.cos(T), R * np.sin(T), np.zeros_like(T)], -1)
    nrm = np.stack([np.cos(P) * np.cos(T), np.cos(P) * np.sin(T), np.sin(P)], -1)
    v = (centre + ring + rr[..., None] * nrm).reshape(-1, 3)
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    i, j = i.ravel(), j.ravel()
    ip, jp = (i + 1) % nu, (j + 1) % nv
    v00, v10, v11, v01 = i * nv + j, ip * nv + j, ip * nv + jp, i * nv + jp
    f = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)])
    return _finish(v, f)


# ------------------------------------------------- spherical-harmonic displaced sphere
def _sh_terms(u: np.ndarray, lmax: int):
    """Yield (l, m, Y_lm(u)) for the real orthonormal spherical harmonics,
    l = 1..lmax, m = -l..l, at unit directions ``u`` (rows)."""
    x = np.clip(u[:, 2], -1.0, 1.0)
    phi = np.arctan2(u[:, 1], u[:, 0])
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    pmm = np.ones_like(x)
    for m in range(lmax + 1):
        # associated Legendre P_l^m (no Condon-Shortley phase), three-term recurrence in l
        if m > 0:
            pmm = pmm * (2 * m - 1) * s
        cm, sm = (np.cos(m * phi), np.sin(m * phi)) if m > 0 else (None, None)
        p_prev, p_cur = None, pmm
        for l in range(m, lmax + 1):
            if l == m + 1:
                p_prev, p_cur = p_cur, x * (2 * m + 1) * p_cur
            elif l > m + 1:
                p_prev, p_cur = p_cur, ((2 * l - 1) * x * p_cur - (l + m - 1) * p_prev) / (l - m)
            if l == 0:
                continue
            N = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                yield l, 0, N * p_cur
            else:
                yield l, m, math.sqrt(2.0) * N * p_cur * cm
                yield l, -m, math.sqrt(2.0) * N * p_cur * sm


def real_sh_basis(u: np.ndarray, lmax: int) -> np.ndarray:
    """Real orthonormal Y_lm as columns, ordered by l, then m ascending."""
    out = np.empty((u.shape[0], (lmax + 1) ** 2 - 1))
    for l, m, y in _sh_terms(u, lmax):
        out[:, l * l - 1 + m + l] = y
    return out


def sh_sphere(level: int, lmax: int, amplitude: float = 0.05, radius: float = 0.35, seed=None,
              centre=CENTRE):
    """Icosphere directions displaced radially: r = radius * (1 + amplitude * g),
    g = sum of a_lm Y_lm (l = 1..lmax, a_lm ~ N(0, 1) from ``seed``), scaled so
    that max |g| over the vertices is 1."""
    u, f = unit_icosphere(level)
    rng = np.random.default_rng(seed)
    nb = (lmax + 1) ** 2 - 1
    a = rng.normal(0.0, 1.0, size=nb)
    g = np.zeros(u.shape[0])
    step = 1 << 15  # chunks small enough to stay in cache
    for s0 in range(0, u.shape[0], step):
        gs = g[s0:s0 + step]
        for l, m, y in _sh_terms(u[s0:s0 + step], lmax):
            gs += a[l * l - 1 + m + l] * y
    g /= np.max(np.abs(g))
    r = radius * (1.0 + amplitude * g)
    return _finish(centre + u * r[:, None], f)


# ------------------------------------------------------------------------ configs
CONFIG_NAMES = {
    1: "cube_64",
    2: "icosphere5_jitter_256",
    3: "noisy_torus_512",
    4: "batch64",
    5: "sh_sphere9_1024",
}


def batch_specs(seed_base: int = SEED_BASE + 1000, n_meshes: int = 64):
    """Recipe of the 64-mesh batch: kind = m mod 3 (icosphere, torus, SH sphere),
    sizes and grids drawn from per-mesh seeds."""
    specs = []
    for m in range(n_meshes):
        rng = np.random.default_rng(seed_base + m)
        kind = m % 3
        N = int(round(math.exp(rng.uniform(math.log(64), math.log(256)))))
        if kind == 0:
            spec = dict(kind="icosphere", level=2 + (m // 3) % 5)
        elif kind == 1:
            F = math.exp(rng.uniform(math.log(2e3), math.log(2e5)))
            nv = max(3, int(round(math.sqrt(F / 4.0))))
            spec = dict(kind="torus", nu=2 * nv, nv=nv)
        else:
            spec = dict(kind="sh", level=3 + (m // 3) % 4, lmax=8, seed=int(rng.integers(0, 2**31)))
        spec.update(N=N, band=3.0, index=m)
        specs.append(spec)
    return specs


def batch_mesh(spec):
    if spec["kind"] == "icosphere":
        return icosphere(spec["level"])
    if spec["kind"] == "torus":
        return torus(nu=spec["nu"], nv=spec["nv"])
    return sh_sphere(spec["level"], spec["lmax"], seed=spec["seed"])


def make_config(k: int):
    """Return (name, meshes, grids) of synthetic configuration ``k`` (1..5).

    1: cube side 0.5, 64^3, band 3.
    2: icosphere level 5, r 0.35, radial N(0, 1e-3) jitter, 256^3, band 4.
    3: torus R 0.3 r 0.12, 600x300 quads, tube-normal U(+-0.01) noise, 512^3, band 3.
    4: 64 meshes of mixed kind and size, each with its own N^3 grid, N in [64, 256], band 3.
    5: icosphere level 9 with degree-16 SH displacement of 5%, 1024^3, band 3.
    """
    seed = SEED_BASE + k
    if k == 1:
        return CONFIG_NAMES[1], [cube()], [Grid.unit(64, 3)]
    if k == 2:
        return CONFIG_NAMES[2], [icosphere(5, 0.35, 1e-3, seed)], [Grid.unit(256, 4)]
    if k == 3:
        return CONFIG_NAMES[3], [torus(600, 300, 0.3, 0.12, 0.01, seed)], [Grid.unit(512, 3)]
    if k == 4:
        specs = batch_specs()
        return CONFIG_NAMES[4], [batch_mesh(s) for s in specs], [Grid.unit(s["N"], s["band"]) for s in specs]
    if k == 5:
        return CONFIG_NAMES[5], [sh_sphere(9, 16, 0.05, 0.35, seed)], [Grid.unit(1024, 3)]
    raise ValueError(f"unknown config {k}")
