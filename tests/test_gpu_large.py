"""Features hundreds of cells across. Eq. 1 defines the exact distance for any
closed surface, whatever the size of its triangles relative to the cells, so
the agreement rules (|d| within 1e-5 h, band membership and sign exact) hold
here too: the cube at 1024^3 (faces 512 cells across) against its closed form
on every cell, coarse icospheres (triangles of about 100 and 190 cells) and a
coarse noisy torus (long concave edges, saddle vertices) against the oracle."""
import numpy as np
import pytest

import meshgen
import oracle
from meshgen import Grid
from parity import assert_parity, compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1903_00353_amd as P  # noqa: E402


def device_band(v, f, g):
    verts, tris = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    feats = P.csc_build_features(verts, tris, g)
    band = P.csc_scan_convert(feats)
    torch.cuda.synchronize()
    return band.cell.cpu().numpy().astype(np.int64), band.sdf.cpu().numpy(), band.feat.cpu().numpy()


def cube_closed_form_band(N, band, side=0.5):
    """Cells of the N^3 unit grid with |SDF| < band*h of the centred cube, and their
    SDF, from the closed form d = |max(q, 0)| + min(max_i q_i, 0), q = |p - 1/2| - side/2,
    evaluated plane by plane in units of h (every q is a half-integer there)."""
    q = np.abs(np.arange(N) + 0.5 - N / 2) - side * N / 2          # per axis, in cells
    qx, qy = q[None, :], q[:, None]                                 # (j, i)
    pos2_xy = np.maximum(qx, 0) ** 2 + np.maximum(qy, 0) ** 2
    max_xy = np.maximum(qx, qy)
    cells, vals = [], []
    planes = {}  # every plane with qz <= -band has the same band cells (d there does not depend on qz)
    for k in range(N):
        qz = q[k]
        if qz >= band:
            continue
        key = qz if qz > -band else None
        if key not in planes:
            d = np.sqrt(pos2_xy + max(qz, 0.0) ** 2) + np.minimum(np.maximum(max_xy, qz), 0)
            jj, ii = np.nonzero(np.abs(d) < band)
            planes[key] = (ii + N * jj, d[jj, ii])
        c, dv = planes[key]
        cells.append(c + N * N * k)
        vals.append(dv)
    return np.concatenate(cells).astype(np.int64), np.concatenate(vals) / N


def test_cube_1024_every_cell():
    v, f = meshgen.cube()
    N = 1024
    g = Grid.unit(N, 3)
    print("[case] cube 1024^3 band 3", flush=True)
    cell, sdf, feat = device_band(v, f, g)
    ref_cell, ref_sdf = cube_closed_form_band(N, 3.0)
    order = np.argsort(cell)
    cell, sdf, feat = cell[order], sdf[order], feat[order]
    assert np.array_equal(cell, ref_cell)           # exact membership (no cell within 0.04 h of an edge)
    err = np.abs(np.abs(sdf.astype(np.float64)) - np.abs(ref_sdf)) * N
    print("max |d| error / h", err.max(), flush=True)
    assert err.max() <= 1e-5
    assert np.array_equal(sdf < 0, ref_sdf < 0)
    om = oracle.OracleMesh(v, f)
    fd = om.feature_dist(g, cell, feat)
    assert np.all(fd <= np.abs(ref_sdf) + 1e-5 / N)


@pytest.mark.parametrize("level,N", [(0, 512), (1, 512)])
def test_coarse_icosphere(level, N):
    v, f = meshgen.icosphere(level, 0.35, 0.0)
    g = Grid.unit(N, 3)
    print(f"[case] icosphere L{level} at {N}^3", flush=True)
    om = oracle.OracleMesh(v, f)
    rep = compare(om, g, om.band(g), *device_band(v, f, g))
    print(rep, flush=True)
    assert_parity(rep)


def test_coarse_noisy_torus():
    v, f = meshgen.torus(nu=10, nv=6, R=0.3, r=0.12, noise=0.02, seed=190300353 + 3000)
    g = Grid.unit(384, 3)
    print("[case] noisy torus 10x6 at 384^3", flush=True)
    om = oracle.OracleMesh(v, f)
    rep = compare(om, g, om.band(g), *device_band(v, f, g))
    print(rep, flush=True)
    assert_parity(rep)
