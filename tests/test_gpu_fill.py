"""Interior fill of the dense field (Section 11.3): off-band cells inside the
solid become -inf, outside ones stay +inf, band cells are untouched. Checked
against the cube's closed form on every cell and against the generalized
winding number of the oracle on sampled cells."""
import numpy as np
import pytest

import meshgen
import oracle
from meshgen import Grid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1903_00353_amd as P  # noqa: E402


def filled(v, f, g):
    verts, tris = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    feats = P.csc_build_features(verts, tris, g)
    n = int(g.n[0]) * int(g.n[1]) * int(g.n[2])
    d = torch.empty(n, dtype=torch.float32, device="cuda")
    band = P.csc_scan_convert(feats, dense=d)
    before = d.clone()
    P.csc_interior_fill(feats, d)
    torch.cuda.synchronize()
    cell = band.cell.cpu().numpy().astype(np.int64)
    return before.cpu().numpy(), d.cpu().numpy(), cell


def check_band_untouched(before, after, cell):
    assert np.array_equal(before[cell], after[cell])
    off = np.ones(after.size, bool)
    off[cell] = False
    assert np.all(np.isinf(after[off]))
    return off


def cube_inside(pts, centre=0.5, half=0.25):
    return np.all(np.abs(pts - centre) < half, axis=1)


def test_cube_every_cell():
    v, f = meshgen.cube()
    g = Grid.unit(64, 3)
    print("[case] cube 64^3", flush=True)
    before, after, cell = filled(v, f, g)
    off = check_band_untouched(before, after, cell)
    idx = np.nonzero(off)[0]
    inside = cube_inside(oracle.cell_centres(g, idx))
    assert inside.any() and (~inside).any()
    assert np.array_equal(after[idx] < 0, inside)


def test_cube_cut_by_grid_boundary():
    """The grid starts inside the solid (z from 0.4): columns through the cube begin
    with unset interior cells, filled from the first band cell after them."""
    v, f = meshgen.cube()
    g = Grid(n=(64, 64, 32), h=1.0 / 64, band=3.0, origin=(0.0, 0.0, 0.4))
    print("[case] cube cut at z=0.4", flush=True)
    before, after, cell = filled(v, f, g)
    off = check_band_untouched(before, after, cell)
    idx = np.nonzero(off)[0]
    pts = oracle.cell_centres(g, idx)
    inside = cube_inside(pts)
    lead = inside & (pts[:, 2] < 0.45)
    assert lead.sum() > 1000  # leading interior cells exist and are covered
    assert np.array_equal(after[idx] < 0, inside)


def sampled_against_winding(v, f, g, n_sample, seed):
    before, after, cell = filled(v, f, g)
    off = check_band_untouched(before, after, cell)
    idx = np.nonzero(off)[0]
    rng = np.random.default_rng(seed)
    inside_all = after[idx] < 0
    # half the sample from each side, so both are exercised
    pick = np.concatenate([rng.choice(idx[inside_all], n_sample // 2, replace=False),
                           rng.choice(idx[~inside_all], n_sample // 2, replace=False)])
    w = oracle.OracleMesh(v, f).winding(oracle.cell_centres(g, pick))
    assert np.all(np.abs(w - np.round(w)) < 1e-6)  # off-band cells are far from the surface
    assert np.array_equal(after[pick] < 0, w > 0.5)
    return inside_all.sum()


def test_torus_sampled():
    """Genus 1: columns through the hole leave and re-enter the solid."""
    v, f = meshgen.torus(120, 60, seed=11)
    g = Grid.unit(128, 3)
    print("[case] torus 120x60 at 128^3", flush=True)
    n_in = sampled_against_winding(v, f, g, 3000, 1)
    assert n_in > 0


def test_jittered_sphere_sampled(configs):
    name, meshes, grids = configs(2)
    v, f = meshes[0]
    print("[case]", name, flush=True)
    sampled_against_winding(v, f, grids[0], 4000, 2)


def test_fill_rejects_batched_handle():
    specs = meshgen.batch_specs()[:2]
    meshes = [meshgen.batch_mesh(s) for s in specs]
    grids = [Grid.unit(s["N"], s["band"]) for s in specs]
    B = P.Batch(meshes, grids)
    d = torch.empty(8, dtype=torch.float32, device="cuda")
    with pytest.raises(P.CscError):
        P.csc_interior_fill(B.f, d)


@pytest.mark.parametrize("band", [0.6, 1.0])
def test_fill_rejects_thin_band(band):
    """With band_cells <= 1 a column can cross the surface between a band cell and
    an unset cell, which would take the wrong side: the call refuses."""
    v, f = meshgen.cube()
    g = Grid.unit(32, band)
    verts, tris = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    feats = P.csc_build_features(verts, tris, g)
    d = torch.empty(g.ncells, dtype=torch.float32, device="cuda")
    P.csc_scan_convert(feats, dense=d)
    with pytest.raises(P.CscError) as ei:
        P.csc_interior_fill(feats, d)
    assert ei.value.code == 1


def test_cube_thin_band_every_cell():
    """The thinnest accepted bands (just over one cell) on the cube, every cell
    against the closed form, with the cube's faces a quarter cell off the centre
    planes (origin shifted)."""
    v, f = meshgen.cube()
    for band in (1.05, 1.5):
        g = Grid(n=(64, 64, 64), h=1.0 / 64, band=band, origin=(0.004, -0.002, 0.0039))
        print("[case] cube thin band", band, flush=True)
        before, after, cell = filled(v, f, g)
        off = check_band_untouched(before, after, cell)
        idx = np.nonzero(off)[0]
        inside = cube_inside(oracle.cell_centres(g, idx))
        assert inside.any() and (~inside).any()
        assert np.array_equal(after[idx] < 0, inside)
