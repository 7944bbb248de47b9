"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed-form distance fields, an independent all-pairs formulation, the winding
number, finite differences, and hand-checked feature numbering."""
import numpy as np
import pytest

import meshgen
import oracle
from meshgen import Grid


def cube_sdf(p, centre=0.5, half=0.25):
    """Closed-form signed distance to the axis-aligned cube [centre-half, centre+half]^3."""
    q = np.abs(p - centre) - half
    return np.linalg.norm(np.maximum(q, 0.0), axis=1) + np.minimum(q.max(axis=1), 0.0)


def test_cube_matches_closed_form():
    v, f = meshgen.cube()
    g = Grid.unit(64, 3)
    om = oracle.OracleMesh(v, f)
    b = om.band(g)
    inb = (b["flags"] & oracle.FLAG_IN_BAND) > 0
    # band from the closed form over the whole grid
    allc = np.arange(g.ncells)
    ref = cube_sdf(oracle.cell_centres(g, allc))
    ref_band = allc[np.abs(ref) < 3.0 / 64]
    assert ref_band.size == 36832
    assert np.array_equal(b["cell"][inb], ref_band)
    assert int((ref[ref_band] > 0).sum()) == 21640 and int((ref[ref_band] < 0).sum()) == 15192
    assert np.max(np.abs(b["sdf"][inb] - ref[ref_band])) <= 1e-12
    # nothing within 1e-6 h of the surface or of the band edge
    assert not np.any(b["flags"] & (oracle.FLAG_NEAR_SURFACE | oracle.FLAG_NEAR_BAND_EDGE))


def test_cube_features_and_pseudonormals():
    v, f = meshgen.cube()
    om = oracle.OracleMesh(v, f)
    assert (om.F, om.E, om.nv) == (12, 18, 8)
    V = om.V
    for k in range(8):
        # angle-weighted pseudonormal at a cube corner: (pi/2) times the sum of the three
        # face normals, whatever the diagonal split (an unweighted mean is not symmetric)
        s = np.sign(V[k] - 0.5)
        assert np.allclose(om.vn[k], np.pi / 2 * s, atol=1e-12)
    for e in range(om.E):
        a, b, fl, fr = om.edges[e]
        assert a < b
        d = np.abs(V[a] - V[b])
        if np.count_nonzero(d) == 1:  # a cube edge: two perpendicular faces
            assert abs(np.linalg.norm(om.en[e]) - np.sqrt(2)) < 1e-12
        else:  # a face diagonal: two coplanar triangles
            assert abs(np.linalg.norm(om.en[e]) - 2.0) < 1e-12


def test_feature_numbering_tetrahedron():
    # hand-numbered tetrahedron: edges are the half-edges 3f+j with start < end, face-major
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float32) * 0.2 + 0.4
    f = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], np.int32)
    om = oracle.OracleMesh(v, f)
    # face 0: (0,2) owned, (2,1) not, (1,0) not; face 1: (0,1) owned, (1,3) owned, (3,0) not;
    # face 2: (0,3) owned, (3,2) not, (2,0) not; face 3: (1,2) owned, (2,3) owned, (3,1) not
    assert om.edges[:, :2].tolist() == [[0, 2], [0, 1], [1, 3], [0, 3], [1, 2], [2, 3]]
    assert om.edges[:, 2].tolist() == [0, 1, 1, 2, 3, 3]
    assert om.edges[:, 3].tolist() == [2, 0, 3, 1, 0, 2]
    assert om.face_edges.reshape(4, 3).tolist() == [[0, 4, 1], [1, 2, 3], [3, 5, 0], [4, 5, 2]]


def test_rejects_open_and_flipped_meshes():
    v, f = meshgen.cube()
    with pytest.raises(ValueError):
        oracle.OracleMesh(v, f[1:])
    f2 = f.copy()
    f2[0] = f2[0, [0, 2, 1]]
    with pytest.raises(ValueError):
        oracle.OracleMesh(v, f2)


@pytest.mark.parametrize("mesh,N", [("cube", 64), ("ico2", 32), ("torus", 28)])
def test_allpairs_matches_culled_oracle(mesh, N):
    """The cull is exact: a literal all-pairs evaluation over the whole grid, with a
    different point-triangle formulation, gives the same band and values."""
    if mesh == "cube":
        v, f = meshgen.cube()
    elif mesh == "ico2":
        v, f = meshgen.icosphere(2, 0.35, 2e-3, seed=7)
    else:
        v, f = meshgen.torus(16, 8, 0.3, 0.12, 0.01, seed=3)
    g = Grid.unit(N, 3)
    om = oracle.OracleMesh(v, f)
    b = om.band(g)
    allc = np.arange(g.ncells)
    d_all = oracle.allpairs_distance(v, f, oracle.cell_centres(g, allc))
    lim = 3.0 / N
    ref_band = allc[d_all < lim]
    inb = (b["flags"] & 1) > 0
    assert np.array_equal(b["cell"][inb], ref_band)
    assert np.max(np.abs(b["d"][inb] - d_all[ref_band])) <= 1e-12
    # and the list mode (every triangle tried, no cull) agrees bit for bit with the band
    d_list, t_list = om.cells_dist(g, b["cell"])
    assert np.array_equal(d_list, b["d"]) and np.array_equal(t_list, b["tri"])


@pytest.mark.parametrize("level", [2, 3, 4])
def test_icosphere_brackets_sphere(level):
    """For a convex polyhedron between concentric spheres of radii r_in and r_out:
    |x-c| - r_out <= SDF(x) <= |x-c| - r_in, and r_out - r_in shrinks ~4x per level."""
    v, f = meshgen.icosphere(level, 0.35)
    g = Grid.unit(64, 3)
    om = oracle.OracleMesh(v, f)
    b = om.band(g)
    c = np.array([0.5, 0.5, 0.5])
    r_out = np.linalg.norm(om.V - c, axis=1).max()
    a = om.V[om.T[:, 0]]
    r_in = np.abs(np.einsum("ij,ij->i", a - c, om.fn)).min()
    rad = np.linalg.norm(oracle.cell_centres(g, b["cell"]) - c, axis=1)
    assert np.all(b["sdf"] >= rad - r_out - 1e-12)
    assert np.all(b["sdf"] <= rad - r_in + 1e-12)


def test_icosphere_converges_to_sphere():
    """The bracket width r_out - r_in shrinks about 4x per subdivision level, so the
    icosphere's SDF converges to |x - c| - r (pinned by the bracket above)."""
    c = np.array([0.5, 0.5, 0.5])
    gaps = []
    for level in range(2, 7):
        v, f = meshgen.icosphere(level, 0.35)
        V = v.astype(np.float64)
        n = np.cross(V[f[:, 1]] - V[f[:, 0]], V[f[:, 2]] - V[f[:, 0]])
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        r_in = np.abs(np.einsum("ij,ij->i", V[f[:, 0]] - c, n)).min()
        gaps.append(np.linalg.norm(V - c, axis=1).max() - r_in)
    ratios = np.array(gaps[1:]) / np.array(gaps[:-1])
    assert np.all((ratios > 0.2) & (ratios < 0.3)), ratios
    assert gaps[-1] < 3e-5


@pytest.mark.parametrize("k", [2, 3])
def test_sign_matches_winding_number(configs, k):
    """Pseudonormal sign agrees with the generalised winding number away from the surface."""
    name, meshes, grids = configs(k)
    v, f = meshes[0]
    g = grids[0]
    om = oracle.OracleMesh(v, f)
    kz = g.n[2] // 2
    b = om.band(g, kz - 2, kz + 2)
    ok = ((b["flags"] & 1) > 0) & (np.abs(b["d"]) > 0.05 * g.h)
    rng = np.random.default_rng(11)
    idx = rng.choice(np.flatnonzero(ok), size=min(1500 if k == 2 else 300, ok.sum()), replace=False)
    w = om.winding(oracle.cell_centres(g, b["cell"][idx]))
    assert np.all((np.abs(w) < 1e-6) | (np.abs(w - 1) < 1e-6))
    assert np.array_equal(b["sdf"][idx] < 0, w > 0.5)


def test_eikonal_on_jittered_sphere(configs):
    """|grad SDF| = 1 (Eq. 2) by central differences on band cells whose neighbours are in the band."""
    name, meshes, grids = configs(2)
    v, f = meshes[0]
    g = grids[0]
    om = oracle.OracleMesh(v, f)
    kz = g.n[2] // 2
    b = om.band(g, kz - 3, kz + 4)
    lut = dict(zip(b["cell"].tolist(), b["sdf"].tolist()))
    n0, n1 = g.n[0], g.n[0] * g.n[1]
    norms = []
    for c in b["cell"][(b["cell"] // n1 == kz)][::3]:
        nb = [c + 1, c - 1, c + n0, c - n0, c + n1, c - n1]
        if all(x in lut for x in nb):
            gr = np.array([lut[nb[0]] - lut[nb[1]], lut[nb[2]] - lut[nb[3]], lut[nb[4]] - lut[nb[5]]]) / (2 * g.h)
            norms.append(np.linalg.norm(gr))
    norms = np.array(norms)
    assert norms.size > 1000
    assert abs(np.median(norms) - 1.0) < 2e-3
    assert np.quantile(norms, 0.98) < 1.0 + 1e-2


def _small_case():
    v, f = meshgen.icosphere(3, 0.3, 3e-3, seed=5)
    return v, f, Grid.unit(48, 3)


def _cells_near(om, g, cells, vi, delta):
    """Cells whose distance can depend on vertex vi: within band*h (+margin) of the
    bounding box of its incident triangles. Every other cell's term cancels exactly."""
    inc = np.flatnonzero((om.T == vi).any(axis=1))
    P = om.V[om.T[inc]].reshape(-1, 3)
    r = g.band * g.h + 2 * delta + 1e-9
    lo, hi = P.min(0) - r, P.max(0) + r
    X = oracle.cell_centres(g, cells)
    return np.flatnonzero(np.all((X >= lo) & (X <= hi), axis=1))


def test_gradient_matches_finite_differences():
    """Closed-form gradient of L = sum_c u_c SDF_c (features fixed) against FP64 central
    differences of the oracle's own distance, sign held at its unperturbed value."""
    v, f, g = _small_case()
    om = oracle.OracleMesh(v, f)
    b = om.band(g)
    keep = ((b["flags"] & 1) > 0) & (b["d"] > 1e-3 * g.h)
    cells, sdf, feat = b["cell"][keep], b["sdf"][keep], b["feat"][keep]
    rng = np.random.default_rng(3)
    u = rng.normal(size=cells.size)
    sgn = np.sign(sdf)
    grad = om.grad(g, cells, feat, sgn, u)
    delta = 1e-3 * g.h
    errs = []
    for s in range(24):
        vi, ax = int(rng.integers(om.nv)), int(rng.integers(3))
        Vp, Vm = om.V.copy(), om.V.copy()
        Vp[vi, ax] += delta
        Vm[vi, ax] -= delta
        sel = _cells_near(om, g, cells, vi, delta)
        dp, _ = om.cells_dist(g, cells[sel], V64=Vp)
        dm, _ = om.cells_dist(g, cells[sel], V64=Vm)
        d0 = b["d"][keep][sel]
        # a cell whose closest point jumps between features inside +-delta (a tie on the
        # medial axis) has a kink: its second difference is O(delta), not O(delta^2)
        kink = np.abs(dp + dm - 2 * d0) > 1e-3 * delta
        ok = ~kink
        fd = np.sum(u[sel][ok] * sgn[sel][ok] * (dp - dm)[ok]) / (2 * delta)
        g1 = om.grad(g, cells[sel][ok], feat[sel][ok], sgn[sel][ok], u[sel][ok])[vi, ax]
        assert abs(g1 - grad[vi, ax]) <= 1e-9 * np.abs(grad).max() or kink.any()
        errs.append(abs(fd - g1) / (1e-12 + np.abs(grad).max()))
    assert max(errs) < 1e-5


def test_gradient_translation_invariant():
    """Moving every vertex by t changes each SDF_c by -grad_c SDF . t, so the summed
    vertex gradient equals the FD derivative of L along a rigid translation."""
    v, f, g = _small_case()
    om = oracle.OracleMesh(v, f)
    b = om.band(g)
    keep = ((b["flags"] & 1) > 0) & (b["d"] > 1e-3 * g.h)
    cells, sdf, feat = b["cell"][keep], b["sdf"][keep], b["feat"][keep]
    u = np.random.default_rng(4).normal(size=cells.size)
    sgn = np.sign(sdf)
    d0 = b["d"][keep]
    delta = 1e-3 * g.h
    for ax in range(3):
        Vp, Vm = om.V.copy(), om.V.copy()
        Vp[:, ax] += delta
        Vm[:, ax] -= delta
        dp, _ = om.cells_dist(g, cells, V64=Vp)
        dm, _ = om.cells_dist(g, cells, V64=Vm)
        ok = np.abs(dp + dm - 2 * d0) <= 1e-3 * delta  # drop medial-axis kinks
        assert ok.mean() > 0.99
        total = om.grad(g, cells[ok], feat[ok], sgn[ok], u[ok]).sum(axis=0)
        fd = np.sum((u * sgn * (dp - dm))[ok]) / (2 * delta)
        # residual: O(delta^2) truncation and shallow kinks below the filter; a wrong
        # sign or a dropped weight would be an O(1) relative error
        assert abs(fd - total[ax]) <= 1e-4 * np.abs(total).max()


def test_feature_distance_of_canonical_feature_is_d(configs):
    """The canonical feature holds the closest point: its own distance equals d."""
    name, meshes, grids = configs(2)
    v, f = meshes[0]
    g = grids[0]
    om = oracle.OracleMesh(v, f)
    kz = g.n[2] // 2
    b = om.band(g, kz, kz + 1)
    fd = om.feature_dist(g, b["cell"], b["feat"])
    assert np.max(np.abs(fd - b["d"])) <= 1e-15
    kinds = np.bincount(np.digitize(b["feat"], [om.F, om.F + om.E]), minlength=3)
    assert np.all(kinds > 0)  # faces, edges and vertices all occur as closest features


def test_feature_distance_every_region():
    """Distance to each single face and edge (every closest-point region of every
    triangle, all orientations) against the independent NumPy formulation, over a
    whole grid around an irregular tetrahedron."""
    v = (np.array([[0.31, 0.28, 0.35], [0.71, 0.33, 0.30], [0.42, 0.74, 0.38], [0.47, 0.45, 0.77]]) ).astype(np.float32)
    f = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], np.int32)
    om = oracle.OracleMesh(v, f)
    g = Grid.unit(24, 3)
    cells = np.arange(g.ncells)
    P = oracle.cell_centres(g, cells)
    for t in range(4):
        d = om.feature_dist(g, cells, np.full(cells.size, t, np.int32))
        ref = oracle.allpairs_distance(v, f[t:t + 1], P)
        assert np.max(np.abs(d - ref)) <= 1e-12, t
    V = v.astype(np.float64)
    for e in range(om.E):
        a, b = V[om.edges[e, 0]], V[om.edges[e, 1]]
        d = om.feature_dist(g, cells, np.full(cells.size, om.F + e, np.int32))
        tt = np.clip((P - a) @ (b - a) / ((b - a) @ (b - a)), 0, 1)
        ref = np.linalg.norm(P - (a + tt[:, None] * (b - a)), axis=1)
        assert np.max(np.abs(d - ref)) <= 1e-12, e


# ---------------------------------------------------------------- soup welding
def _weld_brute(soup):
    """Pairwise definition: corner i is vertex k where k counts the distinct
    positions among corners 0..i (first appearance), equality by value."""
    c = np.asarray(soup, dtype=np.float32).reshape(-1, 3).astype(np.float64)
    ids, reps = [], []
    for i in range(c.shape[0]):
        for k, r in enumerate(reps):
            if np.all(c[r] == c[i]):
                ids.append(k)
                break
        else:
            ids.append(len(reps))
            reps.append(i)
    return c[reps].astype(np.float32), np.array(ids, dtype=np.int32).reshape(-1, 3)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_weld_matches_pairwise_definition(seed):
    rng = np.random.default_rng(seed)
    pool = rng.integers(-3, 4, size=(15, 3)).astype(np.float32) * np.float32(0.25)
    pool[0] = [0.0, -0.0, 0.0]                   # -0 and +0 are one position
    pool[1] = [-0.0, 0.0, -0.0]
    soup = pool[rng.integers(0, 15, size=(40, 3))]
    v, t = oracle.weld_soup(soup)
    vb, tb = _weld_brute(soup)
    assert np.array_equal(t, tb)
    assert np.array_equal(v, vb)
    assert np.all(v[t] == soup)                  # every corner maps to its own position


def test_weld_inverts_flattening():
    """A mesh flattened to a soup welds back to itself when its vertices first
    appear in index order (icosphere: vertex ids grow with face order)."""
    v, f = meshgen.cube()
    soup = v[f]
    vw, tw = oracle.weld_soup(soup)
    assert vw.shape == v.shape and tw.shape == f.shape
    # same mesh up to renumbering: positions of every corner agree
    assert np.array_equal(vw[tw], v[f])
    first = np.unique(f.reshape(-1), return_index=True)[1]
    perm = f.reshape(-1)[np.sort(first)]         # original ids in order of first appearance
    assert np.array_equal(vw, v[perm])
