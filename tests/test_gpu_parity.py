"""Device path against the CPU oracle (agreement rules in tests/parity.py).
Every call goes through the C ABI of libcsc.so via the Python binding."""
import numpy as np
import pytest

import meshgen
import oracle
from meshgen import Grid
from parity import assert_parity, assert_same_sums, compare, vertex_term_scale

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1903_00353_amd as P  # noqa: E402


def run_device(v, f, grid, options=None):
    verts = torch.from_numpy(np.ascontiguousarray(v)).cuda()
    tris = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    feats = P.csc_build_features(verts, tris, grid, options)
    band = P.csc_scan_convert(feats)
    torch.cuda.synchronize()
    return feats, band


def to_np(band):
    return band.cell.cpu().numpy(), band.sdf.cpu().numpy(), band.feat.cpu().numpy()


def check(v, f, grid, options=None, exact=False, k_range=None):
    print(f"[case] F={f.shape[0]} n={grid.n} h={grid.h} band={grid.band} k_range={k_range}", flush=True)
    om = oracle.OracleMesh(v, f)
    o = om.band(grid) if k_range is None else om.band(grid, *k_range)
    feats, band = run_device(v, f, grid, options)
    cell, sdf, feat = to_np(band)
    rep = compare(om, grid, o, cell, sdf, feat, k_range=k_range, exact_membership=exact)
    print(rep, feats.info(), flush=True)
    return rep, feats, band, om, o


def test_cube_exact():
    v, f = meshgen.cube()
    g = Grid.unit(64, 3)
    rep, feats, band, om, o = check(v, f, g, exact=True)
    assert_parity(rep, exact_membership=True)
    assert band.n_band == 36832
    inf = feats.info()
    assert (inf["n_faces"], inf["n_edges"], inf["n_vertices"]) == (12, 18, 8)
    assert (inf["edges_convex"], inf["edges_concave"], inf["edges_flat"]) == (12, 0, 6)
    assert inf["vertices_convex"] == 8 and inf["vertices_saddle"] == 0
    assert inf["n_edge_polyhedra"] == 12 and inf["n_vertex_polyhedra"] == 8


@pytest.mark.parametrize("k,absorb", [(2, 0.0), (3, 0.0), (2, -1.0), (3, 0.24)])
def test_config_parity(configs, k, absorb):
    """Every cell of C2 and C3 with the default absorption of nearly flat edges and
    vertices into their face prisms, with none (every non-flat feature its own
    polyhedron, as in Section 8), and with the largest slack allowed."""
    name, meshes, grids = configs(k)
    v, f = meshes[0]
    rep, feats, band, om, o = check(v, f, grids[0], options=P.make_options(absorb_cells=absorb))
    assert_parity(rep)
    inf = feats.info()
    print("absorbed edges / vertices:", inf["edges_absorbed"], inf["vertices_absorbed"], flush=True)
    if absorb < 0:
        assert inf["edges_absorbed"] == 0 and inf["vertices_absorbed"] == 0
    else:
        assert inf["edges_absorbed"] > 0
    # class statistics: every edge has exactly one class, every vertex with a
    # fan at most one of convex / concave / flat / saddle
    inf = feats.info()
    assert sum(inf[c] for c in ("edges_convex", "edges_concave", "edges_flat", "edges_unknown")) == inf["n_edges"]
    nv_cls = sum(inf[c] for c in ("vertices_convex", "vertices_concave", "vertices_flat", "vertices_saddle"))
    assert 0 < nv_cls <= inf["n_vertices"]


def test_batch_meshes_individually(configs):
    """Meshes of the 64-mesh batch (non-dyadic grids), one of each kind, one at a time."""
    name, meshes, grids = configs(4)
    for m in (0, 1, 2, 31, 61):
        rep, *_ = check(*meshes[m], grids[m])
        assert_parity(rep)


def test_ragged_offset_grid():
    """Non-cubic grid, non-dyadic h, offset origin, mesh partly outside the grid."""
    v, f = meshgen.icosphere(3, 0.3, 2e-3, seed=9)
    g = Grid(n=(37, 50, 29), h=1.0 / 41.0, band=2.5, origin=(0.05, -0.1, 0.12))
    rep, *_ = check(v, f, g)
    assert rep["n_oracle"] > 100
    assert_parity(rep)


@pytest.mark.parametrize("n", [24, 40])
def test_high_degree_fans(n):
    """Apexes with more incident triangles than the vertex pass stages in LDS."""
    v, f = meshgen.bipyramid(n)
    g = Grid.unit(64, 3)
    rep, feats, *_ = check(v, f, g)
    assert rep["n_oracle"] > 1000
    assert_parity(rep)


def test_ruff_vertices(configs):
    """A strongly jittered sphere (radial noise of about one edge length, still an
    embedded surface) has ruff vertices (Section 3.3): some incident normal
    points away from the pseudonormal. The default extrudes hemispheres there
    (Section 4.1.3, proven complete) and must match the oracle. The paper's
    positive-normal cone (ruff_mode 1, Section 3.3: reported to work in practice,
    without a proof) is run as an ablation: on this mesh it leaves no gap either."""
    v, f = meshgen.icosphere(3, 0.35, 0.04, seed=0)
    g = Grid.unit(96, 3)
    rep, feats, *_ = check(v, f, g)
    assert feats.info()["vertices_ruff"] > 0
    assert_parity(rep)
    rep1, *_ = check(v, f, g, options=P.make_options(ruff_mode=1))
    print("ruff_mode 1 (cone):", {k: rep1[k] for k in ("missing", "extra", "max_err_d")}, flush=True)
    assert_parity(rep1)


@pytest.mark.parametrize("cfg", [2, 3])
def test_per_cell_scan_ablation(configs, cfg):
    """Alg. 2 as printed (every box cell tested by itself, scan_mode 1) gives the
    same field as the row intervals: parity against the oracle."""
    name, meshes, grids = configs(cfg)
    v, f = meshes[0]
    k = int(grids[0].n[2]) // 2
    rep, *_ = check(v, f, grids[0], options=P.make_options(scan_mode=1), k_range=(k - 24, k + 24))
    assert rep["n_oracle"] > 1000
    assert_parity(rep)


def test_empty_and_tiny_grids():
    v, f = meshgen.icosphere(2, 0.3)
    g = Grid(n=(16, 16, 16), h=1 / 64, band=3, origin=(5.0, 5.0, 5.0))
    feats, band = run_device(v, f, g)
    assert band.n_band == 0
    g1 = Grid(n=(1, 1, 1), h=0.1, band=3, origin=(0.75, 0.45, 0.45))  # one cell near the sphere
    rep, *_ = check(v, f, g1)
    assert_parity(rep)
    assert rep["n_oracle"] == 1


def test_deterministic(configs):
    name, meshes, grids = configs(2)
    v, f = meshes[0]
    a = to_np(run_device(v, f, grids[0])[1])
    b = to_np(run_device(v, f, grids[0])[1])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_rebuild_in_place():
    """A handle rebuilt for the same mesh gives identical output; rebuilt for a larger
    mesh (arena grows) it matches a fresh handle."""
    v, f = meshgen.icosphere(2, 0.3, 2e-3, seed=2)
    g = Grid.unit(48, 3)
    verts, tris = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    h = P.csc_build_features(verts, tris, g)
    a = to_np(P.csc_scan_convert(h))
    h2 = P.csc_build_features(verts, tris, g, reuse=h)
    assert h2 is h
    b = to_np(P.csc_scan_convert(h))
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    v3, f3 = meshgen.icosphere(4, 0.3, 2e-3, seed=3)
    g3 = Grid.unit(96, 3)
    verts3, tris3 = torch.from_numpy(v3).cuda(), torch.from_numpy(f3).cuda()
    P.csc_build_features(verts3, tris3, g3, reuse=h)
    c = to_np(P.csc_scan_convert(h))
    d = to_np(run_device(v3, f3, g3)[1])
    assert all(np.array_equal(x, y) for x, y in zip(c, d))


def test_dense_output_matches_band():
    v, f = meshgen.cube()
    g = Grid.unit(64, 3)
    verts, tris = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    sdf, feat, cell, dense = P.sdf(verts, tris, g, dense=True)
    d = dense.cpu().numpy().ravel()
    c = cell.cpu().numpy()
    assert np.array_equal(d[c], sdf.cpu().numpy())
    mask = np.ones(d.size, bool)
    mask[c] = False
    assert np.all(np.isinf(d[mask]) & (d[mask] > 0))


def test_saddle_ablation_leaves_holes(configs):
    """Without saddle extrusions (Section 3.2; the paper's rabbit-ear failure) the noisy
    torus is not covered: cells go missing or get values from farther features."""
    name, meshes, grids = configs(3)
    v, f = meshes[0]
    rep, feats, *_ = check(v, f, grids[0], options=P.make_options(saddle_mode=2))
    assert feats.info()["vertices_saddle"] > 0
    assert rep["missing"] > 0 or rep["max_err_d"] > 1e-5


def _bad(kind):
    v, f = meshgen.cube()
    v, f = v.copy(), f.copy()
    if kind == "open":
        f = f[2:]
    elif kind == "flipped":
        f[0] = f[0, [0, 2, 1]]
    elif kind == "index":
        f[3, 1] = 99
    elif kind == "repeat":
        f[3, 1] = f[3, 0]
    elif kind == "nan":
        v[5, 2] = np.nan
    elif kind == "degenerate":
        a, c = f[0, 0], f[0, 2]          # move corner 1 of face 0 onto the midpoint of corners 0 and 2
        v[f[0, 1]] = (v[a] + v[c]) / 2
    return v, f


@pytest.mark.parametrize("kind,code", [("open", 2), ("flipped", 3), ("index", 1), ("repeat", 1), ("nan", 1),
                                       ("degenerate", 4)])
def test_invalid_surfaces_are_rejected(kind, code):
    v, f = _bad(kind)
    verts, tris = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    with pytest.raises(P.CscError) as ei:
        P.csc_build_features(verts, tris, Grid.unit(32, 3))
    assert ei.value.code == code


def test_backward_matches_oracle_gradient(configs):
    name, meshes, grids = configs(2)
    v, f = meshes[0]
    g = grids[0]
    feats, band = run_device(v, f, g)
    cell, sdf, feat = to_np(band)
    gs = torch.from_numpy(2.0 * sdf).cuda()  # d(sum SDF^2)/dSDF
    gv = P.csc_sdf_backward(feats, band, gs).cpu().numpy().astype(np.float64)
    om = oracle.OracleMesh(v, f)
    ref = om.grad(g, cell, feat, np.sign(sdf), 2.0 * sdf.astype(np.float64))
    rel = np.linalg.norm(gv - ref) / np.linalg.norm(ref)
    print("rel l2", rel, "max abs", np.abs(gv - ref).max() / np.abs(ref).max(), flush=True)
    assert rel <= 1e-4
    assert np.abs(gv - ref).max() <= 1e-3 * np.abs(ref).max()


def test_fused_loss_upstream_matches_explicit(configs):
    """grad_sdf None (the loss sum of SDF^2, its upstream 2 SDF formed inside
    the adjoint) accumulates the same terms as an explicit 2 * sdf upstream,
    for one mesh and for a batch: equal up to the order of the float sums."""
    name, meshes, grids = configs(2)
    v, f = meshes[0]
    g = grids[0]
    feats, band = run_device(v, f, g)
    cell, sdf, feat = to_np(band)
    explicit = P.csc_sdf_backward(feats, band, torch.from_numpy(2.0 * sdf).cuda()).cpu().numpy()
    fused = P.csc_sdf_backward(feats, band, None).cpu().numpy()
    om = oracle.OracleMesh(v, f)
    scale = vertex_term_scale(f, om.edges, v.shape[0], feat, 2.0 * sdf)
    assert np.abs(fused).max() > 0
    assert_same_sums(explicit, fused, scale, "single mesh")
    specs = meshgen.batch_specs()[:4]
    bm = [meshgen.batch_mesh(sp) for sp in specs]
    bg = [meshgen.Grid.unit(sp["N"], sp["band"]) for sp in specs]
    B = P.Batch(bm, bg)
    B.step()
    B.check()
    off = B.band_off.cpu().tolist()
    gs = torch.zeros_like(B.out[0])
    gs[:off[-1]] = 2.0 * B.out[0][:off[-1]]
    gv = torch.zeros_like(B.grad_verts)
    P.csc_sdf_backward_batched(B.f, B.out, B.band_off, gs, gv)
    torch.cuda.synchronize()
    vo = 0
    for m, (vm, fm) in enumerate(bm):
        s_m, f_m, _ = (x.cpu().numpy() for x in B.band(m))
        sc = vertex_term_scale(fm, oracle.OracleMesh(vm, fm).edges, vm.shape[0], f_m, 2.0 * s_m)
        assert_same_sums(gv[vo:vo + vm.shape[0]].cpu().numpy(), B.grad(m).cpu().numpy(), sc, m)
        vo += vm.shape[0]


def test_backward_wide_range_upstream(configs):
    """The adjoint sums each block's terms in fixed point scaled to the block's
    largest |dL/dSDF|, and sends terms too small for that scale to the gradient
    as floats. Upstream values spread over 40 decades, with exact zeros, put
    most terms on that second path; every vertex must still match the oracle
    within 1e-5 of its sum of |terms|. An all-zero upstream gives exact zeros."""
    name, meshes, grids = configs(2)
    v, f = meshes[0]
    g = grids[0]
    feats, band = run_device(v, f, g)
    cell, sdf, feat = to_np(band)
    rng = np.random.default_rng(17)
    up = (2.0 * sdf * 10.0 ** rng.uniform(-20, 20, sdf.shape[0])).astype(np.float32)
    up[rng.random(sdf.shape[0]) < 0.1] = 0.0
    print("[case]", name, "wide-range upstream", up.shape, flush=True)
    gv = P.csc_sdf_backward(feats, band, torch.from_numpy(up).cuda()).cpu().numpy().astype(np.float64)
    om = oracle.OracleMesh(v, f)
    ref = om.grad(g, cell, feat, np.sign(sdf), up.astype(np.float64))
    scale = vertex_term_scale(f, om.edges, v.shape[0], feat, up)
    assert np.all(np.isfinite(gv))
    assert_same_sums(gv, ref, scale, "wide-range upstream")
    z = P.csc_sdf_backward(feats, band, torch.zeros_like(band.sdf)).cpu().numpy()
    assert not np.any(z)


def test_backward_matches_finite_differences():
    """Device gradient of L = sum SDF^2 against FP64 central differences of the oracle
    distance over the device band set (cells at a kink excluded from both sides)."""
    v, f = meshgen.icosphere(3, 0.3, 3e-3, seed=5)
    g = Grid.unit(48, 3)
    verts, tris = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    feats = P.csc_build_features(verts, tris, g)
    band = P.csc_scan_convert(feats)
    cell, sdf, feat = to_np(band)
    om = oracle.OracleMesh(v, f)
    d0, _ = om.cells_dist(g, cell)
    rng = np.random.default_rng(17)
    delta = 1e-3 * g.h
    worst = 0.0
    for s in range(32):
        vi, ax = int(rng.integers(om.nv)), int(rng.integers(3))
        Vp, Vm = om.V.copy(), om.V.copy()
        Vp[vi, ax] += delta
        Vm[vi, ax] -= delta
        dp, _ = om.cells_dist(g, cell, V64=Vp)
        dm, _ = om.cells_dist(g, cell, V64=Vm)
        kink = np.abs(dp + dm - 2 * d0) > 1e-3 * delta
        up = np.where(kink, 0.0, 2.0 * sdf).astype(np.float32)
        gv = P.csc_sdf_backward(feats, band, torch.from_numpy(up).cuda()).cpu().numpy()
        fd = np.sum(((dp ** 2 - dm ** 2) / (2 * delta))[~kink])
        err = abs(gv[vi, ax] - fd)
        worst = max(worst, err / (1e-3 * abs(fd) + 1e-5 * 1.0))
        assert err <= 1e-3 * abs(fd) + 1e-5 * max(1.0, abs(fd)), (vi, ax, gv[vi, ax], fd)
    print("worst normalised fd error", worst)


def test_autograd_function():
    v, f = meshgen.icosphere(3, 0.3, 3e-3, seed=5)
    g = Grid.unit(48, 3)
    verts = torch.from_numpy(v).cuda().requires_grad_(True)
    tris = torch.from_numpy(f).cuda()
    sdf, feat, cell = P.CSCFunction.apply(verts, tris, g)
    loss = (sdf.double() ** 2).sum()
    loss.backward()
    feats = P.csc_build_features(verts.detach(), tris, g)
    band = P.csc_scan_convert(feats)
    ref = P.csc_sdf_backward(feats, band, 2.0 * band.sdf)
    scale = vertex_term_scale(f, oracle.OracleMesh(v, f).edges, v.shape[0], band.feat.cpu().numpy(),
                              2.0 * band.sdf.cpu().numpy())
    assert_same_sums(verts.grad.cpu().numpy(), ref.cpu().numpy(), scale)


def test_single_mesh_kept_empty_store():
    """keep_store_empty through the single-mesh entry point: a workspace filled
    with 0xFF once, then scans (one writing the dense field too, one after the
    count diagnostic, one after the vertices moved) that never fill the store
    themselves, each equal bit for bit to a scan that fills its own store."""
    v, f = meshgen.icosphere(4, 0.35, 1e-3, 11)
    g = Grid.unit(96, 3)
    print(f"[case] kept-empty store, single mesh F={f.shape[0]} n={g.n}", flush=True)
    verts, tris = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    kept = P.csc_build_features(verts, tris, g, P.make_options(keep_store_empty=1))
    # room for the bricks the moved vertices reach
    nbytes, _ = P.csc_scan_convert_workspace_for(kept, 2 * int(kept.info()["n_bricks"]))
    ws = torch.full((max(nbytes, 1),), 255, dtype=torch.uint8, device="cuda")

    def reference():
        fresh = P.csc_build_features(verts, tris, g)
        band = to_np(P.csc_scan_convert(fresh))
        fresh.free()
        return band

    n = int(np.prod(g.n))
    for it in range(4):
        if it == 2:
            P.csc_scan_convert_count(kept, ws)
        if it == 3:
            verts.sub_(0.5).mul_(1.01).add_(0.5)
            P.csc_build_features(verts, tris, g, P.make_options(keep_store_empty=1), reuse=kept)
        dense = torch.empty(n, dtype=torch.float32, device="cuda") if it == 1 else None
        band = P.csc_scan_convert(kept, ws, dense=dense)
        got, ref = to_np(band), reference()
        assert all(np.array_equal(a, b) for a, b in zip(got, ref)), it
        if dense is not None:
            d = dense.cpu().numpy()
            assert np.array_equal(d[got[0]], got[1])
