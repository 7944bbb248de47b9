"""Triangle-soup ingestion (Section 7): the device weld equals the oracle's exactly
(integer work: vertex order, triangle indices and positions bit for bit), and the
welded mesh gives the oracle's field."""
import numpy as np
import pytest

import meshgen
import oracle
from meshgen import Grid
from parity import assert_parity, compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1903_00353_amd as P  # noqa: E402


def shuffled_soup(v, f, seed):
    """Faces in random order, each with its corners rotated by a random amount
    (orientation kept)."""
    rng = np.random.default_rng(seed)
    f = f[rng.permutation(f.shape[0])]
    rot = rng.integers(0, 3, f.shape[0])
    f = np.stack([np.roll(row, -r) for row, r in zip(f, rot)]).astype(np.int32)
    return v[f]


def device_weld(soup):
    vw, tw = P.csc_weld_soup(torch.from_numpy(np.ascontiguousarray(soup, dtype=np.float32)).cuda())
    return vw.cpu().numpy(), tw.cpu().numpy()


MESHES = {
    "cube": lambda: meshgen.cube(),
    "icosphere4": lambda: meshgen.icosphere(4, 0.35, 1e-3, seed=3),
    "torus": lambda: meshgen.torus(120, 60, seed=11),
    "bipyramid": lambda: meshgen.bipyramid(24),
}


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("shuffle", [False, True])
def test_weld_equals_oracle(name, shuffle):
    v, f = MESHES[name]()
    soup = shuffled_soup(v, f, 7) if shuffle else v[f]
    print("[case] weld", name, "shuffled" if shuffle else "flat", soup.shape, flush=True)
    vd, td = device_weld(soup)
    vo, to = oracle.weld_soup(soup)
    assert vd.shape == vo.shape == v.shape
    assert np.array_equal(td, to)
    assert np.array_equal(vd.view(np.uint32), vo.view(np.uint32))


def test_weld_large_soup():
    """The flat soup of the L9 icosphere (15.7M corners: enough for the radix
    sort's 8192-pair tiles, used from 12.6M pairs) welds back to that mesh, whose
    2.6M positions are all distinct: vertices numbered by first appearance in
    corner order, positions bit for bit."""
    v, f = meshgen.icosphere(9, 0.35)
    print("[case] weld icosphere L9 soup", f.shape, flush=True)
    vd, td = device_weld(v[f])
    ids, first = np.unique(f.ravel(), return_index=True)
    order = ids[np.argsort(first, kind="stable")]
    rank = np.empty(v.shape[0], np.int64)
    rank[order] = np.arange(order.size)
    assert vd.shape == v.shape
    assert np.array_equal(td, rank[f].astype(np.int32))
    assert np.array_equal(vd.view(np.uint32), v[order].view(np.uint32))


def test_weld_signed_zero_and_single_triangle():
    soup = np.array([[[0.0, 0.5, -0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]],
                     [[-0.0, 0.5, 0.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0]]], dtype=np.float32)
    vd, td = device_weld(soup)
    vo, to = oracle.weld_soup(soup)
    assert vd.shape[0] == 4 and np.array_equal(td, to) and np.array_equal(td, [[0, 1, 2], [0, 2, 3]])
    assert np.array_equal(vd, vo)
    v1, t1 = device_weld(soup[:1])
    assert v1.shape[0] == 3 and np.array_equal(t1, [[0, 1, 2]])


def test_weld_rejects_non_finite():
    soup = np.zeros((2, 3, 3), dtype=np.float32)
    soup[1, 2, 1] = np.nan
    with pytest.raises(P.CscError) as ei:
        device_weld(soup)
    assert ei.value.code == 1


def test_welded_soup_field_matches_oracle():
    """Shuffled soup of the jittered L5 sphere -> weld -> narrow band, against the
    oracle run on the welded mesh (same tolerance as every parity test)."""
    v, f = meshgen.icosphere(5, 0.35, 1e-3, seed=190300355)
    soup = shuffled_soup(v, f, 5)
    vd, td = device_weld(soup)
    g = Grid.unit(128, 3)
    om = oracle.OracleMesh(vd, td)
    o = om.band(g)
    feats = P.csc_build_features(torch.from_numpy(vd).cuda(), torch.from_numpy(td).cuda(), g)
    band = P.csc_scan_convert(feats)
    rep = compare(om, g, o, band.cell.cpu().numpy(), band.sdf.cpu().numpy(), band.feat.cpu().numpy())
    print(rep, flush=True)
    assert rep["n_oracle"] > 10000
    assert_parity(rep)
