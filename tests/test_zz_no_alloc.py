"""csc_weld_soup_noalloc (the weld with the library's static scratch, no
allocation) against csc_weld_soup through the C ABI: bit-identical vertices and
triangles on two calls in a row, the second with a smaller soup (the scratch
keeps the first call's contents), and sizes past the scratch rejected before
anything is queued."""
import ctypes as C

import numpy as np
import pytest

import meshgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1903_00353_amd as P  # noqa: E402


def soup_of(v, f, seed):
    rng = np.random.default_rng(seed)
    f = f[rng.permutation(f.shape[0])]
    return torch.from_numpy(np.ascontiguousarray(v[f], dtype=np.float32)).cuda()


def noalloc(soup):
    nf = soup.shape[0]
    verts = torch.full((3 * nf, 3), float("nan"), dtype=torch.float32, device="cuda")
    tris = torch.full((nf, 3), -1, dtype=torch.int32, device="cuda")
    nv = P.csc_weld_soup_noalloc(soup, verts, tris)
    return verts[:nv].cpu().numpy(), tris.cpu().numpy()


def test_noalloc_weld_matches_weld_twice():
    big = soup_of(*meshgen.icosphere(5, 0.35, 1e-3, seed=4), 1)      # 20,480 triangles
    small = soup_of(*meshgen.torus(40, 20, seed=5), 2)                # 1,600 triangles
    for name, soup in (("icosphere5", big), ("torus40x20", small)):
        print("[case] noalloc weld", name, soup.shape[0], flush=True)
        vr, tr = P.csc_weld_soup(soup)
        vr, tr = vr.cpu().numpy(), tr.cpu().numpy()
        vn, tn = noalloc(soup)
        assert vn.shape == vr.shape and np.array_equal(vn.view(np.uint32), vr.view(np.uint32)), name
        assert np.array_equal(tn, tr), name


def test_noalloc_weld_rejects_oversize_soup():
    mx = P.csc_weld_soup_noalloc_max_faces()
    assert mx > 100000
    fake = C.c_void_p(0x1000)  # never read: the size check comes first
    nv = C.c_int64(-1)
    rc = P.lib().csc_weld_soup_noalloc(fake, mx + 1, fake, fake, C.byref(nv), None)
    assert rc == 8 and nv.value == -1
