"""Comparison of a device band against the CPU oracle under the agreement rules:
  * band membership and sign identical, except cells within 1e-6 h of the
    surface or of the band edge;
  * |d| within 1e-5 h of the FP64 oracle;
  * the device's feature id is one whose own distance is within 1e-5 h of d
    (several features tie where the closest point lies on an edge or vertex).
"""
import numpy as np

import oracle

TOL_D = 1e-5   # in units of h
TOL_FEAT = 1e-5


def compare(om, grid, o, cell, sdf, feat, k_range=None, exact_membership=False):
    """o: oracle band dict (possibly restricted to z-planes k_range=(k0,k1));
    cell/sdf/feat: device results as numpy arrays (any order)."""
    cell = np.asarray(cell, dtype=np.int64)
    sdf = np.asarray(sdf, dtype=np.float64)
    feat = np.asarray(feat, dtype=np.int32)
    if k_range is not None:
        kk = cell // (int(grid.n[0]) * int(grid.n[1]))
        sel = (kk >= k_range[0]) & (kk < k_range[1])
        cell, sdf, feat = cell[sel], sdf[sel], feat[sel]
    order = np.argsort(cell, kind="stable")
    cell, sdf, feat = cell[order], sdf[order], feat[order]
    assert np.all(np.diff(cell) > 0), "duplicate cells in the device band"
    h = float(grid.h)
    oc, od, osdf, ofl = o["cell"], o["d"], o["sdf"], o["flags"]
    exempt = (ofl & (oracle.FLAG_NEAR_SURFACE | oracle.FLAG_NEAR_BAND_EDGE)) > 0
    in_band = (ofl & oracle.FLAG_IN_BAND) > 0
    pos = np.searchsorted(oc, cell)
    pos_c = np.minimum(pos, max(len(oc) - 1, 0))
    found = (pos < len(oc)) & (oc[pos_c] == cell) if len(oc) else np.zeros(len(cell), bool)
    report = {}
    # device cells the oracle does not list at all: not within band*h + 1e-6 h
    extra = cell[~found]
    report["extra"] = int(extra.size)
    # oracle cells (in band, not exempt) missing on the device
    present = np.zeros(len(oc), bool)
    present[pos[found]] = True
    missing = oc[in_band & ~exempt & ~present]
    report["missing"] = int(missing.size)
    # device cells listed by the oracle but outside its band must be exempt
    fi = pos[found]
    wrong_in = (~in_band[fi]) & (~exempt[fi])
    report["wrong_in"] = int(wrong_in.sum())
    if exact_membership:
        report["exempt"] = int(exempt.sum())
    dev_d = np.abs(sdf[found])
    err_d = np.abs(dev_d - od[fi]) / h
    report["max_err_d"] = float(err_d.max()) if err_d.size else 0.0
    sign_ok = (sdf[found] < 0) == (osdf[fi] < 0)
    report["sign_bad"] = int((~sign_ok & ~exempt[fi]).sum())
    fd = om.feature_dist(grid, cell[found], feat[found])
    report["feat_bad"] = int((fd > od[fi] + TOL_FEAT * h).sum())
    report["n_device"] = int(cell.size)
    report["n_oracle"] = int(in_band.sum())
    report["missing_cells"] = missing[:10].tolist()
    report["extra_cells"] = extra[:10].tolist()
    return report


def assert_parity(rep, exact_membership=False):
    msg = str(rep)
    assert rep["extra"] == 0, msg
    assert rep["missing"] == 0, msg
    assert rep["wrong_in"] == 0, msg
    assert rep["max_err_d"] <= TOL_D, msg
    assert rep["sign_bad"] == 0, msg
    assert rep["feat_bad"] == 0, msg
    if exact_membership:
        assert rep["exempt"] == 0 and rep["n_device"] == rep["n_oracle"], msg


def vertex_term_scale(tris, edges, nv, feat, grad_sdf):
    """Per vertex, a bound on the sum of |terms| its adjoint accumulates: every
    band cell adds grad_sdf * w_k * (unit vector) to each vertex k of its feature,
    with weights 0 <= w_k <= 1. feat: the band's mesh-local feature ids (faces,
    then edges, then vertices); edges: (a, b, ...) rows in the same numbering."""
    tris = np.asarray(tris)
    F, E = tris.shape[0], edges.shape[0]
    feat = np.asarray(feat, dtype=np.int64)
    g = np.abs(np.asarray(grad_sdf, dtype=np.float64))
    s = np.zeros(nv)
    fm = feat < F
    for j in range(3):
        np.add.at(s, tris[feat[fm], j], g[fm])
    em = (feat >= F) & (feat < F + E)
    e = feat[em] - F
    np.add.at(s, edges[e, 0], g[em])
    np.add.at(s, edges[e, 1], g[em])
    vm = feat >= F + E
    np.add.at(s, feat[vm] - F - E, g[vm])
    return s


def assert_same_sums(a, b, scale, msg=""):
    """a and b accumulate the same FP32 terms in different orders (float atomics
    land in whatever order the hardware executes them, and the kernel groups
    them into partial sums by block). Reordering a sum of n terms moves it by at
    most about n * 2^-24 * sum |terms|; scale[v] bounds sum |terms| of vertex v
    (vertex_term_scale). Per coordinate: |a - b| <= 1e-5 * scale, which a
    missing or doubled contribution larger than that exceeds."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    sc = np.asarray(scale, dtype=np.float64).reshape(a.shape[0], *([1] * (a.ndim - 1)))
    err = np.abs(a - b)
    bad = err > 1e-5 * sc
    assert not bad.any(), (msg, int(bad.sum()), float(err.max()), float((err / np.maximum(sc, 1e-30)).max()))
