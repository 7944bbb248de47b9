"""Python binding of ``libcsc.so``: the Characteristic/Scan Conversion narrow-band
signed distance field on MI355X (gfx950).

Argument marshalling only: every step of the computation runs in the library's
HIP kernels. PyTorch supplies device memory and the current stream. There is no
fallback: if the library is missing or the device is not gfx950 the calls raise.

Entry points mirror ``include/csc.h``: ``csc_build_features``,
``csc_features_info``, ``csc_scan_convert_workspace``, ``csc_scan_convert``,
``csc_sdf_backward``, ``csc_features_free``, ``csc_error_string``,
``csc_classify_edge``, ``csc_classify_vertex``; plus the conveniences ``sdf``
(one call, returns tensors) and ``CSCFunction`` (autograd with respect to the
vertex positions).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libcsc.so")

CSC_STATUS = {0: "OK", 1: "INVALID_ARG", 2: "NONMANIFOLD", 3: "INCONSISTENT_ORIENTATION", 4: "DEGENERATE_FACE",
              5: "GRID_TOO_LARGE", 6: "OUT_OF_MEMORY", 7: "HIP_ERROR", 8: "WORKSPACE_TOO_SMALL",
              9: "UNSUPPORTED_DEVICE"}


class CscError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = f"{where}: {CSC_STATUS.get(code, code)} ({_lib_error_string(code)})"
        if code == 7:
            msg += f" [{lib().csc_last_hip_error().decode()}]"
        super().__init__(msg)


class csc_grid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("h", C.c_double), ("n", C.c_int32 * 3), ("band_cells", C.c_float)]


class csc_options(C.Structure):
    _fields_ = [("eps_rel", C.c_float), ("ruff_mode", C.c_int32), ("saddle_mode", C.c_int32),
                ("force_both_sides", C.c_int32), ("small_rows", C.c_int32 * 3),
                ("scan_mode", C.c_int32), ("absorb_cells", C.c_float), ("scan_grid", C.c_int32),
                ("geom_blocks", C.c_int32), ("keep_store_empty", C.c_int32)]


class csc_feature_info(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n_vertices", "n_faces", "n_edges", "n_edge_polyhedra", "n_vertex_polyhedra",
        "edges_convex", "edges_concave", "edges_flat", "edges_unknown",
        "vertices_convex", "vertices_concave", "vertices_flat", "vertices_saddle", "vertices_ruff",
        "n_bricks", "max_band_cells", "edges_absorbed", "vertices_absorbed")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


EXPORTS = ["csc_build_features", "csc_features_info", "csc_scan_convert_workspace", "csc_scan_convert",
           "csc_sdf_backward", "csc_features_free", "csc_error_string", "csc_last_hip_error",
           "csc_classify_edge", "csc_classify_vertex", "csc_scan_convert_count", "csc_timing_enable",
           "csc_timing_reset", "csc_timing_read", "csc_timing_stage_name", "csc_build_features_batched",
           "csc_features_sync", "csc_scan_convert_batched", "csc_sdf_backward_batched", "csc_interior_fill",
           "csc_weld_soup", "csc_scan_record_atomics", "csc_atomic_replay", "csc_fadd_rate",
           "csc_weld_soup_noalloc", "csc_weld_soup_noalloc_max_faces", "csc_scan_convert_workspace_for",
           "csc_features_order_faces"]
CSC_BUILD_NO_SYNC = 1
CSC_BUILD_GRAPH_SAFE = 2
N_STAGES = 13

_lib = None


def lib():
    """Load libcsc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1903_00353_amd.build`")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.csc_build_features.restype = C.c_int
    L.csc_build_features.argtypes = [P, C.c_int64, P, C.c_int64, C.POINTER(csc_grid), C.POINTER(csc_options), P,
                                     C.POINTER(C.c_void_p)]
    L.csc_features_info.restype = C.c_int
    L.csc_features_info.argtypes = [P, C.POINTER(csc_feature_info)]
    L.csc_scan_convert_workspace.restype = C.c_int
    L.csc_scan_convert_workspace.argtypes = [P, C.POINTER(C.c_size_t), C.POINTER(C.c_int64)]
    L.csc_scan_convert_workspace_for.restype = C.c_int
    L.csc_scan_convert_workspace_for.argtypes = [P, C.c_int64, C.POINTER(C.c_size_t), C.POINTER(C.c_int64)]
    L.csc_scan_convert.restype = C.c_int
    L.csc_scan_convert.argtypes = [P, P, C.c_size_t, P, P, P, P, P, P]
    L.csc_sdf_backward.restype = C.c_int
    L.csc_sdf_backward.argtypes = [P, P, P, P, C.c_int64, P, P, P, P]
    L.csc_features_order_faces.restype = C.c_int
    L.csc_features_order_faces.argtypes = [P, C.c_int32, P]
    L.csc_scan_convert_count.restype = C.c_int
    L.csc_scan_convert_count.argtypes = [P, P, C.c_size_t, P, P]
    L.csc_timing_enable.restype = C.c_int
    L.csc_timing_enable.argtypes = [C.c_int]
    L.csc_timing_reset.restype = C.c_int
    L.csc_timing_reset.argtypes = []
    L.csc_timing_read.restype = C.c_int
    L.csc_timing_read.argtypes = [P, P, C.c_int32]
    L.csc_timing_stage_name.restype = C.c_char_p
    L.csc_timing_stage_name.argtypes = [C.c_int32]
    L.csc_build_features_batched.restype = C.c_int
    L.csc_build_features_batched.argtypes = [P, P, P, P, C.POINTER(csc_grid), C.c_int32, C.POINTER(csc_options),
                                             C.c_int32, P, C.POINTER(C.c_void_p)]
    L.csc_weld_soup.restype = C.c_int
    L.csc_weld_soup.argtypes = [P, C.c_int64, P, P, C.POINTER(C.c_int64), P]
    L.csc_weld_soup_noalloc.restype = C.c_int
    L.csc_weld_soup_noalloc.argtypes = [P, C.c_int64, P, P, C.POINTER(C.c_int64), P]
    L.csc_weld_soup_noalloc_max_faces.restype = C.c_int64
    L.csc_weld_soup_noalloc_max_faces.argtypes = []
    L.csc_interior_fill.restype = C.c_int
    L.csc_interior_fill.argtypes = [P, P, P]
    L.csc_features_sync.restype = C.c_int
    L.csc_features_sync.argtypes = [P, P]
    L.csc_scan_convert_batched.restype = C.c_int
    L.csc_scan_convert_batched.argtypes = [P, P, C.c_size_t, P, P, P, P, P]
    L.csc_sdf_backward_batched.restype = C.c_int
    L.csc_sdf_backward_batched.argtypes = [P, P, P, P, C.c_int64, P, P, P, P]
    L.csc_scan_record_atomics.restype = C.c_int
    L.csc_scan_record_atomics.argtypes = [P, P, C.c_size_t, C.c_int32, P, P, C.c_int64, C.POINTER(C.c_int64), P]
    L.csc_atomic_replay.restype = C.c_int
    L.csc_atomic_replay.argtypes = [P, P, C.c_int64, P, C.c_int64, C.c_int32, P]
    L.csc_fadd_rate.restype = C.c_int
    L.csc_fadd_rate.argtypes = [P, C.c_int64, C.c_int64, P]
    L.csc_features_free.restype = None
    L.csc_features_free.argtypes = [P]
    L.csc_error_string.restype = C.c_char_p
    L.csc_error_string.argtypes = [C.c_int]
    L.csc_last_hip_error.restype = C.c_char_p
    L.csc_last_hip_error.argtypes = []
    L.csc_classify_edge.restype = C.c_int
    L.csc_classify_edge.argtypes = [P, P, P, P]
    L.csc_classify_vertex.restype = C.c_int
    L.csc_classify_vertex.argtypes = [P, P, C.c_int32, C.POINTER(csc_options), P, P]
    _lib = L
    return L


def _lib_error_string(code: int) -> str:
    return lib().csc_error_string(code).decode()


def csc_error_string(code: int) -> str:
    return _lib_error_string(code)


def make_grid(grid) -> csc_grid:
    """csc_grid from any object with ``n``, ``h``, ``band`` (and optional ``origin``)."""
    g = csc_grid()
    o = getattr(grid, "origin", (0.0, 0.0, 0.0))
    for k in range(3):
        g.origin[k] = float(o[k])
        g.n[k] = int(grid.n[k])
    g.h = float(grid.h)
    g.band_cells = float(grid.band)
    return g


def make_options(eps_rel=1e-3, ruff_mode=0, saddle_mode=0, force_both_sides=0, small_rows=(0, 0, 0),
                 scan_mode=0, absorb_cells=0.0, scan_grid=0, geom_blocks=0, keep_store_empty=0) -> csc_options:
    """absorb_cells: 0 the library's default, negative to give every non-flat
    feature its own polyhedron; scan_grid, geom_blocks: 0 the default schedule;
    keep_store_empty: 1 only for a scan workspace filled with 0xFF bytes once
    and used for nothing else (see csc.h)."""
    o = csc_options(float(eps_rel), int(ruff_mode), int(saddle_mode), int(force_both_sides))
    for k in range(3):
        o.small_rows[k] = int(small_rows[k])
    o.scan_mode = int(scan_mode)
    o.absorb_cells = float(absorb_cells)
    o.scan_grid = int(scan_grid)
    o.geom_blocks = int(geom_blocks)
    o.keep_store_empty = int(keep_store_empty)
    return o


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _check(code: int, where: str):
    if code != 0:
        raise CscError(code, where)


class Features:
    """A built feature handle (``csc_features``). Keeps the mesh tensors alive."""

    def __init__(self, handle: C.c_void_p, verts, tris, grid: csc_grid, options):
        self.handle = handle
        self.verts, self.tris, self.grid, self.options = verts, tris, grid, options

    def info(self) -> dict:
        inf = csc_feature_info()
        _check(lib().csc_features_info(self.handle, C.byref(inf)), "csc_features_info")
        return inf.as_dict()

    def free(self):
        if self.handle:
            lib().csc_features_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _check_mesh(verts, tris):
    import torch
    if not (isinstance(verts, torch.Tensor) and isinstance(tris, torch.Tensor)):
        raise TypeError("verts and tris must be torch tensors")
    if verts.device.type != "cuda" or tris.device.type != "cuda":
        raise ValueError("verts and tris must be device tensors")
    if verts.dtype != torch.float32 or tris.dtype != torch.int32:
        raise TypeError("verts must be float32 and tris int32")
    if verts.dim() != 2 or verts.shape[1] != 3 or tris.dim() != 2 or tris.shape[1] != 3:
        raise ValueError("verts must be [V,3] and tris [F,3]")
    if not (verts.is_contiguous() and tris.is_contiguous()):
        raise ValueError("verts and tris must be contiguous")


def csc_build_features(verts, tris, grid, options=None, stream=None, reuse: Features | None = None) -> Features:
    _check_mesh(verts, tris)
    g = make_grid(grid)
    opt = options if options is not None else make_options()
    prev = reuse.handle if reuse is not None else None
    h = C.c_void_p(prev.value if isinstance(prev, C.c_void_p) else prev)
    code = lib().csc_build_features(_ptr(verts), verts.shape[0], _ptr(tris), tris.shape[0], C.byref(g),
                                    C.byref(opt), _stream(stream), C.byref(h))
    if code != 0:
        if reuse is not None:
            reuse.verts, reuse.tris = verts, tris
        raise CscError(code, "csc_build_features")
    if reuse is not None:
        reuse.handle, reuse.verts, reuse.tris, reuse.grid, reuse.options = h, verts, tris, g, opt
        return reuse
    return Features(h, verts, tris, g, opt)


def csc_scan_convert_workspace(f: Features):
    nbytes, mx = C.c_size_t(), C.c_int64()
    _check(lib().csc_scan_convert_workspace(f.handle, C.byref(nbytes), C.byref(mx)), "csc_scan_convert_workspace")
    return int(nbytes.value), int(mx.value)


def csc_scan_convert_workspace_for(f: Features, n_bricks: int):
    nbytes, mx = C.c_size_t(), C.c_int64()
    _check(lib().csc_scan_convert_workspace_for(f.handle, int(n_bricks), C.byref(nbytes), C.byref(mx)),
           "csc_scan_convert_workspace_for")
    return int(nbytes.value), int(mx.value)


@dataclasses.dataclass
class Band:
    sdf: "object"      # float32 [M]
    feat: "object"     # int32 [M]
    cell: "object"     # int32 [M]
    n_band: int


def csc_scan_convert(f: Features, workspace=None, out=None, dense=None, stream=None, sync_count=True):
    """Run the scan conversion. ``out`` = (sdf, feat, cell, n_band) preallocated
    device tensors of max_band_cells entries (+ an int64 scalar) or None. Returns a
    ``Band`` whose tensors are sliced to the band size (reading it synchronises)
    unless ``sync_count`` is False (then full-length tensors and n_band = -1)."""
    import torch
    nbytes, mx = csc_scan_convert_workspace(f)
    dev = f.verts.device
    if workspace is None:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    if out is None:
        out = (torch.empty(max(mx, 1), dtype=torch.float32, device=dev),
               torch.empty(max(mx, 1), dtype=torch.int32, device=dev),
               torch.empty(max(mx, 1), dtype=torch.int32, device=dev),
               torch.zeros(1, dtype=torch.int64, device=dev))
    sdf, feat, cell, nb = out
    code = lib().csc_scan_convert(f.handle, _ptr(workspace), workspace.numel(), _ptr(sdf), _ptr(feat), _ptr(cell),
                                  _ptr(nb), _ptr(dense), _stream(stream))
    _check(code, "csc_scan_convert")
    if not sync_count:
        return Band(sdf, feat, cell, -1)
    m = int(nb.item())
    return Band(sdf[:m], feat[:m], cell[:m], m)


def csc_sdf_backward(f: Features, band: Band, grad_sdf, grad_verts=None, stream=None, n_band_d=None):
    """Accumulate d(sum grad_sdf * SDF)/d(verts) into grad_verts (new zeros if None).
    ``grad_sdf`` None: the loss sum of SDF^2 (upstream 2 SDF formed in the kernel).
    With ``n_band_d`` (the device count from csc_scan_convert) the band size is read
    on the device and the band tensors may be the full-length outputs."""
    import torch
    if grad_verts is None:
        grad_verts = torch.zeros_like(f.verts)
    n = band.n_band if (band.n_band >= 0 and n_band_d is None) else band.sdf.numel()
    gp = None if grad_sdf is None else _ptr(grad_sdf.contiguous())
    code = lib().csc_sdf_backward(f.handle, _ptr(band.sdf), _ptr(band.feat), _ptr(band.cell), int(n),
                                  _ptr(n_band_d), gp, _ptr(grad_verts), _stream(stream))
    _check(code, "csc_sdf_backward")
    return grad_verts


def csc_scan_convert_count(f: Features, workspace=None, stream=None):
    """Atomics issued by the scans (diagnostic; synchronises): [faces, edges, vertices]
    of the one-thread-per-polyhedron launches, then the same of the overflow launches."""
    import torch
    nbytes, _ = csc_scan_convert_workspace(f)
    if workspace is None:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=f.verts.device)
    counts = (C.c_int64 * 6)()
    _check(lib().csc_scan_convert_count(f.handle, _ptr(workspace), workspace.numel(), counts, _stream(stream)),
           "csc_scan_convert_count")
    return [int(x) for x in counts]


def csc_scan_record_atomics(f: Features, workspace, launch: int = 0, stream=None):
    """Log the packed atomicMin instructions of one scan launch (diagnostic;
    synchronises): returns (log uint32 [rounds*64], mask int64 [rounds]) device
    tensors, one round per wavefront instruction."""
    import torch
    rounds = C.c_int64()
    _check(lib().csc_scan_record_atomics(f.handle, _ptr(workspace), workspace.numel(), int(launch), None, None, 0,
                                         C.byref(rounds), _stream(stream)), "csc_scan_record_atomics")
    n = int(rounds.value)
    log = torch.empty(max(1, 64 * n), dtype=torch.int32, device=workspace.device)
    mask = torch.zeros(max(1, n), dtype=torch.int64, device=workspace.device)
    got = C.c_int64()
    _check(lib().csc_scan_record_atomics(f.handle, _ptr(workspace), workspace.numel(), int(launch), _ptr(log),
                                         _ptr(mask), n, C.byref(got), _stream(stream)), "csc_scan_record_atomics")
    if int(got.value) != n:
        raise RuntimeError(f"csc_scan_record_atomics: {got.value} rounds on the second run, {n} on the first")
    return log[: 64 * n], mask[:n]


def csc_atomic_replay(log, mask, keys, mode: int = 0, stream=None):
    """Queue the replay of a logged atomic stream on ``keys`` (uint64-sized tensor)."""
    _check(lib().csc_atomic_replay(_ptr(log), _ptr(mask), int(mask.numel()), _ptr(keys), int(keys.numel()), int(mode),
                                   _stream(stream)), "csc_atomic_replay")


def csc_fadd_rate(grad, n: int, stream=None):
    """Queue n scattered float atomicAdds (x, y, z of random vertices) into grad [nv, 3]."""
    _check(lib().csc_fadd_rate(_ptr(grad), int(grad.shape[0]), int(n), _stream(stream)), "csc_fadd_rate")


def csc_timing_enable(on: bool = True):
    _check(lib().csc_timing_enable(1 if on else 0), "csc_timing_enable")


def csc_timing_reset():
    _check(lib().csc_timing_reset(), "csc_timing_reset")


def csc_timing_read() -> dict:
    """{stage name: (total ms, calls)} accumulated since the last reset."""
    ms = (C.c_double * N_STAGES)()
    calls = (C.c_int64 * N_STAGES)()
    _check(lib().csc_timing_read(ms, calls, N_STAGES), "csc_timing_read")
    return {lib().csc_timing_stage_name(i).decode(): (float(ms[i]), int(calls[i])) for i in range(N_STAGES)}


def csc_timing_stage_name(i: int) -> str:
    return lib().csc_timing_stage_name(i).decode()


def csc_features_info(f: Features) -> dict:
    return f.info()


def csc_features_sync(f: Features, stream=None):
    _check(lib().csc_features_sync(f.handle, _stream(stream)), "csc_features_sync")


def csc_features_order_faces(f: Features, enable: bool = True, stream=None):
    """Set (or with ``enable=False`` drop) the spatial processing order of the
    face pass, computed from the face positions of the handle's last build and
    kept by later builds into the same handle. A schedule only: the outputs are
    bit for bit the same either way."""
    _check(lib().csc_features_order_faces(f.handle, 1 if enable else 0, _stream(stream)),
           "csc_features_order_faces")


def csc_build_features_batched(verts, tris, nv, nf, grids, options=None, flags=0, stream=None,
                               reuse: Features | None = None) -> Features:
    """verts: [sum nv, 3] float32, tris: [sum nf, 3] int32 (each mesh's own indices),
    nv / nf: per-mesh counts, grids: per-mesh grid objects."""
    _check_mesh(verts, tris)
    n = len(grids)
    if len(nv) != n or len(nf) != n or n == 0:
        raise ValueError("nv, nf and grids must have one entry per mesh")
    g = (csc_grid * n)(*[make_grid(x) for x in grids])
    nva = (C.c_int64 * n)(*[int(x) for x in nv])
    nfa = (C.c_int64 * n)(*[int(x) for x in nf])
    opt = options if options is not None else make_options()
    prev = reuse.handle if reuse is not None else None
    h = C.c_void_p(prev.value if isinstance(prev, C.c_void_p) else prev)
    code = lib().csc_build_features_batched(_ptr(verts), _ptr(tris), nva, nfa, g, n, C.byref(opt), int(flags),
                                            _stream(stream), C.byref(h))
    if code != 0:
        raise CscError(code, "csc_build_features_batched")
    if reuse is not None:
        reuse.handle, reuse.verts, reuse.tris, reuse.grid, reuse.options = h, verts, tris, g, opt
        return reuse
    return Features(h, verts, tris, g, opt)


def csc_scan_convert_batched(f: Features, workspace, out, band_off, stream=None):
    sdf, feat, cell = out
    code = lib().csc_scan_convert_batched(f.handle, _ptr(workspace), workspace.numel(), _ptr(sdf), _ptr(feat),
                                          _ptr(cell), _ptr(band_off), _stream(stream))
    _check(code, "csc_scan_convert_batched")


def csc_sdf_backward_batched(f: Features, out, band_off, grad_sdf, grad_verts, stream=None):
    sdf, feat, cell = out
    code = lib().csc_sdf_backward_batched(f.handle, _ptr(sdf), _ptr(feat), _ptr(cell), int(sdf.numel()),
                                          _ptr(band_off), None if grad_sdf is None else _ptr(grad_sdf),
                                          _ptr(grad_verts), _stream(stream))
    _check(code, "csc_sdf_backward_batched")


class Batch:
    """Many meshes, each with its own grid, processed by one set of launches.

    ``meshes``: list of (verts [nv,3] float32, tris [nf,3] int32) arrays or tensors.
    After ``Batch(...)`` (one synchronised build that sizes every buffer), each
    ``step()`` runs build + scan conversion (+ adjoint of sum SDF^2) without any
    host synchronisation or allocation, so it can be captured in a graph
    (``capture()``) and replayed (``replay()``).

    The band store holds ``headroom`` times the bricks of that first build (at
    most every brick of the grids), so that steps on moved vertices that reach
    new bricks still fit. Bricks past that capacity are dropped and flagged:
    ``check()`` (or ``overflowed()``) after a step or replay whose vertices moved
    tells whether that happened; call it before the next step, whose build
    clears the flag.

    With ``face_order`` the face pass takes the faces in the spatial order of
    that first build (``csc_features_order_faces``), kept by every later step: a
    schedule only, the results are the same bit for bit.

    The batch's workspace is filled with empty keys once and its builds set
    ``keep_store_empty`` (whatever ``options`` says), so that no scan fills the
    key store itself; scan it with nothing but this workspace."""

    def __init__(self, meshes, grids, options=None, device="cuda", backward=True, graph_safe=True, headroom=1.25,
                 face_order=True):
        import torch
        self.grids = list(grids)
        self.nv = [int(m[0].shape[0]) for m in meshes]
        self.nf = [int(m[1].shape[0]) for m in meshes]
        self.verts = torch.cat([torch.as_tensor(m[0], dtype=torch.float32).reshape(-1, 3) for m in meshes]).to(device)
        self.tris = torch.cat([torch.as_tensor(m[1], dtype=torch.int32).reshape(-1, 3) for m in meshes]).to(device)
        self.verts, self.tris = self.verts.contiguous(), self.tris.contiguous()
        self._options = options
        self.flags = CSC_BUILD_GRAPH_SAFE if graph_safe else 0
        self.f = csc_build_features_batched(self.verts, self.tris, self.nv, self.nf, self.grids, options,
                                            flags=self.flags)
        if face_order:
            csc_features_order_faces(self.f)
        nb = int(self.f.info()["n_bricks"])
        nbytes, mx = csc_scan_convert_workspace_for(self.f, int(nb * float(headroom)) + 1)
        # every key empty (all ones) before the first scan; each scan's sign pass leaves it so
        self.workspace = torch.full((max(nbytes, 1),), 255, dtype=torch.uint8, device=device)
        self.out = (torch.empty(max(mx, 1), dtype=torch.float32, device=device),
                    torch.empty(max(mx, 1), dtype=torch.int32, device=device),
                    torch.empty(max(mx, 1), dtype=torch.int32, device=device))
        self.band_off = torch.zeros(len(self.grids) + 1, dtype=torch.int64, device=device)
        self.backward = backward
        self.grad_verts = torch.zeros_like(self.verts)
        self.graph = None

    @property
    def options(self):
        """The build options (the given ones, or the defaults) with keep_store_empty set."""
        o = csc_options()
        if self._options is not None:
            C.memmove(C.byref(o), C.byref(self._options), C.sizeof(csc_options))
        else:
            o = make_options()
        o.keep_store_empty = 1
        return o

    @options.setter
    def options(self, value):
        self._options = value

    def step(self):
        """Build, scan conversion and (if enabled) the adjoint of sum SDF^2 (its
        upstream 2 SDF formed inside the adjoint kernel); queued only."""
        csc_build_features_batched(self.verts, self.tris, self.nv, self.nf, self.grids, self.options,
                                   flags=self.flags | CSC_BUILD_NO_SYNC, reuse=self.f)
        csc_scan_convert_batched(self.f, self.workspace, self.out, self.band_off)
        if self.backward:
            self.grad_verts.zero_()
            csc_sdf_backward_batched(self.f, self.out, self.band_off, None, self.grad_verts)

    def capture(self):
        import torch
        self.step()  # warm up outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def check(self):
        """Synchronise and raise if the last build or scan reported an error
        (CSC_WORKSPACE_TOO_SMALL: bricks past the store's capacity were dropped)."""
        csc_features_sync(self.f)

    def overflowed(self) -> bool:
        """Synchronise; True if the last step needed more bricks than the store holds."""
        try:
            csc_features_sync(self.f)
        except CscError as e:
            if e.code == 8:
                return True
            raise
        return False

    def band(self, m):
        """(sdf, feat, cell) tensors of mesh m (synchronises to read the offsets)."""
        off = self.band_off.cpu().tolist()
        a, b = off[m], off[m + 1]
        return self.out[0][a:b], self.out[1][a:b], self.out[2][a:b]

    def grad(self, m):
        a = sum(self.nv[:m])
        return self.grad_verts[a:a + self.nv[m]]


def csc_features_free(f: Features):
    f.free()


def csc_classify_edge(a, b, c1, c2) -> int:
    arrs = [np.ascontiguousarray(x, dtype=np.float32) for x in (a, b, c1, c2)]
    return int(lib().csc_classify_edge(*[x.ctypes.data_as(C.c_void_p) for x in arrs]))


def csc_classify_vertex(v, ring, options=None):
    """ring: [n][2][3] other corners of each incident triangle (counter-clockwise)."""
    v = np.ascontiguousarray(v, dtype=np.float32)
    ring = np.ascontiguousarray(ring, dtype=np.float32).reshape(-1, 6)
    ax = np.zeros(3)
    ct = C.c_double()
    opt = options if options is not None else make_options()
    bits = lib().csc_classify_vertex(v.ctypes.data_as(C.c_void_p), ring.ctypes.data_as(C.c_void_p), ring.shape[0],
                                     C.byref(opt), ax.ctypes.data_as(C.c_void_p), C.byref(ct))
    return int(bits), ax, float(ct.value)


def csc_weld_soup(soup, stream=None):
    """Indexed mesh from a triangle soup: soup float32 [F, 3, 3] (or [3F, 3]) on the
    device -> (verts float32 [V, 3], tris int32 [F, 3]); synchronises."""
    import torch
    soup = soup.contiguous().reshape(-1, 3, 3)
    if soup.dtype != torch.float32:
        raise TypeError("soup must be float32")
    nf = int(soup.shape[0])
    verts = torch.empty(3 * nf, 3, dtype=torch.float32, device=soup.device)
    tris = torch.empty(nf, 3, dtype=torch.int32, device=soup.device)
    nv = C.c_int64(0)
    _check(lib().csc_weld_soup(_ptr(soup), nf, _ptr(verts), _ptr(tris), C.byref(nv), _stream(stream)),
           "csc_weld_soup")
    return verts[: nv.value], tris


def csc_weld_soup_noalloc(soup, verts, tris, stream=None):
    """csc_weld_soup into caller-provided outputs (verts float32 [>= 3F, 3], tris
    int32 [F, 3]) with the library's static scratch: allocates nothing. Returns
    the vertex count (synchronises)."""
    soup = soup.reshape(-1, 3, 3)
    nv = C.c_int64(0)
    _check(lib().csc_weld_soup_noalloc(_ptr(soup), int(soup.shape[0]), _ptr(verts), _ptr(tris), C.byref(nv),
                                       _stream(stream)), "csc_weld_soup_noalloc")
    return int(nv.value)


def csc_weld_soup_noalloc_max_faces() -> int:
    return int(lib().csc_weld_soup_noalloc_max_faces())


def csc_interior_fill(f: Features, dense, stream=None):
    """Set the off-band cells inside the solid of a dense field written by
    csc_scan_convert to -inf, in place."""
    _check(lib().csc_interior_fill(f.handle, _ptr(dense), _stream(stream)), "csc_interior_fill")
    return dense


def sdf(verts, tris, grid, options=None, dense=False, fill_interior=False):
    """Narrow-band SDF of one mesh: returns (sdf, feat, cell[, dense]) device tensors;
    with fill_interior the dense field holds -inf in the solid's interior beyond the band."""
    import torch
    f = csc_build_features(verts, tris, grid, options)
    d = None
    if dense or fill_interior:
        dense = True
        d = torch.empty(int(grid.n[2]) * int(grid.n[1]) * int(grid.n[0]), dtype=torch.float32, device=verts.device)
    band = csc_scan_convert(f, dense=d)
    if fill_interior:
        csc_interior_fill(f, d)
    out = (band.sdf.clone(), band.feat.clone(), band.cell.clone())
    f.free()
    return out + ((d.view(int(grid.n[2]), int(grid.n[1]), int(grid.n[0])),) if dense else ())


def _autograd():
    import torch

    class CSCFunction(torch.autograd.Function):
        """(verts, tris, grid) -> band SDF values; differentiable in verts only."""

        @staticmethod
        def forward(ctx, verts, tris, grid, options=None):
            f = csc_build_features(verts.detach(), tris, grid, options)
            band = csc_scan_convert(f)
            ctx.f, ctx.band = f, band
            ctx.mark_non_differentiable(band.feat, band.cell)
            return band.sdf, band.feat, band.cell

        @staticmethod
        def backward(ctx, g_sdf, g_feat=None, g_cell=None):
            gv = csc_sdf_backward(ctx.f, ctx.band, g_sdf.contiguous().float())
            return gv, None, None, None

    return CSCFunction


def __getattr__(name):
    if name == "CSCFunction":
        cls = _autograd()
        globals()["CSCFunction"] = cls
        return cls
    raise AttributeError(name)
