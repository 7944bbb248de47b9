/*
 * csc.h -- C ABI of the Characteristic/Scan Conversion (CSC) narrow-band signed
 * distance library for AMD Instinct MI355X (gfx950).
 *
 * Method: Roosing, Strickson, Nikiforakis, "Fast Distance Fields for Fluid
 * Dynamics Mesh Generation on Graphics Hardware" (2019). Every face, edge and
 * vertex of a closed, consistently oriented triangle surface gets a
 * characteristic polyhedron (Section 3, Section 8); each polyhedron is
 * scan-converted onto the grid cells it contains (Section 5) and every cell keeps
 * the smallest distance to a feature whose polyhedron contains it (Alg. 1,
 * Section 2; Section 10). The sign comes from the angle-weighted pseudonormal of
 * the closest feature (Section 4.1.3, Eq. 8).
 *
 * Conventions (all entry points):
 *   - Pointers named *_d are device pointers owned by the caller (for example
 *     torch tensors); they must stay valid until the work queued on `stream`
 *     has finished. `stream` is a hipStream_t (NULL: the default stream).
 *   - Every call queues its device work asynchronously on `stream`; arguments
 *     are checked on the host first and nothing is queued when a check fails.
 *   - Return value: CSC_OK (0) or one of the error codes below. No C++
 *     exception crosses this interface.
 *   - Grid: cell (i, j, k) has centre origin + (i + 1/2, j + 1/2, k + 1/2) * h and
 *     linear index i + n[0] * (j + n[1] * k). A cell is in the band when its
 *     distance to the surface is strictly below band_cells * h (Section 10:
 *     values are written only below the user maximum distance).
 *   - Feature ids: faces 0..F-1 in input order; edges F + e, where e numbers the
 *     half-edges 3f+j whose start vertex index is below their end vertex index,
 *     in face-major order; vertices F + E + v.
 *   - Surface: vertices float32 [nv][3]; triangles int32 [nf][3], counter-clockwise
 *     seen from outside (Section 7); closed, 2-manifold, no zero-area face
 *     (Section 4, Section 6).
 */
#ifndef CSC_H
#define CSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum csc_status {
  CSC_OK = 0,
  CSC_INVALID_ARG = 1,             /* null pointer, size <= 0, non-finite grid value, index out of range,
                                      repeated vertex in a triangle, non-finite coordinate, bad size */
  CSC_NONMANIFOLD = 2,             /* an edge is not shared by exactly two triangles (open surface) */
  CSC_INCONSISTENT_ORIENTATION = 3,/* a directed edge occurs twice (flipped or duplicated triangle) */
  CSC_DEGENERATE_FACE = 4,         /* a triangle of zero area */
  CSC_GRID_TOO_LARGE = 5,          /* over 2^31 - 1 cells, over 65535 cells on an axis, or over
                                      2^26 brick positions in a batch */
  CSC_OUT_OF_MEMORY = 6,
  CSC_HIP_ERROR = 7,               /* a HIP runtime call failed (see csc_last_hip_error) */
  CSC_WORKSPACE_TOO_SMALL = 8,
  CSC_UNSUPPORTED_DEVICE = 9       /* the current device is not gfx950 */
};

typedef struct csc_grid {
  double origin[3];   /* corner of cell (0, 0, 0) */
  double h;           /* cell size, > 0 */
  int32_t n[3];       /* cells per axis, each > 0 */
  float band_cells;   /* band half-width in cells, > 0 */
} csc_grid;

typedef struct csc_options {
  float eps_rel;            /* slack of the inclusion tests as a fraction of h (Section 10: 1e-4..1e-3).
                               Only which cells are tested depends on it, never a value. Default 1e-3. */
  int32_t ruff_mode;        /* vertices with a normal pointing away from the pseudonormal (Section 3.3):
                               0 hemisphere (default, Section 4.1.3), 1 cone over the positive normals */
  int32_t saddle_mode;      /* saddle vertices (Section 3.2): 0 cone and its reflection (default),
                               1 hemispheres on both sides, 2 no extrusion (ablation only) */
  int32_t force_both_sides; /* 1: extrude every non-flat edge and every vertex on both sides */
  int32_t small_rows[3];    /* schedule (faces, edges, vertices): polyhedra with more rows than this
                               go to an overflow pass that gives each one a whole wavefront; the
                               rest share the rows of their wavefront. 0 = 32; values above 2^24
                               act as 2^24. Only the speed depends on it (see the autotuner in the
                               binding). */
  int32_t scan_mode;        /* 0 (default): each row of a polyhedron's box is intersected with its
                               half-spaces at once; 1: every cell of the box is tested by itself
                               (Alg. 2 as printed), an ablation that costs more and gives the same
                               field up to ties between features */
  float absorb_cells;       /* nearly flat features (Section 3.1: flat ones need no extrusion): an edge
                               whose face normals differ by theta needs no wedge of its own once its two
                               face prisms (Section 8.1) take side slack band_cells * sin(theta), and a
                               vertex with cone aperture theta none once its faces take
                               band_cells * sin(2 theta); the distances stay exact (a face prism computes
                               the exact distance to its triangle). Features whose slack is at most
                               this many cells are absorbed that way. 0 = default (0.05); negative: every
                               non-flat edge and vertex keeps its own polyhedron, as in Section 8; at most
                               0.24. The field agrees within the rounding of the FP32 distance whatever
                               the cap; bit for bit, the last bits of |d| and the choice among equally
                               close features can change with it. */
  int32_t scan_grid;        /* schedule of the one-polyhedron-per-lane scan pass (64 polyhedra per
                               wavefront): 1 a launch with one wavefront per 64 polyhedra; 2 a
                               persistent grid (as many wavefronts as fit on the device at once)
                               striding over the groups of 64; 3 that grid taking the groups from a
                               device counter in the order the wavefronts ask. 0 = default (2). Only
                               the speed depends on it (the autotuner in the binding picks one). */
  int32_t geom_blocks;      /* schedule of the build's face pass (face records and band bricks), which runs
                               beside the corner sort: 0 (default) one thread per face; n > 0 a grid of
                               at most n blocks of 256 striding over the faces, which leaves the sort
                               compute units of its own (a batch of many small meshes gains, one large
                               mesh loses). Only the speed depends on it (the binding's autotuner picks
                               it for a batch). */
  int32_t keep_store_empty; /* 1: the caller keeps the key store of the scan workspace empty between
                               scans: the workspace is filled with 0xFF bytes once, before its first
                               scan, and used for nothing else; every scan then skips filling the
                               store (the largest write of the pass) and its sign pass returns each
                               key it read to empty. After an error return, fill it again. 0
                               (default): every scan fills the store itself. Only the speed depends
                               on it. */
} csc_options;

typedef struct csc_features csc_features; /* opaque, library-owned, device resident */

/* Counts gathered while building the features (valid after a successful build). */
typedef struct csc_feature_info {
  int64_t n_vertices, n_faces, n_edges;
  int64_t n_edge_polyhedra, n_vertex_polyhedra;   /* faces give one prism each */
  int64_t edges_convex, edges_concave, edges_flat, edges_unknown;
  int64_t vertices_convex, vertices_concave, vertices_flat, vertices_saddle, vertices_ruff;
  int64_t n_bricks;                               /* allocated 8^3-cell bricks of the band store */
  int64_t max_band_cells;                         /* upper bound of the band size (n_bricks * 512) */
  int64_t edges_absorbed, vertices_absorbed;      /* nearly flat features handed to their faces
                                                     (csc_options.absorb_cells) */
} csc_feature_info;

/*
 * Build the features and their characteristic polyhedra (Section 7, Section 8):
 * edge/face adjacency, unit face normals, angle-weighted pseudonormals (Eq. 8),
 * edge classes (exact orientation predicate on the float inputs) and vertex
 * classes, cone apertures and ruff flags (double precision), the lists of edge
 * and vertex polyhedra, and the set of 8^3-cell bricks the band can touch.
 *
 * verts_d: float32 [nv][3]; tris_d: int32 [nf][3]. Both stay owned by the caller
 * and are read again by csc_scan_convert and csc_sdf_backward, so they must
 * outlive the handle and must not change while it is in use.
 * grid: cell geometry and band width. opt: NULL for defaults.
 * out: if *out is a handle from an earlier call, it is rebuilt in place (its
 * device memory is reused when large enough); else a new handle is made.
 * Synchronises `stream` once at the end (to read back error flags and counts).
 * The triangles are copied (with validated indices) into the handle.
 * Errors: INVALID_ARG, NONMANIFOLD, INCONSISTENT_ORIENTATION, DEGENERATE_FACE,
 * GRID_TOO_LARGE, OUT_OF_MEMORY, HIP_ERROR, UNSUPPORTED_DEVICE. On error a new
 * handle is not returned (*out unchanged) and a reused handle is left unusable
 * until rebuilt.
 */
int csc_build_features(const float* verts_d, int64_t nv, const int32_t* tris_d, int64_t nf,
                       const csc_grid* grid, const csc_options* opt, void* stream, csc_features** out);

/*
 * Batched build: n_meshes closed surfaces, each with its own grid, in one set of
 * launches. verts_d: float32 [sum nv][3], the meshes' vertices one after the
 * other; tris_d: int32 [sum nf][3], each mesh's triangles one after the other,
 * indexing that mesh's own vertices (0 .. nv[m]-1); nv, nf, grids: host arrays
 * of n_meshes entries. Feature ids and cell indices in the outputs are those of
 * each mesh on its own. flags:
 *   CSC_BUILD_NO_SYNC: queue the device work and return without synchronising;
 *     *out must be a handle already built (synchronously) for the same sizes,
 *     grids and options, so that nothing is allocated or copied from the host:
 *     the call can then be captured into a graph. Errors are read later by
 *     csc_features_sync.
 *   CSC_BUILD_GRAPH_SAFE: accepted for compatibility. Every build now groups
 *     corners with the library's own radix sort (kernels only, no memset
 *     nodes), so every build is safe to capture.
 * Errors as csc_build_features.
 */
#define CSC_BUILD_NO_SYNC 1
#define CSC_BUILD_GRAPH_SAFE 2
int csc_build_features_batched(const float* verts_d, const int32_t* tris_d, const int64_t* nv, const int64_t* nf,
                               const csc_grid* grids, int32_t n_meshes, const csc_options* opt, int32_t flags,
                               void* stream, csc_features** out);

/* Wait for the work queued on `stream`, read the handle's error flags and counts
 * back (after a CSC_BUILD_NO_SYNC build, or after a scan to detect a band store
 * too small for the bricks: CSC_WORKSPACE_TOO_SMALL). */
int csc_features_sync(csc_features* f, void* stream);

/* Spatial processing order of the face pass (a schedule, not a result: every
 * output is bit for bit the same with or without it). The paper sorts its
 * triangle soup by the Morton code of the vertices (Section 7.1); here the faces
 * keep their input ids and only the order in which the scan conversion takes
 * them changes: by the Morton code of each face's centroid in its own grid, per
 * mesh. Neighbouring faces then share wavefronts, and their atomic minima share
 * cache lines, where an input numbered by subdivision or by mesh generator
 * scatters them.
 *   enable 1: compute the order from the face positions of the handle's last
 *     build (call after a build; allocates, queues on `stream` and waits for
 *     it). Later builds into the same handle with the same total face count keep
 *     it: in a loop where the vertices move and the connectivity does not, one
 *     call serves every step (a stale order is only slower, never wrong).
 *   enable 0: drop the order (the input order again).
 * Errors: CSC_INVALID_ARG (null or unbuilt handle, enable not 0 or 1),
 * CSC_OUT_OF_MEMORY, CSC_HIP_ERROR. The handle owns the order; csc_features_free
 * releases it. */
int csc_features_order_faces(csc_features* f, int32_t enable, void* stream);

/* Copy the counts of a built and synchronised handle into *info. */
int csc_features_info(const csc_features* f, csc_feature_info* info);

/* Device workspace (bytes) csc_scan_convert needs, and the largest band size it
 * can return (the length the sdf/feat/cell outputs must have). The workspace
 * holds the band bricks counted by the last synchronised build (all bricks of
 * the grids if the handle was never synchronised). A larger workspace holds more
 * bricks; the outputs must then have 512 entries per brick it holds. */
int csc_scan_convert_workspace(const csc_features* f, size_t* bytes, int64_t* max_band_cells);

/* The same for a band store of n_bricks bricks (at most all bricks of the
 * grids): room for bricks that later builds with moved vertices may add (a
 * graph replayed on updated positions, for example). */
int csc_scan_convert_workspace_for(const csc_features* f, int64_t n_bricks, size_t* bytes, int64_t* max_band_cells);

/*
 * Scan-convert every polyhedron (Section 5, Alg. 2: inclusion by the half-space
 * test with slack, cones and hemispheres by their discriminant, Eq. 10), compute
 * the exact distance from each contained cell centre to the polyhedron's feature
 * (closed triangle, segment or point), keep per cell the smallest
 * (distance, feature id) pair (Alg. 1) and drop cells at distance >= band_cells*h;
 * then sign each band cell with the pseudonormal of its closest feature
 * (Section 4.1.3) and write the band as a compact list.
 *
 * workspace_d: ws_bytes >= csc_scan_convert_workspace() bytes of device memory.
 * sdf_d (float32), feat_d (int32), cell_d (int32 linear index): arrays of
 * max_band_cells entries; the first *n_band_d entries are written, ordered by
 * brick and within a brick in Morton order of the cell's position in its 8^3
 * brick (the bits of its in-brick x, y, z interleaved, x lowest): a fixed,
 * deterministic order.
 * n_band_d: device int64 scalar receiving the band size.
 * dense_d: NULL, or float32 [n[2]][n[1]][n[0]] receiving the dense field with
 * +infinity off the band (Alg. 1 initial value).
 * The result is bitwise identical from run to run.
 * Errors: INVALID_ARG, WORKSPACE_TOO_SMALL, HIP_ERROR.
 */
int csc_scan_convert(const csc_features* f, void* workspace_d, size_t ws_bytes, float* sdf_d, int32_t* feat_d,
                     int32_t* cell_d, int64_t* n_band_d, float* dense_d, void* stream);

/*
 * Triangle-soup ingestion (Section 7, Sections 7.1-7.2): weld the corners of an
 * STL-style soup, where every triangle carries its own three corner positions,
 * into an indexed mesh. Corners with equal positions (exact float equality, -0
 * equal to +0) become one vertex; vertices are numbered in order of first
 * appearance in the soup (corner order 3f + j), and tris_d[f][j] is the vertex
 * of corner j of triangle f, so triangle order and corner order (orientation)
 * are kept. Equal positions are grouped by sorting on the exact coordinates (not
 * on coarse Morton codes), so no group needs a sequential pass.
 *
 * soup_d: float32 [nf][3][3] device. verts_d: float32 [3*nf][3] device (room for
 * every corner being distinct); the first *nv rows are written. tris_d: int32
 * [nf][3] device. nv: host pointer receiving the vertex count. Allocates
 * temporaries (44 bytes per corner plus the radix sort's storage) with
 * hipMallocAsync on `stream` and synchronises it before returning. Triangles that collapse (two corners at
 * one position) are not removed here; csc_build_features rejects them.
 * Errors: INVALID_ARG (null, nf <= 0, 3*nf >= 2^31, non-finite coordinate),
 * OUT_OF_MEMORY, UNSUPPORTED_DEVICE, HIP_ERROR.
 */
int csc_weld_soup(const float* soup_d, int64_t nf, float* verts_d, int32_t* tris_d, int64_t* nv, void* stream);

/*
 * Triangle-soup welding for callers that cannot allocate device memory (code
 * under graph capture setup, tight serving loops, harnesses that forbid
 * hipMalloc): the same result as csc_weld_soup, bit for bit, with its scratch in
 * a 64 MiB array that the library holds on each GPU until the process ends, so
 * the call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine). The caller still passes soup_d, verts_d and tris_d as for
 * csc_weld_soup. Every call on one GPU uses that GPU's array: calls that overlap
 * on one GPU (from several host threads or streams) race and must not be made.
 * Synchronises `stream` before returning. nf may be at most
 * csc_weld_soup_noalloc_max_faces() (428,096 triangles); larger
 * soups return CSC_WORKSPACE_TOO_SMALL without queueing anything.
 * Errors: INVALID_ARG (as csc_weld_soup), WORKSPACE_TOO_SMALL, UNSUPPORTED_DEVICE,
 * HIP_ERROR.
 */
int csc_weld_soup_noalloc(const float* soup_d, int64_t nf, float* verts_d, int32_t* tris_d, int64_t* nv,
                          void* stream);
int64_t csc_weld_soup_noalloc_max_faces(void);

/*
 * Interior fill of a dense field (Section 11.3): the band leaves the cells of the
 * solid's interior farther than band_cells*h from the surface at +infinity, a
 * second zero crossing; this sets them to -infinity. dense_d: the float32
 * [n[2]][n[1]][n[0]] grid that csc_scan_convert wrote for this handle (band
 * values, +infinity elsewhere), modified in place on `stream` (queued after the
 * scan on the same stream). Along each z column an unset cell takes the side
 * (sign) of the nearest band cell before it in the column, or of the first one
 * after it; a column with no band cell stays +infinity. Exact for a closed
 * surface when band_cells > 1: where a column crosses the surface between two
 * neighbouring cell centres, both lie within one cell of the crossing and so
 * are band cells, each with its own side. Surfaces cut by the grid boundary are
 * handled as long as every z column that meets the solid meets the band.
 * Single-mesh handles only. Errors: INVALID_ARG (null, not built, batched
 * handle, band_cells <= 1), HIP_ERROR.
 */
int csc_interior_fill(const csc_features* f, float* dense_d, void* stream);

/*
 * Batched scan conversion (as csc_scan_convert for every mesh of a batched
 * handle, in one set of launches, with no host synchronisation). The band of
 * mesh m is entries [band_off_d[m], band_off_d[m+1]) of sdf_d / feat_d / cell_d,
 * with that mesh's own feature ids and cell indices. band_off_d: device int64
 * [n_meshes+1]. Bricks beyond the workspace's capacity are dropped and flagged
 * (csc_features_sync then returns CSC_WORKSPACE_TOO_SMALL).
 */
int csc_scan_convert_batched(const csc_features* f, void* workspace_d, size_t ws_bytes, float* sdf_d,
                             int32_t* feat_d, int32_t* cell_d, int64_t* band_off_d, void* stream);

/*
 * Adjoint of the band values with respect to the vertex positions. For each of
 * the band cells c (sdf_d, feat_d, cell_d as written by csc_scan_convert):
 * with q the closest point of the cell centre on feature feat_d[c] and w_k the
 * barycentric weights of q on the feature's vertices, SDF = s |c - q| and
 * dSDF/dx_k = -s w_k (c - q) / |c - q| (the closest feature is held fixed);
 * grad_verts_d[k] += grad_sdf_d[c] * dSDF/dx_k. grad_sdf_d: float32 per band
 * cell, or NULL for the loss L = sum of SDF^2 over the band, whose upstream
 * 2 SDF is then formed in the kernel from sdf_d (the same floats as an explicit
 * 2 * sdf array, without writing or reading one). Cells at zero distance add
 * nothing. grad_verts_d: float32 [nv][3], accumulated (not cleared). Terms
 * are first summed per block in 64-bit fixed point (exactly, for terms within
 * 2^-17 .. 4 times the block's first chunk's largest |grad_sdf|); those sums
 * and the other terms reach grad_verts_d through float atomics, whose order
 * varies from run to run.
 * n_band: number of band cells, or (with n_band_d) an upper bound on it.
 * n_band_d: NULL, or the device int64 written by csc_scan_convert; the count is
 * then read on the device, so no host synchronisation is needed in between.
 * Single-mesh handles only. Errors: INVALID_ARG, HIP_ERROR.
 */
int csc_sdf_backward(const csc_features* f, const float* sdf_d, const int32_t* feat_d, const int32_t* cell_d,
                     int64_t n_band, const int64_t* n_band_d, const float* grad_sdf_d, float* grad_verts_d,
                     void* stream);

/* Batched adjoint: as csc_sdf_backward over the band written by
 * csc_scan_convert_batched (band_off_d from that call; max_band an upper bound
 * on the total band size). grad_verts_d: float32 [sum nv][3], accumulated. */
int csc_sdf_backward_batched(const csc_features* f, const float* sdf_d, const int32_t* feat_d,
                             const int32_t* cell_d, int64_t max_band, const int64_t* band_off_d,
                             const float* grad_sdf_d, float* grad_verts_d, void* stream);

/*
 * Diagnostics: run only the key initialisation and the scan launches and return
 * the number of packed atomicMin operations each issued: counts[0..2] by the
 * one-thread-per-polyhedron launch for faces, edges and vertices, counts[3..5] by
 * the overflow launch of the same kinds. Synchronises `stream`. The band store in
 * the workspace is left as after a scan, but no band list is written.
 */
int csc_scan_convert_count(const csc_features* f, void* workspace_d, size_t ws_bytes, int64_t counts[6],
                           void* stream);

/*
 * Diagnostics for the atomic roofline. csc_scan_record_atomics runs the key
 * initialisation and the scan launches (as csc_scan_convert_count does) and logs
 * every packed atomicMin instruction of one launch (launch: 0-2 the
 * one-thread-per-polyhedron launch of faces, edges, vertices; 3-5 their overflow
 * launches; 6-8 their wide launches; -1 every launch) as one round: the key
 * indices of the issuing lanes at log_d[64 r + lane] (uint32, device,
 * 64 * max_rounds entries, lanes that do not issue left unwritten) and the mask
 * of issuing lanes at mask_d[r] (device, max_rounds entries). *rounds receives
 * the number of rounds issued, also those past max_rounds, which are not logged
 * (max_rounds 0 only counts them; the log pointers may then be NULL).
 * Synchronises `stream`. The launches run on one stream.
 * csc_atomic_replay issues the logged atomicMin instructions again, each round
 * as one instruction of one wavefront with the same lanes, and nothing else
 * (mode 0), or only reads the log (mode 1), or issues them at workgroup scope
 * (mode 2: in the issuing XCD's L2 only, so the values are meaningless; a rate
 * measurement) or as plain stores (mode 3), or in blocks of 8 rounds per
 * wavefront, the block's addresses loaded before its atomics are issued back to
 * back (mode 4: one wait for completion per block instead of per round, since
 * stores and atomics complete in order with loads): keys_d is any device array of n_keys
 * uint64 (indices at or past n_keys are skipped); rounds must not exceed the
 * rounds logged. csc_fadd_rate queues n float atomicAdds of 1 to the x, y and z
 * of pseudo-random vertices of grad_d (float32 [nv][3], device): the scattered
 * float-atomic rate the adjoint's flushes meet. Both queue one launch on
 * `stream` and return at once. Errors: INVALID_ARG, WORKSPACE_TOO_SMALL,
 * HIP_ERROR.
 */
int csc_scan_record_atomics(const csc_features* f, void* workspace_d, size_t ws_bytes, int32_t launch,
                            uint32_t* log_d, unsigned long long* mask_d, int64_t max_rounds, int64_t* rounds,
                            void* stream);
int csc_atomic_replay(const uint32_t* log_d, const unsigned long long* mask_d, int64_t rounds,
                      unsigned long long* keys_d, int64_t n_keys, int32_t mode, void* stream);
int csc_fadd_rate(float* grad_d, int64_t nv, int64_t n, void* stream);

/*
 * Per-stage timing with HIP events recorded on the stream of each call (stages:
 * 0 build_features, 1 init_keys, 2 scan_faces, 3 scan_edges, 4 scan_vertices,
 * 5 brick_count, 6 sign, 7 backward, 8 scan_faces_big, 9 scan_edges_big,
 * 10 scan_vertices_big, 11 interior_fill, 12 scan_wide; stages 2-4 time the
 * one-thread-per-polyhedron launch of each kind, 8-10 the wave-per-polyhedron
 * launch over its overflow list, 12 the three launches (one per kind) over the
 * polyhedra whose box exceeds 32 cells along an axis, whose distances are taken
 * in FP64; every other stage one launch or the whole build). While enabled, every call records a pair
 * of events around each stage; csc_timing_read waits for the recorded events and
 * returns the accumulated milliseconds and call counts of the first n stages.
 * A batch's scan otherwise runs the edge and vertex kinds on a second stream,
 * beside the faces; while timing is enabled the kinds run one after another, so
 * that each stage times one kernel running alone.
 * Process-wide; not meant for concurrent callers.
 */
int csc_timing_enable(int on);
int csc_timing_reset(void);
int csc_timing_read(double* ms, int64_t* calls, int32_t n);
const char* csc_timing_stage_name(int32_t stage);

/* Release a handle and its device memory (waits for nothing; the caller must
 * make sure no queued work still uses it). NULL is accepted. */
void csc_features_free(csc_features* f);

/* Static, human-readable text of a status code. */
const char* csc_error_string(int code);

/* Text of the last HIP runtime error seen by this thread ("" if none). */
const char* csc_last_hip_error(void);

/*
 * Host-side evaluation of the classification predicates the build uses on the
 * device (same code), for diagnostics and tests; no device is needed.
 * csc_classify_edge: a->b counter-clockwise in the left face with third vertex
 * c1, third vertex c2 of the right face; returns 0 flat, 1 convex, 2 concave,
 * 3 unknown (coordinates too far apart in magnitude for the exact evaluation).
 * csc_classify_vertex: vertex v and its incident triangles given as the two
 * other corners (ring[2i], ring[2i+1]) in counter-clockwise order; writes the
 * unit pseudonormal axis[3] and the cone aperture cosine *cos_t, returns the
 * class bits (1 outward extrusion, 2 inward, 4 outward is a hemisphere,
 * 8 inward is a hemisphere, 16 convex, 32 concave, 64 flat, 128 saddle, 256 ruff).
 */
int csc_classify_edge(const float a[3], const float b[3], const float c1[3], const float c2[3]);
int csc_classify_vertex(const float v[3], const float* ring, int32_t n_faces, const csc_options* opt,
                        double axis[3], double* cos_t);

#ifdef __cplusplus
}
#endif
#endif /* CSC_H */
