/*
 * TEST INFRASTRUCTURE ONLY -- the CPU oracle.
 *
 * Plain, slow, FP64 reference for the narrow-band signed distance field that the
 * Characteristic/Scan Conversion method computes. Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library; the product
 * path never does. It shares no code with the device path.
 *
 * What it computes (plain definitions, not the method's steps):
 *   - d(c) = min over triangles T of the Euclidean distance from the cell centre c
 *     to the closed triangle T (Eq. 1, Section 2; the method reaches this result
 *     exactly, Section 2 and Alg. 1);
 *   - the band: cells with d(c) < band * h (the user maximum, Section 10);
 *   - the sign: with q the closest surface point, s = sign((c - q) . N) where N is
 *     the angle-weighted pseudonormal of the lowest-dimensional feature holding q
 *     (face normal; for an edge the sum of its two face normals; for a vertex
 *     sum_i alpha_i n_i, Eq. 8, Section 4.1.3), interior negative (Section 3.1);
 *   - feature ids: faces 0..F-1, then edges F + e with e counting the half-edges
 *     3f+j whose start vertex index is below their end vertex index in face-major
 *     order, then vertices F + E + v.
 *
 * The only speed-up is an exact cull: a triangle within band*h of c has its
 * bounding box, dilated by band*h, containing c, so cells outside every dilated
 * box are never in the band, and within a box every candidate triangle is tried.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double x, y, z; } vec;

static inline vec vsub(vec a, vec b) { vec r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static inline vec vadd(vec a, vec b) { vec r = {a.x + b.x, a.y + b.y, a.z + b.z}; return r; }
static inline vec vscale(vec a, double s) { vec r = {a.x * s, a.y * s, a.z * s}; return r; }
static inline double vdot(vec a, vec b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline vec vcross(vec a, vec b) {
    vec r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}
static inline double vlen(vec a) { return sqrt(vdot(a, a)); }
static inline vec vload(const double *V, int64_t i) { vec r = {V[3 * i], V[3 * i + 1], V[3 * i + 2]}; return r; }

static inline vec cell_centre(const double o[3], double h, const int32_t n[3], int64_t cell) {
    int64_t i = cell % n[0], j = (cell / n[0]) % n[1], k = cell / ((int64_t)n[0] * n[1]);
    vec c = {o[0] + (i + 0.5) * h, o[1] + (j + 0.5) * h, o[2] + (k + 0.5) * h};
    return c;
}

enum { R_FACE = 0, R_EDGE0 = 1, R_EDGE1 = 2, R_EDGE2 = 3, R_VERT0 = 4, R_VERT1 = 5, R_VERT2 = 6 };

/* Closest point q on the closed triangle (a, b, c) to p, by the Voronoi-region
 * tests of Ericson, Real-Time Collision Detection (2005), section 5.1.5.
 * Writes q and the barycentric weights w (q = w0 a + w1 b + w2 c) and returns the
 * region: face interior, edge j (local edge j joins corner j to corner j+1 mod 3)
 * or vertex j. A point landing exactly on a corner is reported as that vertex. */
static int closest_on_triangle(vec p, vec a, vec b, vec c, vec *q, double w[3]) {
    vec ab = vsub(b, a), ac = vsub(c, a), ap = vsub(p, a);
    double d1 = vdot(ab, ap), d2 = vdot(ac, ap);
    if (d1 <= 0 && d2 <= 0) { w[0] = 1; w[1] = 0; w[2] = 0; *q = a; return R_VERT0; }
    vec bp = vsub(p, b);
    double d3 = vdot(ab, bp), d4 = vdot(ac, bp);
    if (d3 >= 0 && d4 <= d3) { w[0] = 0; w[1] = 1; w[2] = 0; *q = b; return R_VERT1; }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0 && d1 >= 0 && d3 <= 0) {
        double t = d1 / (d1 - d3);
        w[0] = 1 - t; w[1] = t; w[2] = 0; *q = vadd(a, vscale(ab, t));
        return t == 0 ? R_VERT0 : (t == 1 ? R_VERT1 : R_EDGE0);
    }
    vec cp = vsub(p, c);
    double d5 = vdot(ab, cp), d6 = vdot(ac, cp);
    if (d6 >= 0 && d5 <= d6) { w[0] = 0; w[1] = 0; w[2] = 1; *q = c; return R_VERT2; }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0 && d2 >= 0 && d6 <= 0) {
        double t = d2 / (d2 - d6);
        w[0] = 1 - t; w[1] = 0; w[2] = t; *q = vadd(a, vscale(ac, t));
        return t == 0 ? R_VERT0 : (t == 1 ? R_VERT2 : R_EDGE2);
    }
    double va = d3 * d6 - d5 * d4;
    if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
        double t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        w[0] = 0; w[1] = 1 - t; w[2] = t; *q = vadd(b, vscale(vsub(c, b), t));
        return t == 0 ? R_VERT1 : (t == 1 ? R_VERT2 : R_EDGE1);
    }
    double den = 1.0 / (va + vb + vc);
    double v = vb * den, ww = vc * den;
    w[0] = 1 - v - ww; w[1] = v; w[2] = ww;
    *q = vadd(a, vadd(vscale(ab, v), vscale(ac, ww)));
    return R_FACE;
}

/* Closest point on the closed segment [a, b] to p; *t is the weight of b. */
static vec closest_on_segment(vec p, vec a, vec b, double *t) {
    vec ab = vsub(b, a);
    double den = vdot(ab, ab);
    double s = den > 0 ? vdot(vsub(p, a), ab) / den : 0.0;
    if (s < 0) s = 0;
    if (s > 1) s = 1;
    *t = s;
    return vadd(a, vscale(ab, s));
}

/* ----------------------------------------------------------------- features */

typedef struct { uint64_t key; int64_t h; } hkey;

static int cmp_hkey(const void *pa, const void *pb) {
    const hkey *a = (const hkey *)pa, *b = (const hkey *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->h < b->h ? -1 : (a->h > b->h);
}

/* Pair every half-edge with its twin and number the edges.
 * face_edges[3f+j] <- edge index of local edge j of face f;
 * edges[4e..4e+3] <- (a, b, f_left, f_right): a < b, a->b runs counter-clockwise in
 * f_left, b->a in f_right. Returns E, or -1 if some undirected edge does not have
 * exactly two half-edges of opposite direction (open, non-manifold, or flipped). */
int64_t oracle_edges(const int32_t *T, int64_t nf, int64_t nv, int32_t *face_edges, int32_t *edges) {
    int64_t nh = 3 * nf;
    hkey *k = (hkey *)malloc(sizeof(hkey) * (size_t)(nh > 0 ? nh : 1));
    int64_t *twin = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nh > 0 ? nh : 1));
    if (!k || !twin) { free(k); free(twin); return -2; }
    for (int64_t h = 0; h < nh; h++) {
        int64_t f = h / 3, j = h % 3;
        uint64_t u = (uint64_t)T[3 * f + j], w = (uint64_t)T[3 * f + (j + 1) % 3];
        uint64_t lo = u < w ? u : w, hi = u < w ? w : u;
        k[h].key = lo * (uint64_t)nv + hi;
        k[h].h = h;
    }
    qsort(k, (size_t)nh, sizeof(hkey), cmp_hkey);
    int64_t bad = 0;
    for (int64_t s = 0; s < nh;) {
        int64_t e = s + 1;
        while (e < nh && k[e].key == k[s].key) e++;
        if (e - s != 2) { bad = 1; break; }
        int64_t h0 = k[s].h, h1 = k[s + 1].h;
        int32_t a0 = T[h0], b0 = T[3 * (h0 / 3) + (h0 % 3 + 1) % 3];
        int32_t a1 = T[h1], b1 = T[3 * (h1 / 3) + (h1 % 3 + 1) % 3];
        if (!(a0 == b1 && b0 == a1)) { bad = 1; break; }
        twin[h0] = h1; twin[h1] = h0;
        s = e;
    }
    free(k);
    if (bad) { free(twin); return -1; }
    int64_t ne = 0;
    for (int64_t h = 0; h < nh; h++) {
        int64_t f = h / 3, j = h % 3;
        int32_t u = T[3 * f + j], w = T[3 * f + (j + 1) % 3];
        if (u < w) {
            face_edges[h] = (int32_t)ne;
            edges[4 * ne + 0] = u; edges[4 * ne + 1] = w;
            edges[4 * ne + 2] = (int32_t)f; edges[4 * ne + 3] = (int32_t)(twin[h] / 3);
            ne++;
        }
    }
    for (int64_t h = 0; h < nh; h++) {
        int64_t f = h / 3, j = h % 3;
        if (!(T[3 * f + j] < T[3 * f + (j + 1) % 3])) face_edges[h] = face_edges[twin[h]];
    }
    free(twin);
    return ne;
}

/* Unit face normals fn, edge pseudonormals en = n_left + n_right and vertex
 * pseudonormals vn = sum over incident faces of (corner angle) * (unit normal). */
void oracle_normals(const double *V, int64_t nv, const int32_t *T, int64_t nf, const int32_t *edges,
                    int64_t ne, double *fn, double *en, double *vn) {
    memset(vn, 0, sizeof(double) * 3 * (size_t)nv);
    for (int64_t f = 0; f < nf; f++) {
        vec p[3];
        for (int j = 0; j < 3; j++) p[j] = vload(V, T[3 * f + j]);
        vec n = vcross(vsub(p[1], p[0]), vsub(p[2], p[0]));
        n = vscale(n, 1.0 / vlen(n));
        fn[3 * f] = n.x; fn[3 * f + 1] = n.y; fn[3 * f + 2] = n.z;
        for (int j = 0; j < 3; j++) {
            vec e1 = vsub(p[(j + 1) % 3], p[j]), e2 = vsub(p[(j + 2) % 3], p[j]);
            double cs = vdot(e1, e2) / (vlen(e1) * vlen(e2));
            if (cs > 1) cs = 1;
            if (cs < -1) cs = -1;
            double al = acos(cs);
            int64_t v = T[3 * f + j];
            vn[3 * v] += al * n.x; vn[3 * v + 1] += al * n.y; vn[3 * v + 2] += al * n.z;
        }
    }
    for (int64_t e = 0; e < ne; e++) {
        int64_t fl = edges[4 * e + 2], fr = edges[4 * e + 3];
        for (int c = 0; c < 3; c++) en[3 * e + c] = fn[3 * fl + c] + fn[3 * fr + c];
    }
}

/* ------------------------------------------------------------------- band */

typedef struct {
    int64_t count;
    int32_t *cell;   /* linear cell index, ascending */
    double *d;       /* unsigned distance */
    double *sdf;     /* signed distance */
    int32_t *tri;    /* closest triangle (lowest index among exact ties) */
    int32_t *feat;   /* canonical feature id */
    uint8_t *flags;  /* bit0: d < band*h; bit1: d < 1e-6 h; bit2: |d - band*h| < 1e-6 h */
    int32_t threads; /* OpenMP threads used */
} oracle_band_t;

void oracle_band_free(oracle_band_t *b) {
    free(b->cell); free(b->d); free(b->sdf); free(b->tri); free(b->feat); free(b->flags);
    memset(b, 0, sizeof(*b));
}

/* index range [*i0, *i1] of cell centres o + (i + 1/2) h inside [lo, hi], clipped to [0, n) */
static void centre_range(double lo, double hi, double o, double h, int32_t n, int32_t *i0, int32_t *i1) {
    double a = ceil((lo - o) / h - 0.5), b = floor((hi - o) / h - 0.5);
    if (a < 0) a = 0;
    if (b > n - 1) b = n - 1;
    *i0 = (int32_t)a; *i1 = (int32_t)b;
}

/* sign and canonical feature of cell centre p whose closest triangle is t */
static void sign_and_feature(vec p, const double *V, const int32_t *T, int64_t t, const int32_t *face_edges,
                             int64_t nf, int64_t ne, const double *fn, const double *en, const double *vn,
                             double *d, double *s, int32_t *feat) {
    vec a = vload(V, T[3 * t]), b = vload(V, T[3 * t + 1]), c = vload(V, T[3 * t + 2]), q;
    double w[3];
    int r = closest_on_triangle(p, a, b, c, &q, w);
    vec N;
    if (r == R_FACE) { N = vload(fn, t); *feat = (int32_t)t; }
    else if (r <= R_EDGE2) {
        int64_t e = face_edges[3 * t + (r - R_EDGE0)];
        N = vload(en, e); *feat = (int32_t)(nf + e);
    } else {
        int64_t v = T[3 * t + (r - R_VERT0)];
        N = vload(vn, v); *feat = (int32_t)(nf + ne + v);
    }
    vec pq = vsub(p, q);
    *d = vlen(pq);
    *s = vdot(pq, N) >= 0 ? 1.0 : -1.0;
}

/* All cells with d < band*h + 1e-6 h in the z-planes [k0, k1). Output ascending in
 * the linear cell index. Returns 0, or a negative error. */
int oracle_band(const double *V, int64_t nv, const int32_t *T, int64_t nf, const int32_t *face_edges,
                int64_t ne, const double *fn, const double *en, const double *vn, const double origin[3],
                double h, const int32_t n[3], double band, int32_t k0, int32_t k1, oracle_band_t *out) {
    (void)nv;
    memset(out, 0, sizeof(*out));
    if (k0 < 0) k0 = 0;
    if (k1 > n[2]) k1 = n[2];
    const double wh = band * h, tol = 1e-6 * h;
    const double r = wh + 2 * tol; /* cull radius: every cell with d < wh + tol lies inside */
    int32_t *box = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)(nf > 0 ? nf : 1));
    if (!box) return -2;
    int32_t maxspan = 0;
    for (int64_t t = 0; t < nf; t++) {
        vec p0 = vload(V, T[3 * t]), p1 = vload(V, T[3 * t + 1]), p2 = vload(V, T[3 * t + 2]);
        double lo[3] = {fmin(p0.x, fmin(p1.x, p2.x)), fmin(p0.y, fmin(p1.y, p2.y)), fmin(p0.z, fmin(p1.z, p2.z))};
        double hi[3] = {fmax(p0.x, fmax(p1.x, p2.x)), fmax(p0.y, fmax(p1.y, p2.y)), fmax(p0.z, fmax(p1.z, p2.z))};
        for (int ax = 0; ax < 3; ax++)
            centre_range(lo[ax] - r, hi[ax] + r, origin[ax], h, n[ax], &box[6 * t + ax], &box[6 * t + 3 + ax]);
        int32_t span = box[6 * t + 5] - box[6 * t + 2];
        if (span > maxspan) maxspan = span;
    }
    /* bucket triangles by the first z-plane of their box */
    int32_t nk = n[2];
    int64_t *bstart = (int64_t *)calloc((size_t)nk + 1, sizeof(int64_t));
    int64_t *blist = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nf > 0 ? nf : 1));
    for (int64_t t = 0; t < nf; t++)
        if (box[6 * t + 2] <= box[6 * t + 5] && box[6 * t] <= box[6 * t + 3] && box[6 * t + 1] <= box[6 * t + 4])
            bstart[box[6 * t + 2] + 1]++;
    for (int32_t k = 0; k < nk; k++) bstart[k + 1] += bstart[k];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nk + 1));
    memcpy(fill, bstart, sizeof(int64_t) * ((size_t)nk + 1));
    for (int64_t t = 0; t < nf; t++)
        if (box[6 * t + 2] <= box[6 * t + 5] && box[6 * t] <= box[6 * t + 3] && box[6 * t + 1] <= box[6 * t + 4])
            blist[fill[box[6 * t + 2]]++] = t;
    free(fill);

    int32_t nplanes = k1 > k0 ? k1 - k0 : 0;
    int64_t *pcount = (int64_t *)calloc((size_t)nplanes + 1, sizeof(int64_t));
    int32_t **pcell = (int32_t **)calloc((size_t)nplanes + 1, sizeof(int32_t *));
    double **pd = (double **)calloc((size_t)nplanes + 1, sizeof(double *));
    double **psdf = (double **)calloc((size_t)nplanes + 1, sizeof(double *));
    int32_t **ptri = (int32_t **)calloc((size_t)nplanes + 1, sizeof(int32_t *));
    int32_t **pfeat = (int32_t **)calloc((size_t)nplanes + 1, sizeof(int32_t *));
    uint8_t **pflag = (uint8_t **)calloc((size_t)nplanes + 1, sizeof(uint8_t *));
    int64_t plane = (int64_t)n[0] * n[1];
    int nthreads = 1;

#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        nthreads = omp_get_num_threads();
#endif
        double *bd = (double *)malloc(sizeof(double) * (size_t)plane);
        int32_t *bt = (int32_t *)malloc(sizeof(int32_t) * (size_t)plane);
#pragma omp for schedule(dynamic, 1)
        for (int32_t k = k0; k < k1; k++) {
            for (int64_t c = 0; c < plane; c++) { bd[c] = INFINITY; bt[c] = -1; }
            int32_t kb0 = k - maxspan < 0 ? 0 : k - maxspan;
            double pz = origin[2] + (k + 0.5) * h;
            for (int32_t kb = kb0; kb <= k; kb++) {
                for (int64_t s = bstart[kb]; s < bstart[kb + 1]; s++) {
                    int64_t t = blist[s];
                    const int32_t *bx = &box[6 * t];
                    if (bx[5] < k) continue;
                    vec a = vload(V, T[3 * t]), b = vload(V, T[3 * t + 1]), cc = vload(V, T[3 * t + 2]);
                    for (int32_t j = bx[1]; j <= bx[4]; j++) {
                        double py = origin[1] + (j + 0.5) * h;
                        for (int32_t i = bx[0]; i <= bx[3]; i++) {
                            vec p = {origin[0] + (i + 0.5) * h, py, pz}, q;
                            double w[3];
                            closest_on_triangle(p, a, b, cc, &q, w);
                            vec pq = vsub(p, q);
                            double d2 = vdot(pq, pq);
                            int64_t ci = i + (int64_t)n[0] * j;
                            if (d2 < bd[ci] || (d2 == bd[ci] && t < bt[ci])) { bd[ci] = d2; bt[ci] = (int32_t)t; }
                        }
                    }
                }
            }
            int64_t cnt = 0;
            const double lim2 = (wh + tol) * (wh + tol);
            for (int64_t c = 0; c < plane; c++) cnt += (bt[c] >= 0 && bd[c] < lim2);
            int32_t pi = k - k0;
            pcount[pi] = cnt;
            pcell[pi] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt + 1));
            pd[pi] = (double *)malloc(sizeof(double) * (size_t)(cnt + 1));
            psdf[pi] = (double *)malloc(sizeof(double) * (size_t)(cnt + 1));
            ptri[pi] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt + 1));
            pfeat[pi] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt + 1));
            pflag[pi] = (uint8_t *)malloc((size_t)(cnt + 1));
            int64_t o = 0;
            for (int64_t c = 0; c < plane; c++) {
                if (!(bt[c] >= 0 && bd[c] < lim2)) continue;
                int64_t cell = c + plane * k;
                vec p = cell_centre(origin, h, n, cell);
                double d, s;
                int32_t feat;
                sign_and_feature(p, V, T, bt[c], face_edges, nf, ne, fn, en, vn, &d, &s, &feat);
                if (!(d < wh + tol)) continue;
                uint8_t fl = 0;
                if (d < wh) fl |= 1;
                if (d < tol) fl |= 2;
                if (fabs(d - wh) < tol) fl |= 4;
                pcell[pi][o] = (int32_t)cell; pd[pi][o] = d; psdf[pi][o] = s * d;
                ptri[pi][o] = bt[c]; pfeat[pi][o] = feat; pflag[pi][o] = fl;
                o++;
            }
            pcount[pi] = o;
        }
        free(bd); free(bt);
    }
    int64_t total = 0;
    for (int32_t p = 0; p < nplanes; p++) total += pcount[p];
    out->count = total;
    out->threads = nthreads;
    out->cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total + 1));
    out->d = (double *)malloc(sizeof(double) * (size_t)(total + 1));
    out->sdf = (double *)malloc(sizeof(double) * (size_t)(total + 1));
    out->tri = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total + 1));
    out->feat = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total + 1));
    out->flags = (uint8_t *)malloc((size_t)(total + 1));
    int64_t o = 0;
    for (int32_t p = 0; p < nplanes; p++) {
        size_t m = (size_t)pcount[p];
        memcpy(out->cell + o, pcell[p], m * sizeof(int32_t));
        memcpy(out->d + o, pd[p], m * sizeof(double));
        memcpy(out->sdf + o, psdf[p], m * sizeof(double));
        memcpy(out->tri + o, ptri[p], m * sizeof(int32_t));
        memcpy(out->feat + o, pfeat[p], m * sizeof(int32_t));
        memcpy(out->flags + o, pflag[p], m);
        o += (int64_t)m;
        free(pcell[p]); free(pd[p]); free(psdf[p]); free(ptri[p]); free(pfeat[p]); free(pflag[p]);
    }
    free(pcount); free(pcell); free(pd); free(psdf); free(ptri); free(pfeat); free(pflag);
    free(box); free(bstart); free(blist);
    return 0;
}

/* ------------------------------------------------------------- list modes */

/* Unsigned distance from each listed cell centre to the triangles T[sub[0..ns)]
 * (all triangles if sub is NULL), by trying every one of them. */
void oracle_cells_dist(const double *V, const int32_t *T, int64_t nf, const int64_t *sub, int64_t ns,
                       const double origin[3], double h, const int32_t n[3], const int64_t *cells, int64_t count,
                       double *out_d, int32_t *out_tri) {
    int64_t m = sub ? ns : nf;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < count; c++) {
        vec p = cell_centre(origin, h, n, cells[c]);
        double best = INFINITY;
        int32_t bt = -1;
        for (int64_t s = 0; s < m; s++) {
            int64_t t = sub ? sub[s] : s;
            vec q;
            double w[3];
            closest_on_triangle(p, vload(V, T[3 * t]), vload(V, T[3 * t + 1]), vload(V, T[3 * t + 2]), &q, w);
            vec pq = vsub(p, q);
            double d2 = vdot(pq, pq);
            if (d2 < best || (d2 == best && t < bt)) { best = d2; bt = (int32_t)t; }
        }
        out_d[c] = sqrt(best);
        out_tri[c] = bt;
    }
}

/* Closest point and barycentric weights of p on feature id (face, edge or vertex).
 * Returns the number of weighted vertices (3, 2 or 1), their indices in vid. */
static int feature_closest(vec p, const double *V, const int32_t *T, const int32_t *edges, int64_t nf,
                           int64_t ne, int64_t id, vec *q, double w[3], int64_t vid[3]) {
    if (id < nf) {
        for (int j = 0; j < 3; j++) vid[j] = T[3 * id + j];
        closest_on_triangle(p, vload(V, vid[0]), vload(V, vid[1]), vload(V, vid[2]), q, w);
        return 3;
    }
    if (id < nf + ne) {
        int64_t e = id - nf;
        double t;
        vid[0] = edges[4 * e]; vid[1] = edges[4 * e + 1];
        *q = closest_on_segment(p, vload(V, vid[0]), vload(V, vid[1]), &t);
        w[0] = 1 - t; w[1] = t;
        return 2;
    }
    vid[0] = id - nf - ne;
    *q = vload(V, vid[0]);
    w[0] = 1;
    return 1;
}

/* Distance from each listed cell centre to the closed feature feats[c]. */
void oracle_feature_dist(const double *V, const int32_t *T, const int32_t *edges, int64_t nf, int64_t ne,
                         const double origin[3], double h, const int32_t n[3], const int64_t *cells,
                         const int32_t *feats, int64_t count, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < count; c++) {
        vec p = cell_centre(origin, h, n, cells[c]), q;
        double w[3];
        int64_t vid[3];
        feature_closest(p, V, T, edges, nf, ne, feats[c], &q, w, vid);
        out[c] = vlen(vsub(p, q));
    }
}

/* Gradient of sum_c up[c] * SDF(c) with respect to the vertex positions, with the
 * closest feature of each cell held fixed (envelope theorem): SDF = s |c - q| and
 * q = sum_k w_k x_k, so dSDF/dx_k = -s w_k (c - q) / |c - q|. Cells at d = 0 add
 * nothing. grad (nv x 3) is overwritten. Serial, so the sum order is fixed. */
void oracle_grad(const double *V, int64_t nv, const int32_t *T, const int32_t *edges, int64_t nf, int64_t ne,
                 const double origin[3], double h, const int32_t n[3], const int64_t *cells, const int32_t *feats,
                 const double *sign, const double *up, int64_t count, double *grad) {
    memset(grad, 0, sizeof(double) * 3 * (size_t)nv);
    for (int64_t c = 0; c < count; c++) {
        vec p = cell_centre(origin, h, n, cells[c]), q;
        double w[3];
        int64_t vid[3];
        int m = feature_closest(p, V, T, edges, nf, ne, feats[c], &q, w, vid);
        vec pq = vsub(p, q);
        double d = vlen(pq);
        if (!(d > 0)) continue;
        vec g = vscale(pq, sign[c] / d);
        for (int k = 0; k < m; k++) {
            double f = -up[c] * w[k];
            grad[3 * vid[k]] += f * g.x; grad[3 * vid[k] + 1] += f * g.y; grad[3 * vid[k] + 2] += f * g.z;
        }
    }
}

/* Generalised winding number at each point: (1/4pi) * sum of the solid angles the
 * triangles subtend, each by the van Oosterom-Strackee formula (1983). About 1
 * inside a closed outward-oriented surface, about 0 outside. */
void oracle_winding(const double *V, const int32_t *T, int64_t nf, const double *pts, int64_t count, double *out) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < count; c++) {
        vec p = vload(pts, c);
        double acc = 0;
        for (int64_t t = 0; t < nf; t++) {
            vec a = vsub(vload(V, T[3 * t]), p), b = vsub(vload(V, T[3 * t + 1]), p), cc = vsub(vload(V, T[3 * t + 2]), p);
            double la = vlen(a), lb = vlen(b), lc = vlen(cc);
            double num = vdot(a, vcross(b, cc));
            double den = la * lb * lc + vdot(a, b) * lc + vdot(a, cc) * lb + vdot(b, cc) * la;
            acc += 2.0 * atan2(num, den);
        }
        out[c] = acc / (4.0 * M_PI);
    }
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
