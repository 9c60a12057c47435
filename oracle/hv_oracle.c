/*
 * hv_oracle.c -- CPU oracle for per-pixel tile masks.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU path (no headers, no helpers, no constants) and nothing in the
 * product calls it.
 *
 * What it computes (HiVision, arXiv 2005.12489, Sec. 3.2.1 and Algorithm 1,
 * read in binary form):
 *   For tile (z,x,y) and pixel (i,j) (i = column, j = row from the north
 *   edge), with the style's radius or half-width r in pixels, the pixel's
 *   centre c is tested against every indexed object.  D(c) is the Euclidean
 *   distance from c to the nearest object, measured in world pixels of zoom z
 *   (one pixel is the resolution R_z of Algorithm 1, and the radius is
 *   R = N * R_z).  The pixel is lit iff D(c) <= r (the comparisons of
 *   Algorithm 1 are inclusive).
 *
 *   The paper's Algorithm 1 finds objects through R-tree box queries whose
 *   boxes are squares around the pixel (OuterBox) and only then measures
 *   distances ("filter, then refine").  This oracle does the same with one
 *   query box per pixel, the square c +- (r + 1e-5) px, followed by the exact
 *   distance to every object returned.  Like Algorithm 1's InnerBox step with
 *   limit(1), the search stops early once an object certainly lies within r.
 *
 * Readings of the paper made here (it is silent on each):
 *   - Space: Web-Mercator normalised to [0,1]^2, y = 0 at the north edge
 *     (WMTS/XYZ tile rows count from the top).  World size at zoom z is
 *     S = 256 * 2^z pixels, so R_z = 1/S.  Latitude is clamped to
 *     +-85.0511287798066 deg; there is no antimeridian wrap.
 *   - The pixel's own value is that of its centre sample.
 *   - Distance to a segment is the distance to the closed segment; a
 *     zero-length segment is a point.  Polygons arrive already split into
 *     edges (Sec. 3.1), each treated as a segment.
 *   - Tri-state output: pixels whose D lies within 1e-6 px of r are reported
 *     as ambiguous; elsewhere the result is certain at FP64 precision.
 *
 * Index: a serial Sort-Tile-Recursive packed R-tree (Leutenegger, Lopez and
 * Edgington, 1997) with fanout 16 and exact FP64 bounding boxes, built over
 * the objects (points, or segments split from linestrings and polygon edges,
 * as in the paper's RtreeP / RtreeL / RtreeE of Sec. 3.1).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -pthread -lm
 * (no -ffast-math; no FMA contraction, so every product is rounded once).
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_POINTS 0
#define OR_SEGMENTS 1
#define OR_EDGES 2
#define OR_MERC01 0x100

#define OR_FANOUT 16
#define OR_BAND 1e-6          /* ambiguity half-width, px */
#define OR_QUERY_PAD 1e-5     /* query box margin beyond r, px */
#define OR_MAX_LAT 85.0511287798066

static const double OR_PI = 3.14159265358979323846;

typedef struct { double x0, y0, x1, y1; } obox;

typedef struct {
    int kind;
    int64_t n;
    double *ax, *ay, *bx, *by;   /* normalised Mercator; points have b == a */
    int64_t n_nodes;
    obox *box;                   /* node bounding boxes */
    int64_t *first;              /* index into child[] */
    int32_t *count;
    uint8_t *leaf;               /* 1: children are object ids */
    int64_t *child;
    int64_t root;                /* -1 for an empty index */
    int depth;
} or_index;

/* ----------------------------------------------------------- projection */
/* lon/lat in degrees -> normalised Web-Mercator X (east), Y (south). */
static void project_one(double lon, double lat, double *X, double *Y)
{
    if (lat > OR_MAX_LAT) lat = OR_MAX_LAT;
    if (lat < -OR_MAX_LAT) lat = -OR_MAX_LAT;
    double phi = lat * (OR_PI / 180.0);
    *X = (lon + 180.0) / 360.0;
    *Y = 0.5 - log(tan(OR_PI / 4.0 + phi / 2.0)) / (2.0 * OR_PI);
}

int oracle_project(const double *lonlat, int64_t n, double *X, double *Y)
{
    for (int64_t k = 0; k < n; ++k) project_one(lonlat[2 * k], lonlat[2 * k + 1], &X[k], &Y[k]);
    return 0;
}

/* ------------------------------------------------------------ STR build */
typedef struct { obox b; double cx, cy; int64_t id; } entry;

static int cmp_cx(const void *a, const void *b)
{
    double u = ((const entry *)a)->cx, v = ((const entry *)b)->cx;
    return (u > v) - (u < v);
}

static int cmp_cy(const void *a, const void *b)
{
    double u = ((const entry *)a)->cy, v = ((const entry *)b)->cy;
    return (u > v) - (u < v);
}

static obox obj_box(const or_index *ix, int64_t k)
{
    obox b;
    b.x0 = fmin(ix->ax[k], ix->bx[k]);
    b.x1 = fmax(ix->ax[k], ix->bx[k]);
    b.y0 = fmin(ix->ay[k], ix->by[k]);
    b.y1 = fmax(ix->ay[k], ix->by[k]);
    return b;
}

/* Packs `ne` entries into ceil(ne/F) nodes with STR; appends the nodes. */
static int str_level(or_index *ix, entry *e, int64_t ne, int is_leaf,
                     int64_t *node_cap, int64_t *child_cap, int64_t *n_child)
{
    int64_t P = (ne + OR_FANOUT - 1) / OR_FANOUT;
    int64_t Sl = (int64_t)ceil(sqrt((double)P));
    int64_t slice = Sl * OR_FANOUT;
    qsort(e, (size_t)ne, sizeof(entry), cmp_cx);
    for (int64_t s = 0; s < ne; s += slice) {
        int64_t m = ne - s < slice ? ne - s : slice;
        qsort(e + s, (size_t)m, sizeof(entry), cmp_cy);
    }
    for (int64_t s = 0; s < ne; s += OR_FANOUT) {
        int64_t m = ne - s < OR_FANOUT ? ne - s : OR_FANOUT;
        if (ix->n_nodes == *node_cap) {
            *node_cap *= 2;
            ix->box = realloc(ix->box, (size_t)*node_cap * sizeof(obox));
            ix->first = realloc(ix->first, (size_t)*node_cap * sizeof(int64_t));
            ix->count = realloc(ix->count, (size_t)*node_cap * sizeof(int32_t));
            ix->leaf = realloc(ix->leaf, (size_t)*node_cap);
            if (!ix->box || !ix->first || !ix->count || !ix->leaf) return -1;
        }
        while (*n_child + m > *child_cap) {
            *child_cap *= 2;
            ix->child = realloc(ix->child, (size_t)*child_cap * sizeof(int64_t));
            if (!ix->child) return -1;
        }
        int64_t nd = ix->n_nodes++;
        obox b = e[s].b;
        for (int64_t k = 0; k < m; ++k) {
            const obox *c = &e[s + k].b;
            if (c->x0 < b.x0) b.x0 = c->x0;
            if (c->y0 < b.y0) b.y0 = c->y0;
            if (c->x1 > b.x1) b.x1 = c->x1;
            if (c->y1 > b.y1) b.y1 = c->y1;
            ix->child[*n_child + k] = e[s + k].id;
        }
        ix->box[nd] = b;
        ix->first[nd] = *n_child;
        ix->count[nd] = (int32_t)m;
        ix->leaf[nd] = (uint8_t)is_leaf;
        *n_child += m;
    }
    return 0;
}

void oracle_free(void *h)
{
    or_index *ix = (or_index *)h;
    if (!ix) return;
    free(ix->ax); free(ix->ay); free(ix->bx); free(ix->by);
    free(ix->box); free(ix->first); free(ix->count); free(ix->leaf); free(ix->child);
    free(ix);
}

/* objects: points (n,2) lon,lat  or  segments/edges (n,4) lon0,lat0,lon1,lat1;
 * with OR_MERC01 in kind the values are already normalised X,Y. */
void *oracle_build(const double *objects, int kind, int64_t n)
{
    int merc = (kind & OR_MERC01) != 0;
    int k = kind & 0xff;
    if (n < 0 || (k != OR_POINTS && k != OR_SEGMENTS && k != OR_EDGES)) return NULL;
    or_index *ix = calloc(1, sizeof(or_index));
    if (!ix) return NULL;
    ix->kind = k;
    ix->n = n;
    ix->root = -1;
    size_t sz = (size_t)(n > 0 ? n : 1) * sizeof(double);
    ix->ax = malloc(sz); ix->ay = malloc(sz); ix->bx = malloc(sz); ix->by = malloc(sz);
    if (!ix->ax || !ix->ay || !ix->bx || !ix->by) { oracle_free(ix); return NULL; }
    int w = (k == OR_POINTS) ? 2 : 4;
    for (int64_t q = 0; q < n; ++q) {
        const double *o = objects + (size_t)w * q;
        if (merc) {
            ix->ax[q] = o[0]; ix->ay[q] = o[1];
            ix->bx[q] = (w == 4) ? o[2] : o[0];
            ix->by[q] = (w == 4) ? o[3] : o[1];
        } else {
            project_one(o[0], o[1], &ix->ax[q], &ix->ay[q]);
            if (w == 4) project_one(o[2], o[3], &ix->bx[q], &ix->by[q]);
            else { ix->bx[q] = ix->ax[q]; ix->by[q] = ix->ay[q]; }
        }
    }
    if (n == 0) return ix;

    int64_t node_cap = n / 8 + 16, child_cap = n + n / 8 + 16, n_child = 0;
    ix->box = malloc((size_t)node_cap * sizeof(obox));
    ix->first = malloc((size_t)node_cap * sizeof(int64_t));
    ix->count = malloc((size_t)node_cap * sizeof(int32_t));
    ix->leaf = malloc((size_t)node_cap);
    ix->child = malloc((size_t)child_cap * sizeof(int64_t));
    entry *e = malloc((size_t)n * sizeof(entry));
    if (!ix->box || !ix->first || !ix->count || !ix->leaf || !ix->child || !e) {
        free(e); oracle_free(ix); return NULL;
    }
    for (int64_t q = 0; q < n; ++q) {
        e[q].b = obj_box(ix, q);
        e[q].cx = 0.5 * (e[q].b.x0 + e[q].b.x1);
        e[q].cy = 0.5 * (e[q].b.y0 + e[q].b.y1);
        e[q].id = q;
    }
    int64_t ne = n, lvl_first = 0;
    int is_leaf = 1;
    ix->depth = 0;
    for (;;) {
        lvl_first = ix->n_nodes;
        if (str_level(ix, e, ne, is_leaf, &node_cap, &child_cap, &n_child)) {
            free(e); oracle_free(ix); return NULL;
        }
        ix->depth++;
        int64_t made = ix->n_nodes - lvl_first;
        if (made == 1) break;
        for (int64_t q = 0; q < made; ++q) {
            int64_t nd = lvl_first + q;
            e[q].b = ix->box[nd];
            e[q].cx = 0.5 * (e[q].b.x0 + e[q].b.x1);
            e[q].cy = 0.5 * (e[q].b.y0 + e[q].b.y1);
            e[q].id = nd;
        }
        ne = made;
        is_leaf = 0;
    }
    ix->root = ix->n_nodes - 1;
    free(e);
    return ix;
}

int64_t oracle_node_count(const void *h) { return ((const or_index *)h)->n_nodes; }
int oracle_depth(const void *h) { return ((const or_index *)h)->depth; }

/* Root bounding box (normalised); returns 0 for an empty index. */
int oracle_root_box(const void *h, double *out4)
{
    const or_index *ix = (const or_index *)h;
    if (ix->root < 0) return 0;
    out4[0] = ix->box[ix->root].x0; out4[1] = ix->box[ix->root].y0;
    out4[2] = ix->box[ix->root].x1; out4[3] = ix->box[ix->root].y1;
    return 1;
}

/* ------------------------------------------------------------ predicates */
static int box_meets(const obox *a, const obox *b)
{
    return a->x0 <= b->x1 && b->x0 <= a->x1 && a->y0 <= b->y1 && b->y0 <= a->y1;
}

/* Distance (px) from the pixel centre (px,py) to object k, all in the
 * tile-local pixel frame: u = X*S - 256*x, v = Y*S - 256*y. */
static double obj_dist(const or_index *ix, int64_t k, double S, double ox, double oy,
                       double px, double py)
{
    double ax = ix->ax[k] * S - ox, ay = ix->ay[k] * S - oy;
    if (ix->kind == OR_POINTS) {
        double ex = px - ax, ey = py - ay;
        return sqrt(ex * ex + ey * ey);
    }
    double bx = ix->bx[k] * S - ox, by = ix->by[k] * S - oy;
    double dx = bx - ax, dy = by - ay;
    double len2 = dx * dx + dy * dy;
    double t = 0.0;
    if (len2 > 0.0) {
        t = ((px - ax) * dx + (py - ay) * dy) / len2;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    double ex = px - (ax + t * dx), ey = py - (ay + t * dy);
    return sqrt(ex * ex + ey * ey);
}

/* ------------------------------------------------------------ rendering */
enum { C_NODES = 0, C_LIT = 1, C_AMB = 2, C_NBOX_UNLIT = 3, C_UNLIT_CAND = 4, C_NCOUNT = 5 };

typedef struct {
    int64_t *stack; int64_t stack_cap;
    int64_t *pix_ids; int64_t pix_cap;       /* ids meeting c +- r for one pixel */
    int64_t *tile_ids; int64_t tile_cap, tile_n;
} scratch;

static int grow(int64_t **a, int64_t *cap, int64_t need)
{
    if (need <= *cap) return 0;
    int64_t c = *cap ? *cap : 256;
    while (c < need) c *= 2;
    int64_t *p = realloc(*a, (size_t)c * sizeof(int64_t));
    if (!p) return -1;
    *a = p; *cap = c;
    return 0;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t u = *(const int64_t *)a, v = *(const int64_t *)b;
    return (u > v) - (u < v);
}

static int render_tile(const or_index *ix, int z, int64_t tx, int64_t ty, double r,
                       uint8_t *tri, uint8_t *bit, double *dist, int64_t *cnt, scratch *sc)
{
    const double S = 256.0 * ldexp(1.0, z);
    const double ox = 256.0 * (double)tx, oy = 256.0 * (double)ty;
    const double h = r + OR_QUERY_PAD;
    int64_t nodes = 0, lit = 0, amb = 0, nbox_unlit = 0;
    sc->tile_n = 0;
    if (grow(&sc->stack, &sc->stack_cap, (int64_t)OR_FANOUT * (ix->depth + 2))) return -1;
    for (int j = 0; j < 256; ++j) {
        for (int i = 0; i < 256; ++i) {
            const double px = i + 0.5, py = j + 0.5;         /* tile-local centre */
            const double cx = ox + px, cy = oy + py;          /* world pixels */
            obox q = { (cx - h) / S, (cy - h) / S, (cx + h) / S, (cy + h) / S };
            obox qr = { (cx - r) / S, (cy - r) / S, (cx + r) / S, (cy + r) / S };
            double D = INFINITY;
            int64_t npix = 0;
            int certain = 0;
            int64_t sp = 0;
            if (ix->root >= 0) sc->stack[sp++] = ix->root;
            while (sp > 0 && !certain) {
                int64_t nd = sc->stack[--sp];
                ++nodes;
                if (!box_meets(&ix->box[nd], &q)) continue;
                const int64_t *ch = ix->child + ix->first[nd];
                if (!ix->leaf[nd]) {
                    for (int32_t c = 0; c < ix->count[nd]; ++c) sc->stack[sp++] = ch[c];
                    continue;
                }
                for (int32_t c = 0; c < ix->count[nd]; ++c) {
                    int64_t k = ch[c];
                    obox b = obj_box(ix, k);
                    if (!box_meets(&b, &q)) continue;
                    if (box_meets(&b, &qr)) {
                        if (grow(&sc->pix_ids, &sc->pix_cap, npix + 1)) return -1;
                        sc->pix_ids[npix++] = k;
                    }
                    double d = obj_dist(ix, k, S, ox, oy, px, py);
                    if (d < D) D = d;
                    if (D < r - OR_BAND) { certain = 1; break; }
                }
            }
            int b = D <= r;
            uint8_t t = D < r - OR_BAND ? 1 : (D > r + OR_BAND ? 0 : 2);
            size_t p = (size_t)j * 256 + (size_t)i;
            tri[p] = t;
            if (bit) bit[p] = (uint8_t)b;
            if (dist) dist[p] = D;
            lit += b;
            amb += (t == 2);
            if (!b && npix > 0) {
                nbox_unlit += npix;
                if (grow(&sc->tile_ids, &sc->tile_cap, sc->tile_n + npix)) return -1;
                memcpy(sc->tile_ids + sc->tile_n, sc->pix_ids, (size_t)npix * sizeof(int64_t));
                sc->tile_n += npix;
            }
        }
    }
    int64_t uniq = 0;
    if (sc->tile_n > 0) {
        qsort(sc->tile_ids, (size_t)sc->tile_n, sizeof(int64_t), cmp_i64);
        uniq = 1;
        for (int64_t q = 1; q < sc->tile_n; ++q) uniq += sc->tile_ids[q] != sc->tile_ids[q - 1];
    }
    if (cnt) {
        cnt[C_NODES] = nodes; cnt[C_LIT] = lit; cnt[C_AMB] = amb;
        cnt[C_NBOX_UNLIT] = nbox_unlit; cnt[C_UNLIT_CAND] = uniq;
    }
    return 0;
}

typedef struct {
    const or_index *ix;
    const int32_t *tiles;
    const double *r;
    int64_t ntiles;
    uint8_t *tri, *bit;
    double *dist;
    int64_t *cnt;
    int64_t next;          /* shared tile counter */
    int err;
} job;

static void *worker(void *arg)
{
    job *jb = (job *)arg;
    scratch sc;
    memset(&sc, 0, sizeof sc);
    for (;;) {
        int64_t t = __atomic_fetch_add(&jb->next, 1, __ATOMIC_RELAXED);
        if (t >= jb->ntiles) break;
        const int32_t *tl = jb->tiles + 3 * t;
        size_t off = (size_t)t * 65536;
        if (render_tile(jb->ix, tl[0], tl[1], tl[2], jb->r[t], jb->tri + off,
                        jb->bit ? jb->bit + off : NULL, jb->dist ? jb->dist + off : NULL,
                        jb->cnt ? jb->cnt + C_NCOUNT * t : NULL, &sc))
            __atomic_store_n(&jb->err, 1, __ATOMIC_RELAXED);
    }
    free(sc.stack); free(sc.pix_ids); free(sc.tile_ids);
    return NULL;
}

/* tiles: (ntiles,3) int32 z,x,y (0 <= z <= 30, 0 <= x,y < 2^z); r: per-tile
 * radius or half-width in px.  Outputs per tile, 256x256 row-major from the
 * north-west pixel: tri (0 unlit, 1 lit, 2 ambiguous), optional bit = [D<=r],
 * optional dist = D (an upper bound where the search stopped early on a
 * certain hit), optional counters (5 per tile).  Returns 0, or -1 on a bad
 * argument or allocation failure. */
int oracle_render(const void *h, const int32_t *tiles, int64_t ntiles, const double *r,
                  uint8_t *tri, uint8_t *bit, double *dist, int64_t *counters, int nthreads)
{
    const or_index *ix = (const or_index *)h;
    if (!ix || ntiles < 0 || (ntiles > 0 && (!tiles || !r || !tri))) return -1;
    for (int64_t t = 0; t < ntiles; ++t) {
        int32_t z = tiles[3 * t], x = tiles[3 * t + 1], y = tiles[3 * t + 2];
        if (z < 0 || z > 30 || x < 0 || y < 0 || (int64_t)x >= ((int64_t)1 << z) ||
            (int64_t)y >= ((int64_t)1 << z) || !(r[t] > 0.0) || !isfinite(r[t]))
            return -1;
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    job jb = { ix, tiles, r, ntiles, tri, bit, dist, counters, 0, 0 };
    pthread_t th[256];
    int started = 0;
    for (int k = 1; k < nthreads; ++k)
        if (pthread_create(&th[started], NULL, worker, &jb) == 0) ++started;
    worker(&jb);
    for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
    return jb.err ? -1 : 0;
}

/* ---------------------------------------------------- anti-aliased output */
/*
 * Algorithm 1 in full (Sec. 3.2.1) gives every pixel a value 0-4: the number
 * of its four sub-samples, at the pixel centre +- 1/4 px in x and in y, that
 * lie in the rasterised zone of radius r.
 *
 * OR_AA_EXACT -- the plain definition: value = #{ s : D(s) <= r }, D the
 *   distance from sub-sample s to the nearest object.  Each sub-sample gets
 *   its own box query s +- (r + pad).  amb = the number of sub-samples whose
 *   D lies within 1e-6 px of r; lit_sure = the number with D < r - 1e-6.
 *   (Algorithm 1's early answers follow from it: D(P) <= R1 puts every
 *   sub-sample within r, D(P) > R2 puts none.)
 *
 * OR_AA_PAPER -- Algorithm 1's steps as printed, in px (R_z = 1):
 *   R1 = r - sqrt(2)/4, R2 = r + sqrt(2)/4, h = sqrt(2)/2 * R1.
 *   1. An object meeting InnerBox_1 = P +- h answers 4.
 *   2. Otherwise the object nearest to P among those meeting OuterBox_1 =
 *      P +- R1: if it lies within R1 of P, 4.
 *   3. Otherwise the nearest object Tmp among those meeting OuterBox_2 =
 *      P +- R2: if it lies within R2 of P, the number of sub-samples within
 *      r of Tmp.
 *   4. Otherwise 0.
 *   Reading: when several objects are equally near, Tmp is the one with the
 *   smallest input index.  Only the nearest object to the centre is used for
 *   the sub-samples, so this can count fewer sub-samples than OR_AA_EXACT.
 *   amb = 1 for a pixel where a comparison of step 2, 3 or 4 lies within
 *   1e-6 px of its threshold, or where another object is within 1e-6 px of
 *   Tmp's distance; lit_sure is unused (0).
 */
#define OR_AA_EXACT 0
#define OR_AA_PAPER 1

/* Distance from (px,py) to every object meeting the square (px,py) +- h, in
 * the tile-local pixel frame; returns the smallest and, if kmin is not NULL,
 * the smallest input index attaining it, plus the second-smallest distance
 * among other objects in *d2nd (INFINITY if none). */
static double nearest_in_box(const or_index *ix, double S, double ox, double oy, double px, double py,
                             double h, int64_t *kmin, double *d2nd, int64_t *stack)
{
    const double cx = ox + px, cy = oy + py;
    obox q = { (cx - h) / S, (cy - h) / S, (cx + h) / S, (cy + h) / S };
    double D = INFINITY, D2 = INFINITY;
    int64_t best = -1;
    int64_t sp = 0;
    if (ix->root >= 0 && h >= 0.0) stack[sp++] = ix->root;
    while (sp > 0) {
        int64_t nd = stack[--sp];
        if (!box_meets(&ix->box[nd], &q)) continue;
        const int64_t *ch = ix->child + ix->first[nd];
        if (!ix->leaf[nd]) {
            for (int32_t c = 0; c < ix->count[nd]; ++c) stack[sp++] = ch[c];
            continue;
        }
        for (int32_t c = 0; c < ix->count[nd]; ++c) {
            int64_t k = ch[c];
            obox b = obj_box(ix, k);
            if (!box_meets(&b, &q)) continue;
            double d = obj_dist(ix, k, S, ox, oy, px, py);
            if (d < D || (d == D && k < best)) {
                if (best >= 0 && D < D2) D2 = D;
                D = d;
                best = k;
            } else if (d < D2) {
                D2 = d;
            }
        }
    }
    if (kmin) *kmin = best;
    if (d2nd) *d2nd = D2;
    return D;
}

/* True when object k meets the closed square [x0,x1] x [y0,y1] (tile px). */
static int obj_meets_square(const or_index *ix, int64_t k, double S, double ox, double oy,
                            double x0, double y0, double x1, double y1)
{
    double ax = ix->ax[k] * S - ox, ay = ix->ay[k] * S - oy;
    if (ix->kind == OR_POINTS) return ax >= x0 && ax <= x1 && ay >= y0 && ay <= y1;
    double bx = ix->bx[k] * S - ox, by = ix->by[k] * S - oy;
    /* clip the segment a + t (b - a), t in [0, 1], against each slab */
    double t0 = 0.0, t1 = 1.0;
    const double d[2] = { bx - ax, by - ay }, a[2] = { ax, ay }, lo[2] = { x0, y0 }, hi[2] = { x1, y1 };
    for (int c = 0; c < 2; ++c) {
        if (d[c] == 0.0) {
            if (a[c] < lo[c] || a[c] > hi[c]) return 0;
            continue;
        }
        double u = (lo[c] - a[c]) / d[c], v = (hi[c] - a[c]) / d[c];
        if (u > v) { double w = u; u = v; v = w; }
        if (u > t0) t0 = u;
        if (v < t1) t1 = v;
        if (t0 > t1) return 0;
    }
    return 1;
}

static int inner_box_hit(const or_index *ix, double S, double ox, double oy, double px, double py,
                         double h, int64_t *stack)
{
    if (!(h >= 0.0) || ix->root < 0) return 0;
    const double cx = ox + px, cy = oy + py;
    obox q = { (cx - h) / S, (cy - h) / S, (cx + h) / S, (cy + h) / S };
    int64_t sp = 0;
    stack[sp++] = ix->root;
    while (sp > 0) {
        int64_t nd = stack[--sp];
        if (!box_meets(&ix->box[nd], &q)) continue;
        const int64_t *ch = ix->child + ix->first[nd];
        if (!ix->leaf[nd]) {
            for (int32_t c = 0; c < ix->count[nd]; ++c) stack[sp++] = ch[c];
            continue;
        }
        for (int32_t c = 0; c < ix->count[nd]; ++c)
            if (obj_meets_square(ix, ch[c], S, ox, oy, px - h, py - h, px + h, py + h)) return 1;
    }
    return 0;
}

static int render_tile_aa(const or_index *ix, int z, int64_t tx, int64_t ty, double r, int mode,
                          uint8_t *val, uint8_t *amb, uint8_t *sure, int64_t *stack)
{
    const double S = ldexp(256.0, z);
    const double ox = (double)tx * 256.0, oy = (double)ty * 256.0;
    const double q4 = sqrt(2.0) / 4.0;
    const double R1 = r - q4, R2 = r + q4, h = sqrt(2.0) / 2.0 * R1;
    static const double sx[4] = { -0.25, 0.25, -0.25, 0.25 }, sy[4] = { 0.25, 0.25, -0.25, -0.25 };
    for (int j = 0; j < 256; ++j) {
        for (int i = 0; i < 256; ++i) {
            const double px = 0.5 + i, py = 0.5 + j;
            const size_t p = (size_t)(256 * j + i);
            uint8_t v = 0, a = 0, su = 0;
            if (mode == OR_AA_EXACT) {
                for (int s = 0; s < 4; ++s) {
                    double D = nearest_in_box(ix, S, ox, oy, px + sx[s], py + sy[s], r + OR_QUERY_PAD,
                                              NULL, NULL, stack);
                    v += D <= r;
                    a += fabs(D - r) <= OR_BAND;
                    su += D < r - OR_BAND;
                }
            } else {
                if (inner_box_hit(ix, S, ox, oy, px, py, h, stack)) {
                    v = 4;                                            /* step 1 */
                } else {
                    int64_t k = -1;
                    double D2;
                    double D = nearest_in_box(ix, S, ox, oy, px, py, R1, &k, &D2, stack);
                    if (k >= 0 && D <= R1) {
                        v = 4;                                        /* step 2 */
                        a = fabs(D - R1) <= OR_BAND;
                    } else {
                        D = nearest_in_box(ix, S, ox, oy, px, py, R2, &k, &D2, stack);
                        if (k >= 0 && D <= R2) {                      /* step 3 */
                            for (int s = 0; s < 4; ++s) {
                                double d = obj_dist(ix, k, S, ox, oy, px + sx[s], py + sy[s]);
                                v += d <= r;
                                a |= fabs(d - r) <= OR_BAND;
                            }
                            a |= fabs(D - R2) <= OR_BAND || fabs(D - R1) <= OR_BAND || D2 - D <= OR_BAND;
                        } else if (k >= 0) {
                            a = fabs(D - R2) <= OR_BAND;              /* step 4 */
                        }
                    }
                }
            }
            val[p] = v;
            if (amb) amb[p] = a;
            if (sure) sure[p] = su;
        }
    }
    return 0;
}

typedef struct {
    const or_index *ix;
    const int32_t *tiles;
    const double *r;
    int64_t ntiles;
    int mode;
    uint8_t *val, *amb, *sure;
    int64_t next;
    int err;
} job_aa;

static void *worker_aa(void *arg)
{
    job_aa *jb = (job_aa *)arg;
    int64_t *stack = malloc(sizeof(int64_t) * (size_t)OR_FANOUT * (size_t)(jb->ix->depth + 2));
    if (!stack) { __atomic_store_n(&jb->err, 1, __ATOMIC_RELAXED); return NULL; }
    for (;;) {
        int64_t t = __atomic_fetch_add(&jb->next, 1, __ATOMIC_RELAXED);
        if (t >= jb->ntiles) break;
        const int32_t *tl = jb->tiles + 3 * t;
        size_t off = (size_t)t * 65536;
        render_tile_aa(jb->ix, tl[0], tl[1], tl[2], jb->r[t], jb->mode, jb->val + off,
                       jb->amb ? jb->amb + off : NULL, jb->sure ? jb->sure + off : NULL, stack);
    }
    free(stack);
    return NULL;
}

/* Anti-aliased values 0-4 per pixel (see above).  tiles, r as for
 * oracle_render; val (required), amb and sure (optional) are ntiles x 65536
 * bytes, row-major from the north-west pixel.  Returns 0, or -1 on a bad
 * argument or allocation failure. */
int oracle_render_aa(const void *h, const int32_t *tiles, int64_t ntiles, const double *r, int mode,
                     uint8_t *val, uint8_t *amb, uint8_t *sure, int nthreads)
{
    const or_index *ix = (const or_index *)h;
    if (!ix || ntiles < 0 || (ntiles > 0 && (!tiles || !r || !val))) return -1;
    if (mode != OR_AA_EXACT && mode != OR_AA_PAPER) return -1;
    for (int64_t t = 0; t < ntiles; ++t) {
        int32_t z = tiles[3 * t], x = tiles[3 * t + 1], y = tiles[3 * t + 2];
        if (z < 0 || z > 30 || x < 0 || y < 0 || (int64_t)x >= ((int64_t)1 << z) ||
            (int64_t)y >= ((int64_t)1 << z) || !(r[t] > 0.0) || !isfinite(r[t]))
            return -1;
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    job_aa jb = { ix, tiles, r, ntiles, mode, val, amb, sure, 0, 0 };
    pthread_t th[256];
    int started = 0;
    for (int k = 1; k < nthreads; ++k)
        if (pthread_create(&th[started], NULL, worker_aa, &jb) == 0) ++started;
    worker_aa(&jb);
    for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
    return jb.err ? -1 : 0;
}

/* ------------------------------------------------------- polygon filling */
/*
 * SIBF (Sec. 3.2.2, Algorithm 2): a pixel is filled when its centre lies
 * inside some polygon.  The plain definition used here: for every polygon
 * whose bounding box holds the centre c, count the polygon's edges that a
 * ray from c towards +x crosses, with the half-open rule in y (an edge
 * (a, b) is crossed when exactly one of a.y, b.y is greater than c.y, and
 * the crossing lies at x > c.x), so that a vertex on the ray is counted
 * once and edges parallel to x never (Algorithm 2's IsLevel edges and
 * segment cutting do the same).  An odd count puts c inside that polygon
 * (even-odd rule: rings inside rings are holes).  The pixel is filled if c
 * is inside any polygon.
 *
 * Algorithm 2 casts its ray towards the nearer side of the polygon's box;
 * for closed rings the parity does not depend on the direction.
 *
 * Tri-state: 1 when c is inside some polygon and farther than 1e-6 px from
 * its edges; otherwise 2 (ambiguous) when c lies within 1e-6 px of an edge of
 * a candidate polygon; otherwise 0.  bit = [inside some polygon].
 *
 * Polygons: npoly groups of edges, polygon p owning edges [first[p],
 * first[p+1]) of the (n, 4) edge array; each group must form closed rings.
 */
typedef struct {
    or_index *mbr;                 /* STR tree over the polygons' bounding boxes */
    int64_t npoly, n;
    int64_t *first;                /* npoly + 1 */
    double *ax, *ay, *bx, *by;     /* normalised Mercator, input order */
} or_poly;

void oracle_free_polygons(void *h)
{
    or_poly *P = (or_poly *)h;
    if (!P) return;
    if (P->mbr) oracle_free(P->mbr);
    free(P->first); free(P->ax); free(P->ay); free(P->bx); free(P->by);
    free(P);
}

void *oracle_build_polygons(const double *edges, int64_t n, const int64_t *first, int64_t npoly, int merc01)
{
    if (n < 0 || npoly < 0 || (npoly > 0 && !first) || (n > 0 && !edges)) return NULL;
    if (npoly > 0 && (first[0] != 0 || first[npoly] != n)) return NULL;
    for (int64_t p = 0; p < npoly; ++p)
        if (first[p + 1] - first[p] < 3) return NULL;     /* a ring needs three edges */
    or_poly *P = calloc(1, sizeof(or_poly));
    if (!P) return NULL;
    P->npoly = npoly;
    P->n = n;
    size_t sz = (size_t)(n > 0 ? n : 1) * sizeof(double);
    P->first = malloc((size_t)(npoly + 1) * sizeof(int64_t));
    P->ax = malloc(sz); P->ay = malloc(sz); P->bx = malloc(sz); P->by = malloc(sz);
    double *mb = malloc((size_t)(npoly > 0 ? npoly : 1) * 4 * sizeof(double));
    if (!P->first || !P->ax || !P->ay || !P->bx || !P->by || !mb) {
        free(mb); oracle_free_polygons(P); return NULL;
    }
    for (int64_t p = 0; p <= npoly; ++p) P->first[p] = npoly > 0 ? first[p] : 0;
    for (int64_t q = 0; q < n; ++q) {
        const double *o = edges + 4 * q;
        if (merc01) { P->ax[q] = o[0]; P->ay[q] = o[1]; P->bx[q] = o[2]; P->by[q] = o[3]; }
        else { project_one(o[0], o[1], &P->ax[q], &P->ay[q]); project_one(o[2], o[3], &P->bx[q], &P->by[q]); }
    }
    for (int64_t p = 0; p < npoly; ++p) {
        double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
        for (int64_t q = first[p]; q < first[p + 1]; ++q) {
            x0 = fmin(x0, fmin(P->ax[q], P->bx[q])); x1 = fmax(x1, fmax(P->ax[q], P->bx[q]));
            y0 = fmin(y0, fmin(P->ay[q], P->by[q])); y1 = fmax(y1, fmax(P->ay[q], P->by[q]));
        }
        mb[4 * p] = x0; mb[4 * p + 1] = y0; mb[4 * p + 2] = x1; mb[4 * p + 3] = y1;
    }
    /* the box of a diagonal segment is the polygon's box */
    P->mbr = oracle_build(mb, OR_SEGMENTS | OR_MERC01, npoly);
    free(mb);
    if (!P->mbr) { oracle_free_polygons(P); return NULL; }
    return P;
}

/* Distance (px) from (cx, cy) to edge q, tile-local frame. */
static double edge_dist(const or_poly *P, int64_t q, double S, double ox, double oy, double cx, double cy)
{
    double ax = P->ax[q] * S - ox, ay = P->ay[q] * S - oy;
    double bx = P->bx[q] * S - ox, by = P->by[q] * S - oy;
    double dx = bx - ax, dy = by - ay, len2 = dx * dx + dy * dy, t = 0.0;
    if (len2 > 0.0) {
        t = ((cx - ax) * dx + (cy - ay) * dy) / len2;
        if (t < 0.0) t = 0.0;
        t = fmin(t, 1.0);
    }
    double ex = cx - (ax + t * dx), ey = cy - (ay + t * dy);
    return sqrt(ex * ex + ey * ey);
}

static void fill_tile(const or_poly *P, int z, int64_t tx, int64_t ty, uint8_t *tri, uint8_t *bit, int64_t *stack)
{
    const double S = ldexp(256.0, z);
    const double ox = (double)tx * 256.0, oy = (double)ty * 256.0;
    const or_index *M = P->mbr;
    for (int j = 0; j < 256; ++j) {
        for (int i = 0; i < 256; ++i) {
            const double cx = i + 0.5, cy = j + 0.5;            /* tile-local centre */
            const double wx = ox + cx, wy = oy + cy;             /* world pixels */
            const double g = OR_BAND;
            obox q = { (wx - g) / S, (wy - g) / S, (wx + g) / S, (wy + g) / S };
            int inside_sure = 0, inside_any = 0, near = 0;
            int64_t sp = 0;
            if (M->root >= 0) stack[sp++] = M->root;
            while (sp > 0 && !inside_sure) {
                int64_t nd = stack[--sp];
                if (!box_meets(&M->box[nd], &q)) continue;
                const int64_t *ch = M->child + M->first[nd];
                if (!M->leaf[nd]) {
                    for (int32_t c = 0; c < M->count[nd]; ++c) stack[sp++] = ch[c];
                    continue;
                }
                for (int32_t c = 0; c < M->count[nd] && !inside_sure; ++c) {
                    const int64_t p = ch[c];
                    obox b = obj_box(M, p);
                    if (!box_meets(&b, &q)) continue;
                    int par = 0;
                    double dmin = INFINITY;
                    for (int64_t e = P->first[p]; e < P->first[p + 1]; ++e) {
                        double ay = P->ay[e] * S - oy, by = P->by[e] * S - oy;
                        if ((ay > cy) != (by > cy)) {
                            double ax = P->ax[e] * S - ox, bx = P->bx[e] * S - ox;
                            double x = ax + (cy - ay) * (bx - ax) / (by - ay);
                            if (x > cx) par ^= 1;
                        }
                        double d = edge_dist(P, e, S, ox, oy, cx, cy);
                        if (d < dmin) dmin = d;
                    }
                    if (par) inside_any = 1;
                    if (dmin <= OR_BAND) near = 1;
                    else if (par) inside_sure = 1;
                }
            }
            const size_t at = (size_t)j * 256 + (size_t)i;
            tri[at] = inside_sure ? 1 : (near ? 2 : 0);
            if (bit) bit[at] = (uint8_t)(inside_sure || inside_any);
        }
    }
}

typedef struct {
    const or_poly *P;
    const int32_t *tiles;
    int64_t ntiles;
    uint8_t *tri, *bit;
    int64_t next;
    int err;
} job_fill;

static void *worker_fill(void *arg)
{
    job_fill *jb = (job_fill *)arg;
    int64_t *stack = malloc(sizeof(int64_t) * (size_t)OR_FANOUT * (size_t)(jb->P->mbr->depth + 2));
    if (!stack) { __atomic_store_n(&jb->err, 1, __ATOMIC_RELAXED); return NULL; }
    for (;;) {
        int64_t t = __atomic_fetch_add(&jb->next, 1, __ATOMIC_RELAXED);
        if (t >= jb->ntiles) break;
        const int32_t *tl = jb->tiles + 3 * t;
        size_t off = (size_t)t * 65536;
        fill_tile(jb->P, tl[0], tl[1], tl[2], jb->tri + off, jb->bit ? jb->bit + off : NULL, stack);
    }
    free(stack);
    return NULL;
}

/*
 * Work counters of filling one tile, for the fill roofline.  Algorithm 2
 * decides a pixel by the parity of a polygon's edges crossed by a ray from
 * the pixel centre along its row, for each polygon whose box holds the
 * centre.  Per tile:
 *   cnt[0]  candidate polygons: boxes that hold at least one pixel centre;
 *   cnt[1]  needed edges: edges of candidate polygons that a ray on one of
 *           the polygon's centre rows crosses in y (the half-open rule of
 *           the fill above: exactly one end strictly below the row), the
 *           edges whose crossings decide some parity;
 *   cnt[2]  (edge, row) crossings: over those edges, the rows counted;
 *   cnt[3]  (pixel, candidate polygon) pairs: the centres each candidate
 *           polygon's box holds.
 * Algorithmic bytes = 8192 + 32 cnt[1]; flops = 5 cnt[2] (the crossing's x:
 * two differences, a product, a quotient and a sum) + cnt[3] (one parity
 * test per pair).
 */
static void fill_counters_tile(const or_poly *P, int z, int64_t tx, int64_t ty, int64_t *cnt, int64_t *stack)
{
    const double S = ldexp(256.0, z);
    const double ox = (double)tx * 256.0, oy = (double)ty * 256.0;
    const or_index *M = P->mbr;
    /* the tile's pixel centres span [0.5, 255.5] in tile-local px */
    const obox q = { (ox + 0.5) / S, (oy + 0.5) / S, (ox + 255.5) / S, (oy + 255.5) / S };
    int64_t cand = 0, need = 0, pairs = 0, px = 0;
    int64_t sp = 0;
    if (M->root >= 0) stack[sp++] = M->root;
    while (sp > 0) {
        const int64_t nd = stack[--sp];
        if (!box_meets(&M->box[nd], &q)) continue;
        const int64_t *ch = M->child + M->first[nd];
        if (!M->leaf[nd]) {
            for (int32_t c = 0; c < M->count[nd]; ++c) stack[sp++] = ch[c];
            continue;
        }
        for (int32_t c = 0; c < M->count[nd]; ++c) {
            const int64_t p = ch[c];
            const obox b = obj_box(M, p);
            /* centres i + 0.5 inside [bx0, bx1], rows likewise */
            const double bx0 = b.x0 * S - ox, bx1 = b.x1 * S - ox, by0 = b.y0 * S - oy, by1 = b.y1 * S - oy;
            const double fi0 = fmax(ceil(bx0 - 0.5), 0.0), fi1 = fmin(floor(bx1 - 0.5), 255.0);
            const double fj0 = fmax(ceil(by0 - 0.5), 0.0), fj1 = fmin(floor(by1 - 0.5), 255.0);
            if (fi0 > fi1 || fj0 > fj1) continue;
            ++cand;
            px += (int64_t)(fi1 - fi0 + 1.0) * (int64_t)(fj1 - fj0 + 1.0);
            for (int64_t e = P->first[p]; e < P->first[p + 1]; ++e) {
                const double ay = P->ay[e] * S - oy, by = P->by[e] * S - oy;
                if (ay == by) continue;
                const double lo = fmin(ay, by), hi = fmax(ay, by);
                /* rows j with lo <= j + 0.5 < hi */
                const double rj0 = fmax(ceil(lo - 0.5), fj0), rj1 = fmin(ceil(hi - 0.5) - 1.0, fj1);
                if (rj0 > rj1) continue;
                ++need;
                pairs += (int64_t)(rj1 - rj0 + 1.0);
            }
        }
    }
    cnt[0] = cand;
    cnt[1] = need;
    cnt[2] = pairs;
    cnt[3] = px;
}

typedef struct {
    const or_poly *P;
    const int32_t *tiles;
    int64_t ntiles;
    int64_t *cnt;
    int64_t next;
    int err;
} job_fillcnt;

static void *worker_fillcnt(void *arg)
{
    job_fillcnt *jb = (job_fillcnt *)arg;
    int64_t *stack = malloc(sizeof(int64_t) * (size_t)OR_FANOUT * (size_t)(jb->P->mbr->depth + 2));
    if (!stack) { __atomic_store_n(&jb->err, 1, __ATOMIC_RELAXED); return NULL; }
    for (;;) {
        int64_t t = __atomic_fetch_add(&jb->next, 1, __ATOMIC_RELAXED);
        if (t >= jb->ntiles) break;
        const int32_t *tl = jb->tiles + 3 * t;
        fill_counters_tile(jb->P, tl[0], tl[1], tl[2], jb->cnt + 4 * t, stack);
    }
    free(stack);
    return NULL;
}

/* Fill work counters (see fill_counters_tile): cnt is ntiles x 4.
 * Returns 0, or -1 on a bad argument. */
int oracle_fill_counters(const void *h, const int32_t *tiles, int64_t ntiles, int64_t *cnt, int nthreads)
{
    const or_poly *P = (const or_poly *)h;
    if (!P || ntiles < 0 || (ntiles > 0 && (!tiles || !cnt))) return -1;
    for (int64_t t = 0; t < ntiles; ++t) {
        int32_t z = tiles[3 * t], x = tiles[3 * t + 1], y = tiles[3 * t + 2];
        if (z < 0 || z > 30 || x < 0 || y < 0 || (int64_t)x >= ((int64_t)1 << z) || (int64_t)y >= ((int64_t)1 << z))
            return -1;
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    job_fillcnt jb = { P, tiles, ntiles, cnt, 0, 0 };
    pthread_t th[256];
    int started = 0;
    for (int k = 1; k < nthreads; ++k)
        if (pthread_create(&th[started], NULL, worker_fillcnt, &jb) == 0) ++started;
    worker_fillcnt(&jb);
    for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
    return jb.err ? -1 : 0;
}

/* Fill masks of polygons (see above).  tiles as for oracle_render; tri
 * (required) and bit (optional) are ntiles x 65536 bytes, row-major from
 * the north-west pixel.  Returns 0, or -1 on a bad argument. */
int oracle_render_fill(const void *h, const int32_t *tiles, int64_t ntiles, uint8_t *tri, uint8_t *bit, int nthreads)
{
    const or_poly *P = (const or_poly *)h;
    if (!P || ntiles < 0 || (ntiles > 0 && (!tiles || !tri))) return -1;
    for (int64_t t = 0; t < ntiles; ++t) {
        int32_t z = tiles[3 * t], x = tiles[3 * t + 1], y = tiles[3 * t + 2];
        if (z < 0 || z > 30 || x < 0 || y < 0 || (int64_t)x >= ((int64_t)1 << z) || (int64_t)y >= ((int64_t)1 << z))
            return -1;
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    job_fill jb = { P, tiles, ntiles, tri, bit, 0, 0 };
    pthread_t th[256];
    int started = 0;
    for (int k = 1; k < nthreads; ++k)
        if (pthread_create(&th[started], NULL, worker_fill, &jb) == 0) ++started;
    worker_fill(&jb);
    for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
    return jb.err ? -1 : 0;
}
