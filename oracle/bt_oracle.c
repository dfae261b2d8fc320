/*
 * Plain FP64 CPU oracle of the hybrid beam tracer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * that the GPU library is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark load it; the product path never does.
 * It shares no code, header or table with the GPU library.
 *
 * What it computes (paper, Section 2, the hybrid method):
 *   - a source's power is split over beams by direction (solid angle), one
 *     triangular-frustum beam per face of a subdivided icosahedron;
 *   - only the guiding (central) ray of a beam is intersected with the model,
 *     as in ray tracing, so a beam is never split;
 *   - a hit spawns one specular child beam that has lost energy at the surface;
 *   - every microphone inside a beam's frustum receives the beam's
 *     contribution, and a microphone's level is the sum of contributions.
 * Where the paper is silent the readings below are used (beam shape, energy
 * split by solid angle, 1/d^2 spreading from the image apex, energy factor
 * (1 - alpha), frustum caps, tie rules, edge flags).  Each reading is listed
 * beside the function that implements it.
 *
 * Compile with -ffp-contract=off: the exact-antisymmetry argument behind the
 * microphone tie rule needs unfused products.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_LEVEL 9

/* ------------------------------------------------------------------------- */
/* small vector helpers                                                       */
/* ------------------------------------------------------------------------- */

static void v_sub(const double a[3], const double b[3], double r[3]) { r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2]; }
static void v_add(const double a[3], const double b[3], double r[3]) { r[0] = a[0] + b[0]; r[1] = a[1] + b[1]; r[2] = a[2] + b[2]; }
static double v_dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void v_cross(const double a[3], const double b[3], double r[3])
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static double v_norm(const double a[3]) { return sqrt(v_dot(a, a)); }
static void v_normalize(const double a[3], double r[3])
{
    double n = sqrt(v_dot(a, a));
    r[0] = a[0] / n; r[1] = a[1] / n; r[2] = a[2] / n;
}
static void v_copy(const double a[3], double r[3]) { r[0] = a[0]; r[1] = a[1]; r[2] = a[2]; }
static double v_det(const double a[3], const double b[3], const double c[3])
{
    double x[3];
    v_cross(b, c, x);
    return v_dot(a, x);
}

/* ------------------------------------------------------------------------- */
/* Icosphere: the beam directions (paper Section 2: a source's energy is shared */
/* between beams by direction).                                               */
/* Reading: one triangular beam per face of a level-L geodesic icosphere.      */
/*   base vertices: the cyclic permutations (0,a,b), (a,b,0), (b,0,a) of        */
/*     (0, +-1, +-phi), in that permutation order, then a = -1, +1, then        */
/*     b = -phi, +phi; normalised.                                             */
/*   base faces: vertex triples i<j<k at mutual (unnormalised) distance 2, in   */
/*     lexicographic order, with j and k swapped when det(vi,vj,vk) < 0.       */
/*   subdivision: (a,b,c) -> (a,ab,ca), (ab,b,bc), (ca,bc,c), (ab,bc,ca), where  */
/*     xy = normalize(x + y); child index = 4*parent + position.               */
/* ------------------------------------------------------------------------- */

int64_t orc_ico_nfaces(int level)
{
    if (level < 0 || level > ORC_MAX_LEVEL) return -1;
    int64_t n = 20;
    for (int l = 0; l < level; ++l) n *= 4;
    return n;
}

/* dirs: [nfaces][3][3] (d0, d1, d2 of each face), unit vectors, det > 0 */
int orc_icosphere(int level, double *dirs)
{
    if (level < 0 || level > ORC_MAX_LEVEL) return -1;
    const double phi = (1.0 + sqrt(5.0)) / 2.0;
    double raw[12][3];
    int nv = 0;
    for (int perm = 0; perm < 3; ++perm) {
        for (int ia = 0; ia < 2; ++ia) {
            for (int ib = 0; ib < 2; ++ib) {
                double a = ia ? 1.0 : -1.0;
                double b = ib ? phi : -phi;
                double p[3];
                if (perm == 0) { p[0] = 0.0; p[1] = a;   p[2] = b; }
                else if (perm == 1) { p[0] = a; p[1] = b; p[2] = 0.0; }
                else { p[0] = b; p[1] = 0.0; p[2] = a; }
                v_copy(p, raw[nv]);
                nv++;
            }
        }
    }
    double unit[12][3];
    for (int i = 0; i < 12; ++i) v_normalize(raw[i], unit[i]);

    /* 20 base faces */
    int nf = 0;
    double *cur = dirs; /* fill base faces at the front, expand level by level in place from the back */
    int64_t total = orc_ico_nfaces(level);
    double *base = (double *)malloc(sizeof(double) * 9 * 20);
    if (!base) return -2;
    for (int i = 0; i < 12; ++i) {
        for (int j = i + 1; j < 12; ++j) {
            for (int k = j + 1; k < 12; ++k) {
                double dij[3], djk[3], dki[3];
                v_sub(raw[i], raw[j], dij);
                v_sub(raw[j], raw[k], djk);
                v_sub(raw[k], raw[i], dki);
                if (fabs(v_dot(dij, dij) - 4.0) > 1e-9) continue;
                if (fabs(v_dot(djk, djk) - 4.0) > 1e-9) continue;
                if (fabs(v_dot(dki, dki) - 4.0) > 1e-9) continue;
                int a = i, b = j, c = k;
                if (v_det(unit[a], unit[b], unit[c]) < 0.0) { int t = b; b = c; c = t; }
                v_copy(unit[a], base + 9 * nf + 0);
                v_copy(unit[b], base + 9 * nf + 3);
                v_copy(unit[c], base + 9 * nf + 6);
                nf++;
            }
        }
    }
    if (nf != 20) { free(base); return -3; }

    /* level-by-level subdivision; a scratch buffer holds each level */
    double *src = base;
    int64_t n = 20;
    for (int l = 0; l < level; ++l) {
        double *dst = (double *)malloc(sizeof(double) * 9 * (size_t)(n * 4));
        if (!dst) { free(src); return -2; }
        for (int64_t f = 0; f < n; ++f) {
            const double *a = src + 9 * f, *b = a + 3, *c = a + 6;
            double s[3], ab[3], bc[3], ca[3];
            v_add(a, b, s); v_normalize(s, ab);
            v_add(b, c, s); v_normalize(s, bc);
            v_add(c, a, s); v_normalize(s, ca);
            double *o = dst + 9 * (4 * f);
            v_copy(a, o + 0);  v_copy(ab, o + 3);  v_copy(ca, o + 6);   /* (a, ab, ca) */
            v_copy(ab, o + 9); v_copy(b, o + 12);  v_copy(bc, o + 15);  /* (ab, b, bc) */
            v_copy(ca, o + 18); v_copy(bc, o + 21); v_copy(c, o + 24);  /* (ca, bc, c) */
            v_copy(ab, o + 27); v_copy(bc, o + 30); v_copy(ca, o + 33); /* (ab, bc, ca) */
        }
        free(src);
        src = dst;
        n *= 4;
    }
    memcpy(cur, src, sizeof(double) * 9 * (size_t)total);
    free(src);
    return 0;
}

/* Solid angle of the triangular cone (d0, d1, d2), unit vectors
 * (Van Oosterom & Strackee, 1983). */
double orc_solid_angle(const double *d0, const double *d1, const double *d2)
{
    double num = fabs(v_det(d0, d1, d2));
    double den = 1.0 + v_dot(d0, d1) + v_dot(d1, d2) + v_dot(d2, d0);
    return 2.0 * atan2(num, den);
}

/* ------------------------------------------------------------------------- */
/* Scene                                                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    const float *xyz; int64_t n_vert;
    const int32_t *tri; int64_t n_tri;
    const float *alpha;
    const float *src; const float *power; int32_t n_src;
    double mic_x0, mic_y0, mic_z, mic_dx, mic_dy;
    int32_t mic_nx, mic_ny;
    /* optional [n_src][n_faces] relative intensity of each source per icosphere face;
       NULL = omni.  Reading of Section 2's sharing of a source's power between beams by
       direction, for a directional source: beam b of source s gets
       K_b = W_s w_b / sum_f(w_f Omega_f), so its power K_b Omega_b is W_s's share in
       proportion to w_b Omega_b and the beams' powers add up to W_s. */
    const float *src_weight;
    /* microphone layers: layer k sits at height mic_z + k mic_dz, k < mic_nz (a volumetric
       grid filling a box, as in Section 4's experiment; mic_nz = 1 is a planar grid).
       Microphone (i, j, k) has index (k mic_ny + j) mic_nx + i. */
    double mic_dz;
    int32_t mic_nz;
    /* explicit microphone points (float [mic_n][3]); when set they replace the grid and
       every point is tested against every segment */
    const float *mic_xyz;
    int64_t mic_n;
} orc_scene;

typedef struct {
    int32_t level, depth;
    double t_min;        /* hits at t <= t_min are ignored (self-intersection guard) */
    double delta;        /* edge / tie flag distance, metres */
    double m_air;        /* air attenuation exp(-m_air d); 0 = off */
    double e_min;        /* beams with K*Omega <= e_min are not reflected further; 0 = off */
    int32_t use_bvh;     /* 0: all-triangle brute force, 1: the oracle's own BVH */
    int32_t mic_mode;    /* 0: test every microphone, 1: per-row grid rasterisation */
    int32_t n_threads;
    int64_t beam_begin, beam_end;  /* initial beams traced: global ids [begin, end) */
} orc_params;

enum { C_SEGMENTS = 0, C_NODE_VISITS, C_TRI_TESTS, C_MIC_UPDATES, C_MIC_TESTS, C_HITS, C_FLAGGED_SEG, C_CHILD, C_NCOUNTERS = 16 };

typedef struct {
    int32_t *hit;       /* [n_beams0][depth+1]: -2 not traced, -1 miss, else triangle id; may be NULL */
    uint8_t *flag;      /* same shape: 1 if this segment or an ancestor is flagged; may be NULL */
    double *t_hit;      /* same shape; may be NULL */
    int64_t *count;     /* [depth+1] beams traced per generation */
    int64_t *flagged;   /* [depth+1] flagged beams per generation */
    double *power;      /* [depth+1] sum over traced beams of K * Omega (watts) */
    double *e_strict;   /* [n_mic] energy from unflagged, unambiguous (segment, mic) pairs */
    double *e_flag;     /* [n_mic] energy from flagged segments or ambiguous pairs */
    int64_t counters[C_NCOUNTERS];
} orc_result;

static void tri_verts(const orc_scene *s, int64_t t, double v0[3], double v1[3], double v2[3])
{
    const int32_t *ix = s->tri + 3 * t;
    for (int k = 0; k < 3; ++k) {
        v0[k] = (double)s->xyz[3 * (int64_t)ix[0] + k];
        v1[k] = (double)s->xyz[3 * (int64_t)ix[1] + k];
        v2[k] = (double)s->xyz[3 * (int64_t)ix[2] + k];
    }
}

/* Unnormalised plane normal N = (v1 - v0) x (v2 - v0) and its anchor v0. */
static void tri_plane(const orc_scene *s, int64_t t, double N[3], double P[3])
{
    double v0[3], v1[3], v2[3], e1[3], e2[3];
    tri_verts(s, t, v0, v1, v2);
    v_sub(v1, v0, e1);
    v_sub(v2, v0, e2);
    v_cross(e1, e2, N);
    v_copy(v0, P);
}

/* ------------------------------------------------------------------------- */
/* Ray / triangle (paper Section 2: intersections are handled as in ray        */
/* tracing, for the guiding ray only).  Moller-Trumbore (1997), two-sided.     */
/* Returns 0 when the ray is parallel to the plane (det == 0).  Otherwise      */
/* *t is the plane parameter and *sd the signed in-plane distance of the      */
/* plane point to the triangle boundary: >= 0 inside (distance to the nearest */
/* edge), < 0 outside (minus the Euclidean distance to the triangle).         */
/* ------------------------------------------------------------------------- */

static double seg_dist(const double p[3], const double a[3], const double b[3])
{
    double ab[3], ap[3], q[3], r[3];
    v_sub(b, a, ab);
    v_sub(p, a, ap);
    double l2 = v_dot(ab, ab);
    double u = l2 > 0.0 ? v_dot(ap, ab) / l2 : 0.0;
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
    q[0] = a[0] + u * ab[0]; q[1] = a[1] + u * ab[1]; q[2] = a[2] + u * ab[2];
    v_sub(p, q, r);
    return v_norm(r);
}

static int ray_tri(const double o[3], const double c[3], const double v0[3], const double v1[3],
                   const double v2[3], double *t, double *sd)
{
    double e1[3], e2[3], p[3], T[3], q[3];
    v_sub(v1, v0, e1);
    v_sub(v2, v0, e2);
    v_cross(c, e2, p);
    double det = v_dot(e1, p);
    if (det == 0.0) return 0;
    v_sub(o, v0, T);
    double u = v_dot(T, p) / det;
    v_cross(T, e1, q);
    double v = v_dot(c, q) / det;
    *t = v_dot(e2, q) / det;
    double w = (1.0 - u) - v;
    double N[3], e12[3];
    v_cross(e1, e2, N);
    double twice_area = v_norm(N);
    v_sub(v2, v1, e12);
    double s0 = w * twice_area / v_norm(e12);  /* distance to edge v1-v2 */
    double s1 = u * twice_area / v_norm(e2);   /* distance to edge v0-v2 */
    double s2 = v * twice_area / v_norm(e1);   /* distance to edge v0-v1 */
    double m = s0 < s1 ? s0 : s1;
    if (s2 < m) m = s2;
    if (m >= 0.0) { *sd = m; return 1; }
    double P[3];
    P[0] = o[0] + (*t) * c[0]; P[1] = o[1] + (*t) * c[1]; P[2] = o[2] + (*t) * c[2];
    double d0 = seg_dist(P, v0, v1), d1 = seg_dist(P, v1, v2), d2 = seg_dist(P, v2, v0);
    double d = d0 < d1 ? d0 : d1;
    if (d2 < d) d = d2;
    *sd = -d;
    return 1;
}

/* ------------------------------------------------------------------------- */
/* The oracle's own acceleration hierarchy (paper Sections 2-3 mention a        */
/* hierarchical structure for intersection detection).  Binary BVH, binned    */
/* SAH with 16 bins per axis, leaves of at most 4 triangles, boxes grown by a */
/* margin (delta + 1e-6 m) so that flag candidates are never culled.          */
/* ------------------------------------------------------------------------- */

typedef struct { double lo[3], hi[3]; int32_t left, right, first, count; } onode;
typedef struct { onode *nodes; int64_t n_nodes, cap; int32_t *order; int max_depth; } obvh;

typedef struct { double lo[3], hi[3]; double cen[3]; } tbox;

static void box_empty(double lo[3], double hi[3]) { for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; } }
static void box_grow(double lo[3], double hi[3], const double plo[3], const double phi[3])
{
    for (int k = 0; k < 3; ++k) { if (plo[k] < lo[k]) lo[k] = plo[k]; if (phi[k] > hi[k]) hi[k] = phi[k]; }
}
static double box_area(const double lo[3], const double hi[3])
{
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    if (dx < 0 || dy < 0 || dz < 0) return 0.0;
    return 2.0 * (dx * dy + dy * dz + dz * dx);
}

static int64_t bvh_new_node(obvh *b)
{
    if (b->n_nodes == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->nodes = (onode *)realloc(b->nodes, sizeof(onode) * (size_t)b->cap);
    }
    return b->n_nodes++;
}

static void bvh_build_rec(obvh *b, const tbox *tb, int64_t node, int32_t first, int32_t count, double margin, int depth)
{
    onode *nd = &b->nodes[node];
    double lo[3], hi[3], clo[3], chi[3];
    box_empty(lo, hi);
    box_empty(clo, chi);
    for (int32_t i = first; i < first + count; ++i) {
        const tbox *t = &tb[b->order[i]];
        box_grow(lo, hi, t->lo, t->hi);
        box_grow(clo, chi, t->cen, t->cen);
    }
    for (int k = 0; k < 3; ++k) { nd->lo[k] = lo[k] - margin; nd->hi[k] = hi[k] + margin; }
    if (depth > b->max_depth) b->max_depth = depth;
    if (count <= 4) { nd->left = nd->right = -1; nd->first = first; nd->count = count; return; }

    enum { NB = 16 };
    double best_cost = INFINITY;
    int best_axis = -1, best_split = -1;
    for (int ax = 0; ax < 3; ++ax) {
        double ext = chi[ax] - clo[ax];
        if (!(ext > 0.0)) continue;
        int64_t cnt[NB] = {0};
        double blo[NB][3], bhi[NB][3];
        for (int i = 0; i < NB; ++i) box_empty(blo[i], bhi[i]);
        for (int32_t i = first; i < first + count; ++i) {
            const tbox *t = &tb[b->order[i]];
            int bi = (int)((t->cen[ax] - clo[ax]) / ext * NB);
            if (bi >= NB) bi = NB - 1;
            if (bi < 0) bi = 0;
            cnt[bi]++;
            box_grow(blo[bi], bhi[bi], t->lo, t->hi);
        }
        for (int s = 1; s < NB; ++s) {
            double llo[3], lhi[3], rlo[3], rhi[3];
            int64_t nl = 0, nr = 0;
            box_empty(llo, lhi); box_empty(rlo, rhi);
            for (int i = 0; i < s; ++i) { nl += cnt[i]; if (cnt[i]) box_grow(llo, lhi, blo[i], bhi[i]); }
            for (int i = s; i < NB; ++i) { nr += cnt[i]; if (cnt[i]) box_grow(rlo, rhi, blo[i], bhi[i]); }
            if (nl == 0 || nr == 0) continue;
            double cost = box_area(llo, lhi) * (double)nl + box_area(rlo, rhi) * (double)nr;
            if (cost < best_cost) { best_cost = cost; best_axis = ax; best_split = s; }
        }
    }
    int32_t mid;
    if (best_axis < 0) {
        mid = first + count / 2;  /* all centroids coincide: split the index range */
    } else {
        double ext = chi[best_axis] - clo[best_axis];
        int32_t i = first, j = first + count - 1;
        while (i <= j) {
            const tbox *t = &tb[b->order[i]];
            int bi = (int)((t->cen[best_axis] - clo[best_axis]) / ext * NB);
            if (bi >= NB) bi = NB - 1;
            if (bi < 0) bi = 0;
            if (bi < best_split) { i++; }
            else { int32_t tmp = b->order[i]; b->order[i] = b->order[j]; b->order[j] = tmp; j--; }
        }
        mid = i;
    }
    int64_t l = bvh_new_node(b);
    int64_t r = bvh_new_node(b);
    nd = &b->nodes[node];  /* realloc may have moved the array */
    nd->left = (int32_t)l; nd->right = (int32_t)r; nd->first = 0; nd->count = 0;
    bvh_build_rec(b, tb, l, first, mid - first, margin, depth + 1);
    bvh_build_rec(b, tb, r, mid, first + count - mid, margin, depth + 1);
}

static obvh *bvh_build(const orc_scene *s, double margin)
{
    obvh *b = (obvh *)calloc(1, sizeof(obvh));
    if (!b) return NULL;
    b->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(s->n_tri > 0 ? s->n_tri : 1));
    tbox *tb = (tbox *)malloc(sizeof(tbox) * (size_t)(s->n_tri > 0 ? s->n_tri : 1));
    for (int64_t t = 0; t < s->n_tri; ++t) {
        double v0[3], v1[3], v2[3];
        tri_verts(s, t, v0, v1, v2);
        box_empty(tb[t].lo, tb[t].hi);
        box_grow(tb[t].lo, tb[t].hi, v0, v0);
        box_grow(tb[t].lo, tb[t].hi, v1, v1);
        box_grow(tb[t].lo, tb[t].hi, v2, v2);
        for (int k = 0; k < 3; ++k) tb[t].cen[k] = 0.5 * (tb[t].lo[k] + tb[t].hi[k]);
        b->order[t] = (int32_t)t;
    }
    if (s->n_tri > 0) {
        int64_t root = bvh_new_node(b);
        bvh_build_rec(b, tb, root, 0, (int32_t)s->n_tri, margin, 0);
    }
    free(tb);
    return b;
}

static void bvh_free(obvh *b)
{
    if (!b) return;
    free(b->nodes);
    free(b->order);
    free(b);
}

/* Parameter interval of the ray inside a box, intersected with [t0, t1]. */
static int ray_box(const double o[3], const double c[3], const double lo[3], const double hi[3],
                   double t0, double t1, double *tnear)
{
    for (int k = 0; k < 3; ++k) {
        if (c[k] == 0.0) {
            if (o[k] < lo[k] || o[k] > hi[k]) return 0;
            continue;
        }
        double ta = (lo[k] - o[k]) / c[k];
        double tb = (hi[k] - o[k]) / c[k];
        if (ta > tb) { double x = ta; ta = tb; tb = x; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    *tnear = t0;
    return 1;
}

/* ------------------------------------------------------------------------- */
/* Closest hit of one guiding ray with flags.                                  */
/* Reading: closest hit over t in (t_min, inf), two-sided, the triangle the    */
/* ray starts on excluded, equal t broken by the lowest triangle index.        */
/* The segment is flagged when its result is sensitive at the delta scale:     */
/*   - the hit point is within delta of an edge of the hit triangle, or        */
/*   - t* - t_min < delta, or                                                  */
/*   - another triangle (not the hit, not the start) has its plane point       */
/*     within delta of itself (inside or outside) at some t in                 */
/*     (t_min - delta, t* + delta)  (near misses, second-nearest hits, ties).  */
/* ------------------------------------------------------------------------- */

typedef struct { int32_t hit; double t; int flag; int64_t node_visits, tri_tests; } orc_hitres;

static void closest_hit(const orc_scene *s, const obvh *b, const double o[3], const double c[3],
                        int32_t start, double t_min, double delta, orc_hitres *res)
{
    double best_t = INFINITY;
    int32_t best = -1;
    double best_sd = 0.0;
    res->node_visits = 0;
    res->tri_tests = 0;

    /* pass 1: closest valid hit */
    if (!b) {
        for (int64_t t = 0; t < s->n_tri; ++t) {
            if (t == start) continue;
            double v0[3], v1[3], v2[3], tt, sd;
            tri_verts(s, t, v0, v1, v2);
            res->tri_tests++;
            if (!ray_tri(o, c, v0, v1, v2, &tt, &sd)) continue;
            if (tt > t_min && sd >= 0.0 && (tt < best_t || (tt == best_t && t < best))) {
                best_t = tt; best = (int32_t)t; best_sd = sd;
            }
        }
    } else if (b->n_nodes > 0) {
        /* stack of (node, entry t); a node is re-checked against the current best on pop */
        int32_t stack[128];
        double stack_t[128];
        int sp = 0;
        double tr0;
        if (ray_box(o, c, b->nodes[0].lo, b->nodes[0].hi, t_min, best_t, &tr0)) { stack[sp] = 0; stack_t[sp] = tr0; sp++; }
        while (sp > 0) {
            sp--;
            const onode *nd = &b->nodes[stack[sp]];
            if (stack_t[sp] > best_t) continue;
            if (nd->count > 0) {
                for (int32_t i = nd->first; i < nd->first + nd->count; ++i) {
                    int32_t t = b->order[i];
                    if (t == start) continue;
                    double v0[3], v1[3], v2[3], tt, sd;
                    tri_verts(s, t, v0, v1, v2);
                    res->tri_tests++;
                    if (!ray_tri(o, c, v0, v1, v2, &tt, &sd)) continue;
                    if (tt > t_min && sd >= 0.0 && (tt < best_t || (tt == best_t && t < best))) {
                        best_t = tt; best = t; best_sd = sd;
                    }
                }
            } else {
                /* one node visit = both child boxes tested; nearer child is visited first */
                res->node_visits++;
                const onode *L = &b->nodes[nd->left], *R = &b->nodes[nd->right];
                double tl, tr;
                int hl = ray_box(o, c, L->lo, L->hi, t_min, best_t, &tl);
                int hr = ray_box(o, c, R->lo, R->hi, t_min, best_t, &tr);
                if (hl && hr) {
                    if (tl <= tr) { stack[sp] = nd->right; stack_t[sp] = tr; sp++; stack[sp] = nd->left; stack_t[sp] = tl; sp++; }
                    else { stack[sp] = nd->left; stack_t[sp] = tl; sp++; stack[sp] = nd->right; stack_t[sp] = tr; sp++; }
                } else if (hl) { stack[sp] = nd->left; stack_t[sp] = tl; sp++; }
                else if (hr) { stack[sp] = nd->right; stack_t[sp] = tr; sp++; }
            }
        }
    }

    /* pass 2: flag window */
    int flag = 0;
    if (best >= 0 && (best_sd < delta || best_t - t_min < delta)) flag = 1;
    double w_lo = t_min - delta, w_hi = best_t + delta;
    if (!flag) {
        if (!b) {
            for (int64_t t = 0; t < s->n_tri && !flag; ++t) {
                if (t == start || t == best) continue;
                double v0[3], v1[3], v2[3], tt, sd;
                tri_verts(s, t, v0, v1, v2);
                if (!ray_tri(o, c, v0, v1, v2, &tt, &sd)) continue;
                if (tt > w_lo && tt < w_hi && sd > -delta) flag = 1;
            }
        } else if (b->n_nodes > 0) {
            int32_t stack[128];
            int sp = 0;
            stack[sp++] = 0;
            while (sp > 0 && !flag) {
                const onode *nd = &b->nodes[stack[--sp]];
                double tn;
                if (!ray_box(o, c, nd->lo, nd->hi, w_lo, w_hi, &tn)) continue;
                if (nd->count > 0) {
                    for (int32_t i = nd->first; i < nd->first + nd->count; ++i) {
                        int32_t t = b->order[i];
                        if (t == start || t == best) continue;
                        double v0[3], v1[3], v2[3], tt, sd;
                        tri_verts(s, t, v0, v1, v2);
                        if (!ray_tri(o, c, v0, v1, v2, &tt, &sd)) continue;
                        if (tt > w_lo && tt < w_hi && sd > -delta) { flag = 1; break; }
                    }
                } else {
                    const onode *L = &b->nodes[nd->left], *R = &b->nodes[nd->right];
                    if (ray_box(o, c, L->lo, L->hi, w_lo, w_hi, &tn)) stack[sp++] = nd->left;
                    if (ray_box(o, c, R->lo, R->hi, w_lo, w_hi, &tn)) stack[sp++] = nd->right;
                }
            }
        }
    }
    res->hit = best;
    res->t = best_t;
    res->flag = flag;
}

/* ------------------------------------------------------------------------- */
/* Microphone in beam (paper Section 2: microphones measure the sum of the    */
/* contributions that reach them).  Reading: a microphone m belongs to a       */
/* segment iff                                                                  */
/*   for i = 0,1,2, with n_i = d_i x d_(i+1) and s_i = n_i . (m - A):           */
/*     s_i > 0, or s_i == 0 and n_i is lexicographically positive              */
/*   and (generation 0, or strictly on the outgoing side of the plane the beam */
/*     was reflected from)                                                     */
/*   and (the guiding ray escaped, or m is on the incoming side of the hit      */
/*     triangle's plane, the plane itself included).                          */
/* Adjacent beams hold exactly opposite side normals, so a point of a shared  */
/* face has exactly one owner.  A pair is ambiguous when every active test   */
/* passes within -delta and one is within delta of its plane.                */
/* ------------------------------------------------------------------------- */

typedef struct {
    double A[3], d[3][3], o[3], c[3];
    double K, omega;
    int32_t start, depth, near_sign;  /* near plane: triangle `start`, outgoing side sign */
    int flag;
} obeam;

typedef struct {
    double n[3][3];      /* side normals */
    double nlen[3];
    int has_near, has_far;
    double Nn[3], Pn[3], Nn_len; int near_sign;
    double Nf[3], Pf[3], Nf_len; int far_sign;
} ofrustum;

static int lex_positive(const double n[3])
{
    if (n[0] != 0.0) return n[0] > 0.0;
    if (n[1] != 0.0) return n[1] > 0.0;
    return n[2] > 0.0;
}

static void make_frustum(const orc_scene *s, const obeam *bm, int32_t hit, const double c[3], ofrustum *f)
{
    for (int i = 0; i < 3; ++i) {
        v_cross(bm->d[i], bm->d[(i + 1) % 3], f->n[i]);
        f->nlen[i] = v_norm(f->n[i]);
    }
    f->has_near = bm->depth > 0;
    if (f->has_near) {
        tri_plane(s, bm->start, f->Nn, f->Pn);
        f->Nn_len = v_norm(f->Nn);
        f->near_sign = bm->near_sign;
    }
    f->has_far = hit >= 0;
    if (f->has_far) {
        tri_plane(s, hit, f->Nf, f->Pf);
        f->Nf_len = v_norm(f->Nf);
        f->far_sign = v_dot(c, f->Nf) > 0.0 ? 1 : -1;
    }
}

/* returns 1 if inside; *amb set when the pair is ambiguous at distance delta */
static int mic_inside(const ofrustum *f, const double A[3], const double m[3], double delta, int *amb)
{
    double r[3];
    int inside = 1, near_any = 0, far_out = 0;
    v_sub(m, A, r);
    for (int i = 0; i < 3; ++i) {
        double si = v_dot(f->n[i], r);
        int in = si > 0.0 || (si == 0.0 && lex_positive(f->n[i]));
        if (!in) inside = 0;
        double dist = si / f->nlen[i];
        if (dist <= -delta) far_out = 1;
        if (fabs(dist) < delta) near_any = 1;
    }
    if (f->has_near) {
        double q[3];
        v_sub(m, f->Pn, q);
        double sn = (double)f->near_sign * v_dot(f->Nn, q);
        if (!(sn > 0.0)) inside = 0;
        double dist = sn / f->Nn_len;
        if (dist <= -delta) far_out = 1;
        if (fabs(dist) < delta) near_any = 1;
    }
    if (f->has_far) {
        double q[3];
        v_sub(m, f->Pf, q);
        double sf = -(double)f->far_sign * v_dot(f->Nf, q);  /* >= 0 on the incoming side */
        if (!(sf >= 0.0)) inside = 0;
        double dist = sf / f->Nf_len;
        if (dist <= -delta) far_out = 1;
        if (fabs(dist) < delta) near_any = 1;
    }
    *amb = (!far_out && near_any);
    return inside;
}

/* 2D half-plane a x + b y + k >= 0 on the microphone plane, from a keep-side
 * normal g through point P, relaxed by eps metres. */
typedef struct { double a, b, k; } hplane;

static hplane make_hplane(const double g[3], const double P[3], double z, double eps)
{
    hplane h;
    h.a = g[0];
    h.b = g[1];
    h.k = g[2] * (z - P[2]) - g[0] * P[0] - g[1] * P[1] + eps * v_norm(g);
    return h;
}

/* Sutherland-Hodgman clip of a convex polygon by one half-plane. */
static int clip_poly(const double *px, const double *py, int n, hplane h, double *qx, double *qy)
{
    int m = 0;
    for (int i = 0; i < n; ++i) {
        int j = (i + 1) % n;
        double fi = h.a * px[i] + h.b * py[i] + h.k;
        double fj = h.a * px[j] + h.b * py[j] + h.k;
        if (fi >= 0.0) { qx[m] = px[i]; qy[m] = py[i]; m++; }
        if ((fi >= 0.0) != (fj >= 0.0)) {
            double u = fi / (fi - fj);
            qx[m] = px[i] + u * (px[j] - px[i]);
            qy[m] = py[i] + u * (py[j] - py[i]);
            m++;
        }
    }
    return m;
}

typedef struct {
    double *e_strict, *e_flag;
    int64_t *counters;
} oaccum;

static void add_contribution(const orc_scene *s, const orc_params *p, const obeam *bm, int64_t mic,
                             const double m[3], int ambiguous, oaccum *acc)
{
    double r[3];
    v_sub(m, bm->A, r);
    double d2 = v_dot(r, r);
    double d = sqrt(d2);
    double e = bm->K * exp(-p->m_air * d) / d2;  /* reading: intensity K / d^2 from the (image) apex */
    (void)s;
    if (bm->flag || ambiguous) acc->e_flag[mic] += e;
    else acc->e_strict[mic] += e;
    acc->counters[C_MIC_UPDATES]++;
}

/* Microphones of layer k inside the segment's frustum: the grid rectangle at that height
 * is clipped by the (relaxed) keep half-planes, then the rows inside the clipped polygon
 * are scanned, one row and one column of slack on each side; membership is decided by
 * the exact plane tests. */
static void accumulate_layer(const orc_scene *s, const orc_params *p, const obeam *bm, const ofrustum *f,
                             int64_t k, oaccum *acc)
{
    const double z = s->mic_z + (double)k * s->mic_dz;
    const int64_t layer0 = k * (int64_t)s->mic_ny;
    const double eps = 1e-6;
    hplane hp[5];
    int nh = 0;
    for (int i = 0; i < 3; ++i) hp[nh++] = make_hplane(f->n[i], bm->A, z, eps);
    if (f->has_near) {
        double g[3] = { f->near_sign * f->Nn[0], f->near_sign * f->Nn[1], f->near_sign * f->Nn[2] };
        hp[nh++] = make_hplane(g, f->Pn, z, eps);
    }
    if (f->has_far) {
        double g[3] = { -f->far_sign * f->Nf[0], -f->far_sign * f->Nf[1], -f->far_sign * f->Nf[2] };
        hp[nh++] = make_hplane(g, f->Pf, z, eps);
    }
    double xlo = s->mic_x0 - 0.5 * s->mic_dx, xhi = s->mic_x0 + ((double)s->mic_nx - 0.5) * s->mic_dx;
    double ylo = s->mic_y0 - 0.5 * s->mic_dy, yhi = s->mic_y0 + ((double)s->mic_ny - 0.5) * s->mic_dy;
    double px[16], py[16], qx[16], qy[16];
    int n = 4;
    px[0] = xlo; py[0] = ylo; px[1] = xhi; py[1] = ylo; px[2] = xhi; py[2] = yhi; px[3] = xlo; py[3] = yhi;
    for (int h = 0; h < nh && n > 0; ++h) {
        n = clip_poly(px, py, n, hp[h], qx, qy);
        memcpy(px, qx, sizeof(double) * (size_t)n);
        memcpy(py, qy, sizeof(double) * (size_t)n);
    }
    if (n == 0) return;
    double pymin = INFINITY, pymax = -INFINITY;
    for (int i = 0; i < n; ++i) { if (py[i] < pymin) pymin = py[i]; if (py[i] > pymax) pymax = py[i]; }
    int64_t j0 = (int64_t)ceil((pymin - s->mic_y0) / s->mic_dy) - 1;
    int64_t j1 = (int64_t)floor((pymax - s->mic_y0) / s->mic_dy) + 1;
    if (j0 < 0) j0 = 0;
    if (j1 > s->mic_ny - 1) j1 = s->mic_ny - 1;
    for (int64_t j = j0; j <= j1; ++j) {
        double y = s->mic_y0 + (double)j * s->mic_dy;
        double lo = -INFINITY, hi = INFINITY;
        int empty = 0;
        for (int h = 0; h < nh; ++h) {
            double rest = hp[h].b * y + hp[h].k;  /* a x + rest >= 0 */
            if (hp[h].a > 0.0) { double x = -rest / hp[h].a; if (x > lo) lo = x; }
            else if (hp[h].a < 0.0) { double x = -rest / hp[h].a; if (x < hi) hi = x; }
            else if (rest < 0.0) { empty = 1; }
        }
        if (empty || lo > hi) continue;
        double flo = (lo - s->mic_x0) / s->mic_dx, fhi = (hi - s->mic_x0) / s->mic_dx;
        if (flo > (double)s->mic_nx || fhi < -1.0) continue;
        int64_t i0 = flo < -1.0 ? 0 : (int64_t)ceil(flo) - 1;
        int64_t i1 = fhi > (double)s->mic_nx ? s->mic_nx - 1 : (int64_t)floor(fhi) + 1;
        if (i0 < 0) i0 = 0;
        if (i1 > s->mic_nx - 1) i1 = s->mic_nx - 1;
        for (int64_t i = i0; i <= i1; ++i) {
            double m[3] = { s->mic_x0 + (double)i * s->mic_dx, y, z };
            int amb;
            acc->counters[C_MIC_TESTS]++;
            if (mic_inside(f, bm->A, m, p->delta, &amb)) add_contribution(s, p, bm, (layer0 + j) * s->mic_nx + i, m, amb, acc);
        }
    }
}

static void accumulate_mics(const orc_scene *s, const orc_params *p, const obeam *bm, int32_t hit, oaccum *acc)
{
    ofrustum f;
    make_frustum(s, bm, hit, bm->c, &f);
    const int64_t nz = s->mic_nz > 0 ? s->mic_nz : 1;
    if (s->mic_xyz) {
        for (int64_t mi = 0; mi < s->mic_n; ++mi) {
            double m[3] = { (double)s->mic_xyz[3 * mi], (double)s->mic_xyz[3 * mi + 1], (double)s->mic_xyz[3 * mi + 2] };
            int amb;
            acc->counters[C_MIC_TESTS]++;
            if (mic_inside(&f, bm->A, m, p->delta, &amb)) add_contribution(s, p, bm, mi, m, amb, acc);
        }
        return;
    }
    if (p->mic_mode == 0) {
        /* every microphone of every layer */
        const int64_t nmic = (int64_t)s->mic_nx * s->mic_ny * nz;
        for (int64_t mi = 0; mi < nmic; ++mi) {
            int64_t i = mi % s->mic_nx, j = (mi / s->mic_nx) % s->mic_ny, k = mi / ((int64_t)s->mic_nx * s->mic_ny);
            double m[3] = { s->mic_x0 + (double)i * s->mic_dx, s->mic_y0 + (double)j * s->mic_dy,
                            s->mic_z + (double)k * s->mic_dz };
            int amb;
            acc->counters[C_MIC_TESTS]++;
            if (mic_inside(&f, bm->A, m, p->delta, &amb)) add_contribution(s, p, bm, mi, m, amb, acc);
        }
        return;
    }
    /* grid rasterisation, layer by layer */
    for (int64_t k = 0; k < nz; ++k) accumulate_layer(s, p, bm, &f, k, acc);
}

/* ------------------------------------------------------------------------- */
/* Specular reflection without splitting (paper Section 2: a reflected beam    */
/* loses energy; the hybrid method never splits a beam).  Reading: mirror the  */
/* apex, edge directions and guiding direction in the hit plane, restore a    */
/* positive orientation by swapping d1 and d2, restart the ray at the hit      */
/* point, scale the intensity constant by (1 - alpha).                        */
/* ------------------------------------------------------------------------- */

static void mirror_dir(const double v[3], const double n[3], double r[3])
{
    double k = 2.0 * v_dot(v, n);
    r[0] = v[0] - k * n[0]; r[1] = v[1] - k * n[1]; r[2] = v[2] - k * n[2];
}

static void reflect(const orc_scene *s, const obeam *bm, int32_t hit, double t, obeam *ch)
{
    double N[3], P[3], n[3], q[3];
    tri_plane(s, hit, N, P);
    v_normalize(N, n);
    v_sub(bm->A, P, q);
    double k = 2.0 * v_dot(q, n);
    ch->A[0] = bm->A[0] - k * n[0]; ch->A[1] = bm->A[1] - k * n[1]; ch->A[2] = bm->A[2] - k * n[2];
    mirror_dir(bm->d[0], n, ch->d[0]);
    mirror_dir(bm->d[2], n, ch->d[1]);
    mirror_dir(bm->d[1], n, ch->d[2]);
    mirror_dir(bm->c, n, ch->c);
    ch->o[0] = bm->o[0] + t * bm->c[0];
    ch->o[1] = bm->o[1] + t * bm->c[1];
    ch->o[2] = bm->o[2] + t * bm->c[2];
    ch->K = bm->K * (1.0 - (double)s->alpha[hit]);
    ch->omega = bm->omega;
    ch->start = hit;
    ch->depth = bm->depth + 1;
    ch->near_sign = v_dot(bm->c, N) > 0.0 ? -1 : 1;
    ch->flag = bm->flag;
}

/* ------------------------------------------------------------------------- */
/* Driver: follow every initial beam through its reflections.                 */
/* ------------------------------------------------------------------------- */

typedef struct {
    const orc_scene *s;
    const orc_params *p;
    const obvh *bvh;
    const double *dirs;
    int64_t nf;
    const double *wnorm;  /* [n_src] sum over faces of weight x solid angle (directional sources) */
    int64_t b0, b1;
    orc_result *res;
    double *e_strict, *e_flag;
    int64_t counters[C_NCOUNTERS];
    int64_t *count, *flagged;
    double *power;
} oworker;

static void *run_worker(void *arg)
{
    oworker *w = (oworker *)arg;
    const orc_scene *s = w->s;
    const orc_params *p = w->p;
    int D = p->depth;
    oaccum acc = { w->e_strict, w->e_flag, w->counters };
    for (int64_t gb = w->b0; gb < w->b1; ++gb) {
        int64_t src = gb / w->nf, face = gb % w->nf;
        const double *fd = w->dirs + 9 * face;
        obeam bm;
        for (int k = 0; k < 3; ++k) {
            bm.A[k] = (double)s->src[3 * src + k];
            bm.o[k] = bm.A[k];
            bm.d[0][k] = fd[k]; bm.d[1][k] = fd[3 + k]; bm.d[2][k] = fd[6 + k];
        }
        double sum[3], sum01[3];
        v_add(bm.d[0], bm.d[1], sum01);
        v_add(sum01, bm.d[2], sum);
        v_normalize(sum, bm.c);
        bm.omega = orc_solid_angle(bm.d[0], bm.d[1], bm.d[2]);
        if (s->src_weight) {
            const double wn = w->wnorm[src];
            bm.K = wn > 0.0 ? (double)s->power[src] * (double)s->src_weight[src * w->nf + face] / wn : 0.0;
        } else {
            bm.K = (double)s->power[src] / (4.0 * M_PI);   /* reading: omni source, power W * Omega / (4 pi) */
        }
        bm.start = -1; bm.depth = 0; bm.near_sign = 0; bm.flag = 0;
        for (int g = 0; g <= D; ++g) {
            orc_hitres hr;
            closest_hit(s, w->bvh, bm.o, bm.c, bm.start, p->t_min, p->delta, &hr);
            w->counters[C_SEGMENTS]++;
            w->counters[C_NODE_VISITS] += hr.node_visits;
            w->counters[C_TRI_TESTS] += hr.tri_tests;
            if (hr.flag) { bm.flag = 1; w->counters[C_FLAGGED_SEG]++; }
            w->count[g]++;
            if (bm.flag) w->flagged[g]++;
            w->power[g] += bm.K * bm.omega;
            if (w->res->hit) w->res->hit[gb * (D + 1) + g] = hr.hit;
            if (w->res->flag) w->res->flag[gb * (D + 1) + g] = (uint8_t)bm.flag;
            if (w->res->t_hit) w->res->t_hit[gb * (D + 1) + g] = hr.t;
            accumulate_mics(s, p, &bm, hr.hit, &acc);
            if (hr.hit < 0) break;
            w->counters[C_HITS]++;
            if (g == D) break;
            if (p->e_min > 0.0 && bm.K * bm.omega * (1.0 - (double)s->alpha[hr.hit]) <= p->e_min) break;
            obeam ch;
            reflect(s, &bm, hr.hit, hr.t, &ch);
            w->counters[C_CHILD]++;
            bm = ch;
        }
    }
    return NULL;
}

int orc_trace(const orc_scene *s, const orc_params *p, orc_result *res)
{
    int64_t nf = orc_ico_nfaces(p->level);
    if (nf < 0 || p->depth < 0 || s->n_src < 0) return -1;
    int64_t nb = nf * s->n_src;
    int64_t b0 = p->beam_begin < 0 ? 0 : p->beam_begin;
    int64_t b1 = p->beam_end > nb || p->beam_end < 0 ? nb : p->beam_end;
    int D = p->depth;
    int64_t nmic = s->mic_xyz ? s->mic_n : (int64_t)s->mic_nx * s->mic_ny * (s->mic_nz > 0 ? s->mic_nz : 1);
    double *dirs = (double *)malloc(sizeof(double) * 9 * (size_t)nf);
    if (!dirs) return -2;
    if (orc_icosphere(p->level, dirs) != 0) { free(dirs); return -3; }
    double *wnorm = NULL;
    if (s->src_weight) {
        wnorm = (double *)calloc((size_t)(s->n_src > 0 ? s->n_src : 1), sizeof(double));
        if (!wnorm) { free(dirs); return -2; }
        for (int64_t f = 0; f < nf; ++f) {
            const double *fd = dirs + 9 * f;
            const double om = orc_solid_angle(fd, fd + 3, fd + 6);
            for (int32_t k = 0; k < s->n_src; ++k) wnorm[k] += (double)s->src_weight[k * nf + f] * om;
        }
    }
    obvh *bvh = p->use_bvh ? bvh_build(s, p->delta + 1e-6) : NULL;
    int T = p->n_threads > 0 ? p->n_threads : 1;
    if (T > b1 - b0 && b1 > b0) T = (int)(b1 - b0);
    if (T < 1) T = 1;
    oworker *w = (oworker *)calloc((size_t)T, sizeof(oworker));
    pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
    for (int k = 0; k < T; ++k) {
        w[k].s = s; w[k].p = p; w[k].bvh = bvh; w[k].dirs = dirs; w[k].nf = nf; w[k].res = res; w[k].wnorm = wnorm;
        w[k].b0 = b0 + (b1 - b0) * k / T;
        w[k].b1 = b0 + (b1 - b0) * (k + 1) / T;
        w[k].e_strict = (double *)calloc((size_t)(nmic > 0 ? nmic : 1), sizeof(double));
        w[k].e_flag = (double *)calloc((size_t)(nmic > 0 ? nmic : 1), sizeof(double));
        w[k].count = (int64_t *)calloc((size_t)D + 1, sizeof(int64_t));
        w[k].flagged = (int64_t *)calloc((size_t)D + 1, sizeof(int64_t));
        w[k].power = (double *)calloc((size_t)D + 1, sizeof(double));
    }
    if (T == 1) run_worker(&w[0]);
    else {
        for (int k = 0; k < T; ++k) pthread_create(&th[k], NULL, run_worker, &w[k]);
        for (int k = 0; k < T; ++k) pthread_join(th[k], NULL);
    }
    /* reduce in thread order */
    for (int k = 0; k < T; ++k) {
        for (int64_t m = 0; m < nmic; ++m) {
            if (res->e_strict) res->e_strict[m] += w[k].e_strict[m];
            if (res->e_flag) res->e_flag[m] += w[k].e_flag[m];
        }
        for (int g = 0; g <= D; ++g) {
            if (res->count) res->count[g] += w[k].count[g];
            if (res->flagged) res->flagged[g] += w[k].flagged[g];
            if (res->power) res->power[g] += w[k].power[g];
        }
        for (int c = 0; c < C_NCOUNTERS; ++c) res->counters[c] += w[k].counters[c];
        free(w[k].e_strict); free(w[k].e_flag); free(w[k].count); free(w[k].flagged); free(w[k].power);
    }
    free(w);
    free(th);
    bvh_free(bvh);
    free(wnorm);
    free(dirs);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Single-ray entry point for brute-force / BVH cross-checks.                  */
/* ------------------------------------------------------------------------- */

int orc_closest_hits(const orc_scene *s, int use_bvh, const double *orig, const double *dir,
                     const int32_t *start, int64_t n, double t_min, double delta,
                     int32_t *hit, double *t_hit, uint8_t *flag, int64_t *node_visits, int64_t *tri_tests)
{
    obvh *bvh = use_bvh ? bvh_build(s, delta + 1e-6) : NULL;
    for (int64_t r = 0; r < n; ++r) {
        orc_hitres hr;
        closest_hit(s, bvh, orig + 3 * r, dir + 3 * r, start ? start[r] : -1, t_min, delta, &hr);
        hit[r] = hr.hit;
        if (t_hit) t_hit[r] = hr.t;
        if (flag) flag[r] = (uint8_t)hr.flag;
        if (node_visits) node_visits[r] = hr.node_visits;
        if (tri_tests) tri_tests[r] = hr.tri_tests;
    }
    bvh_free(bvh);
    return 0;
}

int orc_bvh_depth(const orc_scene *s, double margin)
{
    obvh *b = bvh_build(s, margin);
    int d = b ? b->max_depth : -1;
    bvh_free(b);
    return d;
}
