// Guiding-ray trace: closest hit through the per-tile hierarchies over the tiles a ray
// crosses, with edge/tie flags (k_trace walks them in each lane; k_tbin, k_tscan,
// k_tscatter and k_ttrace hand rays between per-tile queues instead); the generation's
// children, flags and power per wave and children per block (k_tcount); the specular
// reflection and compaction of the children into the next generation's queue, each block
// finding its queue offset from the counts of the blocks before it, and the generation's
// totals (k_reflect).
//
// Precision: boxes are tested in FP32 against boxes grown by a margin that covers the
// rounding of the ray.  A slab parameter is one FMA, l (1/c) - fl(o (1/c)); in distance
// along the ray it lies within about 8 x 2^-24 of the largest coordinate magnitude of its
// exact value, inside the margin's 12 x 2^-24 of that magnitude.  Every triangle first
// goes through a conservative FP32 Moller-Trumbore filter, and only triangles that may be
// a hit or a flag candidate are decided by the exact FP64 test (FP32 vertices widened
// exactly, FP64 ray).  The FP64 ray is read from the queue where it is needed rather than
// held in registers, which keeps the traversal loop small enough for more waves per SIMD.
#include "bt_device.h"

namespace bt {

__device__ __forceinline__ float f32_down(double x)
{
    float f = (float)x;
    if ((double)f > x) f = nextafterf(f, -INFINITY);
    return f;
}
__device__ __forceinline__ float f32_up(double x)
{
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

// Where the ray's FP64 origin and direction live (the input queue), so that the rare
// exact tests reload them instead of keeping 12 registers busy during traversal.
struct RaySrc {
    const double *o;   // queue + D_O * cap
    const double *c;   // queue + D_C * cap
    long long cap;
    int i;             // queue index (< 2^31): one register stays live, not a 64-bit pair
};

__device__ __forceinline__ void load_ray64(RaySrc src, V3 &o, V3 &c)
{
    // launder the index so the loads are not hoisted out of the traversal loop
    int i = src.i;
    asm volatile("" : "+v"(i));
    const double *ox = src.o, *oy = src.o + src.cap, *oz = src.o + 2 * src.cap;
    const double *cx = src.c, *cy = src.c + src.cap, *cz = src.c + 2 * src.cap;
    o = {ox[i], oy[i], oz[i]};
    c = {cx[i], cy[i], cz[i]};
}

struct RayState {
    float ox, oy, oz;     // FP32 rounded origin
    float cx, cy, cz;     // FP32 rounded direction
    float ix, iy, iz;     // FP32 reciprocal direction (|c| clamped away from 0)
    float oix, oiy, oiz;  // origin times reciprocal: a slab parameter is fma(l, i, -o i)
    float o_l1;           // |ox| + |oy| + |oz|, bounds the origin's rounding
    int start;
    double best_t;
    int best_id;
    int best_near;        // hit point within delta of an edge, or t* - t_min < delta
    double c1_t, c2_t;    // two smallest flag-candidate parameters
    int c1_id;
    unsigned node_visits, tri_tests;
};

// Distance from P to segment [a, b].
__device__ double seg_dist(V3 p, V3 a, V3 b)
{
    const V3 ab = b - a, ap = p - a;
    const double l2 = dot(ab, ab);
    double u = l2 > 0.0 ? dot(ap, ab) / l2 : 0.0;
    u = fmin(fmax(u, 0.0), 1.0);
    const V3 r = p - (a + u * ab);
    return sqrt(dot(r, r));
}

// Signed in-plane distance of the plane point to the triangle boundary (>= 0 inside:
// distance to the nearest edge; < 0 outside: minus the distance to the triangle).
__device__ double exact_signed_dist(V3 P, double u, double v, double w, V3 v0, V3 v1, V3 v2)
{
    const V3 e1 = v1 - v0, e2 = v2 - v0, e12 = v2 - v1;
    const V3 N = cross(e1, e2);
    const double a2 = sqrt(dot(N, N));
    const double s0 = w * a2 / sqrt(dot(e12, e12));
    const double s1 = u * a2 / sqrt(dot(e2, e2));
    const double s2 = v * a2 / sqrt(dot(e1, e1));
    const double m = fmin(s0, fmin(s1, s2));
    if (m >= 0.0) return m;
    return -fmin(seg_dist(P, v0, v1), fmin(seg_dist(P, v1, v2), seg_dist(P, v2, v0)));
}

// Conservative FP32 filter.  Each FP32 quantity (det, the barycentric numerators, the
// parameter numerator) deviates from its exact value by far less than
// B = 2^-18 x (product of the L1 magnitudes of its operands), including the rounding of
// the ray origin and direction.  The triangle is skipped only when, under those bounds,
// its plane point is surely more than delta outside an edge or surely outside the
// parameter window (lo, hi).
__device__ __forceinline__ bool maybe_candidate(const float4 &a, const float4 &b, const float4 &cc,
                                                const RayState &r, float lo, float hi, float dh_num)
{
    const float e1x = a.w - a.x, e1y = b.x - a.y, e1z = b.y - a.z;
    const float e2x = b.z - a.x, e2y = b.w - a.y, e2z = cc.x - a.z;
    const float tx = r.ox - a.x, ty = r.oy - a.y, tz = r.oz - a.z;
    const float px = r.cy * e2z - r.cz * e2y, py = r.cz * e2x - r.cx * e2z, pz = r.cx * e2y - r.cy * e2x;
    const float qx = ty * e1z - tz * e1y, qy = tz * e1x - tx * e1z, qz = tx * e1y - ty * e1x;
    float det = e1x * px + e1y * py + e1z * pz;
    float un = tx * px + ty * py + tz * pz;
    float vn = r.cx * qx + r.cy * qy + r.cz * qz;
    float tn = e2x * qx + e2y * qy + e2z * qz;
    const float k = 0x1p-18f;
    const float l1 = fabsf(e1x) + fabsf(e1y) + fabsf(e1z), l2 = fabsf(e2x) + fabsf(e2y) + fabsf(e2z);
    const float lt = fabsf(tx) + fabsf(ty) + fabsf(tz) + r.o_l1;
    const float bd = k * l1 * l2, bu = k * lt * l2, bv = k * lt * l1, bt = k * lt * l1 * l2;
    if (!(fabsf(det) > bd)) return true;  // grazing or sign uncertain: decide exactly
    if (det < 0.0f) {
        det = -det;
        un = -un;
        vn = -vn;
        tn = -tn;
    }
    const float wn = det - un - vn, bw = bd + bu + bv;
    const float slack = (dh_num / cc.z) * (det + bd);  // (delta / h_min) * max |det|
    if (un + bu < -slack || vn + bv < -slack || wn + bw < -slack) return false;
    if (lo > -INFINITY && tn + bt <= lo * (lo >= 0.0f ? det - bd : det + bd)) return false;
    if (hi < INFINITY && hi >= 0.0f && tn - bt >= hi * (det + bd)) return false;
    return true;
}

// Test the triangle references [first, first + count) over the tile window.
//   valid hit:   t in (hit_lo, t_hi], inside, better than the current best
//   candidate:   t in (cand_lo, t_hi], t < best_t + delta, within delta of the triangle
__device__ __forceinline__ void test_leaf(const float4 *__restrict__ tris, int first, int count, RayState &r,
                                          RaySrc src, double hit_lo, double cand_lo, float flo, double t_hi,
                                          double t_min, double delta)
{
    for (int k = first; k < first + count; ++k) {
        const float4 a = tris[3 * k], b = tris[3 * k + 1], cc = tris[3 * k + 2];
        const int id = __float_as_int(cc.y);
        if (id == r.start) continue;
        r.tri_tests++;
        const double upper = fmin(t_hi, r.best_t + delta);
        if (!maybe_candidate(a, b, cc, r, flo, f32_up(upper), (float)delta)) continue;
        V3 o, c;
        load_ray64(src, o, c);
        const V3 v0 = {a.x, a.y, a.z}, v1 = {a.w, b.x, b.y}, v2 = {b.z, b.w, cc.x};
        const V3 e1 = v1 - v0, e2 = v2 - v0;
        const V3 p = cross(c, e2);
        const double det = dot(e1, p);
        if (det == 0.0) continue;
        const double inv = 1.0 / det;
        const V3 T = o - v0;
        const V3 q = cross(T, e1);
        const double t = dot(e2, q) * inv;
        if (!(t > cand_lo && t <= t_hi && t < r.best_t + delta)) continue;
        const double u = dot(T, p) * inv;
        const double v = dot(c, q) * inv;
        const double w = (1.0 - u) - v;
        const double wmin = fmin(u, fmin(v, w));
        const double hmin = (double)cc.z;
        double sd;
        if (wmin >= 0.0 && wmin * hmin >= delta) {
            sd = delta;  // inside and at least delta from every edge
        } else if (wmin < 0.0 && -wmin * hmin >= delta) {
            continue;    // outside by at least delta
        } else {
            sd = exact_signed_dist(o + t * c, u, v, w, v0, v1, v2);
            if (sd <= -delta) continue;
        }
        // flag candidate: keep the two smallest parameters (ties by id for the first)
        if (t < r.c1_t || (t == r.c1_t && id < r.c1_id)) {
            r.c2_t = r.c1_t;
            r.c1_t = t;
            r.c1_id = id;
        } else if (t < r.c2_t) {
            r.c2_t = t;
        }
        if (sd >= 0.0 && t > hit_lo && (t < r.best_t || (t == r.best_t && id < r.best_id))) {
            r.best_t = t;
            r.best_id = id;
            r.best_near = (sd < delta) || (t - t_min < delta);
        }
    }
}

__device__ __forceinline__ void box2(const float4 &nx, const float4 &ny, const float4 &nz, const RayState &r,
                                     float tlo, float thi, float &t0, float &t1, bool &h0, bool &h1)
{
    const float ax0 = (nx.x - r.ox) * r.ix, bx0 = (nx.z - r.ox) * r.ix;
    const float ay0 = (ny.x - r.oy) * r.iy, by0 = (ny.z - r.oy) * r.iy;
    const float az0 = (nz.x - r.oz) * r.iz, bz0 = (nz.z - r.oz) * r.iz;
    const float mn0 = fmaxf(fmaxf(fminf(ax0, bx0), fminf(ay0, by0)), fmaxf(fminf(az0, bz0), tlo));
    const float mx0 = fminf(fminf(fmaxf(ax0, bx0), fmaxf(ay0, by0)), fminf(fmaxf(az0, bz0), thi));
    const float ax1 = (nx.y - r.ox) * r.ix, bx1 = (nx.w - r.ox) * r.ix;
    const float ay1 = (ny.y - r.oy) * r.iy, by1 = (ny.w - r.oy) * r.iy;
    const float az1 = (nz.y - r.oz) * r.iz, bz1 = (nz.w - r.oz) * r.iz;
    const float mn1 = fmaxf(fmaxf(fminf(ax1, bx1), fminf(ay1, by1)), fmaxf(fminf(az1, bz1), tlo));
    const float mx1 = fminf(fminf(fmaxf(ax1, bx1), fmaxf(ay1, by1)), fminf(fmaxf(az1, bz1), thi));
    h0 = mn0 <= mx0;
    h1 = mn1 <= mx1;
    t0 = mn0;
    t1 = mn1;
}

__device__ __forceinline__ bool box1(const float *bx, const RayState &r, float tlo, float thi)
{
    const float ax = (bx[0] - r.ox) * r.ix, bxx = (bx[3] - r.ox) * r.ix;
    const float ay = (bx[1] - r.oy) * r.iy, by = (bx[4] - r.oy) * r.iy;
    const float az = (bx[2] - r.oz) * r.iz, bz = (bx[5] - r.oz) * r.iz;
    const float mn = fmaxf(fmaxf(fminf(ax, bxx), fminf(ay, by)), fmaxf(fminf(az, bz), tlo));
    const float mx = fminf(fminf(fmaxf(ax, bxx), fmaxf(ay, by)), fminf(fmaxf(az, bz), thi));
    return mn <= mx;
}

// Traverse one tile's hierarchy over the ray window (t_lo, t_hi].
// The walk of a tile's hierarchy is "while-while": a lane descends interior nodes until it
// stands at a leaf (or has nothing left), and the wave tests its lanes' leaves together
// once every lane is there.  Leaf tests are the long code path; taking them in one pass
// keeps most lanes of the wave busy in it instead of a few lanes in every node step.
constexpr int kDone = (int)0x80000000;  // no leaf reference can take this value (< 2^28 refs)
constexpr int kTraceBlock = 64 * kWavesPerBlock;  // k_trace's block size (its launch uses it)
static_assert(kTraceBlock == 256, "k_trace's LDS stacks are laid out for 256 lanes");

// Traverse one tile's hierarchy over the ray window (t_lo, t_hi].
__device__ void traverse_tile(const DevMesh &M, int tile, RayState &r, RaySrc src, double t_lo, double t_hi,
                              double t_min, double delta, int *stk)
{
    const int root = M.tile_root[tile];
    if (root == kEmptyRoot) return;
    const double hit_lo = fmax(t_lo, t_min);
    const double cand_lo = fmax(t_lo, t_min - delta);
    const float flo = f32_down(cand_lo);
    // FP32 upper end of the box window, refreshed after every leaf (which may lower best_t)
    float fhi = f32_up(fmin(t_hi, r.best_t + delta));
    if (!box1(M.tile_box + 6 * tile, r, flo, fhi)) return;
    // the lane's stack: entry e at lane_stk[e * kTraceBlock] (a shift, not a multiply)
    int *lane_stk = stk + threadIdx.x;
    int sp = 0;
    int ref = root;
    while (true) {
        while (ref >= 0) {
            const float4 *nd = M.nodes + 8 * (long long)ref;
            const float4 lx = nd[0], hx = nd[1], ly = nd[2], hy = nd[3], lz = nd[4], hz = nd[5], rr = nd[6];
            r.node_visits++;
            float t[4];
            int c[4];
            const float lxa[4] = {lx.x, lx.y, lx.z, lx.w}, hxa[4] = {hx.x, hx.y, hx.z, hx.w};
            const float lya[4] = {ly.x, ly.y, ly.z, ly.w}, hya[4] = {hy.x, hy.y, hy.z, hy.w};
            const float lza[4] = {lz.x, lz.y, lz.z, lz.w}, hza[4] = {hz.x, hz.y, hz.z, hz.w};
            const int ca[4] = {__float_as_int(rr.x), __float_as_int(rr.y), __float_as_int(rr.z), __float_as_int(rr.w)};
            int nh = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float ax = fmaf(lxa[k], r.ix, -r.oix), bx = fmaf(hxa[k], r.ix, -r.oix);
                const float ay = fmaf(lya[k], r.iy, -r.oiy), by = fmaf(hya[k], r.iy, -r.oiy);
                const float az = fmaf(lza[k], r.iz, -r.oiz), bz = fmaf(hza[k], r.iz, -r.oiz);
                const float mn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), flo));
                const float mx = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), fhi));
                const bool h = mn <= mx;  // unused slots never pass (kEmptyChild)
                t[k] = h ? mn : INFINITY;
                c[k] = ca[k];
                nh += h ? 1 : 0;
            }
            // order the children by entry parameter (misses last)
#define BT_CSWAP(i, j)                                              \
    if (t[j] < t[i]) {                                              \
        const float tt = t[i]; t[i] = t[j]; t[j] = tt;              \
        const int cc = c[i]; c[i] = c[j]; c[j] = cc;                \
    }
            BT_CSWAP(0, 1) BT_CSWAP(2, 3) BT_CSWAP(0, 2) BT_CSWAP(1, 3) BT_CSWAP(1, 2)
#undef BT_CSWAP
            if (nh > 0) {
                // the nearest next, the others pushed farthest first
                if (nh > 3) lane_stk[(sp++) * kTraceBlock] = c[3];
                if (nh > 2) lane_stk[(sp++) * kTraceBlock] = c[2];
                if (nh > 1) lane_stk[(sp++) * kTraceBlock] = c[1];
                ref = c[0];
            } else if (sp > 0) {
                sp--;
                ref = lane_stk[sp * kTraceBlock];
            } else {
                ref = kDone;
            }
        }
        if (ref == kDone) break;
        const int v = ~ref;
        test_leaf(M.tris, v >> 3, v & 7, r, src, hit_lo, cand_lo, flo, t_hi, t_min, delta);
        fhi = f32_up(fmin(t_hi, r.best_t + delta));
        if (sp == 0) break;
        sp--;
        ref = lane_stk[sp * kTraceBlock];
    }
}

// ---------------------------------------------------------------------------------------
// Tile windows.  A ray's parameter range inside the mesh's box, (t_start, tx], is cut by
// the interior tile boundaries it crosses into consecutive half-open windows (t_lo, t_hi],
// one per tile; t_hi is the nearer of the tile's x and y boundaries ahead (or tx), computed
// from the tile index alone, so every path that reaches a tile computes the same window
// end.  The first tile's window starts at t_start (a ray may start on a boundary).
// ---------------------------------------------------------------------------------------
// The ray's range in the mesh's box and the tile of its start point; false when the ray
// misses the box.
__device__ bool ray_box(const DevMesh &M, V3 o, V3 c, double t_min, double delta, double &t_start, double &tx,
                        int &ix, int &iy)
{
    double te = -INFINITY;
    tx = INFINITY;
    bool ok = true;
    const double o3[3] = {o.x, o.y, o.z}, c3[3] = {c.x, c.y, c.z};
    const double lo3[3] = {M.gx0, M.gy0, M.zmin}, hi3[3] = {M.gx1, M.gy1, M.zmax};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (c3[k] != 0.0) {
            const double ta = (lo3[k] - o3[k]) / c3[k], tb = (hi3[k] - o3[k]) / c3[k];
            te = fmax(te, fmin(ta, tb));
            tx = fmin(tx, fmax(ta, tb));
        } else if (o3[k] < lo3[k] || o3[k] > hi3[k]) {
            ok = false;
        }
    }
    t_start = fmax(te, t_min - delta);
    if (!ok || !(t_start <= tx)) return false;
    const double px = o.x + t_start * c.x, py = o.y + t_start * c.y;
    ix = (int)floor((px - M.gx0) / M.tw);
    iy = (int)floor((py - M.gy0) / M.th);
    ix = ix < 0 ? 0 : (ix >= M.tiles_x ? M.tiles_x - 1 : ix);
    iy = iy < 0 ? 0 : (iy >= M.tiles_y ? M.tiles_y - 1 : iy);
    return true;
}

// End of tile (ix, iy)'s window and the tile entered there (both axes step when the
// ray leaves through a corner).  Only interior boundaries count: the outer ones are the
// box exit tx.
__device__ __forceinline__ double tile_exit(const DevMesh &M, V3 o, V3 c, int ix, int iy, double tx, int &nix,
                                            int &niy)
{
    double X = INFINITY, Y = INFINITY;
    if (c.x > 0.0 && ix < M.tiles_x - 1) X = (M.gx0 + (double)(ix + 1) * M.tw - o.x) / c.x;
    else if (c.x < 0.0 && ix > 0) X = (M.gx0 + (double)ix * M.tw - o.x) / c.x;
    if (c.y > 0.0 && iy < M.tiles_y - 1) Y = (M.gy0 + (double)(iy + 1) * M.th - o.y) / c.y;
    else if (c.y < 0.0 && iy > 0) Y = (M.gy0 + (double)iy * M.th - o.y) / c.y;
    nix = ix + ((X <= Y && X < INFINITY) ? (c.x > 0.0 ? 1 : -1) : 0);
    niy = iy + ((Y <= X && Y < INFINITY) ? (c.y > 0.0 ? 1 : -1) : 0);
    return fmin(fmin(X, Y), tx);
}

// Traverse tiles in order from (ix, iy), whose window starts at t_lo, until the ray is
// resolved (a hit with no other triangle within delta beyond the window, or the box
// exit).  Only the tile index, t_lo and tx stay live across a tile's traversal; the FP64
// ray is reloaded to find the next window.
__device__ void walk_tiles(const DevMesh &M, RayState &r, RaySrc src, int ix, int iy, double t_lo, double tx,
                           double t_min, double delta, int *stk)
{
    for (int guard = 0; guard < M.tiles_x + M.tiles_y; ++guard) {
        int nix, niy;
        double t_hi;
        {
            V3 o, c;
            load_ray64(src, o, c);
            t_hi = tile_exit(M, o, c, ix, iy, tx, nix, niy);
        }
        if (t_hi > t_lo) traverse_tile(M, iy * M.tiles_x + ix, r, src, t_lo, t_hi, t_min, delta, stk);
        if (t_hi >= tx || t_hi >= r.best_t + delta) break;
        ix = nix;
        iy = niy;
        t_lo = t_hi;
    }
}

// A child is spawned by a hit with depth < max_depth whose power after absorption exceeds
// e_min (when set), decided in FP64 from the beam's FP64 power P.  The child-counting
// kernels and k_reflect apply this rule.
__device__ __forceinline__ bool spawns_child(const DevMesh &M, const TraceArgs &a, int hit, int meta, double P)
{
    const int max_depth = a.scenarios ? meta_max_depth(meta) : a.max_depth;
    if (hit < 0 || (meta & 0xff) >= max_depth) return false;
    return !(a.e_min > 0.0) || (P * (1.0 - (double)M.alpha[hit]) > a.e_min);
}

// Ray state of queue record i, with nothing found yet.
__device__ __forceinline__ void ray_init(RayState &r, RaySrc src, int start)
{
    V3 o, c;
    load_ray64(src, o, c);
    r.ox = (float)o.x;
    r.oy = (float)o.y;
    r.oz = (float)o.z;
    r.cx = (float)c.x;
    r.cy = (float)c.y;
    r.cz = (float)c.z;
    r.o_l1 = fabsf(r.ox) + fabsf(r.oy) + fabsf(r.oz);
    const double tiny = 1e-20;
    r.ix = (float)(1.0 / (fabs(c.x) < tiny ? copysign(tiny, c.x) : c.x));
    r.iy = (float)(1.0 / (fabs(c.y) < tiny ? copysign(tiny, c.y) : c.y));
    r.iz = (float)(1.0 / (fabs(c.z) < tiny ? copysign(tiny, c.z) : c.z));
    r.oix = r.ox * r.ix;
    r.oiy = r.oy * r.iy;
    r.oiz = r.oz * r.iz;
    r.start = start;
    r.best_t = INFINITY;
    r.best_id = -1;
    r.best_near = 0;
    r.c1_t = INFINITY;
    r.c2_t = INFINITY;
    r.c1_id = -1;
    r.node_visits = 0;
    r.tri_tests = 0;
}

// The resolved segment of record i: hit, parameter and flag (own or inherited), and the
// optional per-(initial beam, generation) parity outputs.  Returns the flag.
__device__ __forceinline__ int finish_ray(const RayState &r, const DevQueue &in, DevSegs segs, const TraceArgs &a,
                                          long long i)
{
    const long long icap = in.cap;
    const int meta = in.ints[I_META * icap + i];
    const int hit = r.best_id;
    int own_flag;
    if (hit >= 0) own_flag = r.best_near || (r.c1_id != hit) || (r.c2_t < r.best_t + a.delta);
    else own_flag = r.c1_t < INFINITY;
    const int flag_total = ((meta & kMetaFlag) != 0) || own_flag;
    segs.hit[i] = hit;
    segs.t[i] = r.best_t;
    segs.flag[i] = flag_total;
    if (a.hit_out || a.flag_out || a.t_out) {
        const long long oidx = (long long)in.ints[I_ID * icap + i] * (a.max_depth + 1) + a.gen;
        if (a.hit_out) a.hit_out[oidx] = hit;
        if (a.flag_out) a.flag_out[oidx] = (uint8_t)flag_total;
        if (a.t_out) a.t_out[oidx] = r.best_t;
    }
    return flag_total;
}

// The tile table (roots and root boxes) staged in LDS for up to 256 tiles, so that a tile
// change waits on no global load.
constexpr int kLdsTiles = 64;
struct TileTable {
    int root[kLdsTiles];
    float box[6 * kLdsTiles];
};
__device__ __forceinline__ DevMesh stage_tiles(const DevMesh &M, TileTable &t)
{
    DevMesh Ml = M;
    const int n_tiles = M.tiles_x * M.tiles_y;
    if (n_tiles <= kLdsTiles) {
        for (int k = threadIdx.x; k < n_tiles; k += blockDim.x) t.root[k] = M.tile_root[k];
        for (int k = threadIdx.x; k < 6 * n_tiles; k += blockDim.x) t.box[k] = M.tile_box[k];
        __syncthreads();
        Ml.tile_root = t.root;
        Ml.tile_box = t.box;
    }
    return Ml;
}

// In-lane walk: each lane resolves its ray through every tile it crosses and writes its
// segment; the generation's children, flags and power are counted by k_tcount.
__global__ void __launch_bounds__(kTraceBlock, 4) k_trace(DevMesh M, DevQueue in, DevSegs segs, DevCounters *ctr, TraceArgs a,
                                               WaveScratch ws)
{
    __shared__ int stk[kStack * kTraceBlock];
    __shared__ TileTable tt_lds;
    __shared__ unsigned s_nv[kTraceBlock], s_tt[kTraceBlock];  // per-lane totals (not in registers)
    const DevMesh Ml = stage_tiles(M, tt_lds);
    const unsigned long long n = ctr->count[a.gen];
    const long long s0 = (long long)gen_start(ctr, a.gen);
    const int lane = lane_id();
    const long long icap = in.cap;
    s_nv[threadIdx.x] = 0;
    s_tt[threadIdx.x] = 0;
    for (unsigned long long base = wave_first_batch(); base < n; base += wave_batch_stride()) {
        const bool active = (long long)base + lane < (long long)n;
        const long long i = s0 + (long long)base + lane;
        const RaySrc src{in.dbl + D_O * icap, in.dbl + D_C * icap, icap, active ? (int)i : 0};
        if (active) {
            RayState r;
            ray_init(r, src, in.ints[I_START * icap + i]);
            {
                double t_start, tx;
                int ix, iy;
                bool inside;
                {
                    V3 o, c;
                    load_ray64(src, o, c);
                    inside = ray_box(Ml, o, c, a.t_min, a.delta, t_start, tx, ix, iy);
                }
                if (inside) walk_tiles(Ml, r, src, ix, iy, t_start, tx, a.t_min, a.delta, stk);
            }
            finish_ray(r, in, segs, a, i);
            s_nv[threadIdx.x] += r.node_visits;
            s_tt[threadIdx.x] += r.tri_tests;
        }
    }
    const unsigned long long snv = wave_sum_u64(s_nv[threadIdx.x]), stt = wave_sum_u64(s_tt[threadIdx.x]);
    if (lane == 0) {
        const unsigned long long w = wave_first_batch() >> 6;
        ws.stats[3 * w + 1] = snv;
        ws.stats[3 * w + 2] = stt;
    }
}

// ---------------------------------------------------------------------------------------
// Per-tile beam queues (the paper's sub-domain decomposition, Section 3, kept as an
// on-GPU partition: each sub-domain owns a queue of the beams inside it, and a beam
// leaving a sub-domain without a hit is handed to the queue of the sub-domain it enters).
// A generation is traced in rounds:
//   k_tbin:     every ray's entry tile; rays missing the mesh's box are resolved at once;
//               the others become round-0 items of their tile
//   k_tscan, k_tscatter: the round's items ordered by tile (counting sort, no atomics)
//   k_ttrace:   the ordered items split into equal shares, one per XCD, so that each
//               XCD's L2 holds the hierarchies of few tiles; a ray whose window ends
//               unresolved becomes, with its partial result, an item of the next round
//               queued for the tile it enters; in the last queued round it walks its
//               remaining tiles in its own lane
//   k_tcount:   children, flags and power per wave in the static partition k_reflect uses
// Items are (position in the generation, tile | first-window bit << 16 | near bit << 17);
// a handed-off ray's partial result lives in the segment record (best hit and parameter)
// and in the per-position arrays of TileWork (flag candidates and the window start).
// ---------------------------------------------------------------------------------------
constexpr int kItemFirst = 1 << 16;
constexpr int kItemNear = 1 << 17;

__device__ __forceinline__ unsigned long long lanes_below() { return (1ull << lane_id()) - 1ull; }

// Producer side: the lanes with `want` add their items to wave w's region and to its
// per-tile counts (both owned by the wave, so no atomics).  `n_out` is the wave's item
// count so far (uniform).
__device__ __forceinline__ void wave_produce(const TileWork &tw, long long w, bool want, int tile, int2 item,
                                             int &n_out)
{
    const unsigned long long m = __ballot(want);
    if (m == 0) return;
    if (want) {
        const long long k = (long long)n_out + __popcll(m & lanes_below());
        if (k < tw.region) tw.stage[w * tw.region + k] = item;
    }
    n_out += __popcll(m);
    unsigned long long rem = m;
    while (rem) {
        const int leader = __ffsll((long long)rem) - 1;
        const int t = __shfl(tile, leader, 64);
        const unsigned long long same = __ballot(want && tile == t);
        if (lane_id() == leader) tw.cnt[(long long)t * tw.n_waves + w] += __popcll(same);
        rem &= ~same;
    }
}

__device__ __forceinline__ long long global_wave() { return ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; }

__global__ void __launch_bounds__(256) k_tbin(DevMesh M, DevQueue in, DevSegs segs, DevCounters *ctr, TraceArgs a,
                                              WaveScratch ws, TileWork tw)
{
    const unsigned long long n0 = ctr->count[a.gen];
    const unsigned long long n = (long long)n0 > tw.cap ? (unsigned long long)tw.cap : n0;
    const long long s0 = (long long)gen_start(ctr, a.gen);
    const int lane = lane_id();
    const long long icap = in.cap;
    const long long w = global_wave();
    int n_out = 0;
    for (unsigned long long base = wave_first_batch(); base < n; base += wave_batch_stride()) {
        const bool active = (long long)base + lane < (long long)n;
        const long long i = s0 + (long long)base + lane;
        int tile = -1;
        if (active) {
            V3 o = ld3(in.dbl + D_O * icap, icap, i), c = ld3(in.dbl + D_C * icap, icap, i);
            double t_start, tx;
            int ix, iy;
            if (ray_box(M, o, c, a.t_min, a.delta, t_start, tx, ix, iy)) {
                tile = iy * M.tiles_x + ix;
            } else {
                // misses the mesh's box: resolved (escape, nothing near)
                RayState r;
                r.best_t = INFINITY;
                r.best_id = -1;
                r.best_near = 0;
                r.c1_t = r.c2_t = INFINITY;
                r.c1_id = -1;
                finish_ray(r, in, segs, a, i);
            }
        }
        wave_produce(tw, w, tile >= 0, tile, make_int2((int)(base + lane), tile | kItemFirst), n_out);
    }
    if (lane == 0) {
        tw.stage_n[w] = n_out;
        ws.stats[3 * w + 1] = 0;   // node visits and triangle tests, added to by the rounds
        ws.stats[3 * w + 2] = 0;
    }
}

// Block t: exclusive scan of tile t's counts over the producer waves, the tile's total;
// the counts are cleared for the next round.
constexpr int kScanBlock = 1024;
__global__ void __launch_bounds__(kScanBlock) k_tscan(TileWork tw)
{
    __shared__ int s_wsum[kScanBlock / 64];
    const int t = blockIdx.x;
    const int W = tw.n_waves;
    int *cnt = tw.cnt + (long long)t * W;
    int *off = tw.off + (long long)t * W;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int per = (W + kScanBlock - 1) / kScanBlock;
    const int b0 = threadIdx.x * per, b1 = min(b0 + per, W);
    int sum = 0;
    for (int k = b0; k < b1; ++k) sum += cnt[k];
    int incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) s_wsum[wv] = incl;
    __syncthreads();
    int run = incl - sum, tot = 0;
    for (int k = 0; k < kScanBlock / 64; ++k) {
        if (k < wv) run += s_wsum[k];
        tot += s_wsum[k];
    }
    for (int k = b0; k < b1; ++k) {
        const int c = cnt[k];
        off[k] = run;
        run += c;
        cnt[k] = 0;
    }
    if (threadIdx.x == 0) tw.total[t] = tot;
}

// Wave w places the items of producer region w: tile start (scan of the totals) + the
// wave's offset within the tile + the item's rank among the region's items of that tile.
__global__ void __launch_bounds__(256) k_tscatter(TileWork tw)
{
    __shared__ int s_start[kMaxQueueTiles + 1];
    __shared__ int s_run[4][kMaxQueueTiles];
    const int T = tw.n_tiles, W = tw.n_waves;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < T; ++t) {
            s_start[t] = run;
            run += tw.total[t];
        }
        s_start[T] = run;
        if (blockIdx.x == 0) *tw.n_items = run;
    }
    for (int k = lane; k < T; k += 64) s_run[wv][k] = 0;
    __syncthreads();
    const long long w = global_wave();
    if (w >= W) return;
    const int n = (int)min((long long)tw.stage_n[w], tw.region);
    for (int base = 0; base < n; base += 64) {
        const bool active = base + lane < n;
        const int2 item = active ? tw.stage[w * tw.region + base + lane] : make_int2(0, 0);
        const int tile = active ? (item.y & 0xffff) : -1;
        unsigned long long rem = __ballot(active);
        while (rem) {
            const int leader = __ffsll((long long)rem) - 1;
            const int t = __shfl(tile, leader, 64);
            const unsigned long long same = __ballot(active && tile == t);
            if (active && tile == t) {
                const long long pos = (long long)s_start[t] + tw.off[(long long)t * W + w] + s_run[wv][t] +
                                      __popcll(same & lanes_below());
                if (pos < tw.cap) tw.list[pos] = item;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == leader) s_run[wv][t] += __popcll(same);
            __builtin_amdgcn_wave_barrier();
            rem &= ~same;
        }
    }
}

__global__ void __launch_bounds__(kTraceBlock, 4) k_ttrace(DevMesh M, DevQueue in, DevSegs segs, DevCounters *ctr,
                                                          TraceArgs a, WaveScratch ws, TileWork tw, int last)
{
    __shared__ int stk[kStack * kTraceBlock];
    __shared__ TileTable tt_lds;
    const DevMesh Ml = stage_tiles(M, tt_lds);
    const long long n = min((long long)*tw.n_items, tw.cap);
    const long long s0 = (long long)gen_start(ctr, a.gen);
    const int lane = lane_id();
    const long long icap = in.cap;
    const long long w = global_wave();
    // blocks are dispatched to the XCDs in turn: XCD x runs blocks x, x + 8, ... and
    // takes the x-th share of the tile-ordered list
    const int groups = (gridDim.x % kXcds) == 0 ? kXcds : 1;
    const int xcd = (int)blockIdx.x % groups;
    const long long wave_in_xcd = (long long)(blockIdx.x / groups) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const long long waves_per_xcd = (long long)(gridDim.x / groups) * (blockDim.x >> 6);
    const long long share = ((n + groups - 1) / groups + 63) / 64 * 64;
    const long long lo = (long long)xcd * share, hi = min(n, lo + share);
    unsigned nv = 0, tt = 0;
    int n_out = 0;
    for (long long base = lo + 64 * wave_in_xcd; base < hi; base += 64 * waves_per_xcd) {
        const bool active = base + lane < hi;
        const int2 item = active ? tw.list[base + lane] : make_int2(0, 0);
        const long long pos = item.x;
        const long long i = s0 + pos;
        const RaySrc src{in.dbl + D_O * icap, in.dbl + D_C * icap, icap, active ? (int)i : 0};
        bool hand_off = false;
        int next = 0;
        if (active) {
            RayState r;
            ray_init(r, src, in.ints[I_START * icap + i]);
            const int tile = item.y & 0xffff;
            int ix = tile % Ml.tiles_x, iy = tile / Ml.tiles_x;
            double t_lo, tx;
            {
                V3 o, c;
                load_ray64(src, o, c);
                double t_start;
                int sx, sy;
                ray_box(Ml, o, c, a.t_min, a.delta, t_start, tx, sx, sy);
                t_lo = t_start;
            }
            if (!(item.y & kItemFirst)) {
                // carried over from the previous round
                r.best_t = segs.t[i];
                r.best_id = segs.hit[i];
                r.best_near = (item.y & kItemNear) ? 1 : 0;
                r.c1_t = tw.c1t[pos];
                r.c2_t = tw.c2t[pos];
                r.c1_id = tw.c1id[pos];
                t_lo = tw.lo[pos];
            }
            int nix, niy;
            double t_hi;
            {
                V3 o, c;
                load_ray64(src, o, c);
                t_hi = tile_exit(Ml, o, c, ix, iy, tx, nix, niy);
            }
            if (t_hi > t_lo) traverse_tile(Ml, tile, r, src, t_lo, t_hi, a.t_min, a.delta, stk);
            const bool done = t_hi >= tx || t_hi >= r.best_t + a.delta;
            if (!done && !last) {
                // hand off to the queue of the tile it enters, with its partial result
                hand_off = true;
                next = niy * Ml.tiles_x + nix;
                segs.t[i] = r.best_t;
                segs.hit[i] = r.best_id;
                tw.c1t[pos] = r.c1_t;
                tw.c2t[pos] = r.c2_t;
                tw.c1id[pos] = r.c1_id;
                tw.lo[pos] = t_hi;
                next |= r.best_near ? kItemNear : 0;
            } else {
                if (!done) walk_tiles(Ml, r, src, nix, niy, t_hi, tx, a.t_min, a.delta, stk);
                finish_ray(r, in, segs, a, i);
            }
            nv += r.node_visits;
            tt += r.tri_tests;
        }
        if (!last) wave_produce(tw, w, hand_off, next & 0xffff, make_int2((int)pos, next), n_out);
    }
    const unsigned long long snv = wave_sum_u64(nv), stt = wave_sum_u64(tt);
    if (lane == 0) {
        if (!last) tw.stage_n[w] = n_out;
        ws.stats[3 * w + 1] += snv;
        ws.stats[3 * w + 2] += stt;
    }
}

// Children, flags and power of the generation per wave, and children per block, in the
// static partition that k_reflect uses.
__global__ void __launch_bounds__(64 * kWavesPerBlock) k_tcount(DevMesh M, DevQueue in, DevSegs segs, DevCounters *ctr, TraceArgs a,
                                                WaveScratch ws)
{
    const unsigned long long n = ctr->count[a.gen];
    const long long s0 = (long long)gen_start(ctr, a.gen);
    const int lane = lane_id();
    const long long icap = in.cap;
    unsigned children = 0, flagged = 0;
    double power = 0.0;
    for (unsigned long long base = wave_first_batch(); base < n; base += wave_batch_stride()) {
        if ((long long)base + lane < (long long)n) {
            const long long i = s0 + (long long)base + lane;
            const double P = in.dbl[D_P * icap + i];
            children += spawns_child(M, a, segs.hit[i], in.ints[I_META * icap + i], P);
            flagged += segs.flag[i] != 0;
            power += P;
        }
    }
    const unsigned long long sc = wave_sum_u64(children), sf = wave_sum_u64(flagged);
    const double sp = wave_sum_f64(power);
    __shared__ unsigned long long s_rec[kWavesPerBlock][4];
    __shared__ double s_pow[kWavesPerBlock];
    if (lane == 0) {
        const unsigned long long w = wave_first_batch() >> 6;
        ws.children[w] = sc;
        ws.stats[3 * w] = sf;
        ws.power[w] = sp;
        const int wv = (int)threadIdx.x >> 6;
        s_rec[wv][0] = sc;
        s_rec[wv][1] = sf;
        s_rec[wv][2] = ws.stats[3 * w + 1];   // the trace's node visits and triangle tests
        s_rec[wv][3] = ws.stats[3 * w + 2];
        s_pow[wv] = sp;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned long long b = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) b += s_rec[k][threadIdx.x];
        ws.block_rec[4 * (long long)blockIdx.x + threadIdx.x] = b;
    } else if (threadIdx.x == 4) {
        double b = 0.0;
        for (int k = 0; k < kWavesPerBlock; ++k) b += s_pow[k];
        ws.block_power[blockIdx.x] = b;
    }
}

// The generation's totals, summed by one block over k_tcount's block records in a fixed
// order (so they are the same on every run): children (the next generation's size),
// flagged segments, power, and the traversal counters.
__device__ void generation_totals(DevCounters *ctr, const TraceArgs &a, const WaveScratch &ws)
{
    constexpr int kThreads = 64 * kWavesPerBlock;
    __shared__ unsigned long long s_tot[4][kWavesPerBlock];
    __shared__ double s_pow[kWavesPerBlock];
    const int nb = ws.n_waves / kWavesPerBlock, lane = lane_id(), wv = (int)threadIdx.x >> 6;
    unsigned long long t[4] = {0, 0, 0, 0};
    double p = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) {
#pragma unroll
        for (int k = 0; k < 4; ++k) t[k] += ws.block_rec[4 * (long long)b + k];
        p += ws.block_power[b];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = wave_sum_u64(t[k]);
    p = wave_sum_f64(p);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s_tot[k][wv] = t[k];
        s_pow[wv] = p;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tt[4] = {0, 0, 0, 0};
        double tp = 0.0;
        for (int w = 0; w < kWavesPerBlock; ++w) {
            for (int k = 0; k < 4; ++k) tt[k] += s_tot[k][w];
            tp += s_pow[w];
        }
        ctr->count[a.gen + 1] = tt[0];
        ctr->flagged[a.gen] = tt[1];
        ctr->power[a.gen] = tp;
        ctr->node_visits += tt[2];
        ctr->tri_tests += tt[3];
    }
}

// First queue position, in the next generation, of this wave's children: the children of
// the blocks before this one (k_tcount's block records, summed by the whole block, their
// loads issued together) and of this block's earlier waves.  Children keep the order of
// the waves, so the next generation's order is deterministic.
__device__ unsigned long long child_offset(const WaveScratch &ws)
{
    constexpr int kThreads = 64 * kWavesPerBlock;
    constexpr int kUnroll = 4;
    __shared__ unsigned long long s_part[kWavesPerBlock], s_wc[kWavesPerBlock];
    const int lane = lane_id(), wv = (int)threadIdx.x >> 6;
    const int nb = (int)blockIdx.x;
    unsigned long long part = 0;
    for (int b0 = threadIdx.x; b0 < nb; b0 += kUnroll * kThreads) {
        unsigned long long v[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k)
            v[k] = b0 + k * kThreads < nb ? ws.block_rec[4 * (long long)(b0 + k * kThreads)] : 0ull;
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) part += v[k];
    }
    part = wave_sum_u64(part);
    if (lane == 0) {
        s_part[wv] = part;
        s_wc[wv] = ws.children[(long long)nb * kWavesPerBlock + wv];
    }
    __syncthreads();
    unsigned long long off = 0;
    for (int k = 0; k < kWavesPerBlock; ++k) off += s_part[k] + (k < wv ? s_wc[k] : 0ull);
    return off;
}

// Specular reflection without splitting: every hit with depth < max_depth (and, when set,
// power above e_min) spawns one child mirrored in the hit triangle's plane (apex, edge and
// guiding directions; d1 and d2 swapped to keep det > 0), starting at the hit point with
// K (1 - alpha).  Children are compacted into the next generation with a wave ballot and
// a popcount prefix from the wave's offset.  When the set classifies its beams, each
// child's planar microphone class is written while it is in registers.  Block 0 also
// writes the generation's totals (the next generation's size among them).
__global__ void __launch_bounds__(64 * kWavesPerBlock) k_reflect(DevMesh M, DevQueue q, DevSegs segs,
                                                                 DevCounters *ctr, TraceArgs a, WaveScratch ws)
{
    const unsigned long long n = ctr->count[a.gen];
    const long long s0 = (long long)gen_start(ctr, a.gen);
    const long long s1 = (long long)gen_start(ctr, a.gen + 1);  // the children's generation starts here
    const int lane = lane_id();
    const DevQueue &in = q, &out = q;
    const long long icap = q.cap, ocap = q.cap;
    if (blockIdx.x == 0) generation_totals(ctr, a, ws);
    // this wave's children go to [offset, offset + children) of the next generation, in
    // batch order (the same static partition as k_trace, which counted them)
    unsigned long long obase = child_offset(ws);
    for (unsigned long long base = wave_first_batch(); base < n; base += wave_batch_stride()) {
        const long long i = s0 + (long long)base + lane;
        int child = 0, hit = -1, meta = 0;
        float Kc = 0.f;
        double Pc = 0.0;
        if ((long long)base + lane < (long long)n) {
            hit = segs.hit[i];
            meta = in.ints[I_META * icap + i];
            const double P = in.dbl[D_P * icap + i];
            child = spawns_child(M, a, hit, meta, P);
            if (child) {
                const float al = M.alpha[hit];
                Kc = in.flt[F_K * icap + i] * (1.0f - al);
                Pc = P * (1.0 - (double)al);
            }
        }
        const unsigned long long mask = __ballot(child);
        if (mask == 0) continue;
        V3 A2, o2, c2, m0, m1, m2;
        int meta2 = 0, id = 0;
        if (child) {
            V3 v0, v1, v2;
            tri_vertices(M.tri_g, hit, v0, v1, v2);
            const V3 N = cross(v1 - v0, v2 - v0);
            const V3 nn = unit(N);
            const V3 A = ld3(in.dbl + D_A * icap, icap, i);
            const V3 o = ld3(in.dbl + D_O * icap, icap, i), c = ld3(in.dbl + D_C * icap, icap, i);
            const double t = segs.t[i];
            A2 = A - (2.0 * dot(A - v0, nn)) * nn;
            o2 = o + t * c;
            c2 = mirror(c, nn);
            m0 = mirror(ld3(in.dbl + D_D0 * icap, icap, i), nn);
            m1 = mirror(ld3(in.dbl + D_D2 * icap, icap, i), nn);  // d1 and d2 swap: det stays > 0
            m2 = mirror(ld3(in.dbl + D_D1 * icap, icap, i), nn);
            // the child lives on the side the parent came from
            meta2 = (meta & kMetaInherited) | ((meta & 0xff) + 1) | (dot(c, N) > 0.0 ? kMetaNegNear : 0) |
                    (segs.flag[i] ? kMetaFlag : 0);
            id = in.ints[I_ID * icap + i];
        }
        const unsigned long long my_base = obase;
        obase += (unsigned long long)__popcll(mask);
        if (child) {
            const long long j = s1 + (long long)my_base + __popcll(mask & ((1ull << lane) - 1ull));
            st3(out.dbl + D_A * ocap, ocap, j, A2);
            st3(out.dbl + D_D0 * ocap, ocap, j, m0);
            st3(out.dbl + D_D1 * ocap, ocap, j, m1);
            st3(out.dbl + D_D2 * ocap, ocap, j, m2);
            st3(out.dbl + D_O * ocap, ocap, j, o2);
            st3(out.dbl + D_C * ocap, ocap, j, c2);
            out.flt[F_K * ocap + j] = Kc;
            out.dbl[D_P * ocap + j] = Pc;
            out.ints[I_ID * ocap + j] = id;
            out.ints[I_START * ocap + j] = hit;
            out.ints[I_META * ocap + j] = meta2;
            if (a.cg.cls) a.cg.cls[j] = plane_class(a.cg, A2, m0, m1, m2);
        }
    }
}

hipError_t launch_trace(const DevMesh &m, DevQueue q, DevSegs segs, DevCounters *ctr, const TraceArgs &a,
                        WaveScratch ws, const TileWork *tw, int n_cu, hipStream_t s)
{
    // the statically partitioned kernels (k_trace / k_tbin / k_tcount and k_reflect) and
    // the queued rounds must use the same grid: wave w owns the same batches, records and
    // producer region in all of them
    (void)n_cu;
    const int blocks = ws.n_waves / kWavesPerBlock;
    if (blocks <= 0 || blocks * kWavesPerBlock != ws.n_waves) return hipErrorInvalidValue;
    hipError_t e;
    if (tw) {
        const int T = m.tiles_x * m.tiles_y;
        if (tw->n_tiles != T || T > kMaxQueueTiles || tw->rounds < 1 || tw->rounds > kMaxQueueRounds ||
            tw->n_waves != ws.n_waves)
            return hipErrorInvalidValue;
        k_tbin<<<blocks, 256, 0, s>>>(m, q, segs, ctr, a, ws, *tw);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int r = 0; r < tw->rounds; ++r) {
            k_tscan<<<T, kScanBlock, 0, s>>>(*tw);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            k_tscatter<<<blocks, 256, 0, s>>>(*tw);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            k_ttrace<<<blocks, kTraceBlock, 0, s>>>(m, q, segs, ctr, a, ws, *tw, r + 1 == tw->rounds);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        k_tcount<<<blocks, 64 * kWavesPerBlock, 0, s>>>(m, q, segs, ctr, a, ws);
    } else {
        k_trace<<<blocks, kTraceBlock, 0, s>>>(m, q, segs, ctr, a, ws);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_tcount<<<blocks, 64 * kWavesPerBlock, 0, s>>>(m, q, segs, ctr, a, ws);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_reflect<<<blocks, 64 * kWavesPerBlock, 0, s>>>(m, q, segs, ctr, a, ws);
    return hipGetLastError();
}

}  // namespace bt
