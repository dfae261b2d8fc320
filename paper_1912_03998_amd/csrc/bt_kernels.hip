// HIP kernels of the hybrid beam tracer for gfx950 (CDNA4, wave64).
//
// Emission, guiding-ray traversal with sub-domain hand-off, fused reflection and
// queue compaction, microphone-in-frustum accumulation and levels.  Built with
// -ffp-contract=off: the microphone tie rule relies on exactly antisymmetric cross
// products of shared beam edges.
#include <hip/hip_runtime.h>
#include <math.h>

#include "bt_internal.h"

namespace bt {

// ---------------------------------------------------------------------------------------
// small FP64 vector helpers
// ---------------------------------------------------------------------------------------
struct V3 {
    double x, y, z;
};
__device__ __forceinline__ V3 v3(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(double k, V3 a) { return {k * a.x, k * a.y, k * a.z}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 unit(V3 a)
{
    double n = sqrt(dot(a, a));
    return {a.x / n, a.y / n, a.z / n};
}
__device__ __forceinline__ V3 mirror(V3 v, V3 n) { return v - (2.0 * dot(v, n)) * n; }

__device__ __forceinline__ V3 ld3(const double *p, long long cap, long long i)
{
    return {p[i], p[cap + i], p[2 * cap + i]};
}
__device__ __forceinline__ void st3(double *p, long long cap, long long i, V3 v)
{
    p[i] = v.x;
    p[cap + i] = v.y;
    p[2 * cap + i] = v.z;
}
__device__ __forceinline__ void tri_vertices(const float *tri_g, int id, V3 &v0, V3 &v1, V3 &v2)
{
    const float *p = tri_g + 9 * (long long)id;
    v0 = {p[0], p[1], p[2]};
    v1 = {p[3], p[4], p[5]};
    v2 = {p[6], p[7], p[8]};
}

// ---------------------------------------------------------------------------------------
// wave64 reductions
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_sum_f64(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Grab the next 64 work items for this wave from a cursor; returns the wave's base.
__device__ __forceinline__ unsigned long long wave_grab(unsigned long long *cursor)
{
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(cursor, 64ull);
    return __shfl(base, 0, 64);
}

// ---------------------------------------------------------------------------------------
// counters
// ---------------------------------------------------------------------------------------
__global__ void k_init_counters(DevCounters *ctr, long long n0)
{
    unsigned long long *w = reinterpret_cast<unsigned long long *>(ctr);
    const int nw = (int)(sizeof(DevCounters) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0ull;  // doubles: +0.0 bits
    __syncthreads();
    if (threadIdx.x == 0) ctr->count[0] = (unsigned long long)n0;
}

hipError_t launch_init_counters(DevCounters *ctr, long long n0, hipStream_t s)
{
    k_init_counters<<<1, 256, 0, s>>>(ctr, n0);
    return hipGetLastError();
}

__global__ void k_fill(double *p, long long n, double v)
{
    long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill(double *p, long long n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_fill<<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Emission: one beam per (source, icosphere face).  The face's three directions are
// found by walking the subdivision from its base icosahedron face: at every level the
// edge midpoints are normalize(x + y) and the child at position j of (a, b, c) is
// (a, ab, ca), (ab, b, bc), (ca, bc, c) or (ab, bc, ca).
// ---------------------------------------------------------------------------------------
__global__ void k_emit(const double *__restrict__ base20, const float *__restrict__ src,
                       const float *__restrict__ power, int n_src, int level, long long nf, DevQueue q)
{
    long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    long long total = nf * n_src;
    if (b >= total) return;
    long long s = b / nf, f = b - s * nf;
    int bf = (int)(f >> (2 * level));
    const double *bp = base20 + 9 * bf;
    V3 a = {bp[0], bp[1], bp[2]}, bb = {bp[3], bp[4], bp[5]}, c = {bp[6], bp[7], bp[8]};
    for (int l = level - 1; l >= 0; --l) {
        int j = (int)((f >> (2 * l)) & 3);
        V3 ab = unit(a + bb), bc = unit(bb + c), ca = unit(c + a);
        if (j == 0) { bb = ab; c = ca; }
        else if (j == 1) { a = ab; c = bc; }
        else if (j == 2) { a = ca; bb = bc; }
        else { a = ab; bb = bc; c = ca; }
    }
    V3 cc = unit((a + bb) + c);
    double num = fabs(dot(a, cross(bb, c)));
    double den = 1.0 + dot(a, bb) + dot(bb, c) + dot(c, a);
    double omega = 2.0 * atan2(num, den);
    V3 S = {src[3 * s], src[3 * s + 1], src[3 * s + 2]};
    const long long cap = q.cap;
    st3(q.dbl + D_A * cap, cap, b, S);
    st3(q.dbl + D_D0 * cap, cap, b, a);
    st3(q.dbl + D_D1 * cap, cap, b, bb);
    st3(q.dbl + D_D2 * cap, cap, b, c);
    st3(q.dbl + D_O * cap, cap, b, S);
    st3(q.dbl + D_C * cap, cap, b, cc);
    q.flt[F_K * cap + b] = (float)((double)power[s] / (4.0 * M_PI));
    q.flt[F_OMEGA * cap + b] = (float)omega;
    q.ints[I_ID * cap + b] = (int)b;
    q.ints[I_START * cap + b] = -1;
    q.ints[I_META * cap + b] = 0;
}

hipError_t launch_emit(const double *base20, const float *src, const float *power, int n_src, int level,
                       DevQueue q, hipStream_t s)
{
    long long nf = 20ll << (2 * level);
    long long total = nf * n_src;
    if (total <= 0) return hipSuccess;
    k_emit<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(base20, src, power, n_src, level, nf, q);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Traversal
// ---------------------------------------------------------------------------------------
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

struct RayState {
    V3 o, c;              // FP64 ray
    float ox, oy, oz;     // FP32 copies for box tests
    float ix, iy, iz;     // FP32 reciprocal direction (|c| clamped away from 0)
    int start;
    // result and flag candidates
    double best_t;
    int best_id;
    int best_near;        // hit point within delta of an edge, or t* - t_min < delta
    double c1_t, c2_t;    // two smallest candidate parameters
    int c1_id;
    unsigned node_visits, tri_tests;
};

// Distance from P to segment [a, b].
__device__ double seg_dist(V3 p, V3 a, V3 b)
{
    V3 ab = b - a, ap = p - a;
    double l2 = dot(ab, ab);
    double u = l2 > 0.0 ? dot(ap, ab) / l2 : 0.0;
    u = fmin(fmax(u, 0.0), 1.0);
    V3 q = a + u * ab;
    V3 r = p - q;
    return sqrt(dot(r, r));
}

// Exact signed boundary distance of the plane point (slow path, near an edge only).
__device__ double exact_signed_dist(const RayState &r, double t, double u, double v, double w, V3 v0, V3 v1, V3 v2)
{
    V3 e1 = v1 - v0, e2 = v2 - v0, e12 = v2 - v1;
    double a2 = sqrt(dot(cross(e1, e2), cross(e1, e2)));
    double s0 = w * a2 / sqrt(dot(e12, e12));
    double s1 = u * a2 / sqrt(dot(e2, e2));
    double s2 = v * a2 / sqrt(dot(e1, e1));
    double m = fmin(s0, fmin(s1, s2));
    if (m >= 0.0) return m;
    V3 P = r.o + t * r.c;
    double d = fmin(seg_dist(P, v0, v1), fmin(seg_dist(P, v1, v2), seg_dist(P, v2, v0)));
    return -d;
}

// Test the triangle references [first, first + count) over the tile window.
//   valid hit:   t in (hit_lo, t_hi], inside, better than the current best
//   candidate:   t in (cand_lo, t_hi], t < best_t + delta, within delta of the triangle
__device__ __forceinline__ void test_leaf(const float4 *__restrict__ tris, int first, int count, RayState &r,
                                          double hit_lo, double cand_lo, double t_hi, double t_min, double delta)
{
    for (int k = first; k < first + count; ++k) {
        float4 a = tris[3 * k], b = tris[3 * k + 1], cc = tris[3 * k + 2];
        int id = __float_as_int(cc.y);
        if (id == r.start) continue;
        r.tri_tests++;
        V3 v0 = {a.x, a.y, a.z}, v1 = {a.w, b.x, b.y}, v2 = {b.z, b.w, cc.x};
        V3 e1 = v1 - v0, e2 = v2 - v0;
        V3 p = cross(r.c, e2);
        double det = dot(e1, p);
        if (det == 0.0) continue;
        double inv = 1.0 / det;
        V3 T = r.o - v0;
        V3 q = cross(T, e1);
        double t = dot(e2, q) * inv;
        if (!(t > cand_lo && t <= t_hi && t < r.best_t + delta)) continue;
        double u = dot(T, p) * inv;
        double v = dot(r.c, q) * inv;
        double w = (1.0 - u) - v;
        double wmin = fmin(u, fmin(v, w));
        double hmin = (double)cc.z;
        double sd;
        if (wmin >= 0.0 && wmin * hmin >= delta) {
            sd = delta;  // inside and at least delta from every edge
        } else if (wmin < 0.0 && -wmin * hmin >= delta) {
            continue;    // outside by at least delta
        } else {
            sd = exact_signed_dist(r, t, u, v, w, v0, v1, v2);
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

__device__ __forceinline__ bool box2(const float4 &nx, const float4 &ny, const float4 &nz, const RayState &r,
                                     float tlo, float thi, float &t0, float &t1, bool &h0, bool &h1)
{
    // child 0
    float ax0 = (nx.x - r.ox) * r.ix, bx0 = (nx.z - r.ox) * r.ix;
    float ay0 = (ny.x - r.oy) * r.iy, by0 = (ny.z - r.oy) * r.iy;
    float az0 = (nz.x - r.oz) * r.iz, bz0 = (nz.z - r.oz) * r.iz;
    float mn0 = fmaxf(fmaxf(fminf(ax0, bx0), fminf(ay0, by0)), fmaxf(fminf(az0, bz0), tlo));
    float mx0 = fminf(fminf(fmaxf(ax0, bx0), fmaxf(ay0, by0)), fminf(fmaxf(az0, bz0), thi));
    // child 1
    float ax1 = (nx.y - r.ox) * r.ix, bx1 = (nx.w - r.ox) * r.ix;
    float ay1 = (ny.y - r.oy) * r.iy, by1 = (ny.w - r.oy) * r.iy;
    float az1 = (nz.y - r.oz) * r.iz, bz1 = (nz.w - r.oz) * r.iz;
    float mn1 = fmaxf(fmaxf(fminf(ax1, bx1), fminf(ay1, by1)), fmaxf(fminf(az1, bz1), tlo));
    float mx1 = fminf(fminf(fmaxf(ax1, bx1), fmaxf(ay1, by1)), fminf(fmaxf(az1, bz1), thi));
    h0 = mn0 <= mx0;
    h1 = mn1 <= mx1;
    t0 = mn0;
    t1 = mn1;
    return h0 || h1;
}

__device__ __forceinline__ bool box1(const float *bx, const RayState &r, float tlo, float thi)
{
    float ax = (bx[0] - r.ox) * r.ix, bxx = (bx[3] - r.ox) * r.ix;
    float ay = (bx[1] - r.oy) * r.iy, by = (bx[4] - r.oy) * r.iy;
    float az = (bx[2] - r.oz) * r.iz, bz = (bx[5] - r.oz) * r.iz;
    float mn = fmaxf(fmaxf(fminf(ax, bxx), fminf(ay, by)), fmaxf(fminf(az, bz), tlo));
    float mx = fminf(fminf(fmaxf(ax, bxx), fmaxf(ay, by)), fminf(fmaxf(az, bz), thi));
    return mn <= mx;
}

// Traverse one tile's hierarchy over the ray window (t_lo, t_hi].
__device__ void traverse_tile(const DevMesh &M, int tile, RayState &r, double t_lo, double t_hi, double t_min,
                              double delta, int *stk)
{
    int root = M.tile_root[tile];
    if (root == kEmptyRoot) return;
    const double hit_lo = fmax(t_lo, t_min);
    const double cand_lo = fmax(t_lo, t_min - delta);
    float flo = f32_down(cand_lo);
    float fhi = f32_up(fmin(t_hi, r.best_t + delta));
    if (!box1(M.tile_box + 6 * tile, r, flo, fhi)) return;
    const int bdim = blockDim.x;
    const int tid = threadIdx.x;
    int sp = 0;
    int ref = root;
    while (true) {
        if (ref >= 0) {
            const float4 *nd = M.nodes + 4 * (long long)ref;
            float4 nx = nd[0], ny = nd[1], nz = nd[2], nr = nd[3];
            r.node_visits++;
            float t0, t1;
            bool h0, h1;
            fhi = f32_up(fmin(t_hi, r.best_t + delta));
            box2(nx, ny, nz, r, flo, fhi, t0, t1, h0, h1);
            int c0 = __float_as_int(nr.x), c1 = __float_as_int(nr.y);
            if (h0 && h1) {
                int nearc = t0 <= t1 ? c0 : c1;
                int farc = t0 <= t1 ? c1 : c0;
                stk[sp * bdim + tid] = farc;
                sp++;
                ref = nearc;
                continue;
            } else if (h0) {
                ref = c0;
                continue;
            } else if (h1) {
                ref = c1;
                continue;
            }
        } else {
            int v = ~ref;
            test_leaf(M.tris, v >> 3, v & 7, r, hit_lo, cand_lo, t_hi, t_min, delta);
        }
        if (sp == 0) break;
        sp--;
        ref = stk[sp * bdim + tid];
    }
}

// Walk the tiles crossed by the ray in order and traverse each over its window.
__device__ void trace_ray(const DevMesh &M, RayState &r, double t_min, double delta, int *stk)
{
    // parameter range of the ray inside the grid footprint and the z slab
    double te = -INFINITY, tx = INFINITY;
    bool ok = true;
    {
        const double o3[3] = {r.o.x, r.o.y, r.o.z}, c3[3] = {r.c.x, r.c.y, r.c.z};
        const double lo3[3] = {M.gx0, M.gy0, M.zmin}, hi3[3] = {M.gx1, M.gy1, M.zmax};
        for (int k = 0; k < 3; ++k) {
            if (c3[k] != 0.0) {
                double ta = (lo3[k] - o3[k]) / c3[k], tb = (hi3[k] - o3[k]) / c3[k];
                te = fmax(te, fmin(ta, tb));
                tx = fmin(tx, fmax(ta, tb));
            } else if (o3[k] < lo3[k] || o3[k] > hi3[k]) {
                ok = false;
            }
        }
    }
    double t_start = fmax(te, t_min - delta);
    if (!ok || !(t_start <= tx)) return;
    int ix, iy;
    {
        double px = r.o.x + t_start * r.c.x, py = r.o.y + t_start * r.c.y;
        ix = (int)floor((px - M.gx0) / M.tw);
        iy = (int)floor((py - M.gy0) / M.th);
        ix = ix < 0 ? 0 : (ix >= M.tiles_x ? M.tiles_x - 1 : ix);
        iy = iy < 0 ? 0 : (iy >= M.tiles_y ? M.tiles_y - 1 : iy);
    }
    const int sx = r.c.x > 0.0 ? 1 : (r.c.x < 0.0 ? -1 : 0);
    const int sy = r.c.y > 0.0 ? 1 : (r.c.y < 0.0 ? -1 : 0);
    auto next_x = [&](int i) -> double {
        if (sx == 0) return INFINITY;
        double X = M.gx0 + (double)(sx > 0 ? i + 1 : i) * M.tw;
        return (X - r.o.x) / r.c.x;
    };
    auto next_y = [&](int j) -> double {
        if (sy == 0) return INFINITY;
        double Y = M.gy0 + (double)(sy > 0 ? j + 1 : j) * M.th;
        return (Y - r.o.y) / r.c.y;
    };
    double tnx = M.tiles_x > 1 ? next_x(ix) : INFINITY;
    double tny = M.tiles_y > 1 ? next_y(iy) : INFINITY;
    double t_lo = t_start;
    for (int guard = 0; guard < 4 * (M.tiles_x + M.tiles_y) + 4; ++guard) {
        double t_hi = fmin(fmin(tnx, tny), tx);
        if (t_hi > t_lo) traverse_tile(M, iy * M.tiles_x + ix, r, t_lo, t_hi, t_min, delta, stk);
        if (t_hi >= tx) break;
        if (t_hi >= r.best_t + delta) break;
        bool stepx = tnx <= tny, stepy = tny <= tnx;
        if (stepx) {
            ix += sx;
            tnx = (ix >= 0 && ix < M.tiles_x - 1 && sx > 0) || (ix > 0 && ix < M.tiles_x && sx < 0) ? next_x(ix)
                                                                                                   : INFINITY;
        }
        if (stepy) {
            iy += sy;
            tny = (iy >= 0 && iy < M.tiles_y - 1 && sy > 0) || (iy > 0 && iy < M.tiles_y && sy < 0) ? next_y(iy)
                                                                                                   : INFINITY;
        }
        if (ix < 0 || ix >= M.tiles_x || iy < 0 || iy >= M.tiles_y) break;
        t_lo = t_hi;
    }
}

__global__ void __launch_bounds__(256) k_trace(DevMesh M, DevQueue in, DevQueue out, DevSegs segs,
                                               DevCounters *ctr, TraceArgs a)
{
    __shared__ int stk[kStack * 256];
    const unsigned long long n = ctr->count[a.gen];
    const int lane = lane_id();
    const long long icap = in.cap, ocap = out.cap;
    const int D1 = a.max_depth + 1;
    while (true) {
        unsigned long long base = wave_grab(&ctr->work_trace[a.gen]);
        if (base >= n) break;
        long long i = (long long)base + lane;
        bool active = i < (long long)n;
        int child = 0;
        int flag_total = 0;
        double power_term = 0.0;
        unsigned nv = 0, tt = 0;
        // beam state needed by the epilogue
        V3 A, d0, d1, d2;
        int meta = 0, id = 0, depth = 0;
        float K = 0.f, om = 0.f;
        RayState r;
        if (active) {
            r.o = ld3(in.dbl + D_O * icap, icap, i);
            r.c = ld3(in.dbl + D_C * icap, icap, i);
            r.start = in.ints[I_START * icap + i];
            meta = in.ints[I_META * icap + i];
            id = in.ints[I_ID * icap + i];
            K = in.flt[F_K * icap + i];
            om = in.flt[F_OMEGA * icap + i];
            depth = meta & 0xff;
            r.ox = (float)r.o.x;
            r.oy = (float)r.o.y;
            r.oz = (float)r.o.z;
            const double tiny = 1e-20;
            double cx = fabs(r.c.x) < tiny ? copysign(tiny, r.c.x) : r.c.x;
            double cy = fabs(r.c.y) < tiny ? copysign(tiny, r.c.y) : r.c.y;
            double cz = fabs(r.c.z) < tiny ? copysign(tiny, r.c.z) : r.c.z;
            r.ix = (float)(1.0 / cx);
            r.iy = (float)(1.0 / cy);
            r.iz = (float)(1.0 / cz);
            r.best_t = INFINITY;
            r.best_id = -1;
            r.best_near = 0;
            r.c1_t = INFINITY;
            r.c2_t = INFINITY;
            r.c1_id = -1;
            r.node_visits = 0;
            r.tri_tests = 0;
            trace_ray(M, r, a.t_min, a.delta, stk);
            int hit = r.best_id;
            int own_flag;
            if (hit >= 0) own_flag = r.best_near || (r.c1_id != hit) || (r.c2_t < r.best_t + a.delta);
            else own_flag = r.c1_t < INFINITY;
            flag_total = ((meta & kMetaFlag) != 0) || own_flag;
            segs.hit[i] = hit;
            segs.t[i] = r.best_t;
            segs.flag[i] = flag_total;
            long long oidx = (long long)id * D1 + a.gen;
            if (a.hit_out) a.hit_out[oidx] = hit;
            if (a.flag_out) a.flag_out[oidx] = (uint8_t)flag_total;
            if (a.t_out) a.t_out[oidx] = r.best_t;
            power_term = (double)K * (double)om;
            nv = r.node_visits;
            tt = r.tri_tests;
            if (hit >= 0 && depth < a.max_depth) {
                float Kc = K * (1.0f - M.alpha[hit]);
                child = !(a.e_min > 0.0) || ((double)Kc * (double)om > a.e_min);
            }
            if (child) {
                A = ld3(in.dbl + D_A * icap, icap, i);
                d0 = ld3(in.dbl + D_D0 * icap, icap, i);
                d1 = ld3(in.dbl + D_D1 * icap, icap, i);
                d2 = ld3(in.dbl + D_D2 * icap, icap, i);
            }
        }
        // wave-aggregated counters
        unsigned long long fl = wave_sum_u64((unsigned long long)(active && flag_total));
        double pw = wave_sum_f64(power_term);
        unsigned long long snv = wave_sum_u64(nv), stt = wave_sum_u64(tt);
        // wave-aggregated append of children into the next generation
        unsigned long long mask = __ballot(child);
        unsigned long long obase = 0;
        if (lane == 0) {
            if (fl) atomicAdd(&ctr->flagged[a.gen], fl);
            atomicAdd(&ctr->power[a.gen], pw);
            atomicAdd(&ctr->node_visits, snv);
            atomicAdd(&ctr->tri_tests, stt);
            if (mask) obase = atomicAdd(&ctr->count[a.gen + 1], (unsigned long long)__popcll(mask));
        }
        obase = __shfl(obase, 0, 64);
        if (child) {
            long long j = (long long)obase + __popcll(mask & ((1ull << lane) - 1ull));
            int hit = r.best_id;
            V3 v0, v1, v2;
            tri_vertices(M.tri_g, hit, v0, v1, v2);
            V3 N = cross(v1 - v0, v2 - v0);
            V3 nn = unit(N);
            V3 Ac = A - (2.0 * dot(A - v0, nn)) * nn;
            V3 oc = r.o + r.best_t * r.c;
            st3(out.dbl + D_A * ocap, ocap, j, Ac);
            st3(out.dbl + D_D0 * ocap, ocap, j, mirror(d0, nn));
            st3(out.dbl + D_D1 * ocap, ocap, j, mirror(d2, nn));  // swap restores orientation
            st3(out.dbl + D_D2 * ocap, ocap, j, mirror(d1, nn));
            st3(out.dbl + D_O * ocap, ocap, j, oc);
            st3(out.dbl + D_C * ocap, ocap, j, mirror(r.c, nn));
            out.flt[F_K * ocap + j] = K * (1.0f - M.alpha[hit]);
            out.flt[F_OMEGA * ocap + j] = om;
            out.ints[I_ID * ocap + j] = id;
            out.ints[I_START * ocap + j] = hit;
            int neg_near = dot(r.c, N) > 0.0;  // the child lives on the side the parent came from
            out.ints[I_META * ocap + j] = (depth + 1) | (neg_near ? kMetaNegNear : 0) | (flag_total ? kMetaFlag : 0);
        }
    }
}

hipError_t launch_trace(const DevMesh &m, DevQueue in, DevQueue out, DevSegs segs, DevCounters *ctr,
                        const TraceArgs &a, int n_cu, hipStream_t s)
{
    int blocks = n_cu * 8;
    k_trace<<<blocks, 256, 0, s>>>(m, in, out, segs, ctr, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Microphones
//
// A segment's frustum meets the microphone plane z = zm in a convex polygon: three side
// half-planes through the (image) apex, the reflecting plane (outgoing side, strict) and
// the hit plane (incoming side, closed).  The kernels first bound the polygon's rows,
// then enumerate candidate microphones row by row (one column of slack on each side)
// and decide membership with the exact plane tests.
//   k_mics:      one lane per segment; footprints of <= kInlineRows rows are finished
//                in place, wider ones are split into (segment, row) work items
//   k_mic_rows:  one lane per (segment, row) work item
//   k_mics_big:  one wave per segment, for segments whose rows did not fit the item
//                buffer (overflow fallback)
// ---------------------------------------------------------------------------------------
struct Frustum {
    V3 A;
    V3 n[3];
    double amb2[3];     // delta^2 |n_k|^2: |s| < delta |n| <=> s^2 < amb2
    bool has_near, has_far;
    V3 Nn, Pn;
    double near_sign, amb2_near;
    V3 Nf, Pf;
    double far_sign, amb2_far;
    float K;
    int flag;
};

struct HalfPlane {
    double a, b, k;  // a x + b y + k >= 0 on the microphone plane
};

__device__ __forceinline__ bool lex_positive(V3 n)
{
    if (n.x != 0.0) return n.x > 0.0;
    if (n.y != 0.0) return n.y > 0.0;
    return n.z > 0.0;
}

// Keep-side half-plane g . (p - P) >= 0 on z = zm, relaxed by eps * |g|_1 (>= eps |g|).
__device__ __forceinline__ HalfPlane make_hp(V3 g, V3 P, double z, double eps)
{
    HalfPlane h;
    h.a = g.x;
    h.b = g.y;
    h.k = g.z * (z - P.z) - g.x * P.x - g.y * P.y + eps * (fabs(g.x) + fabs(g.y) + fabs(g.z));
    return h;
}

__device__ void load_frustum(const DevMesh &M, const DevQueue &q, const DevSegs &segs, long long i, double delta,
                             Frustum &f)
{
    const long long cap = q.cap;
    const double d2 = delta * delta;
    f.A = ld3(q.dbl + D_A * cap, cap, i);
    V3 d[3] = {ld3(q.dbl + D_D0 * cap, cap, i), ld3(q.dbl + D_D1 * cap, cap, i), ld3(q.dbl + D_D2 * cap, cap, i)};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        f.n[k] = cross(d[k], d[(k + 1) % 3]);
        f.amb2[k] = d2 * dot(f.n[k], f.n[k]);
    }
    int meta = q.ints[I_META * cap + i];
    int start = q.ints[I_START * cap + i];
    int hit = segs.hit[i];
    f.K = q.flt[F_K * cap + i];
    f.flag = segs.flag[i];
    f.has_near = (meta & 0xff) > 0;
    if (f.has_near) {
        V3 v0, v1, v2;
        tri_vertices(M.tri_g, start, v0, v1, v2);
        f.Nn = cross(v1 - v0, v2 - v0);
        f.Pn = v0;
        f.near_sign = (meta & kMetaNegNear) ? -1.0 : 1.0;
        f.amb2_near = d2 * dot(f.Nn, f.Nn);
    }
    f.has_far = hit >= 0;
    if (f.has_far) {
        V3 v0, v1, v2;
        tri_vertices(M.tri_g, hit, v0, v1, v2);
        f.Nf = cross(v1 - v0, v2 - v0);
        f.Pf = v0;
        V3 c = ld3(q.dbl + D_C * cap, cap, i);
        f.far_sign = dot(c, f.Nf) > 0.0 ? 1.0 : -1.0;
        f.amb2_far = d2 * dot(f.Nf, f.Nf);
    }
}

// The frustum's half-planes plus the grid rectangle (grown by half a cell) as 9 lines;
// unused slots are the always-true constraint 0 x + 0 y + 1 >= 0.
__device__ __forceinline__ void footprint_lines(const Frustum &f, const DevMics &mc, HalfPlane *L)
{
    const double eps = 1e-6;
#pragma unroll
    for (int k = 0; k < 3; ++k) L[k] = make_hp(f.n[k], f.A, mc.z, eps);
    L[3] = f.has_near ? make_hp(f.near_sign * f.Nn, f.Pn, mc.z, eps) : HalfPlane{0.0, 0.0, 1.0};
    L[4] = f.has_far ? make_hp((-f.far_sign) * f.Nf, f.Pf, mc.z, eps) : HalfPlane{0.0, 0.0, 1.0};
    double xlo = mc.x0 - 0.5 * mc.dx, xhi = mc.x0 + ((double)mc.nx - 0.5) * mc.dx;
    double ylo = mc.y0 - 0.5 * mc.dy, yhi = mc.y0 + ((double)mc.ny - 0.5) * mc.dy;
    L[5] = HalfPlane{1.0, 0.0, -xlo};
    L[6] = HalfPlane{-1.0, 0.0, xhi};
    L[7] = HalfPlane{0.0, 1.0, -ylo};
    L[8] = HalfPlane{0.0, -1.0, yhi};
}

// Row range of the footprint polygon: every constraint line is clipped by all the
// others (parametrically, comparing fractions without dividing); the endpoints of the
// surviving edges bound the polygon's y-extent.  One row of slack on each side.
__device__ bool footprint_rows(const HalfPlane *L, const DevMics &mc, int &j0, int &j1)
{
    double ymn = INFINITY, ymx = -INFINITY;
#pragma unroll
    for (int h = 0; h < 9; ++h) {
        const double a = L[h].a, b = L[h].b, k = L[h].k;
        const double nn = a * a + b * b;
        if (nn == 0.0) continue;
        const double px = -k * a / nn, py = -k * b / nn;  // point on the line
        const double dx = -b, dy = a;                     // direction along it
        // t >= lo_n / lo_d and t <= hi_n / hi_d with positive denominators
        double lo_n = -1.0, lo_d = 0.0, hi_n = 1.0, hi_d = 0.0;  // -inf, +inf
        bool empty = false;
#pragma unroll
        for (int g = 0; g < 9; ++g) {
            if (g == h) continue;
            const double den = L[g].a * dx + L[g].b * dy;
            const double num = -(L[g].a * px + L[g].b * py + L[g].k);  // need den * t >= num
            if (den > 0.0) {
                if (lo_d == 0.0 || num * lo_d > lo_n * den) { lo_n = num; lo_d = den; }
            } else if (den < 0.0) {
                if (hi_d == 0.0 || (-num) * hi_d < hi_n * (-den)) { hi_n = -num; hi_d = -den; }
            } else if (num > 0.0) {
                empty = true;
            }
        }
        if (empty || lo_d == 0.0 || hi_d == 0.0) continue;  // (bounded by the rectangle otherwise)
        const double tlo = lo_n / lo_d, thi = hi_n / hi_d;
        if (!(tlo <= thi)) continue;
        const double y0 = py + tlo * dy, y1 = py + thi * dy;
        ymn = fmin(ymn, fmin(y0, y1));
        ymx = fmax(ymx, fmax(y0, y1));
    }
    if (!(ymn <= ymx)) return false;
    double fj0 = ceil((ymn - mc.y0) / mc.dy) - 1.0, fj1 = floor((ymx - mc.y0) / mc.dy) + 1.0;
    fj0 = fmax(fj0, 0.0);
    fj1 = fmin(fj1, (double)(mc.ny - 1));
    if (!(fj0 <= fj1)) return false;
    j0 = (int)fj0;
    j1 = (int)fj1;
    return true;
}

// Column range of row j inside the relaxed frustum half-planes (one column of slack).
__device__ __forceinline__ bool row_cols(const HalfPlane *L, const DevMics &mc, int j, int &i0, int &i1)
{
    const double y = mc.y0 + (double)j * mc.dy;
    double lo = -INFINITY, hi = INFINITY;
#pragma unroll
    for (int h = 0; h < 5; ++h) {
        const double rest = L[h].b * y + L[h].k;
        if (L[h].a > 0.0) lo = fmax(lo, -rest / L[h].a);
        else if (L[h].a < 0.0) hi = fmin(hi, -rest / L[h].a);
        else if (rest < 0.0) return false;
    }
    if (!(lo <= hi)) return false;
    const double flo = (lo - mc.x0) / mc.dx, fhi = (hi - mc.x0) / mc.dx;
    if (flo > (double)mc.nx || fhi < -1.0) return false;
    const double a0 = fmax(ceil(flo) - 1.0, 0.0), a1 = fmin(floor(fhi) + 1.0, (double)(mc.nx - 1));
    if (!(a0 <= a1)) return false;
    i0 = (int)a0;
    i1 = (int)a1;
    return true;
}

// Membership of grid microphone (i, j) and its contribution; returns 1 if accumulated.
// Ambiguous: every active test passes within -delta and one is within delta of its plane.
__device__ __forceinline__ int mic_apply(const Frustum &f, const DevMics &mc, int i, int j, double air_m)
{
    const V3 m = {mc.x0 + (double)i * mc.dx, mc.y0 + (double)j * mc.dy, mc.z};
    const V3 r = m - f.A;
    bool inside = true, far_out = false, near_any = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double s = dot(f.n[k], r);
        inside = inside && (s > 0.0 || (s == 0.0 && lex_positive(f.n[k])));
        const double s2 = s * s;
        far_out = far_out || (s < 0.0 && s2 >= f.amb2[k]);
        near_any = near_any || s2 < f.amb2[k];
    }
    if (f.has_near) {
        const double s = f.near_sign * dot(f.Nn, m - f.Pn);
        inside = inside && s > 0.0;
        const double s2 = s * s;
        far_out = far_out || (s < 0.0 && s2 >= f.amb2_near);
        near_any = near_any || s2 < f.amb2_near;
    }
    if (f.has_far) {
        const double s = -f.far_sign * dot(f.Nf, m - f.Pf);
        inside = inside && s >= 0.0;
        const double s2 = s * s;
        far_out = far_out || (s < 0.0 && s2 >= f.amb2_far);
        near_any = near_any || s2 < f.amb2_far;
    }
    if (!inside) return 0;
    const double d2 = dot(r, r);
    float e = f.K / (float)d2;
    if (air_m > 0.0) e *= expf(-(float)(air_m * sqrt(d2)));
    const bool amb = !far_out && near_any;
    const long long idx = (long long)j * mc.nx + i;
    atomicAdd((f.flag || amb) ? &mc.e_flag[idx] : &mc.e_strict[idx], (double)e);
    return 1;
}

constexpr int kInlineRows = 4;

__device__ __forceinline__ void flush_mic_counters(DevCounters *ctr, unsigned tests, unsigned updates)
{
    unsigned long long st = wave_sum_u64(tests), su = wave_sum_u64(updates);
    if (lane_id() == 0) {
        if (st) atomicAdd(&ctr->mic_tests, st);
        if (su) atomicAdd(&ctr->mic_updates, su);
    }
}

__global__ void __launch_bounds__(256) k_mics(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr, DevMics mc,
                                              TraceArgs a, MicWork w)
{
    const unsigned long long n = ctr->count[a.gen];
    const int lane = lane_id();
    while (true) {
        const unsigned long long base = wave_grab(&ctr->work_mic[a.gen]);
        if (base >= n) break;
        const long long i = (long long)base + lane;
        unsigned tests = 0, updates = 0;
        int nrows = 0, j0 = 0, j1 = -1;
        bool wide = false;
        if (i < (long long)n) {
            Frustum f;
            load_frustum(M, q, segs, i, a.delta, f);
            HalfPlane L[9];
            footprint_lines(f, mc, L);
            if (footprint_rows(L, mc, j0, j1)) {
                nrows = j1 - j0 + 1;
                if (nrows <= kInlineRows) {
                    for (int j = j0; j <= j1; ++j) {
                        int c0, c1;
                        if (!row_cols(L, mc, j, c0, c1)) continue;
                        for (int c = c0; c <= c1; ++c) {
                            tests++;
                            updates += mic_apply(f, mc, c, j, a.air_m);
                        }
                    }
                } else {
                    wide = true;
                }
            }
        }
        // wide footprints: reserve one work item per row (wave-aggregated)
        const int want = wide ? nrows : 0;
        int incl = want;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        const int total = __shfl(incl, 63, 64);
        unsigned long long rbase = 0;
        if (lane == 0 && total > 0) rbase = atomicAdd(&ctr->n_rows[a.gen], (unsigned long long)total);
        rbase = __shfl(rbase, 0, 64);
        bool to_big = false;
        if (wide) {
            const unsigned long long first = rbase + (unsigned long long)(incl - want);
            if (first + (unsigned long long)want <= (unsigned long long)w.rows_cap) {
                for (int r = 0; r < want; ++r) w.rows[first + r] = make_int2((int)i, j0 + r);
            } else {
                // does not fit: the whole segment goes to the wave path; slots of its
                // reservation that lie inside the buffer are marked empty
                for (unsigned long long r = first; r < (unsigned long long)w.rows_cap; ++r)
                    w.rows[r] = make_int2(-1, 0);
                to_big = true;
            }
        }
        const unsigned long long bm = __ballot(to_big);
        unsigned long long bbase = 0;
        if (lane == 0 && bm) bbase = atomicAdd(&ctr->n_big[a.gen], (unsigned long long)__popcll(bm));
        bbase = __shfl(bbase, 0, 64);
        if (to_big) w.big_list[bbase + __popcll(bm & ((1ull << lane) - 1ull))] = (int)i;
        flush_mic_counters(ctr, tests, updates);
    }
}

__global__ void __launch_bounds__(256) k_mic_rows(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr, DevMics mc,
                                                  TraceArgs a, MicWork w)
{
    unsigned long long n = ctr->n_rows[a.gen];
    if (n > (unsigned long long)w.rows_cap) n = (unsigned long long)w.rows_cap;
    while (true) {
        const unsigned long long base = wave_grab(&ctr->work_rows[a.gen]);
        if (base >= n) break;
        const unsigned long long r = base + (unsigned long long)lane_id();
        unsigned tests = 0, updates = 0;
        const int2 it = r < n ? w.rows[r] : make_int2(-1, 0);
        if (it.x >= 0) {
            Frustum f;
            load_frustum(M, q, segs, it.x, a.delta, f);
            HalfPlane L[9];
            footprint_lines(f, mc, L);
            int c0, c1;
            if (row_cols(L, mc, it.y, c0, c1)) {
                for (int c = c0; c <= c1; ++c) {
                    tests++;
                    updates += mic_apply(f, mc, c, it.y, a.air_m);
                }
            }
        }
        flush_mic_counters(ctr, tests, updates);
    }
}

__global__ void __launch_bounds__(256) k_mics_big(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr,
                                                  DevMics mc, TraceArgs a, MicWork w)
{
    const unsigned long long n = ctr->n_big[a.gen];
    const int lane = lane_id();
    const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int n_waves = (int)((gridDim.x * blockDim.x) >> 6);
    for (unsigned long long s = (unsigned long long)wave; s < n; s += (unsigned long long)n_waves) {
        const long long i = w.big_list[s];
        Frustum f;
        load_frustum(M, q, segs, i, a.delta, f);
        HalfPlane L[9];
        footprint_lines(f, mc, L);
        int j0, j1;
        unsigned tests = 0, updates = 0;
        if (footprint_rows(L, mc, j0, j1)) {
            for (int j = j0 + lane; j <= j1; j += 64) {
                int c0, c1;
                if (!row_cols(L, mc, j, c0, c1)) continue;
                for (int c = c0; c <= c1; ++c) {
                    tests++;
                    updates += mic_apply(f, mc, c, j, a.air_m);
                }
            }
        }
        flush_mic_counters(ctr, tests, updates);
    }
}

hipError_t launch_mics(const DevMesh &m, DevQueue q, DevSegs segs, DevCounters *ctr, DevMics mics,
                       const TraceArgs &a, MicWork w, int n_cu, hipStream_t s)
{
    k_mics<<<n_cu * 8, 256, 0, s>>>(m, q, segs, ctr, mics, a, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_mic_rows<<<n_cu * 8, 256, 0, s>>>(m, q, segs, ctr, mics, a, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_mics_big<<<n_cu * 4, 256, 0, s>>>(m, q, segs, ctr, mics, a, w);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Levels: L = 10 log10((strict + flag) / 1e-12)
// ---------------------------------------------------------------------------------------
__global__ void k_levels(const double *es, const double *ef, double *level, long long n)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double e = es[i] + ef[i];
    level[i] = e > 0.0 ? 10.0 * log10(e / 1e-12) : -INFINITY;
}

hipError_t launch_levels(const double *es, const double *ef, double *level, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_levels<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(es, ef, level, n);
    return hipGetLastError();
}

}  // namespace bt
