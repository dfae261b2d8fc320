// Host side of the C ABI declared in include/bt.h: contexts, validation, the per-tile
// BVH build, queue management and kernel sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bt.h"
#include "bt_host.h"

using namespace bt;

// ---------------------------------------------------------------------------------------
// errors and memory
// ---------------------------------------------------------------------------------------
bt_status fail(bt_ctx *ctx, bt_status s, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return s;
}

static bt_status why(std::string &msg, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    msg = buf;
    return BT_EINVAL;
}

bt_status check_mesh_args(const float *xyz, int64_t n_vert, const int32_t *tri, const float *absorption, int64_t n_tri,
                          int32_t tiles_x, int32_t tiles_y, std::string &msg)
{
    if (n_vert < 0 || n_tri < 0 || n_tri > (1ll << 27))
        return why(msg, "bad sizes n_vert=%lld n_tri=%lld", (long long)n_vert, (long long)n_tri);
    if (n_tri > 0 && (!xyz || !tri || !absorption)) return why(msg, "NULL mesh array");
    if (tiles_x < 1 || tiles_y < 1 || tiles_x > 64 || tiles_y > 64)
        return why(msg, "tiles must be in 1..64 (got %d x %d)", tiles_x, tiles_y);
    for (int64_t t = 0; t < n_tri; ++t) {
        double v[3][3];
        for (int k = 0; k < 3; ++k) {
            const int32_t id = tri[3 * t + k];
            if (id < 0 || id >= n_vert) return why(msg, "triangle %lld has vertex index %d out of range", (long long)t, id);
            for (int c = 0; c < 3; ++c) {
                const float x = xyz[3 * (int64_t)id + c];
                if (!std::isfinite(x)) return why(msg, "vertex %d is not finite", id);
                v[k][c] = x;
            }
        }
        const float a = absorption[t];
        if (!(a >= 0.0f && a <= 1.0f)) return why(msg, "absorption of triangle %lld not in [0, 1]", (long long)t);
        double e1[3], e2[3];
        for (int c = 0; c < 3; ++c) { e1[c] = v[1][c] - v[0][c]; e2[c] = v[2][c] - v[0][c]; }
        const double nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2];
        const double nz = e1[0] * e2[1] - e1[1] * e2[0];
        if (!(nx * nx + ny * ny + nz * nz > 0.0)) return why(msg, "triangle %lld has zero area", (long long)t);
    }
    return BT_OK;
}

bt_status check_source_args(const float *src_xyz, const float *src_power, const float *src_weight, int32_t n_src,
                            int32_t level, bool two_slot, std::string &msg)
{
    if (n_src < 0 || (n_src > 0 && (!src_xyz || !src_power))) return why(msg, "bad sources");
    if (level < 0 || level > BT_MAX_LEVEL) return why(msg, "level %d not in 0..%d", level, BT_MAX_LEVEL);
    const long long nf = 20ll << (2 * level);
    const long long n0 = nf * n_src;
    if (n0 * (two_slot ? 2 : 1) > (1ll << 31) - 1) return why(msg, "too many beams (%lld)", n0);
    if (src_weight)
        for (long long k = 0; k < n0; ++k)
            if (!(src_weight[k] >= 0.f) || !std::isfinite(src_weight[k]))
                return why(msg, "weight %lld (source %lld, face %lld) invalid", k, k / nf, k % nf);
    for (int i = 0; i < n_src; ++i) {
        for (int c = 0; c < 3; ++c)
            if (!std::isfinite(src_xyz[3 * i + c])) return why(msg, "source %d not finite", i);
        if (!(src_power[i] >= 0.f) || !std::isfinite(src_power[i])) return why(msg, "source %d power invalid", i);
    }
    return BT_OK;
}

bt_status check_grid_args(float x0, float y0, float z0, float dx, float dy, float dz, int32_t nx, int32_t ny,
                          int32_t nz, std::string &msg)
{
    if (nx < 1 || ny < 1 || nz < 1 || (int64_t)nx * ny * nz > (1ll << 31))
        return why(msg, "bad microphone grid %d x %d x %d", nx, ny, nz);
    if (nz > 1 && (nx >= (1 << 24) || ny >= (1 << 24) || nz >= (1 << 25)))  // FP32-exact lattice indices;
        return why(msg, "volumetric grid %d x %d x %d: nx, ny must be below 2^24 and nz below 2^25", nx, ny,
                   nz);  // layer numbers packed beside 6-bit slots
    if (!std::isfinite(x0) || !std::isfinite(y0) || !std::isfinite(z0) || !(dx > 0.f) || !(dy > 0.f) ||
        !std::isfinite(dx) || !std::isfinite(dy) || (nz > 1 && (!(dz > 0.f) || !std::isfinite(dz))))
        return why(msg, "bad microphone grid geometry");
    return BT_OK;
}

bt_status check_param_args(const bt_params *p, double delta_cap, std::string &msg)
{
    if (!p) return why(msg, "params is NULL");
    if (p->max_depth < 0 || p->max_depth > BT_MAX_DEPTH)
        return why(msg, "max_depth %d not in 0..%d", p->max_depth, BT_MAX_DEPTH);
    if (!(p->t_min >= 0.0) || !std::isfinite(p->t_min)) return why(msg, "t_min invalid");
    if (!(p->edge_delta >= 0.0) || !(p->edge_delta <= delta_cap)) return why(msg, "edge_delta must be in [0, %g]", delta_cap);
    if (!(p->air_m >= 0.0) || !std::isfinite(p->air_m)) return why(msg, "air_m invalid");
    if (!(p->e_min >= 0.0)) return why(msg, "e_min invalid");
    if (p->queue_rounds < 0 || p->queue_rounds > kMaxQueueRounds)
        return why(msg, "queue_rounds %d not in 0..%d", p->queue_rounds, kMaxQueueRounds);
    if (p->run_records < 0 || p->run_records > (1ll << 31) - 1)
        return why(msg, "run_records %lld not in 0..2^31 - 1", (long long)p->run_records);
    return BT_OK;
}

static bt_status to_caller(bt_status s, const std::string &msg, char *out, size_t out_len)
{
    if (out && out_len > 0) {
        const size_t n = std::min(out_len - 1, msg.size());
        std::memcpy(out, msg.data(), n);
        out[n] = 0;
    }
    return s;
}

extern "C" bt_status bt_validate_mesh(const float *xyz, int64_t n_vert, const int32_t *tri, const float *absorption,
                                      int64_t n_tri, int32_t tiles_x, int32_t tiles_y, char *msg, size_t msg_len)
{
    std::string m;
    return to_caller(check_mesh_args(xyz, n_vert, tri, absorption, n_tri, tiles_x, tiles_y, m), m, msg, msg_len);
}

extern "C" bt_status bt_validate_sources(const float *src_xyz, const float *src_power, const float *src_weight,
                                         int32_t n_src, int32_t level, char *msg, size_t msg_len)
{
    std::string m;
    return to_caller(check_source_args(src_xyz, src_power, src_weight, n_src, level, false, m), m, msg, msg_len);
}

extern "C" bt_status bt_validate_grid(float x0, float y0, float z0, float dx, float dy, float dz, int32_t nx, int32_t ny,
                                      int32_t nz, char *msg, size_t msg_len)
{
    std::string m;
    return to_caller(check_grid_args(x0, y0, z0, dx, dy, dz, nx, ny, nz, m), m, msg, msg_len);
}

extern "C" bt_status bt_validate_params(const bt_params *p, char *msg, size_t msg_len)
{
    std::string m;
    return to_caller(check_param_args(p, kDeltaCap, m), m, msg, msg_len);
}

bt_status hip_fail(bt_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, BT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bt_status dev_alloc(bt_ctx *ctx, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    if (ctx->budget && ctx->used + bytes > ctx->budget)
        return fail(ctx, BT_ENOMEM, "HBM budget exceeded: %zu + %zu > %zu bytes", ctx->used, bytes, ctx->budget);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, BT_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    ctx->used += bytes;
    return BT_OK;
}

void dev_free(bt_ctx *ctx, void *p, size_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    if (bytes == 0) bytes = 256;
    if (ctx) ctx->used -= std::min(ctx->used, bytes);
}

// ---------------------------------------------------------------------------------------
// misc API
// ---------------------------------------------------------------------------------------
extern "C" void bt_params_default(bt_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->max_depth = 3;
    p->t_min = 1e-3;
    p->edge_delta = 1e-5;
    p->air_m = 0.0;
    p->e_min = 0.0;
    p->queue_rounds = 0;   // the in-lane walk measures faster on the district workload
}

extern "C" const char *bt_status_str(bt_status s)
{
    switch (s) {
    case BT_OK: return "ok";
    case BT_PENDING: return "pending";
    case BT_EINVAL: return "invalid argument";
    case BT_ENOMEM: return "out of memory / budget";
    case BT_EDEVICE: return "device error";
    case BT_EOVERFLOW: return "internal capacity exceeded";
    case BT_ENOTFOUND: return "not found";
    case BT_ESTATE: return "call out of order";
    }
    return "unknown status";
}

extern "C" const char *bt_last_error(const bt_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// The 20 base faces of the icosahedron used for beam directions: vertices are the cyclic
// permutations (0,a,b), (a,b,0), (b,0,a) of (0, +-1, +-phi) listed by permutation, then
// a, then b; faces are the vertex triples at mutual distance 2 in lexicographic order,
// oriented outward (det > 0) by swapping their last two vertices when needed.
static void icosahedron_faces(double out[20 * 9])
{
    const double phi = (1.0 + std::sqrt(5.0)) / 2.0;
    double raw[12][3], u[12][3];
    int nv = 0;
    for (int perm = 0; perm < 3; ++perm)
        for (double a : {-1.0, 1.0})
            for (double b : {-phi, phi}) {
                double x = perm == 0 ? 0.0 : (perm == 1 ? a : b);
                double y = perm == 0 ? a : (perm == 1 ? b : 0.0);
                double z = perm == 0 ? b : (perm == 1 ? 0.0 : a);
                raw[nv][0] = x; raw[nv][1] = y; raw[nv][2] = z;
                double n = std::sqrt(x * x + y * y + z * z);
                u[nv][0] = x / n; u[nv][1] = y / n; u[nv][2] = z / n;
                nv++;
            }
    auto d2 = [&](int i, int j) {
        double dx = raw[i][0] - raw[j][0], dy = raw[i][1] - raw[j][1], dz = raw[i][2] - raw[j][2];
        return dx * dx + dy * dy + dz * dz;
    };
    int nf = 0;
    for (int i = 0; i < 12; ++i)
        for (int j = i + 1; j < 12; ++j)
            for (int k = j + 1; k < 12; ++k) {
                if (std::fabs(d2(i, j) - 4.0) > 1e-9 || std::fabs(d2(j, k) - 4.0) > 1e-9 ||
                    std::fabs(d2(k, i) - 4.0) > 1e-9)
                    continue;
                const double *A = u[i], *B = u[j], *C = u[k];
                double det = A[0] * (B[1] * C[2] - B[2] * C[1]) + A[1] * (B[2] * C[0] - B[0] * C[2]) +
                             A[2] * (B[0] * C[1] - B[1] * C[0]);
                const double *f[3] = {A, det < 0.0 ? C : B, det < 0.0 ? B : C};
                for (int v = 0; v < 3; ++v)
                    for (int c = 0; c < 3; ++c) out[9 * nf + 3 * v + c] = f[v][c];
                nf++;
            }
}

extern "C" bt_status bt_create(int device, size_t hbm_budget_bytes, void *hip_stream, bt_ctx **out)
{
    if (!out) return BT_EINVAL;
    *out = nullptr;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev) {
        (void)hipGetLastError();
        return BT_EINVAL;
    }
    bt_ctx *ctx = new bt_ctx();
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) { delete ctx; return BT_EDEVICE; }
    // the device's static work area, looked up once per device with the device current
    if (static_scratch(device, &ctx->scratch) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return BT_EDEVICE;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        ctx->n_cu = ncu;
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) { delete ctx; return BT_EDEVICE; }
        ctx->own_stream = true;
    }
    double base[20 * 9];
    icosahedron_faces(base);
    if (dev_alloc(ctx, (void **)&ctx->base20, sizeof base) != BT_OK ||
        hipMemcpy(ctx->base20, base, sizeof base, hipMemcpyHostToDevice) != hipSuccess) {
        bt_destroy(ctx);
        return BT_EDEVICE;
    }
    *out = ctx;
    return BT_OK;
}

extern "C" bt_status bt_destroy(bt_ctx *ctx)
{
    if (!ctx) return BT_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto &kv : ctx->requests) {
        Request *r = kv.second;
        if (r->done) (void)hipEventDestroy(r->done);
        bt_mics_free(r->mics);
        bt_beams_free(r->beams);
        delete r;
    }
    batch_work_free(ctx);
    for (int l = 0; l <= BT_MAX_LEVEL; ++l) {
        const long long nf = 20ll << (2 * l);
        dev_free(ctx, ctx->face_dirs[l], (size_t)nf * 12 * sizeof(double));
        dev_free(ctx, ctx->face_om[l], (size_t)nf * sizeof(double));
    }
    dev_free(ctx, ctx->base20, 20 * 9 * sizeof(double));
    for (int k = 0; k < kMaxParts; ++k) {
        if (ctx->part_stream[k]) {
            (void)hipStreamSynchronize(ctx->part_stream[k]);
            (void)hipStreamDestroy(ctx->part_stream[k]);
        }
        if (ctx->join_ev[k]) (void)hipEventDestroy(ctx->join_ev[k]);
    }
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return BT_OK;
}

extern "C" bt_status bt_memory_used(const bt_ctx *ctx, size_t *bytes)
{
    if (!ctx || !bytes) return BT_EINVAL;
    *bytes = ctx->used;
    return BT_OK;
}

// ---------------------------------------------------------------------------------------
// BVH build (host): binned SAH over triangle boxes, 32 bins per axis, leaves of up to 2
// triangles (up to 7 where the SAH prefers a leaf or the depth limit forces one),
// flattened so each interior node holds both child boxes.
// ---------------------------------------------------------------------------------------
namespace {

struct Box {
    float lo[3], hi[3];
    void empty()
    {
        for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    }
    void grow(const Box &b)
    {
        for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], b.lo[k]); hi[k] = std::max(hi[k], b.hi[k]); }
    }
    double area() const
    {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = std::max(0.0, (double)hi[k] - (double)lo[k]);
        return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
    }
};

struct Prim {
    Box box;     // already grown by the margin
    float cen[3];
    int id;
};

struct Builder {
    std::vector<Prim> &prims;
    std::vector<float4> &nodes;   // 4 float4 per interior node
    std::vector<float4> &tris;    // 3 float4 per triangle reference
    const std::vector<float4> &tri_rec;  // per global triangle, 3 float4
    int max_depth = 0;
    bool overflow = false;

    static int leaf_ref(int first, int count) { return ~((first << 3) | count); }

    int make_leaf(int b, int e)
    {
        int first = (int)(tris.size() / 3);
        for (int i = b; i < e; ++i) {
            const float4 *t = &tri_rec[3 * (size_t)prims[i].id];
            tris.push_back(t[0]);
            tris.push_back(t[1]);
            tris.push_back(t[2]);
        }
        return leaf_ref(first, e - b);
    }

    Box range_box(int b, int e) const
    {
        Box bx;
        bx.empty();
        for (int i = b; i < e; ++i) bx.grow(prims[i].box);
        return bx;
    }

    // Returns the child reference of the subtree over prims[b, e).
    int build(int b, int e, int depth)
    {
        max_depth = std::max(max_depth, depth);
        int n = e - b;
        // two-triangle leaves: with leaves tested together by the wave, a deeper tree of
        // small leaves beat 1-, 4- and 7-triangle leaves on the district (measured)
        if (n <= 2) return make_leaf(b, e);
        if (depth >= kStack - 1) {
            if (n <= 7) return make_leaf(b, e);
            overflow = true;
            return make_leaf(b, b + 1);
        }
        float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int i = b; i < e; ++i)
            for (int k = 0; k < 3; ++k) { clo[k] = std::min(clo[k], prims[i].cen[k]); chi[k] = std::max(chi[k], prims[i].cen[k]); }
        enum { NB = 32 };
        double best = INFINITY;
        int best_axis = -1, best_bin = -1;
        for (int ax = 0; ax < 3; ++ax) {
            double ext = (double)chi[ax] - (double)clo[ax];
            if (!(ext > 0.0)) continue;
            Box bb[NB];
            int cnt[NB] = {0};
            for (int i = 0; i < NB; ++i) bb[i].empty();
            for (int i = b; i < e; ++i) {
                int k = (int)(((double)prims[i].cen[ax] - clo[ax]) / ext * NB);
                k = std::min(std::max(k, 0), NB - 1);
                cnt[k]++;
                bb[k].grow(prims[i].box);
            }
            double rarea[NB];
            int rcnt[NB];
            Box acc;
            acc.empty();
            int c = 0;
            for (int i = NB - 1; i >= 1; --i) {
                acc.grow(bb[i]);
                c += cnt[i];
                rarea[i] = acc.area();
                rcnt[i] = c;
            }
            acc.empty();
            c = 0;
            for (int i = 0; i < NB - 1; ++i) {
                acc.grow(bb[i]);
                c += cnt[i];
                if (c == 0 || rcnt[i + 1] == 0) continue;
                double cost = acc.area() * c + rarea[i + 1] * rcnt[i + 1];
                if (cost < best) { best = cost; best_axis = ax; best_bin = i + 1; }
            }
        }
        int mid;
        if (best_axis < 0) {
            mid = b + n / 2;
        } else {
            Box all = range_box(b, e);
            double leaf_cost = all.area() * n;
            if (n <= 7 && best >= leaf_cost) return make_leaf(b, e);
            double ext = (double)chi[best_axis] - (double)clo[best_axis];
            auto it = std::partition(prims.begin() + b, prims.begin() + e, [&](const Prim &p) {
                int k = (int)(((double)p.cen[best_axis] - clo[best_axis]) / ext * NB);
                k = std::min(std::max(k, 0), NB - 1);
                return k < best_bin;
            });
            mid = (int)(it - prims.begin());
            if (mid == b || mid == e) mid = b + n / 2;
        }
        int idx = (int)(nodes.size() / 4);
        nodes.resize(nodes.size() + 4);
        Box lb = range_box(b, mid), rb = range_box(mid, e);
        int l = build(b, mid, depth + 1);
        int r = build(mid, e, depth + 1);
        float4 *nd = &nodes[4 * (size_t)idx];
        nd[0] = make_float4(lb.lo[0], rb.lo[0], lb.hi[0], rb.hi[0]);
        nd[1] = make_float4(lb.lo[1], rb.lo[1], lb.hi[1], rb.hi[1]);
        nd[2] = make_float4(lb.lo[2], rb.lo[2], lb.hi[2], rb.hi[2]);
        float fl, fr;
        std::memcpy(&fl, &l, 4);
        std::memcpy(&fr, &r, 4);
        nd[3] = make_float4(fl, fr, 0.f, 0.f);
        return idx;
    }
};

// Collapse of a binary hierarchy (4 float4 per node) into a 4-wide one (8 float4 per
// node: lo x, hi x, lo y, hi y, lo z, hi z of the four children, their references, and
// padding).  A node takes its two children and keeps replacing the interior child with
// the largest box area by that child's two children until it has four or only leaves.
// Unused slots hold a box no ray window reaches and the empty reference.
struct Collapse {
    const std::vector<float4> &bin;
    std::vector<float4> &out;
    int max_push = 0;   // most entries the traversal stack can hold on any root-leaf path
    struct Child {
        float lo[3], hi[3];
        int ref;
    };
    static double area(const Child &c)
    {
        const double x = (double)c.hi[0] - c.lo[0], y = (double)c.hi[1] - c.lo[1], z = (double)c.hi[2] - c.lo[2];
        return x * y + y * z + z * x;
    }
    void children(int b, Child &l, Child &r) const
    {
        const float4 *nd = &bin[4 * (size_t)b];
        l.lo[0] = nd[0].x; r.lo[0] = nd[0].y; l.hi[0] = nd[0].z; r.hi[0] = nd[0].w;
        l.lo[1] = nd[1].x; r.lo[1] = nd[1].y; l.hi[1] = nd[1].z; r.hi[1] = nd[1].w;
        l.lo[2] = nd[2].x; r.lo[2] = nd[2].y; l.hi[2] = nd[2].z; r.hi[2] = nd[2].w;
        std::memcpy(&l.ref, &nd[3].x, 4);
        std::memcpy(&r.ref, &nd[3].y, 4);
    }
    std::vector<int> height;   // binary height of each binary node's subtree (leaf = 0)
    int height_of(int ref)
    {
        if (ref < 0) return 0;
        if (height[ref] >= 0) return height[ref];
        Child l, r;
        children(ref, l, r);
        return height[ref] = 1 + std::max(height_of(l.ref), height_of(r.ref));
    }
    // budget: stack entries still free on the way here; invariant: height_of(ref) <= budget
    // (a binary walk of the subtree pushes at most its height)
    int collapse(int ref, int pushed)
    {
        if (ref < 0) return ref;
        if (height.empty()) height.assign(bin.size() / 4, -1);
        const int budget = kStack - pushed;
        Child c[4];
        int n = 2;
        children(ref, c[0], c[1]);
        while (n < 4) {
            int best = -1;
            double ba = -1.0;
            for (int k = 0; k < n; ++k)
                if (c[k].ref >= 0 && area(c[k]) > ba) { ba = area(c[k]); best = k; }
            if (best < 0) break;
            Child a, b;
            children(c[best].ref, a, b);
            // one more child costs one more stack entry: take it only if every child's
            // subtree still fits the entries left below this node
            const int hmax = std::max({height_of(a.ref), height_of(b.ref), [&] {
                int h = 0;
                for (int k = 0; k < n; ++k) if (k != best) h = std::max(h, height_of(c[k].ref));
                return h;
            }()});
            if (hmax > budget - n) break;
            c[best] = a;
            c[n++] = b;
        }
        const int idx = (int)(out.size() / 8);
        out.resize(out.size() + 8);
        max_push = std::max(max_push, pushed + n - 1);
        int refs[4] = {kEmptyChild, kEmptyChild, kEmptyChild, kEmptyChild};
        for (int k = 0; k < n; ++k) refs[k] = collapse(c[k].ref, pushed + n - 1);
        float v[6][4];
        for (int k = 0; k < 4; ++k)
            for (int a = 0; a < 3; ++a) {
                v[2 * a][k] = k < n ? c[k].lo[a] : 1e30f;
                v[2 * a + 1][k] = k < n ? c[k].hi[a] : 1e30f;
            }
        float4 *nd = &out[8 * (size_t)idx];
        for (int q = 0; q < 6; ++q) nd[q] = make_float4(v[q][0], v[q][1], v[q][2], v[q][3]);
        float fr[4];
        std::memcpy(fr, refs, sizeof fr);
        nd[6] = make_float4(fr[0], fr[1], fr[2], fr[3]);
        nd[7] = make_float4(0.f, 0.f, 0.f, 0.f);
        return idx;
    }
};

float round_down_f(double x)
{
    float f = (float)x;
    if ((double)f > x) f = std::nextafter(f, -INFINITY);
    return f;
}
float round_up_f(double x)
{
    float f = (float)x;
    if ((double)f < x) f = std::nextafter(f, INFINITY);
    return f;
}

}  // namespace

extern "C" bt_status bt_build_mesh(bt_ctx *ctx, const float *xyz, int64_t n_vert, const int32_t *tri,
                                   const float *absorption, int64_t n_tri, int32_t tiles_x, int32_t tiles_y,
                                   bt_mesh **out)
{
    if (!ctx) return BT_EINVAL;
    if (!out) return fail(ctx, BT_EINVAL, "out is NULL");
    *out = nullptr;
    {
        std::string msg;
        bt_status s = check_mesh_args(xyz, n_vert, tri, absorption, n_tri, tiles_x, tiles_y, msg);
        if (s != BT_OK) return fail(ctx, s, "%s", msg.c_str());
    }
    (void)hipSetDevice(ctx->device);

    // per-triangle records
    const double delta_cap = kDeltaCap;
    double r_mesh = 0.0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t t = 0; t < n_tri; ++t) {
        for (int k = 0; k < 3; ++k) {
            int32_t v = tri[3 * t + k];
            if (v < 0 || v >= n_vert) return fail(ctx, BT_EINVAL, "triangle %lld has vertex index %d out of range", (long long)t, v);
            for (int c = 0; c < 3; ++c) {
                float x = xyz[3 * (int64_t)v + c];
                if (!std::isfinite(x)) return fail(ctx, BT_EINVAL, "vertex %d is not finite", v);
                r_mesh = std::max(r_mesh, (double)std::fabs(x));
                lo[c] = std::min(lo[c], (double)x);
                hi[c] = std::max(hi[c], (double)x);
            }
        }
        float a = absorption[t];
        if (!(a >= 0.0f && a <= 1.0f)) return fail(ctx, BT_EINVAL, "absorption of triangle %lld not in [0, 1]", (long long)t);
    }
    const double r_eff = 2.0 * r_mesh + 10.0;
    const double margin = delta_cap + 12.0 * r_eff * std::ldexp(1.0, -24);

    std::vector<float> tri_g((size_t)n_tri * 9);
    std::vector<float4> tri_rec((size_t)n_tri * 3);
    std::vector<Prim> all((size_t)n_tri);
    for (int64_t t = 0; t < n_tri; ++t) {
        double v[3][3];
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 3; ++c) {
                float x = xyz[3 * (int64_t)tri[3 * t + k] + c];
                tri_g[9 * t + 3 * k + c] = x;
                v[k][c] = x;
            }
        double e1[3], e2[3], e3[3], N[3];
        for (int c = 0; c < 3; ++c) { e1[c] = v[1][c] - v[0][c]; e2[c] = v[2][c] - v[0][c]; e3[c] = v[2][c] - v[1][c]; }
        N[0] = e1[1] * e2[2] - e1[2] * e2[1];
        N[1] = e1[2] * e2[0] - e1[0] * e2[2];
        N[2] = e1[0] * e2[1] - e1[1] * e2[0];
        double a2 = std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        if (!(a2 > 0.0)) return fail(ctx, BT_EINVAL, "triangle %lld has zero area", (long long)t);
        double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        double l2 = std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
        double l3 = std::sqrt(e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]);
        double hmin = a2 / std::max(l1, std::max(l2, l3)) * (1.0 - 1e-12);
        float idf;
        int idi = (int)t;
        std::memcpy(&idf, &idi, 4);
        tri_rec[3 * t + 0] = make_float4((float)v[0][0], (float)v[0][1], (float)v[0][2], (float)v[1][0]);
        tri_rec[3 * t + 1] = make_float4((float)v[1][1], (float)v[1][2], (float)v[2][0], (float)v[2][1]);
        tri_rec[3 * t + 2] = make_float4((float)v[2][2], idf, round_down_f(hmin), 0.f);
        Prim &p = all[t];
        p.id = (int)t;
        for (int c = 0; c < 3; ++c) {
            double mn = std::min(v[0][c], std::min(v[1][c], v[2][c]));
            double mx = std::max(v[0][c], std::max(v[1][c], v[2][c]));
            p.box.lo[c] = round_down_f(mn - margin);
            p.box.hi[c] = round_up_f(mx + margin);
            p.cen[c] = (float)(0.5 * (mn + mx));
        }
    }

    // tile grid over the (grown) xy footprint
    DevMesh dm{};
    dm.tiles_x = tiles_x;
    dm.tiles_y = tiles_y;
    dm.n_tri = (int)n_tri;
    if (n_tri > 0) {
        dm.gx0 = lo[0] - margin; dm.gx1 = hi[0] + margin;
        dm.gy0 = lo[1] - margin; dm.gy1 = hi[1] + margin;
        dm.zmin = lo[2] - margin; dm.zmax = hi[2] + margin;
    } else {
        dm.gx0 = 0.0; dm.gx1 = 1.0; dm.gy0 = 0.0; dm.gy1 = 1.0; dm.zmin = 1.0; dm.zmax = -1.0;
    }
    dm.tw = (dm.gx1 - dm.gx0) / tiles_x;
    dm.th = (dm.gy1 - dm.gy0) / tiles_y;

    std::vector<float4> nodes, trefs, nodes4;
    int max_push = 0;
    std::vector<int> roots((size_t)tiles_x * tiles_y, kEmptyRoot);
    std::vector<float> tboxes((size_t)tiles_x * tiles_y * 6, 0.f);
    int max_depth = 0;
    bool overflow = false;
    for (int ty = 0; ty < tiles_y; ++ty)
        for (int tx = 0; tx < tiles_x; ++tx) {
            double x0 = dm.gx0 + tx * dm.tw, x1 = dm.gx0 + (tx + 1) * dm.tw;
            double y0 = dm.gy0 + ty * dm.th, y1 = dm.gy0 + (ty + 1) * dm.th;
            if (tx == tiles_x - 1) x1 = dm.gx1;
            if (ty == tiles_y - 1) y1 = dm.gy1;
            std::vector<Prim> prims;
            for (const Prim &p : all)
                if ((double)p.box.lo[0] <= x1 + margin && (double)p.box.hi[0] >= x0 - margin &&
                    (double)p.box.lo[1] <= y1 + margin && (double)p.box.hi[1] >= y0 - margin)
                    prims.push_back(p);
            int tile = ty * tiles_x + tx;
            if (prims.empty()) continue;
            Builder b{prims, nodes, trefs, tri_rec};
            {
                const int root2 = b.build(0, (int)prims.size(), 0);
                Collapse cl{nodes, nodes4};
                roots[tile] = cl.collapse(root2, 0);
                max_push = std::max(max_push, cl.max_push);
            }
            max_depth = std::max(max_depth, b.max_depth);
            overflow = overflow || b.overflow;
            Box rb;
            rb.empty();
            for (const Prim &p : prims) rb.grow(p.box);
            for (int c = 0; c < 3; ++c) { tboxes[6 * tile + c] = rb.lo[c]; tboxes[6 * tile + 3 + c] = rb.hi[c]; }
        }
    if (overflow || max_push > kStack)
        return fail(ctx, BT_EOVERFLOW, "BVH deeper than the %d-entry traversal stack", kStack);
    if (trefs.size() / 3 >= (1u << 28)) return fail(ctx, BT_EOVERFLOW, "too many triangle references");

    bt_mesh *m = new bt_mesh();
    m->ctx = ctx;
    m->n_nodes = (int64_t)(nodes4.size() / 8);
    m->n_refs = (int64_t)(trefs.size() / 3);
    m->max_depth = max_depth;
    m->delta_cap = delta_cap;
    m->r_eff = r_eff;
    const void *src[6] = {nodes4.data(), trefs.data(), tri_g.data(), absorption, roots.data(), tboxes.data()};
    size_t sz[6] = {nodes4.size() * sizeof(float4), trefs.size() * sizeof(float4), tri_g.size() * sizeof(float),
                    (size_t)n_tri * sizeof(float), roots.size() * sizeof(int), tboxes.size() * sizeof(float)};
    for (int i = 0; i < 6; ++i) {
        bt_status s = dev_alloc(ctx, &m->bufs[i], sz[i]);
        if (s != BT_OK) { bt_mesh_free(m); return s; }
        m->sizes[i] = sz[i];
        if (sz[i] && hipMemcpy(m->bufs[i], src[i], sz[i], hipMemcpyHostToDevice) != hipSuccess) {
            bt_mesh_free(m);
            return fail(ctx, BT_EDEVICE, "mesh upload failed");
        }
    }
    dm.nodes = (const float4 *)m->bufs[0];
    dm.tris = (const float4 *)m->bufs[1];
    dm.tri_g = (const float *)m->bufs[2];
    dm.alpha = (const float *)m->bufs[3];
    dm.tile_root = (const int *)m->bufs[4];
    dm.tile_box = (const float *)m->bufs[5];
    m->dev = dm;
    *out = m;
    return BT_OK;
}

extern "C" bt_status bt_mesh_free(bt_mesh *m)
{
    if (!m) return BT_EINVAL;
    for (int i = 0; i < 6; ++i) dev_free(m->ctx, m->bufs[i], m->sizes[i]);
    delete m;
    return BT_OK;
}

extern "C" bt_status bt_mesh_info(const bt_mesh *m, int64_t *n_nodes, int32_t *max_depth, int64_t *n_tri_refs)
{
    if (!m) return BT_EINVAL;
    if (n_nodes) *n_nodes = m->n_nodes;
    if (max_depth) *max_depth = m->max_depth;
    if (n_tri_refs) *n_tri_refs = m->n_refs;
    return BT_OK;
}

// ---------------------------------------------------------------------------------------
// microphones
// ---------------------------------------------------------------------------------------
extern "C" bt_status bt_mics_grid3d(bt_ctx *ctx, float x0, float y0, float z0, float dx, float dy, float dz,
                                    int32_t nx, int32_t ny, int32_t nz, bt_mics **out)
{
    if (!ctx) return BT_EINVAL;
    if (!out) return fail(ctx, BT_EINVAL, "out is NULL");
    *out = nullptr;
    {
        std::string msg;
        bt_status s = check_grid_args(x0, y0, z0, dx, dy, dz, nx, ny, nz, msg);
        if (s != BT_OK) return fail(ctx, s, "%s", msg.c_str());
    }
    (void)hipSetDevice(ctx->device);
    bt_mics *m = new bt_mics();
    m->ctx = ctx;
    long long n = (long long)nx * ny * nz;
    m->bytes = (size_t)n * sizeof(double) * 3;
    void *p = nullptr;
    bt_status s = dev_alloc(ctx, &p, m->bytes);
    if (s != BT_OK) { delete m; return s; }
    m->dev.x0 = x0; m->dev.y0 = y0; m->dev.z = z0; m->dev.dx = dx; m->dev.dy = dy;
    m->dev.nx = nx; m->dev.ny = ny;
    m->dev.nz = nz;
    m->dev.dz = nz > 1 ? (double)dz : 0.0;
    m->dev.fx0 = x0;
    m->dev.fy0 = y0;
    m->dev.fidx = (float)(1.0 / (double)dx);
    m->dev.fidy = (float)(1.0 / (double)dy);
    m->dev.fnx1 = (float)(nx - 1);
    m->dev.fny1 = (float)(ny - 1);
    m->dev.e_strict = (double *)p;
    m->dev.e_flag = m->dev.e_strict + n;
    m->level = m->dev.e_flag + n;
    m->n_out = n;
    s = bt_mics_reset(ctx, m);
    if (s != BT_OK) { bt_mics_free(m); return s; }
    *out = m;
    return BT_OK;
}

// Energies a set holds: a grid's (also for a subset of it) or one per explicit point.
static long long mic_energies(const bt_mics *m)
{
    return m->points ? m->pts.n : (long long)m->dev.nx * m->dev.ny * m->dev.nz;
}

extern "C" bt_status bt_mics_subset(bt_ctx *ctx, const bt_mics *grid, const int32_t *idx, int64_t n, bt_mics **out)
{
    if (!ctx) return BT_EINVAL;
    if (!out) return fail(ctx, BT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!grid || grid->points || grid->sel) return fail(ctx, BT_EINVAL, "a subset is taken of a grid set");
    if (n < 1 || !idx) return fail(ctx, BT_EINVAL, "empty or NULL subset");
    const long long N = mic_energies(grid);
    for (int64_t k = 0; k < n; ++k)
        if (idx[k] < 0 || idx[k] >= N) return fail(ctx, BT_EINVAL, "subset index %d not in [0, %lld)", idx[k], N);
    (void)hipSetDevice(ctx->device);
    bt_mics *m = new bt_mics();
    m->ctx = ctx;
    m->dev = grid->dev;
    m->bytes = (size_t)N * sizeof(double) * 3;
    m->mask_bytes = (size_t)((N + 31) / 32) * sizeof(unsigned);
    void *p = nullptr, *q = nullptr, *r = nullptr, *t = nullptr;
    bt_status s = dev_alloc(ctx, &p, m->bytes);
    if (s == BT_OK) s = dev_alloc(ctx, &q, m->mask_bytes);
    if (s == BT_OK) s = dev_alloc(ctx, &r, (size_t)n * sizeof(long long));
    if (s == BT_OK) s = dev_alloc(ctx, &t, (size_t)n * 3 * sizeof(double));
    m->dev.e_strict = (double *)p;
    m->mask = (unsigned *)q;
    m->sel = (long long *)r;
    m->sel_buf = (double *)t;
    m->n_out = n;
    if (s != BT_OK) { bt_mics_free(m); return s; }
    m->dev.e_flag = m->dev.e_strict + N;
    m->level = m->dev.e_flag + N;
    m->dev.mask = m->mask;
    std::vector<unsigned> bits((size_t)((N + 31) / 32), 0u);
    std::vector<long long> sel((size_t)n);
    for (int64_t k = 0; k < n; ++k) {
        bits[(size_t)(idx[k] >> 5)] |= 1u << (idx[k] & 31);
        sel[(size_t)k] = idx[k];
    }
    if (hipMemcpy(m->mask, bits.data(), m->mask_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->sel, sel.data(), (size_t)n * sizeof(long long), hipMemcpyHostToDevice) != hipSuccess) {
        bt_mics_free(m);
        return fail(ctx, BT_EDEVICE, "subset upload failed");
    }
    if ((s = bt_mics_reset(ctx, m)) != BT_OK) { bt_mics_free(m); return s; }
    *out = m;
    return BT_OK;
}

extern "C" bt_status bt_mics_points(bt_ctx *ctx, const float *xyz, int64_t n, bt_mics **out)
{
    if (!ctx) return BT_EINVAL;
    if (!out) return fail(ctx, BT_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !xyz || n >= (1ll << 31)) return fail(ctx, BT_EINVAL, "bad microphone point count %lld", (long long)n);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = 0; k < n; ++k)
        for (int c = 0; c < 3; ++c) {
            const float v = xyz[3 * k + c];
            if (!std::isfinite(v)) return fail(ctx, BT_EINVAL, "microphone point %lld is not finite", (long long)k);
            lo[c] = std::min(lo[c], (double)v);
            hi[c] = std::max(hi[c], (double)v);
        }
    // buckets in xy of about two points each (smaller buckets fit thin beams' regions
    // better, larger ones need fewer bucket rows per beam); one spare column and row, so
    // that no point's bucket is clamped
    const double sx = hi[0] - lo[0], sy = hi[1] - lo[1];
    double bh = std::sqrt(std::max(sx * sy, 0.0) / std::max((double)n / 2.0, 1.0));
    bh = std::max(bh, std::max(std::max(sx, sy) / 4096.0, 1e-3));
    const int nbx = (int)std::floor(sx / bh) + 2, nby = (int)std::floor(sy / bh) + 2;
    const long long nb = (long long)nbx * nby;
    std::vector<int> cell((size_t)nb + 1, 0), key((size_t)n);
    for (int64_t k = 0; k < n; ++k) {
        const int bi = (int)std::floor(((double)xyz[3 * k] - lo[0]) / bh);
        const int bj = (int)std::floor(((double)xyz[3 * k + 1] - lo[1]) / bh);
        key[(size_t)k] = bj * nbx + bi;
        cell[(size_t)key[(size_t)k] + 1]++;
    }
    for (long long b = 0; b < nb; ++b) cell[(size_t)b + 1] += cell[(size_t)b];
    std::vector<double> pos((size_t)n * 3);
    std::vector<int> orig((size_t)n), fill(cell.begin(), cell.end() - 1);
    for (int64_t k = 0; k < n; ++k) {
        const int at = fill[(size_t)key[(size_t)k]]++;
        pos[(size_t)at] = xyz[3 * k];
        pos[(size_t)n + at] = xyz[3 * k + 1];
        pos[2 * (size_t)n + at] = xyz[3 * k + 2];
        orig[(size_t)at] = (int)k;
    }
    (void)hipSetDevice(ctx->device);
    bt_mics *m = new bt_mics();
    m->ctx = ctx;
    m->points = true;
    m->n_out = n;
    m->bytes = (size_t)n * sizeof(double) * 3;
    m->pts_bytes = (size_t)n * 3 * sizeof(double) + (size_t)n * sizeof(int) + (size_t)(nb + 1) * sizeof(int);
    void *p = nullptr, *q = nullptr;
    bt_status s = dev_alloc(ctx, &p, m->bytes);
    if (s == BT_OK) s = dev_alloc(ctx, &q, m->pts_bytes);
    m->dev.e_strict = (double *)p;
    m->pts_buf = q;
    if (s != BT_OK) { bt_mics_free(m); return s; }
    m->dev.e_flag = m->dev.e_strict + n;
    m->level = m->dev.e_flag + n;
    char *b = (char *)q;
    DevPoints &P = m->pts;
    P.px = (const double *)b;
    P.py = P.px + n;
    P.pz = P.py + n;
    P.orig = (const int *)(b + (size_t)n * 3 * sizeof(double));
    P.cell = P.orig + n;
    P.bx0 = lo[0];
    P.by0 = lo[1];
    P.bh = bh;
    P.nbx = nbx;
    P.nby = nby;
    P.zlo = lo[2];
    P.zhi = hi[2];
    P.n = n;
    if (hipMemcpy(b, pos.data(), (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy((void *)P.orig, orig.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy((void *)P.cell, cell.data(), (size_t)(nb + 1) * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
        bt_mics_free(m);
        return fail(ctx, BT_EDEVICE, "microphone point upload failed");
    }
    if ((s = bt_mics_reset(ctx, m)) != BT_OK) { bt_mics_free(m); return s; }
    *out = m;
    return BT_OK;
}

extern "C" bt_status bt_mics_grid(bt_ctx *ctx, float x0, float y0, float z, float dx, float dy, int32_t nx, int32_t ny,
                                  bt_mics **out)
{
    return bt_mics_grid3d(ctx, x0, y0, z, dx, dy, 0.f, nx, ny, 1, out);
}

extern "C" bt_status bt_mics_reset(bt_ctx *ctx, bt_mics *m)
{
    if (!ctx || !m) return BT_EINVAL;
    HIP_TRY(ctx, launch_fill(m->dev.e_strict, 2 * mic_energies(m), 0.0, ctx->stream));
    return BT_OK;
}

bt_status mics_fit(bt_ctx *ctx, bt_mics **m, float x0, float y0, float z, float dx, float dy, int32_t nx, int32_t ny)
{
    const long long n = (long long)nx * ny;
    if (*m && (size_t)n * sizeof(double) * 3 <= (*m)->bytes) {
        bt_mics *g = *m;
        g->dev.x0 = x0; g->dev.y0 = y0; g->dev.z = z; g->dev.dx = dx; g->dev.dy = dy;
        g->dev.nx = nx; g->dev.ny = ny;
        g->dev.nz = 1; g->dev.dz = 0.0;
        g->n_out = n;
        g->dev.e_flag = g->dev.e_strict + n;
        g->level = g->dev.e_flag + n;
        return bt_mics_reset(ctx, g);
    }
    if (*m) {
        bt_mics_free(*m);
        *m = nullptr;
    }
    return bt_mics_grid(ctx, x0, y0, z, dx, dy, nx, ny, m);
}

extern "C" bt_status bt_mics_free(bt_mics *m)
{
    if (!m) return BT_EINVAL;
    dev_free(m->ctx, m->dev.e_strict, m->bytes);
    dev_free(m->ctx, m->mask, m->mask_bytes);
    dev_free(m->ctx, m->sel, (size_t)m->n_out * sizeof(long long));
    dev_free(m->ctx, m->sel_buf, (size_t)m->n_out * 3 * sizeof(double));
    dev_free(m->ctx, m->pts_buf, m->pts_bytes);
    delete m;
    return BT_OK;
}

// ---------------------------------------------------------------------------------------
// beams
// ---------------------------------------------------------------------------------------
// Integers in the segment-list buffer of a queue of capacity n: the wave-path overflow
// list (n), then the general-path list, whose per-wave regions hold 64 items per batch
// (at most n + 64 (W + 1)).
size_t list_ints(long long n, int n_waves)
{
    return (size_t)(2 * n + 64 * ((long long)n_waves + 1));
}

// Per-wave scratch of a beam set for a grid of W = n_cu * blocks_per_cu * kWavesPerBlock
// waves: children, offsets, 3 stats, power (8 B each) and general counts (4 B).
bt_status alloc_wave_scratch(bt_ctx *ctx, bt_beams *b, int blocks_per_cu)
{
    const int W = ctx->n_cu * blocks_per_cu * kWavesPerBlock;
    const size_t bytes = (size_t)W * (7 * 8 + 4 + 4);
    bt_status s = dev_alloc(ctx, &b->ws_buf, bytes);
    if (s != BT_OK) return s;
    b->ws_bytes = bytes;
    char *p = (char *)b->ws_buf;
    b->ws.children = (unsigned long long *)p;
    b->ws.block_rec = b->ws.children + W;                      // [W / kWavesPerBlock][4]
    b->ws.stats = b->ws.block_rec + W;
    b->ws.power = (double *)(b->ws.stats + 3 * (size_t)W);
    b->ws.block_power = b->ws.power + W;                       // [W / kWavesPerBlock], W reserved
    b->ws.general = (unsigned int *)(b->ws.block_power + W);
    b->ws.rows_n = b->ws.general + W;
    b->ws.n_waves = W;
    b->ws_cap_waves = W;
    return BT_OK;
}

// The grid of the set's statically partitioned kernels: blocks_per_cu workgroups of
// kWavesPerBlock waves per compute unit, at most the waves its arrays were sized for.
static void set_wave_grid(bt_ctx *ctx, bt_beams *b, int blocks_per_cu)
{
    const int W = ctx->n_cu * std::max(blocks_per_cu, 1) * kWavesPerBlock;
    b->ws.n_waves = std::min(W, b->ws_cap_waves);
}

void queue_free(bt_ctx *ctx, DevQueue &q)
{
    dev_free(ctx, q.dbl, (size_t)q.cap * D_N * sizeof(double));
    dev_free(ctx, q.flt, (size_t)q.cap * F_N * sizeof(float));
    dev_free(ctx, q.ints, (size_t)q.cap * I_N * sizeof(int));
    q = DevQueue{};
}

void beams_release(bt_beams *b)
{
    bt_ctx *ctx = b->ctx;
    queue_free(ctx, b->q);
    dev_free(ctx, b->segs.hit, (size_t)b->cap * sizeof(int));
    dev_free(ctx, b->segs.t, (size_t)b->cap * sizeof(double));
    dev_free(ctx, b->segs.flag, (size_t)b->cap * sizeof(int));
    b->segs = DevSegs{};
    dev_free(ctx, b->big_list, list_ints(b->cap, b->ws_cap_waves) * sizeof(int));
    b->big_list = nullptr;
    b->cap = 0;
    dev_free(ctx, b->rows, (size_t)b->rows_cap * sizeof(int2));
    b->rows = nullptr;
    b->rows_cap = 0;
    dev_free(ctx, b->spans, (size_t)b->spans_cap * sizeof(int4));
    b->spans = nullptr;
    b->spans_cap = 0;
    dev_free(ctx, b->layers, (size_t)b->layers_cap * sizeof(int2));
    b->layers = nullptr;
    b->layers_cap = 0;
    dev_free(ctx, b->layer_cnt, (size_t)kLayerRegions * kLayerCntStride * sizeof(unsigned));
    b->layer_cnt = nullptr;
    b->work_n0 = 0;
    dev_free(ctx, b->tw_buf, b->tw_bytes);
    b->tw_buf = nullptr;
    b->tw_bytes = 0;
    b->tw = TileWork{};
    dev_free(ctx, b->cgrid.cls, (size_t)b->cls_cap * sizeof(int2));
    b->cgrid = ClassGrid{};
    b->cls_cap = 0;
    b->bound = false;
    b->class_gens = 0;
}

bt_status reserve_tiles(bt_ctx *ctx, bt_beams *b, long long n)
{
    n = std::max(n, 1ll);
    const int W = b->ws.n_waves;
    if (W <= 0) return fail(ctx, BT_EINVAL, "beam set without a wave grid");
    if (b->tw_buf && b->tw.cap >= n && b->tw.n_waves == W) return BT_OK;
    dev_free(ctx, b->tw_buf, b->tw_bytes);
    b->tw_buf = nullptr;
    b->tw_bytes = 0;
    b->tw = TileWork{};
    // a producer wave handles at most ceil(n / (64 W)) + 2 batches of 64 (static
    // partition, or its XCD's share of the ordered list)
    const long long region = 64 * ((n + 64ll * W - 1) / (64ll * W) + 2);
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t b_stage = up((size_t)W * region * sizeof(int2)), b_stage_n = up((size_t)W * sizeof(int));
    const size_t b_cnt = up((size_t)kMaxQueueTiles * W * sizeof(int)), b_tot = up((kMaxQueueTiles + 1) * sizeof(int));
    const size_t b_list = up((size_t)n * sizeof(int2)), b_dbl = up((size_t)n * sizeof(double));
    const size_t b_int = up((size_t)n * sizeof(int));
    const size_t bytes = b_stage + b_stage_n + 2 * b_cnt + b_tot + b_list + 3 * b_dbl + b_int;
    bt_status s = dev_alloc(ctx, &b->tw_buf, bytes);
    if (s != BT_OK) return s;
    b->tw_bytes = bytes;
    char *p = (char *)b->tw_buf;
    b->tw.stage = (int2 *)p;
    p += b_stage;
    b->tw.stage_n = (int *)p;
    p += b_stage_n;
    b->tw.cnt = (int *)p;
    p += b_cnt;
    b->tw.off = (int *)p;
    p += b_cnt;
    b->tw.total = (int *)p;
    b->tw.n_items = b->tw.total + kMaxQueueTiles;
    p += b_tot;
    b->tw.list = (int2 *)p;
    p += b_list;
    b->tw.lo = (double *)p;
    p += b_dbl;
    b->tw.c1t = (double *)p;
    p += b_dbl;
    b->tw.c2t = (double *)p;
    p += b_dbl;
    b->tw.c1id = (int *)p;
    b->tw.cap = n;
    b->tw.region = region;
    b->tw.n_waves = W;
    // the per-(tile, wave) counts start at zero; every scan clears them again
    HIP_TRY(ctx, launch_zero_ints(b->tw.cnt, (long long)kMaxQueueTiles * W, ctx->stream));
    return BT_OK;
}

const TileWork *trace_tiles(bt_beams *b, const bt_mesh *mesh, const TraceArgs &a)
{
    // partitions of more than kMaxQueueTiles tiles walk their tiles in-lane
    if (a.queue_rounds <= 0 || !b->tw_buf || mesh->dev.tiles_x * mesh->dev.tiles_y > kMaxQueueTiles) return nullptr;
    b->tw.n_tiles = mesh->dev.tiles_x * mesh->dev.tiles_y;
    b->tw.rounds = a.queue_rounds;
    return &b->tw;
}

// (segment, layer) item buffer of the volumetric microphone pass, sized from the
// generation-0 count: 4 per initial beam covers the tall district workload (1.2 per beam)
// with room; items past a full buffer are done in place by the lane that found them.
static bt_status reserve_layers(bt_ctx *ctx, bt_beams *b)
{
    long long want = std::max(4 * b->n0, 1ll << 20);
    if (const char *env = std::getenv("BT_MIC_LAYER_CAPACITY")) {  // testing the full-buffer path
        long long v = std::atoll(env);
        if (v > 0) want = v;
    }
    if (b->layers && b->layers_cap == want) return BT_OK;
    dev_free(ctx, b->layers, (size_t)b->layers_cap * sizeof(int2));
    b->layers = nullptr;
    b->layers_cap = 0;
    if (!b->layer_cnt &&
        dev_alloc(ctx, (void **)&b->layer_cnt, (size_t)kLayerRegions * kLayerCntStride * sizeof(unsigned)) != BT_OK)
        return BT_ENOMEM;
    bt_status s = dev_alloc(ctx, (void **)&b->layers, (size_t)want * sizeof(int2));
    if (s != BT_OK) return s;
    b->layers_cap = want;
    return BT_OK;
}

// Queue, segment and overflow-list capacity of at least n records.  When the arrays
// move, the first `keep` queue records (every field) are carried over on the stream.
bt_status reserve_queue(bt_ctx *ctx, bt_beams *b, long long n, long long keep)
{
    if (n <= b->cap) return BT_OK;
    DevQueue nq{};
    bt_status s;
    if ((s = dev_alloc(ctx, (void **)&nq.dbl, (size_t)n * D_N * sizeof(double))) != BT_OK ||
        (s = dev_alloc(ctx, (void **)&nq.flt, (size_t)n * F_N * sizeof(float))) != BT_OK ||
        (s = dev_alloc(ctx, (void **)&nq.ints, (size_t)n * I_N * sizeof(int))) != BT_OK) {
        nq.cap = n;
        queue_free(ctx, nq);
        return s;
    }
    nq.cap = n;
    if (keep > 0) {
        for (int k = 0; k < D_N; ++k)
            HIP_TRY(ctx, hipMemcpyAsync(nq.dbl + k * n, b->q.dbl + k * b->q.cap, (size_t)keep * sizeof(double),
                                        hipMemcpyDeviceToDevice, ctx->stream));
        for (int k = 0; k < F_N; ++k)
            HIP_TRY(ctx, hipMemcpyAsync(nq.flt + k * n, b->q.flt + k * b->q.cap, (size_t)keep * sizeof(float),
                                        hipMemcpyDeviceToDevice, ctx->stream));
        for (int k = 0; k < I_N; ++k)
            HIP_TRY(ctx, hipMemcpyAsync(nq.ints + k * n, b->q.ints + k * b->q.cap, (size_t)keep * sizeof(int),
                                        hipMemcpyDeviceToDevice, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // the old arrays are freed next
    }
    if (b->cgrid.cls) {
        // the class array follows the queue (its kept records' classes too)
        int2 *nc = nullptr;
        if ((s = dev_alloc(ctx, (void **)&nc, (size_t)n * sizeof(int2))) != BT_OK) {
            queue_free(ctx, nq);
            return s;
        }
        if (keep > 0) {
            HIP_TRY(ctx, hipMemcpyAsync(nc, b->cgrid.cls, (size_t)keep * sizeof(int2), hipMemcpyDeviceToDevice,
                                        ctx->stream));
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        }
        dev_free(ctx, b->cgrid.cls, (size_t)b->cls_cap * sizeof(int2));
        b->cgrid.cls = nc;
        b->cls_cap = n;
    }
    queue_free(ctx, b->q);
    b->q = nq;
    dev_free(ctx, b->segs.hit, (size_t)b->cap * sizeof(int));
    dev_free(ctx, b->segs.t, (size_t)b->cap * sizeof(double));
    dev_free(ctx, b->segs.flag, (size_t)b->cap * sizeof(int));
    dev_free(ctx, b->big_list, list_ints(b->cap, b->ws_cap_waves) * sizeof(int));
    b->segs = DevSegs{};
    b->big_list = nullptr;
    b->cap = 0;
    if ((s = dev_alloc(ctx, (void **)&b->segs.hit, (size_t)n * sizeof(int))) != BT_OK) return s;
    if ((s = dev_alloc(ctx, (void **)&b->segs.t, (size_t)n * sizeof(double))) != BT_OK) return s;
    if ((s = dev_alloc(ctx, (void **)&b->segs.flag, (size_t)n * sizeof(int))) != BT_OK) return s;
    if ((s = dev_alloc(ctx, (void **)&b->big_list, list_ints(n, b->ws_cap_waves) * sizeof(int))) != BT_OK) return s;
    b->cap = n;
    return BT_OK;
}

// Work-item buffers of the microphone stage, sized from the generation-0 count.
bt_status reserve_work(bt_ctx *ctx, bt_beams *b, long long n0)
{
    if (n0 <= b->work_n0) return BT_OK;
    dev_free(ctx, b->rows, (size_t)b->rows_cap * sizeof(int2));
    dev_free(ctx, b->spans, (size_t)b->spans_cap * sizeof(int4));
    b->rows = nullptr;
    b->spans = nullptr;
    b->rows_cap = b->spans_cap = 0;
    bt_status s;
    // row work items of wide footprints over all generations, in equal per-wave regions:
    // 4 per initial beam gives every wave room for about three times the district
    // workload's mean (1.2 per beam); a wave whose region is full sends its further wide
    // segments to the one-wave-per-segment path
    long long rows_cap = std::max(4 * n0, 1ll << 20);
    if (const char *env = std::getenv("BT_MIC_ROW_CAPACITY")) {  // testing the overflow path
        long long v = std::atoll(env);
        if (v > 0) rows_cap = v;
    }
    if ((s = dev_alloc(ctx, (void **)&b->rows, (size_t)rows_cap * sizeof(int2))) != BT_OK) return s;
    b->rows_cap = rows_cap;
    // column spans of long rows; a full buffer makes the row's lane process it in place
    long long spans_cap = std::max(n0, 1ll << 20);
    if (const char *env = std::getenv("BT_MIC_SPAN_CAPACITY")) {  // testing the full-buffer path
        long long v = std::atoll(env);
        if (v > 0) spans_cap = v;
    }
    if ((s = dev_alloc(ctx, (void **)&b->spans, (size_t)spans_cap * sizeof(int4))) != BT_OK) return s;
    b->spans_cap = spans_cap;
    b->work_n0 = n0;
    return BT_OK;
}

// Generation 0 of a beam set; src_weight NULL (omni sources) or host float[n_src][nf].
// two_slot: the set keeps two generation slots of n0 records (each generation must be
// accumulated before the next is traced) instead of every generation.
// An empty beam set of the context (counters and per-wave scratch only).
static bt_status new_beams(bt_ctx *ctx, bt_beams **out)
{
    bt_beams *b = new bt_beams();
    b->ctx = ctx;
    bt_status s = dev_alloc(ctx, (void **)&b->ctr, sizeof(DevCounters));
    if (s == BT_OK) s = alloc_wave_scratch(ctx, b, kBlocksPerCU);
    // counters start at zero (no beams), so statistics of a set never emitted are zeros
    if (s == BT_OK && launch_init_counters(b->ctr, 0, 0, ctx->stream) != hipSuccess)
        s = hip_fail(ctx, hipGetLastError(), "launch_init_counters");
    if (s != BT_OK) {
        bt_beams_free(b);
        return s;
    }
    *out = b;
    return BT_OK;
}

// The classification grid of the set's new records (none unless bound).
static ClassGrid class_target(const bt_beams *b)
{
    if (!b->bound) return ClassGrid{};
    return b->cgrid;
}

// Bind set b to classification grid g (allocating its class array), or unbind it.
static bt_status bind_set(bt_ctx *ctx, bt_beams *b, const ClassGrid *g)
{
    if (!g) {
        b->bound = false;
        return BT_OK;
    }
    const ClassGrid &c = b->cgrid;
    const bool same = c.cls && c.x0 == g->x0 && c.y0 == g->y0 && c.z == g->z && c.dx == g->dx && c.dy == g->dy &&
                      c.nx == g->nx && c.ny == g->ny;
    if (!same) b->class_gens = 0;   // the records' classes refer to another grid
    if (!b->cgrid.cls || b->cls_cap < b->cap) {
        dev_free(ctx, b->cgrid.cls, (size_t)b->cls_cap * sizeof(int2));
        b->cgrid.cls = nullptr;
        b->cls_cap = 0;
        b->class_gens = 0;
        const long long n = std::max(b->cap, 1ll);
        bt_status s = dev_alloc(ctx, (void **)&b->cgrid.cls, (size_t)n * sizeof(int2));
        if (s != BT_OK) return s;
        b->cls_cap = n;
    }
    int2 *cls = b->cgrid.cls;
    b->cgrid = *g;
    b->cgrid.cls = cls;
    b->bound = true;
    return BT_OK;
}

// Generation 0 of one set (a partition) from n_src sources, enqueued on the context's
// stream; src_weight NULL (omni sources) or host float[n_src][nf].  two_slot: the set
// keeps two generation slots of n0 records (each generation must be accumulated before
// the next is traced) instead of every generation.  The caller synchronises before the
// host inputs are released.
static bt_status emit_set(bt_ctx *ctx, bt_beams *b, const float *src_xyz, const float *src_power,
                          const float *src_weight, int32_t n_src, int32_t level, bool two_slot)
{
    const long long nf = 20ll << (2 * level);
    const long long n0 = nf * n_src;
    double r_src = 0.0;
    for (int i = 0; i < n_src; ++i)
        for (int c = 0; c < 3; ++c) r_src = std::max(r_src, (double)std::fabs(src_xyz[3 * i + c]));
    // room for every generation of the previous run's depth (grown at the first trace if
    // the depth is larger), or for two generations
    const long long want = std::max(n0, 1ll) * (two_slot ? 2ll : (long long)(b->depth_hint + 1));
    bt_status s = reserve_queue(ctx, b, want <= (1ll << 31) - 1 ? want : std::max(n0, 1ll), 0);
    if (s == BT_OK) s = reserve_work(ctx, b, std::max(n0, 1ll));
    if (s == BT_OK && n_src > b->src_cap) {
        dev_free(ctx, b->src_dev, (size_t)b->src_cap * 3 * sizeof(float));
        dev_free(ctx, b->pow_dev, (size_t)b->src_cap * sizeof(float));
        dev_free(ctx, b->norm_dev, (size_t)b->src_cap * sizeof(double));
        b->src_dev = b->pow_dev = nullptr;
        b->norm_dev = nullptr;
        b->src_cap = 0;
        s = dev_alloc(ctx, (void **)&b->src_dev, (size_t)n_src * 3 * sizeof(float));
        if (s == BT_OK) s = dev_alloc(ctx, (void **)&b->pow_dev, (size_t)n_src * sizeof(float));
        if (s == BT_OK) s = dev_alloc(ctx, (void **)&b->norm_dev, (size_t)n_src * sizeof(double));
        if (s == BT_OK) b->src_cap = n_src;
    }
    if (s == BT_OK && src_weight && n0 > b->wt_cap) {
        dev_free(ctx, b->wt_dev, (size_t)b->wt_cap * sizeof(float));
        b->wt_dev = nullptr;
        b->wt_cap = 0;
        s = dev_alloc(ctx, (void **)&b->wt_dev, (size_t)n0 * sizeof(float));
        if (s == BT_OK) b->wt_cap = n0;
    }
    if (s != BT_OK) return s;
    if (n_src > 0) {
        HIP_TRY(ctx, hipMemcpyAsync(b->src_dev, src_xyz, (size_t)n_src * 3 * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(b->pow_dev, src_power, (size_t)n_src * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
        if (src_weight)
            HIP_TRY(ctx, hipMemcpyAsync(b->wt_dev, src_weight, (size_t)n0 * sizeof(float), hipMemcpyHostToDevice,
                                        ctx->stream));
    }
    HIP_TRY(ctx, launch_init_counters(b->ctr, n0, two_slot ? std::max(n0, 1ll) : 0, ctx->stream));
    if (!ctx->face_dirs[level]) {
        // the level's face directions, computed once per context
        if ((s = dev_alloc(ctx, (void **)&ctx->face_dirs[level], (size_t)nf * 12 * sizeof(double))) != BT_OK) return s;
        if ((s = dev_alloc(ctx, (void **)&ctx->face_om[level], (size_t)nf * sizeof(double))) != BT_OK) return s;
        HIP_TRY(ctx, launch_faces(ctx->base20, level, ctx->face_dirs[level], ctx->face_om[level], ctx->stream));
    }
    HIP_TRY(ctx, launch_emit(ctx->face_dirs[level], ctx->face_om[level], b->src_dev, b->pow_dev,
                             src_weight ? b->wt_dev : nullptr, b->norm_dev, n_src, level, b->q, class_target(b),
                             ctx->stream));
    b->class_gens = b->bound ? 1ull : 0ull;
    b->gen = 0;
    b->acc_gen = 0;
    b->max_depth = -1;
    b->n0 = n0;
    b->ring = two_slot ? std::max(n0, 1ll) : 0;
    b->prior = bt_stats{};
    b->r_src = r_src;
    b->emitted = true;
    b->mesh = nullptr;
    return BT_OK;
}

// Partition k of a set (0: the set itself).
static inline bt_beams *part_of(bt_beams *b, int k) { return k == 0 ? b : b->part[k - 1]; }
static inline const bt_beams *part_of(const bt_beams *b, int k) { return k == 0 ? b : b->part[k - 1]; }

// Generation 0 of a beam set.  With two or more sources and the context's partition count
// above 1, the sources are split into min(parts, n_src) contiguous groups of near-equal
// size, each emitted into a partition of its own (a set with its own queue, counters and
// work lists; partition 0 is the set itself) that later calls trace on a stream of its
// own.  A partition's beams keep their order and are numbered from 0; beam0 places them
// in the emission (their parity-output rows).
static bt_status emit_beams(bt_ctx *ctx, const float *src_xyz, const float *src_power, const float *src_weight,
                            int32_t n_src, int32_t level, bt_beams **inout, bool two_slot = false)
{
    if (!ctx) return BT_EINVAL;
    if (!inout) return fail(ctx, BT_EINVAL, "inout is NULL");
    {
        std::string msg;
        bt_status s = check_source_args(src_xyz, src_power, src_weight, n_src, level, two_slot, msg);
        if (s != BT_OK) return fail(ctx, s, "%s", msg.c_str());
    }
    (void)hipSetDevice(ctx->device);
    bt_beams *b = *inout;
    bool fresh = false;
    if (!b) {
        bt_status s = new_beams(ctx, &b);
        if (s != BT_OK) return s;
        fresh = true;
    }
    const long long nf = 20ll << (2 * level);
    const int K = n_src >= 2 ? std::min(ctx->parts, (int)n_src) : 1;
    // the partitions' kernels run side by side: each gets 1/K of the grid one set uses
    // (measured on the district with two partitions: 4 workgroups per CU each 5.58 ms per
    // step, 8 each 5.80, 2 each 6.58)
    const int bpc = std::max(1, kBlocksPerCU / K);
    // until every partition is emitted, the set holds no emission (a failed call leaves it
    // so: it must be emitted again before it is traced)
    b->emitted = false;
    b->n_parts = 1;
    bt_status s = BT_OK;
    for (int k = 1; k < K && s == BT_OK; ++k) {
        if (!b->part[k - 1]) s = new_beams(ctx, &b->part[k - 1]);
        if (s == BT_OK) {
            bt_beams *q = b->part[k - 1];
            q->depth_hint = b->depth_hint;
            s = bind_set(ctx, q, b->bound ? &b->cgrid : nullptr);
        }
    }
    for (int k = 0; k < K && s == BT_OK; ++k) {
        const long long s0 = (long long)n_src * k / K, s1 = (long long)n_src * (k + 1) / K;
        bt_beams *q = part_of(b, k);
        set_wave_grid(ctx, q, bpc);
        s = emit_set(ctx, q, src_xyz + 3 * s0, src_power + s0, src_weight ? src_weight + s0 * nf : nullptr,
                     (int32_t)(s1 - s0), level, two_slot);
        q->beam0 = s0 * nf;
    }
    if (s != BT_OK) {
        b->emitted = false;
        if (fresh) bt_beams_free(b);
        return s;
    }
    b->n_parts = K;
    // host inputs are borrowed for the call only
    if (n_src > 0) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    *inout = b;
    return BT_OK;
}

extern "C" bt_status bt_emit_beams(bt_ctx *ctx, const float *src_xyz, const float *src_power, int32_t n_src,
                                   int32_t level, bt_beams **inout)
{
    return emit_beams(ctx, src_xyz, src_power, nullptr, n_src, level, inout);
}

extern "C" bt_status bt_emit_beams_directional(bt_ctx *ctx, const float *src_xyz, const float *src_power,
                                               const float *src_weight, int32_t n_src, int32_t level,
                                               bt_beams **inout)
{
    if (ctx && !src_weight) return fail(ctx, BT_EINVAL, "src_weight is NULL");
    return emit_beams(ctx, src_xyz, src_power, src_weight, n_src, level, inout);
}

extern "C" bt_status bt_beams_free(bt_beams *b)
{
    if (!b) return BT_EINVAL;
    for (bt_beams *&q : b->part) {
        if (q) bt_beams_free(q);
        q = nullptr;
    }
    beams_release(b);
    dev_free(b->ctx, b->ctr, sizeof(DevCounters));
    dev_free(b->ctx, b->ws_buf, b->ws_bytes);
    dev_free(b->ctx, b->src_dev, (size_t)b->src_cap * 3 * sizeof(float));
    dev_free(b->ctx, b->pow_dev, (size_t)b->src_cap * sizeof(float));
    dev_free(b->ctx, b->norm_dev, (size_t)b->src_cap * sizeof(double));
    dev_free(b->ctx, b->wt_dev, (size_t)b->wt_cap * sizeof(float));
    delete b;
    return BT_OK;
}

extern "C" bt_status bt_beams_stats(bt_ctx *ctx, const bt_beams *b, bt_stats *out)
{
    if (!ctx || !b || !out) return BT_EINVAL;
    // the counters of every partition (each partition's work is joined to the context's
    // stream by the call that enqueued it)
    const int K = b->n_parts;
    std::vector<DevCounters> hv(K);
    for (int k = 0; k < K; ++k)
        HIP_TRY(ctx, hipMemcpyAsync(&hv[k], part_of(b, k)->ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    std::memset(out, 0, sizeof *out);
    out->generations = b->gen;
    for (int k = 0; k < K; ++k) {
        const DevCounters &h = hv[k];
        const bt_beams *q = part_of(b, k);
        for (int g = 0; g <= BT_MAX_DEPTH; ++g) {
            if (g < q->gen) {
                out->count[g] += (int64_t)h.count[g];
                out->flagged[g] += (int64_t)h.flagged[g];
                out->power[g] += h.power[g];
                out->segments += (int64_t)h.count[g];
            }
        }
        out->node_visits += (int64_t)h.node_visits;
        out->tri_tests += (int64_t)h.tri_tests;
        out->mic_tests += (int64_t)mic_stat_total(h, MS_TESTS);
        out->mic_updates += (int64_t)mic_stat_total(h, MS_UPDATES);
        out->mic_layer_visits += (int64_t)mic_stat_total(h, MS_LAYERS);
        out->mic_classified += (int64_t)mic_stat_total(h, MS_CLASSIFIED);
        for (int g = 0; g <= BT_MAX_DEPTH; ++g) out->mic_general += (int64_t)h.n_layers[g];
        out->mic_fallback += (int64_t)mic_stat_total(h, MS_LAYER_FALLBACK);
    }
    // earlier source chunks of a bt_run
    const bt_stats &q = b->prior;
    out->generations = std::max(out->generations, q.generations);
    for (int g = 0; g <= BT_MAX_DEPTH; ++g) {
        out->count[g] += q.count[g];
        out->flagged[g] += q.flagged[g];
        out->power[g] += q.power[g];
    }
    out->segments += q.segments;
    out->node_visits += q.node_visits;
    out->tri_tests += q.tri_tests;
    out->mic_tests += q.mic_tests;
    out->mic_updates += q.mic_updates;
    out->mic_classified += q.mic_classified;
    out->mic_layer_visits += q.mic_layer_visits;
    out->mic_general += q.mic_general;
    out->mic_fallback += q.mic_fallback;
    return BT_OK;
}

bt_status check_params(bt_ctx *ctx, const bt_mesh *mesh, const bt_params *p)
{
    std::string msg;
    bt_status s = check_param_args(p, mesh->delta_cap, msg);
    if (s != BT_OK) return fail(ctx, s, "%s", msg.c_str());
    return BT_OK;
}

TraceArgs make_args(const bt_params *p, int gen)
{
    TraceArgs a{};
    a.gen = gen;
    a.max_depth = p->max_depth;
    a.t_min = p->t_min;
    a.delta = p->edge_delta;
    a.delta2 = p->edge_delta * p->edge_delta;
    a.air_m = p->air_m;
    a.e_min = p->e_min;
    a.queue_rounds = p->queue_rounds;
    a.hit_out = p->hit_out;
    a.flag_out = p->flag_out;
    a.t_out = p->t_out;
    return a;
}

// ---------------------------------------------------------------------------------------
// Partition streams.  A call on a partitioned set forks the context's stream: each
// partition stream first waits for the work enqueued on the context's stream so far,
// partition k's work goes to partition stream k, and before the call returns the
// context's stream waits for every partition stream, so the call's work is ordered on the
// context's stream as the ABI states.  The partition streams are created together, one
// after the other, so that the runtime spreads them over distinct hardware queues (two
// busy streams on one in-order hardware queue would run one after the other, with every
// small kernel's fixed cost paid twice); the context's own stream, idle while they run,
// may share a queue with one of them.
// ---------------------------------------------------------------------------------------
hipError_t partition_streams(bt_ctx *ctx)
{
    if (ctx->fork_ev) return hipSuccess;
    hipError_t e = hipSuccess;
    for (int k = 0; k < kMaxParts && e == hipSuccess; ++k) {
        // default priority, like the context's stream
        e = hipStreamCreateWithFlags(&ctx->part_stream[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->join_ev[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        for (int k = 0; k < kMaxParts; ++k) {
            if (ctx->part_stream[k]) (void)hipStreamDestroy(ctx->part_stream[k]);
            if (ctx->join_ev[k]) (void)hipEventDestroy(ctx->join_ev[k]);
            ctx->part_stream[k] = nullptr;
            ctx->join_ev[k] = nullptr;
        }
        ctx->fork_ev = nullptr;
    }
    return e;
}

class StreamFork {
public:
    StreamFork(bt_ctx *ctx, int n) : ctx_(ctx), n_(n) {}
    StreamFork(const StreamFork &) = delete;
    StreamFork &operator=(const StreamFork &) = delete;
    ~StreamFork() { (void)join(); }
    hipError_t begin()
    {
        if (n_ <= 1) return hipSuccess;
        hipError_t e = partition_streams(ctx_);
        if (e != hipSuccess) return e;
        if ((e = hipEventRecord(ctx_->fork_ev, ctx_->stream)) != hipSuccess) return e;
        forked_ = true;   // from here on, join() orders the context's stream after every partition stream
        for (int k = 0; k < n_; ++k)
            if ((e = hipStreamWaitEvent(ctx_->part_stream[k], ctx_->fork_ev, 0)) != hipSuccess) return e;
        return hipSuccess;
    }
    hipStream_t stream(int k) const { return forked_ ? ctx_->part_stream[k] : ctx_->stream; }
    // The context's stream waits for every partition stream (on failure to order them by
    // an event, the host waits for the partition stream instead).
    hipError_t join()
    {
        if (!forked_) return hipSuccess;
        forked_ = false;
        hipError_t first = hipSuccess;
        for (int k = 0; k < n_; ++k) {
            hipError_t e = hipEventRecord(ctx_->join_ev[k], ctx_->part_stream[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(ctx_->stream, ctx_->join_ev[k], 0);
            if (e != hipSuccess) {
                (void)hipStreamSynchronize(ctx_->part_stream[k]);
                if (first == hipSuccess) first = e;
            }
        }
        return first;
    }

private:
    bt_ctx *ctx_;
    int n_;
    bool forked_ = false;
};

extern "C" bt_status bt_set_partitions(bt_ctx *ctx, int32_t k)
{
    if (!ctx) return BT_EINVAL;
    if (k < 1 || k > kMaxParts) return fail(ctx, BT_EINVAL, "partitions %d not in 1..%d", k, kMaxParts);
    ctx->parts = k;
    return BT_OK;
}

// A partition's parameters: its parity-output rows start at its first beam's.
static bt_params part_params(const bt_params *p, const bt_beams *b)
{
    bt_params q = *p;
    const long long row0 = b->beam0 * (long long)(p->max_depth + 1);
    if (q.hit_out) q.hit_out += row0;
    if (q.flag_out) q.flag_out += row0;
    if (q.t_out) q.t_out += row0;
    return q;
}

// Checks and buffers before set (partition) b's next generation is traced; nothing is
// enqueued but the queue's growth on the context's stream.
static bt_status trace_prepare(bt_ctx *ctx, const bt_mesh *mesh, bt_beams *b, const bt_params *p)
{
    if (!b->emitted) return fail(ctx, BT_ESTATE, "the beam set holds no emission (emit beams first)");
    if (b->mesh && b->mesh != mesh)
        return fail(ctx, BT_EINVAL, "the beam set's generations were traced with another mesh");
    if (b->max_depth >= 0 && b->max_depth != p->max_depth)
        return fail(ctx, BT_EINVAL, "max_depth changed between generations (%d -> %d)", b->max_depth, p->max_depth);
    if (b->gen > p->max_depth) return fail(ctx, BT_ESTATE, "all %d generations already traced", p->max_depth + 1);
    if (b->r_src > mesh->r_eff) return fail(ctx, BT_EINVAL, "a source lies outside the region the mesh margins cover (|x| <= %g)", mesh->r_eff);
    if (b->ring && b->acc_gen < b->gen)
        return fail(ctx, BT_ESTATE, "two-slot beam set: accumulate generation %d before tracing the next", b->gen - 1);
    bt_status s;
    if (b->gen == 0 && !b->ring) {
        // every generation stays resident: at most n0 records each
        const long long total = std::max(b->n0, 1ll) * (long long)(p->max_depth + 1);
        if (total > (1ll << 31) - 1)
            return fail(ctx, BT_EINVAL, "n_beams0 * (max_depth + 1) = %lld exceeds 2^31 - 1", total);
        if ((s = reserve_queue(ctx, b, total, b->n0)) != BT_OK) return s;
        b->depth_hint = p->max_depth;
    }
    if (p->queue_rounds > 0 && (s = reserve_tiles(ctx, b, b->n0)) != BT_OK) return s;
    return BT_OK;
}

// Enqueue the trace of set (partition) b's next generation on stream st.
static bt_status trace_enqueue(bt_ctx *ctx, const bt_mesh *mesh, bt_beams *b, const bt_params *p, hipStream_t st)
{
    const int g = b->gen;
    b->max_depth = p->max_depth;
    b->mesh = mesh;
    const bt_params q = part_params(p, b);
    TraceArgs a = make_args(&q, g);
    a.cg = class_target(b);
    HIP_TRY(ctx, launch_trace(mesh->dev, b->q, b->segs, b->ctr, a, b->ws, trace_tiles(b, mesh, a), ctx->n_cu, st));
    b->gen = g + 1;
    if (g + 1 < 64) {
        if (b->bound) b->class_gens |= 1ull << (g + 1);
        else b->class_gens &= ~(1ull << (g + 1));
    }
    return BT_OK;
}

extern "C" bt_status bt_trace(bt_ctx *ctx, const bt_mesh *mesh, bt_beams *b, const bt_params *p, int64_t *n_next)
{
    if (!ctx) return BT_EINVAL;
    if (!mesh || !b) return fail(ctx, BT_EINVAL, "NULL mesh or beams");
    bt_status s = check_params(ctx, mesh, p);
    if (s != BT_OK) return s;
    (void)hipSetDevice(ctx->device);
    const int K = b->n_parts;
    for (int k = 0; k < K; ++k)
        if ((s = trace_prepare(ctx, mesh, part_of(b, k), p)) != BT_OK) return s;
    const int g = b->gen;
    {
        StreamFork f(ctx, K);
        HIP_TRY(ctx, f.begin());
        for (int k = 0; k < K; ++k)
            if ((s = trace_enqueue(ctx, mesh, part_of(b, k), p, f.stream(k))) != BT_OK) return s;
        HIP_TRY(ctx, f.join());
    }
    if (n_next) {
        unsigned long long c[kMaxParts] = {};
        for (int k = 0; k < K; ++k)
            HIP_TRY(ctx, hipMemcpyAsync(&c[k], &part_of(b, k)->ctr->count[g + 1], sizeof c[k], hipMemcpyDeviceToHost,
                                        ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        unsigned long long t = 0;
        for (int k = 0; k < K; ++k) t += c[k];
        *n_next = (int64_t)t;
    }
    return BT_OK;
}

extern "C" bt_status bt_trace_all(bt_ctx *ctx, const bt_mesh *mesh, bt_beams *b, const bt_params *p)
{
    if (!ctx) return BT_EINVAL;
    if (!mesh || !b) return fail(ctx, BT_EINVAL, "NULL mesh or beams");
    bt_status s = check_params(ctx, mesh, p);
    if (s != BT_OK) return s;
    if (b->ring) return fail(ctx, BT_ESTATE, "a two-slot beam set traces one generation per accumulation");
    (void)hipSetDevice(ctx->device);
    const int K = b->n_parts;
    for (int k = 0; k < K; ++k)
        if ((s = trace_prepare(ctx, mesh, part_of(b, k), p)) != BT_OK) return s;
    const int n_gen = p->max_depth + 1 - b->gen;
    StreamFork f(ctx, K);
    HIP_TRY(ctx, f.begin());
    // generation by generation, so that each stream is fed in turn; the streams do not
    // wait for each other until the join
    for (int i = 0; i < n_gen; ++i)
        for (int k = 0; k < K; ++k)
            if ((s = trace_enqueue(ctx, mesh, part_of(b, k), p, f.stream(k))) != BT_OK) return s;
    HIP_TRY(ctx, f.join());
    return BT_OK;
}

// The records' planar classes, when every generation of the pass [acc_gen, gen) was
// classified against this microphone set's grid (a planar grid or a subset of one);
// otherwise NULL and the pass decides from each frustum.  The decisions are the same.
static const int2 *pass_classes(const bt_beams *b, const bt_mics *m)
{
    if (!b->cgrid.cls || m->points || m->dev.nz != 1 || b->gen > 63) return nullptr;
    const ClassGrid &g = b->cgrid;
    if (g.x0 != m->dev.x0 || g.y0 != m->dev.y0 || g.z != m->dev.z || g.dx != m->dev.dx || g.dy != m->dev.dy ||
        g.nx != m->dev.nx || g.ny != m->dev.ny)
        return nullptr;
    for (int k = b->acc_gen; k < b->gen; ++k)
        if (!((b->class_gens >> k) & 1ull)) return nullptr;
    return g.cls;
}

extern "C" bt_status bt_beams_bind_mics(bt_ctx *ctx, bt_beams **beams, const bt_mics *mics)
{
    if (!ctx) return BT_EINVAL;
    if (!beams) return fail(ctx, BT_EINVAL, "beams is NULL");
    if (mics && (mics->points || mics->dev.nz != 1))
        return fail(ctx, BT_EINVAL, "only a planar grid (or a subset of one) classifies beams");
    if (mics && (mics->dev.nx >= kClassMaxDim || mics->dev.ny >= kClassMaxDim))
        return fail(ctx, BT_EINVAL, "grid of %d x %d microphones: at most %d per side classify beams", mics->dev.nx,
                    mics->dev.ny, kClassMaxDim - 1);
    (void)hipSetDevice(ctx->device);
    bt_status s;
    if (!*beams && (s = new_beams(ctx, beams)) != BT_OK) return s;
    bt_beams *b = *beams;
    ClassGrid g{};
    if (mics) {
        const DevMics &m = mics->dev;
        g.x0 = m.x0;
        g.y0 = m.y0;
        g.z = m.z;
        g.dx = m.dx;
        g.dy = m.dy;
        g.nx = m.nx;
        g.ny = m.ny;
    }
    // the set and every partition it holds (later emissions bind new partitions alike)
    for (int k = 0; k < kMaxParts; ++k) {
        bt_beams *q = part_of(b, k);
        if (q && (s = bind_set(ctx, q, mics ? &g : nullptr)) != BT_OK) return s;
    }
    return BT_OK;
}

// Buffers of set (partition) b's microphone pass (allocation only).
static bt_status accumulate_prepare(bt_ctx *ctx, bt_beams *b, const bt_mics *mics)
{
    if (!mics->points && mics->dev.nz > 1) return reserve_layers(ctx, b);
    return BT_OK;
}

// Enqueue the microphone pass over set (partition) b's generations traced since its
// previous pass, on stream st, with its own work lists.
static bt_status accumulate_enqueue(bt_ctx *ctx, const bt_mesh *mesh, bt_beams *b, const bt_params *p, bt_mics *mics,
                                    hipStream_t st)
{
    if (b->acc_gen == b->gen) return BT_OK;
    TraceArgs a = make_args(p, b->acc_gen);
    a.gen_end = b->gen;
    a.mic_cls = pass_classes(b, mics);
    if (mics->points) {
        HIP_TRY(ctx, launch_mics_points(mesh->dev, b->q, b->segs, b->ctr, mics->dev, mics->pts, a, ctx->n_cu, st));
    } else {
        MicWork w{b->rows, b->rows_cap, b->spans, b->spans_cap, b->big_list + b->cap, b->big_list, b->layers,
                  b->layers_cap, b->layer_cnt};
        HIP_TRY(ctx, launch_mics(mesh->dev, b->q, b->segs, b->ctr, mics->dev, a, w, b->ws, ctx->n_cu, st));
    }
    b->acc_gen = b->gen;
    return BT_OK;
}

extern "C" bt_status bt_accumulate_mics(bt_ctx *ctx, const bt_mesh *mesh, bt_beams *b, const bt_params *p,
                                        bt_mics *mics)
{
    if (!ctx) return BT_EINVAL;
    if (!mesh || !b || !mics) return fail(ctx, BT_EINVAL, "NULL mesh, beams or mics");
    bt_status s = check_params(ctx, mesh, p);
    if (s != BT_OK) return s;
    if (!b->emitted) return fail(ctx, BT_ESTATE, "the beam set holds no emission (emit beams first)");
    if (b->gen == 0) return fail(ctx, BT_ESTATE, "no generation traced yet");
    if (b->mesh != mesh) return fail(ctx, BT_EINVAL, "the beam set was traced with another mesh");
    if (b->acc_gen == b->gen) return BT_OK;  // nothing traced since the last call
    (void)hipSetDevice(ctx->device);
    // all generations traced since the previous call, in one pass per partition; the
    // partitions' passes run on their own streams (their contributions meet only in the
    // microphones' FP64 atomic additions)
    const int K = b->n_parts;
    for (int k = 0; k < K; ++k)
        if ((s = accumulate_prepare(ctx, part_of(b, k), mics)) != BT_OK) return s;
    StreamFork f(ctx, K);
    HIP_TRY(ctx, f.begin());
    for (int k = 0; k < K; ++k)
        if ((s = accumulate_enqueue(ctx, mesh, part_of(b, k), p, mics, f.stream(k))) != BT_OK) return s;
    HIP_TRY(ctx, f.join());
    return BT_OK;
}

// The allocation-free variant: the same kernels, with their work lists in the device's
// static work area instead of the beam set's buffers.
extern "C" bt_status bt_accumulate_mics_static(bt_ctx *ctx, const bt_mesh *mesh, bt_beams *b, const bt_params *p,
                                               bt_mics *mics)
{
    if (!ctx) return BT_EINVAL;
    if (!mesh || !b || !mics) return fail(ctx, BT_EINVAL, "NULL mesh, beams or mics");
    bt_status s = check_params(ctx, mesh, p);
    if (s != BT_OK) return s;
    if (!b->emitted) return fail(ctx, BT_ESTATE, "the beam set holds no emission (emit beams first)");
    if (b->gen == 0) return fail(ctx, BT_ESTATE, "no generation traced yet");
    if (b->mesh != mesh) return fail(ctx, BT_EINVAL, "the beam set was traced with another mesh");
    if (b->acc_gen == b->gen) return BT_OK;  // nothing traced since the last call
    if (!ctx->scratch) return fail(ctx, BT_EDEVICE, "no static work area on device %d", ctx->device);
    (void)hipSetDevice(ctx->device);
    // the partitions share the device's static area, so their passes run one after the
    // other on the context's stream; every partition is checked before any is enqueued
    const int K = b->n_parts;
    const int W = b->ws.n_waves;
    if (W > kStaticMaxWaves) return fail(ctx, BT_EINVAL, "%d waves exceed the static work area's %d", W, kStaticMaxWaves);
    const long long n_max = (kStaticListInts - 64ll * (W + 1)) / 2;
    for (int k = 0; k < K && !mics->points; ++k) {
        // segments of this pass: at most n0 per generation
        const bt_beams *q = part_of(b, k);
        const long long n_bound = std::max(q->n0, 1ll) * (long long)(q->gen - q->acc_gen);
        if (n_bound > n_max)
            return fail(ctx, BT_EINVAL,
                        "this pass may hold %lld segments (%lld generation-0 beams x %d generations), more than the "
                        "static work area's %lld; accumulate after fewer generations",
                        n_bound, q->n0, q->gen - q->acc_gen, n_max);
    }
    for (int k = 0; k < K; ++k) {
        bt_beams *q = part_of(b, k);
        TraceArgs a = make_args(p, q->acc_gen);
        a.gen_end = q->gen;
        a.mic_cls = pass_classes(q, mics);
        if (mics->points) {   // the point kernel uses no work lists
            HIP_TRY(ctx, launch_mics_points(mesh->dev, q->q, q->segs, q->ctr, mics->dev, mics->pts, a, ctx->n_cu,
                                            ctx->stream));
        } else {
            const long long n_bound = std::max(q->n0, 1ll) * (long long)(q->gen - q->acc_gen);
            char *base = (char *)ctx->scratch;
            WaveScratch ws = q->ws;
            ws.general = (unsigned *)base;
            int *lists = (int *)(base + kStaticListsOffset);
            MicWork w{(int2 *)(base + kStaticRowsOffset), kStaticRows, (int4 *)(base + kStaticSpansOffset),
                      kStaticSpans, lists + n_bound, lists, (int2 *)(base + kStaticLayersOffset), kStaticLayers,
                      (unsigned *)(base + kStaticLayerCntOffset)};
            HIP_TRY(ctx, launch_mics(mesh->dev, q->q, q->segs, q->ctr, mics->dev, a, w, ws, ctx->n_cu, ctx->stream));
        }
        q->acc_gen = q->gen;
    }
    return BT_OK;
}

extern "C" bt_status bt_levels(bt_ctx *ctx, const bt_mics *m, double *strict_out, double *flag_out, double *level_db_out)
{
    if (!ctx || !m) return BT_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (m->sel) {   // a subset: its points, in subset order
        const long long n = m->n_out;
        const size_t bytes = (size_t)n * sizeof(double);
        HIP_TRY(ctx, launch_select(m->dev.e_strict, m->dev.e_flag, m->sel, n, m->sel_buf, m->sel_buf + n,
                                   m->sel_buf + 2 * n, ctx->stream));
        if (strict_out) HIP_TRY(ctx, hipMemcpyAsync(strict_out, m->sel_buf, bytes, hipMemcpyDefault, ctx->stream));
        if (flag_out) HIP_TRY(ctx, hipMemcpyAsync(flag_out, m->sel_buf + n, bytes, hipMemcpyDefault, ctx->stream));
        if (level_db_out)
            HIP_TRY(ctx, hipMemcpyAsync(level_db_out, m->sel_buf + 2 * n, bytes, hipMemcpyDefault, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        return BT_OK;
    }
    long long n = mic_energies(m);
    size_t bytes = (size_t)n * sizeof(double);
    if (level_db_out) {
        HIP_TRY(ctx, launch_levels(m->dev.e_strict, m->dev.e_flag, m->level, n, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(level_db_out, m->level, bytes, hipMemcpyDefault, ctx->stream));
    }
    if (strict_out) HIP_TRY(ctx, hipMemcpyAsync(strict_out, m->dev.e_strict, bytes, hipMemcpyDefault, ctx->stream));
    if (flag_out) HIP_TRY(ctx, hipMemcpyAsync(flag_out, m->dev.e_flag, bytes, hipMemcpyDefault, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return BT_OK;
}

// Generation-0 beams of a bt_run source chunk at most (a chunk in two generation slots
// holds twice this), and the default record budget for keeping every generation.
constexpr long long kRunChunkBeams = 1ll << 24;
constexpr long long kRunResidentRecords = 1ll << 26;

extern "C" bt_status bt_run(bt_ctx *ctx, const bt_mesh *mesh, const float *src_xyz, const float *src_power,
                            int32_t n_src, int32_t level, const bt_params *p, bt_mics *mics, bt_beams **beams)
{
    if (!ctx) return BT_EINVAL;
    if (!mesh || !mics || !beams) return fail(ctx, BT_EINVAL, "NULL mesh, mics or beams");
    bt_status s = check_params(ctx, mesh, p);
    if (s != BT_OK) return s;
    if (level < 0 || level > BT_MAX_LEVEL) return fail(ctx, BT_EINVAL, "level %d not in 0..%d", level, BT_MAX_LEVEL);
    if (n_src < 0 || (n_src > 0 && (!src_xyz || !src_power))) return fail(ctx, BT_EINVAL, "bad sources");
    // Sources in chunks of at most kRunChunkBeams generation-0 beams (at least one source).
    // The run keeps every generation when the largest chunk's records fit the record budget
    // (one microphone pass per chunk), else two generation slots (a pass per generation),
    // so memory is bounded whatever the number of sources, depth or level.  Parity outputs
    // keep their global rows.
    const long long nf = 20ll << (2 * level);
    const long long per = std::max(1ll, kRunChunkBeams / nf);
    const long long budget = p->run_records > 0 ? p->run_records : kRunResidentRecords;
    const long long largest = std::max(1ll, std::min<long long>(per, n_src));
    const bool resident = largest * nf * (long long)(p->max_depth + 1) <= budget;
    // beams classified against a planar grid as they are created (the microphone pass
    // then dismisses most of them without reading their frustums)
    const bool planar = !mics->points && mics->dev.nz == 1 && mics->dev.nx < kClassMaxDim &&
                        mics->dev.ny < kClassMaxDim;
    if ((s = bt_beams_bind_mics(ctx, beams, planar ? mics : nullptr)) != BT_OK) return s;
    bt_stats total{};
    for (long long c0 = 0; c0 < std::max<long long>(n_src, 1); c0 += per) {
        const int32_t nc = (int32_t)std::min<long long>(per, (long long)n_src - c0);
        if (c0 > 0) {
            // the finished chunk's statistics carry over (one synchronisation per chunk)
            bt_stats st;
            if ((s = bt_beams_stats(ctx, *beams, &st)) != BT_OK) return s;
            total = st;
        }
        if (resident && *beams) (*beams)->depth_hint = p->max_depth;   // size the queue at emission
        s = emit_beams(ctx, nc > 0 ? src_xyz + 3 * c0 : src_xyz, nc > 0 ? src_power + c0 : src_power, nullptr,
                       std::max(nc, 0), level, beams, !resident);
        if (s != BT_OK) return s;
        bt_beams *b = *beams;
        b->prior = total;
        bt_params pc = *p;
        const long long row0 = c0 * nf * (long long)(p->max_depth + 1);
        if (p->hit_out) pc.hit_out = p->hit_out + row0;
        if (p->flag_out) pc.flag_out = p->flag_out + row0;
        if (p->t_out) pc.t_out = p->t_out + row0;
        // each partition of the chunk runs its whole method on its own stream: every
        // generation's trace, and its microphone pass after each generation (two slots)
        // or once after the last (resident); the streams meet again at the chunk's end
        const int K = b->n_parts;
        for (int k = 0; k < K; ++k) {
            if ((s = trace_prepare(ctx, mesh, part_of(b, k), &pc)) != BT_OK) return s;
            if ((s = accumulate_prepare(ctx, part_of(b, k), mics)) != BT_OK) return s;
        }
        {
            StreamFork f(ctx, K);
            HIP_TRY(ctx, f.begin());
            for (int g = 0; g <= p->max_depth; ++g)
                for (int k = 0; k < K; ++k) {
                    if ((s = trace_enqueue(ctx, mesh, part_of(b, k), &pc, f.stream(k))) != BT_OK) return s;
                    if (!resident && (s = accumulate_enqueue(ctx, mesh, part_of(b, k), &pc, mics, f.stream(k))) != BT_OK)
                        return s;
                }
            if (resident)
                for (int k = 0; k < K; ++k)
                    if ((s = accumulate_enqueue(ctx, mesh, part_of(b, k), &pc, mics, f.stream(k))) != BT_OK) return s;
            HIP_TRY(ctx, f.join());
        }
        if (nc <= 0) break;
    }
    return BT_OK;
}

// ---------------------------------------------------------------------------------------
// request interface: each submission is enqueued on the context stream at once (one
// request per launch sequence); bt_poll reports completion through an event.
// ---------------------------------------------------------------------------------------
extern "C" bt_status bt_submit(bt_ctx *ctx, const bt_mesh *mesh, const bt_request *req, uint64_t *ticket)
{
    if (!ctx) return BT_EINVAL;
    if (!mesh || !req || !ticket) return fail(ctx, BT_EINVAL, "NULL mesh, request or ticket");
    std::lock_guard<std::mutex> lk(ctx->mtx);
    if (req->n_src < 0 || (req->n_src > 0 && (!req->src_xyz || !req->src_power)))
        return fail(ctx, BT_EINVAL, "bad request sources");
    bt_params p;
    bt_params_default(&p);
    p.max_depth = req->max_depth;
    bt_status s = check_params(ctx, mesh, &p);
    if (s != BT_OK) return s;
    Request *r = new Request();
    r->req = *req;
    r->src.assign(req->src_xyz, req->src_xyz + 3 * (size_t)req->n_src);
    r->pw.assign(req->src_power, req->src_power + (size_t)req->n_src);
    s = bt_mics_grid(ctx, req->mic_x0, req->mic_y0, req->mic_z, req->mic_dx, req->mic_dy, req->mic_nx, req->mic_ny,
                     &r->mics);
    if (s == BT_OK) s = bt_run(ctx, mesh, r->src.data(), r->pw.data(), req->n_src, req->level, &p, r->mics, &r->beams);
    if (s == BT_OK && hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess) s = BT_EDEVICE;
    if (s == BT_OK && hipEventRecord(r->done, ctx->stream) != hipSuccess) s = BT_EDEVICE;
    if (s != BT_OK) {
        if (r->done) (void)hipEventDestroy(r->done);
        if (r->mics) bt_mics_free(r->mics);
        if (r->beams) bt_beams_free(r->beams);
        delete r;
        return s;
    }
    *ticket = ctx->next_ticket++;
    ctx->requests[*ticket] = r;
    return BT_OK;
}

extern "C" bt_status bt_poll(bt_ctx *ctx, uint64_t ticket, bt_result *out)
{
    if (!ctx) return BT_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mtx);
    auto it = ctx->requests.find(ticket);
    if (it == ctx->requests.end()) return fail(ctx, BT_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    hipError_t q = hipEventQuery(r->done);
    if (q == hipErrorNotReady) return BT_PENDING;
    if (q != hipSuccess) return hip_fail(ctx, q, "hipEventQuery");
    if (!out) return fail(ctx, BT_EINVAL, "out is NULL");
    long long n = (long long)r->req.mic_nx * r->req.mic_ny;
    std::vector<double> es((size_t)n), ef((size_t)n);
    bt_status s = bt_levels(ctx, r->mics, es.data(), ef.data(), nullptr);
    if (s != BT_OK) return s;
    bt_stats st;
    if ((s = bt_beams_stats(ctx, r->beams, &st)) != BT_OK) return s;
    if (out->energy)
        for (long long i = 0; i < n; ++i) out->energy[i] = es[i] + ef[i];
    if (out->flag_energy) std::memcpy(out->flag_energy, ef.data(), (size_t)n * sizeof(double));
    out->segments = st.segments;
    out->mic_updates = st.mic_updates;
    (void)hipEventDestroy(r->done);
    bt_mics_free(r->mics);
    bt_beams_free(r->beams);
    delete r;
    ctx->requests.erase(it);
    return BT_OK;
}

extern "C" bt_status bt_cancel(bt_ctx *ctx, uint64_t ticket)
{
    if (!ctx) return BT_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mtx);
    auto it = ctx->requests.find(ticket);
    if (it == ctx->requests.end()) return fail(ctx, BT_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    (void)hipEventSynchronize(r->done);  // device work cannot be withdrawn once enqueued
    (void)hipEventDestroy(r->done);
    bt_mics_free(r->mics);
    bt_beams_free(r->beams);
    delete r;
    ctx->requests.erase(it);
    return BT_OK;
}
