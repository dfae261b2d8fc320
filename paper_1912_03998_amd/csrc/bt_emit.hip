// Emission (single sets and scenario tables), counter initialisation, fills, levels and
// output gathers (subsets, batch outputs).
#include "bt_device.h"

namespace bt {

// ---------------------------------------------------------------------------------------
// counters
// ---------------------------------------------------------------------------------------
__global__ void k_init_counters(DevCounters *ctr, long long n0, long long ring)
{
    unsigned long long *w = reinterpret_cast<unsigned long long *>(ctr);
    const int nw = (int)(sizeof(DevCounters) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0ull;  // doubles: +0.0 bits
    __syncthreads();
    if (threadIdx.x == 0) {
        ctr->count[0] = (unsigned long long)n0;
        ctr->ring = (unsigned long long)ring;
    }
}

hipError_t launch_init_counters(DevCounters *ctr, long long n0, long long ring, hipStream_t s)
{
    k_init_counters<<<1, 256, 0, s>>>(ctr, n0, ring);
    return hipGetLastError();
}

__global__ void k_fill(double *p, long long n, double v)
{
    long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_zero_ints(int *p, long long n)
{
    long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

hipError_t launch_zero_ints(int *p, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    k_zero_ints<<<(unsigned)blocks, 256, 0, s>>>(p, n);
    return hipGetLastError();
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
// Face `f` of the level-`level` icosphere: its three edge directions, the guiding
// direction and the solid angle.
__device__ void face_of(const double *__restrict__ base20, int level, long long f, V3 &a, V3 &bb, V3 &c, V3 &cc,
                        double &om)
{
    int bf = (int)(f >> (2 * level));
    const double *bp = base20 + 9 * bf;
    a = {bp[0], bp[1], bp[2]};
    bb = {bp[3], bp[4], bp[5]};
    c = {bp[6], bp[7], bp[8]};
    for (int l = level - 1; l >= 0; --l) {
        int k = (int)((f >> (2 * l)) & 3);
        V3 ab = unit(a + bb), bc = unit(bb + c), ca = unit(c + a);
        if (k == 0) { bb = ab; c = ca; }
        else if (k == 1) { a = ab; c = bc; }
        else if (k == 2) { a = ca; bb = bc; }
        else { a = ab; bb = bc; c = ca; }
    }
    cc = unit((a + bb) + c);
    double num = fabs(dot(a, cross(bb, c)));
    double den = 1.0 + dot(a, bb) + dot(bb, c) + dot(c, a);
    om = 2.0 * atan2(num, den);
}

// A generation-0 beam record at queue index j: apex and origin at the source S, the face's
// directions, intensity constant K (W/sr) and power P = K Omega (W).
__device__ __forceinline__ void store_beam(DevQueue q, long long j, V3 S, V3 a, V3 bb, V3 c, V3 cc, double K,
                                           double om, int meta, int id)
{
    const long long cap = q.cap;
    st3(q.dbl + D_A * cap, cap, j, S);
    st3(q.dbl + D_D0 * cap, cap, j, a);
    st3(q.dbl + D_D1 * cap, cap, j, bb);
    st3(q.dbl + D_D2 * cap, cap, j, c);
    st3(q.dbl + D_O * cap, cap, j, S);
    st3(q.dbl + D_C * cap, cap, j, cc);
    q.flt[F_K * cap + j] = (float)K;
    q.dbl[D_P * cap + j] = K * om;
    q.ints[I_ID * cap + j] = id;
    q.ints[I_START * cap + j] = -1;
    q.ints[I_META * cap + j] = meta;
}

// Beam `f` (face index) of a level-`level` source at S with power W, written at queue
// index j.
__device__ void emit_one(const double *__restrict__ base20, int level, long long f, V3 S, float W, int meta, int id,
                         DevQueue q, long long j)
{
    V3 a, bb, c, cc;
    double om;
    face_of(base20, level, f, a, bb, c, cc, om);
    store_beam(q, j, S, a, bb, c, cc, (double)W / (4.0 * M_PI), om, meta, id);
}

// The face table of one level, computed once: dirs[k * nf + f] for k = 0..11 (d0, d1, d2,
// c) and om[f].
__global__ void k_faces(const double *__restrict__ base20, int level, long long nf, double *dirs, double *om)
{
    const long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    V3 a, bb, c, cc;
    face_of(base20, level, f, a, bb, c, cc, om[f]);
    st3(dirs, nf, f, a);
    st3(dirs + 3 * nf, nf, f, bb);
    st3(dirs + 6 * nf, nf, f, c);
    st3(dirs + 9 * nf, nf, f, cc);
}

hipError_t launch_faces(const double *base20, int level, double *dirs, double *om, hipStream_t s)
{
    const long long nf = 20ll << (2 * level);
    k_faces<<<(unsigned)((nf + 255) / 256), 256, 0, s>>>(base20, level, nf, dirs, om);
    return hipGetLastError();
}

// Generation 0 of one beam set: beam b = s nf + f is face f of source s, copied from the
// level's face table.  An omni source has K = W / (4 pi); a directional one (weights
// w[s nf + f]) K = W w / norm[s], norm[s] = sum over faces of w Omega, so that its beams'
// powers K Omega add up to W.
__global__ void k_emit(const double *__restrict__ dirs, const double *__restrict__ fom, const float *__restrict__ src,
                       const float *__restrict__ power, const float *__restrict__ wt, const double *__restrict__ norm,
                       int n_src, long long nf, DevQueue q, ClassGrid cg)
{
    long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    long long total = nf * n_src;
    if (b >= total) return;
    long long s = b / nf, f = b - s * nf;
    const V3 S = {src[3 * s], src[3 * s + 1], src[3 * s + 2]};
    double K;
    if (wt) K = norm[s] > 0.0 ? (double)power[s] * (double)wt[b] / norm[s] : 0.0;
    else K = (double)power[s] / (4.0 * M_PI);
    const V3 d0 = ld3(dirs, nf, f), d1 = ld3(dirs + 3 * nf, nf, f), d2 = ld3(dirs + 6 * nf, nf, f);
    store_beam(q, b, S, d0, d1, d2, ld3(dirs + 9 * nf, nf, f), K, fom[f], 0, (int)b);
    if (cg.cls) cg.cls[b] = plane_class(cg, S, d0, d1, d2);
}

// norm[s] = sum over faces f of wt[s nf + f] Omega_f (FP64, one block per source, a fixed
// reduction order).
__global__ void __launch_bounds__(256) k_source_norms(const double *__restrict__ fom, const float *__restrict__ wt,
                                                      long long nf, double *norm)
{
    __shared__ double part[256];
    const long long s = blockIdx.x;
    double acc = 0.0;
    for (long long f = threadIdx.x; f < nf; f += blockDim.x) acc += (double)wt[s * nf + f] * fom[f];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) norm[s] = part[0];
}

hipError_t launch_emit(const double *dirs, const double *om, const float *src, const float *power, const float *wt,
                       double *norm, int n_src, int level, DevQueue q, ClassGrid cg, hipStream_t s)
{
    long long nf = 20ll << (2 * level);
    long long total = nf * n_src;
    if (total <= 0) return hipSuccess;
    if (wt) {
        k_source_norms<<<(unsigned)n_src, 256, 0, s>>>(om, wt, nf, norm);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_emit<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(dirs, om, src, power, wt, norm, n_src, nf, q, cg);
    return hipGetLastError();
}

// Beams of an emission table appended to generation `gen` after its current count[gen]
// beams; the grid strides over the table's beams.
__global__ void k_emit_table(const double *__restrict__ base20, EmitTable t, DevQueue q, const DevCounters *ctr,
                             int gen)
{
    const long long total = t.dims[0];
    const int n = (int)t.dims[1];
    if (n <= 0) return;
    const long long base = (long long)(gen_start(ctr, gen) + ctr->count[gen]);
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < total; b += stride) {
        // the source whose beam range holds b: first[lo] <= b < first[hi + 1]
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (t.first[mid] <= b) lo = mid;
            else hi = mid - 1;
        }
        const long long f = b - t.first[lo];
        const V3 S = {t.src[3 * lo], t.src[3 * lo + 1], t.src[3 * lo + 2]};
        emit_one(base20, t.level[lo], f, S, t.power[lo], t.meta[lo], t.id0[lo] + (int)f, q, base + b);
    }
}

__global__ void k_count_add(DevCounters *ctr, int gen, const long long *n)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->count[gen] += (unsigned long long)n[0];
}

hipError_t launch_emit_table(const double *base20, const EmitTable &t, long long max_total, DevQueue q,
                             DevCounters *ctr, int gen, hipStream_t s)
{
    long long blocks = (max_total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_emit_table<<<(unsigned)blocks, 256, 0, s>>>(base20, t, q, ctr, gen);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_count_add<<<1, 64, 0, s>>>(ctr, gen, t.dims);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Batch chunks: zero the energies, and gather each scenario's outputs (strict + flag,
// and flag) from its grid arrays; sizes come from the chunk descriptor.
// ---------------------------------------------------------------------------------------
__global__ void k_fill_desc(double *p, const BatchDesc *d)
{
    const long long n = d->n_fill;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

__global__ void k_gather(const double *__restrict__ e, const long long *__restrict__ idx, const BatchDesc *d,
                         double *__restrict__ out_e, double *__restrict__ out_f)
{
    const long long n = d->n_out, es = d->e_stride;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += stride) {
        const long long i = idx[k];
        const double f = e[es + i];
        out_e[k] = e[i] + f;
        out_f[k] = f;
    }
}

hipError_t launch_fill_desc(double *p, const BatchDesc *d, long long max_n, hipStream_t s)
{
    long long blocks = (max_n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    k_fill_desc<<<(unsigned)blocks, 256, 0, s>>>(p, d);
    return hipGetLastError();
}

hipError_t launch_gather(const double *e, const long long *idx, const BatchDesc *d, long long max_n, double *out_e,
                         double *out_f, hipStream_t s)
{
    long long blocks = (max_n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    k_gather<<<(unsigned)blocks, 256, 0, s>>>(e, idx, d, out_e, out_f);
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

// A subset of a grid: its points' strict and flag energies and levels, in subset order.
__global__ void k_select(const double *__restrict__ es, const double *__restrict__ ef,
                         const long long *__restrict__ sel, long long n, double *__restrict__ out_s,
                         double *__restrict__ out_f, double *__restrict__ out_level)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += stride) {
        const long long i = sel[k];
        const double a = es[i], b = ef[i], e = a + b;
        out_s[k] = a;
        out_f[k] = b;
        out_level[k] = e > 0.0 ? 10.0 * log10(e / 1e-12) : -INFINITY;
    }
}

hipError_t launch_select(const double *es, const double *ef, const long long *sel, long long n, double *out_s,
                         double *out_f, double *out_level, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_select<<<(unsigned)blocks, 256, 0, s>>>(es, ef, sel, n, out_s, out_f, out_level);
    return hipGetLastError();
}

}  // namespace bt
