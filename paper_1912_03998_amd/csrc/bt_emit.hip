// Emission, counter initialisation, fills and levels.
#include "bt_device.h"

namespace bt {

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
