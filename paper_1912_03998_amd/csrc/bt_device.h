// Device-side helpers shared by the HIP kernels of the hybrid beam tracer (gfx950,
// CDNA4, wave64): FP64 vector algebra, SoA queue access, wave64 reductions and the
// static work partition.
#pragma once

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

// Static work partition: wave w of the grid takes the 64-item batches w, w + W, w + 2W...
// (W = waves in the grid).  Device-scope atomics on a shared cursor cost a round trip past
// the XCD's L2 and serialise thousands of waves on one address, so none are used to hand
// out work.
__device__ __forceinline__ unsigned long long wave_first_batch()
{
    return ((unsigned long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6 << 6;
}
__device__ __forceinline__ unsigned long long wave_batch_stride()
{
    return (unsigned long long)gridDim.x * blockDim.x;
}

// First queue index of generation g: the sizes of the generations before it (resident
// layout), or its slot (two-slot layout).
__device__ __forceinline__ unsigned long long gen_start(const DevCounters *ctr, int g)
{
    if (ctr->ring) return (unsigned long long)(g & 1) * ctr->ring;
    unsigned long long s = 0;
    for (int k = 0; k < g; ++k) s += ctr->count[k];
    return s;
}
// Segments of generations [g0, g1) (contiguous in the queue; one generation in the
// two-slot layout).
__device__ __forceinline__ unsigned long long gen_count(const DevCounters *ctr, int g0, int g1)
{
    unsigned long long s = 0;
    for (int k = g0; k < g1; ++k) s += ctr->count[k];
    return s;
}

// ---------------------------------------------------------------------------------------
// Planar microphone fast path.  A frustum with apex A and edge directions d0, d1, d2 on
// the grid plane z (lattice x0 + i dx, y0 + j dy, i < nx, j < ny): 0 = no microphone can
// be inside it, 1 = the candidates are the lattice box [i0, i1] x [j0, j1] (at most
// kPlaneBox points), 2 = the clipped footprint is needed.  When all three edge rays cross
// the plane ahead of the apex, the frustum meets the plane inside the triangle of the
// three crossing points (the caps only cut it down), so the lattice points of that
// triangle's bounding box are the only candidates.  It depends on the frustum alone (not
// on the hit), so the kernels that create a beam can decide it while the beam is in
// registers, and the microphone pass gets the same decision from the stored record.
// ---------------------------------------------------------------------------------------
constexpr int kPlaneBox = 32;

__device__ __forceinline__ int plane_decide(V3 A, V3 d0, V3 d1, V3 d2, double x0, double y0, double z, double dx,
                                            double dy, int nx, int ny, int &i0, int &i1, int &j0, int &j1)
{
    const double zr = z - A.z;
    bool proper = zr != 0.0;
    // the frustum lies in the cone of its edge directions from the apex; when the apex is
    // off the microphone plane (by far more than the plane tests' rounding) and no edge
    // direction turns towards the plane, no microphone can be inside
    bool away = zr > 1e-6 || zr < -1e-6;
    // The crossing points are only used to bound the candidate lattice, so they are found
    // in FP32: each coordinate is within 16 x 2^-24 of `mag` (the largest magnitude
    // involved) of its exact value, and the box is widened by 1e-5 mag.  The exact FP64
    // membership test decides every candidate.
    const float zrf = (float)zr, axf = (float)A.x, ayf = (float)A.y;
    float xmn = INFINITY, xmx = -INFINITY, ymn = INFINITY, ymx = -INFINITY;
    float mag = fmaxf(fabsf(axf), fabsf(ayf));
    const V3 d[3] = {d0, d1, d2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        proper = proper && (zr > 0.0 ? d[k].z > 0.0 : d[k].z < 0.0);
        away = away && (zr > 0.0 ? d[k].z <= 0.0 : d[k].z >= 0.0);
        const float s = zrf / (float)d[k].z;
        proper = proper && isfinite(s);  // FP32 overflow: the general path decides
        const float sx = s * (float)d[k].x, sy = s * (float)d[k].y;
        const float px = axf + sx, py = ayf + sy;
        xmn = fminf(xmn, px); xmx = fmaxf(xmx, px);
        ymn = fminf(ymn, py); ymx = fmaxf(ymx, py);
        mag = fmaxf(mag, fmaxf(fabsf(sx), fabsf(sy)));
    }
    if (away) return 0;
    if (!proper) return 2;
    // lattice range by a reciprocal multiply, widened by 1e-9 cells for its rounding
    const double relax = 1e-6 + 1e-5 * (double)mag;
    const double idx = 1.0 / dx, idy = 1.0 / dy;
    const double fi0 = fmax(ceil(((double)xmn - relax - x0) * idx - 1e-9), 0.0);
    const double fi1 = fmin(floor(((double)xmx + relax - x0) * idx + 1e-9), (double)(nx - 1));
    const double fj0 = fmax(ceil(((double)ymn - relax - y0) * idy - 1e-9), 0.0);
    const double fj1 = fmin(floor(((double)ymx + relax - y0) * idy + 1e-9), (double)(ny - 1));
    if (!(fi0 <= fi1 && fj0 <= fj1)) return 0;  // no lattice point under the footprint
    if ((fi1 - fi0 + 1.0) * (fj1 - fj0 + 1.0) > (double)kPlaneBox) return 2;
    i0 = (int)fi0; i1 = (int)fi1; j0 = (int)fj0; j1 = (int)fj1;
    return 1;
}

// The decision stored per record: (-1, 0) none inside, (-2, 0) clipped footprint, else
// the box as (i0 + (i1 - i0) 2^26, j0 + (j1 - j0) 2^26) (grids narrower than 2^26, box
// sides of at most kPlaneBox points).
__device__ __forceinline__ int2 plane_code(int kind, int i0, int i1, int j0, int j1)
{
    if (kind == 0) return make_int2(-1, 0);
    if (kind == 2) return make_int2(-2, 0);
    return make_int2(i0 | ((i1 - i0) << 26), j0 | ((j1 - j0) << 26));
}
__device__ __forceinline__ int plane_uncode(int2 c, int &i0, int &i1, int &j0, int &j1)
{
    if (c.x == -1) return 0;
    if (c.x == -2) return 2;
    i0 = c.x & (kClassMaxDim - 1);
    i1 = i0 + (c.x >> 26);
    j0 = c.y & (kClassMaxDim - 1);
    j1 = j0 + (c.y >> 26);
    return 1;
}
// The decision for a beam being created, against a classification grid.
__device__ __forceinline__ int2 plane_class(const ClassGrid &g, V3 A, V3 d0, V3 d1, V3 d2)
{
    int i0 = 0, i1 = -1, j0 = 0, j1 = -1;
    const int kind = plane_decide(A, d0, d1, d2, g.x0, g.y0, g.z, g.dx, g.dy, g.nx, g.ny, i0, i1, j0, j1);
    return plane_code(kind, i0, i1, j0, j1);
}

}  // namespace bt
