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

}  // namespace bt
