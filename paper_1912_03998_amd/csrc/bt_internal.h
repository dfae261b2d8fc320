// Internal layouts shared by the host code (bt_host.cpp) and the kernels (bt_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bt.h"

namespace bt {

// ---------------------------------------------------------------------------------------
// Mesh in HBM
//
// Nodes: binary BVH, one node = 64 B = 4 float4 holding BOTH children's boxes, so a node
// fetch tests two boxes (x, y, z rows are [lo0, lo1, hi0, hi1]):
//   n[0] = (lo0.x, lo1.x, hi0.x, hi1.x)
//   n[1] = (lo0.y, lo1.y, hi0.y, hi1.y)
//   n[2] = (lo0.z, lo1.z, hi0.z, hi1.z)
//   n[3] = (ref0, ref1, -, -) as int bits
// A child reference >= 0 is an interior node; < 0 is a leaf: v = ~ref, first = v >> 3,
// count = v & 7 (count <= 7), `first` indexing the triangle-reference array.
// Boxes are grown by a margin covering FP32 rounding of the ray and the flag distance.
//
// Triangle references: 48 B = 3 float4, duplicated per sub-domain (tile):
//   t[0] = (v0.x, v0.y, v0.z, v1.x)
//   t[1] = (v1.y, v1.z, v2.x, v2.y)
//   t[2] = (v2.z, global id bits, h_min, 0)   h_min = smallest altitude, rounded down
// Global triangles (by id): float[9] vertices, float absorption.
// ---------------------------------------------------------------------------------------

constexpr int kStack = 32;          // traversal stack entries per lane (>= BVH depth)
constexpr int kEmptyRoot = 0x7fffffff;

struct DevMesh {
    const float4 *nodes;
    const float4 *tris;
    const float *tri_g;       // [n_tri][9]
    const float *alpha;       // [n_tri]
    const int *tile_root;     // [tiles] root reference or kEmptyRoot
    const float *tile_box;    // [tiles][6] root box lo.xyz, hi.xyz (grown)
    int tiles_x, tiles_y;
    double gx0, gy0, tw, th;  // tile grid origin and tile size (xy footprint of the mesh)
    double gx1, gy1;
    double zmin, zmax;        // z slab of the whole mesh (grown)
    int n_tri;
};

// Beam queue, structure of arrays with capacity `cap`.  All generations of a beam set
// stay resident: generation g occupies [start_g, start_g + count_g) with
// start_g = count_0 + ... + count_(g-1), so the capacity is n0 * (max_depth + 1) records.
//   dbl[k * cap + i], k = 0..17: A.xyz, d0.xyz, d1.xyz, d2.xyz, o.xyz, c.xyz
//   flt[k * cap + i], k = 0..1: K (W/sr), Omega (sr)
//   ints[k * cap + i], k = 0..2: initial beam id, start triangle, meta
// meta: bits 0-7 depth, bit 8 near side is negative, bit 9 flagged (inherited)
enum { D_A = 0, D_D0 = 3, D_D1 = 6, D_D2 = 9, D_O = 12, D_C = 15, D_N = 18 };
enum { F_K = 0, F_OMEGA = 1, F_N = 2 };
enum { I_ID = 0, I_START = 1, I_META = 2, I_N = 3 };
constexpr int kMetaNegNear = 1 << 8;
constexpr int kMetaFlag = 1 << 9;

struct DevQueue {
    double *dbl;
    float *flt;
    int *ints;
    long long cap;
};

// Traced segments, indexed like the queue.
struct DevSegs {
    int *hit;        // hit triangle id or -1
    double *t;       // hit parameter or +inf
    int *flag;       // 1 = flagged (inherited or own)
};

// Device-side counters of one beam set, zeroed at emission.
struct DevCounters {
    unsigned long long count[BT_MAX_DEPTH + 2];      // beams per generation
    unsigned long long flagged[BT_MAX_DEPTH + 2];
    double power[BT_MAX_DEPTH + 2];
    unsigned long long n_big[BT_MAX_DEPTH + 2];      // segments for the wave-per-segment fallback
    unsigned long long n_rows[BT_MAX_DEPTH + 2];     // (segment, row) work items requested
    unsigned long long n_spans[BT_MAX_DEPTH + 2];    // (segment, row, columns) work items
    unsigned long long node_visits, tri_tests, mic_tests, mic_updates;
};

struct DevMics {
    double x0, y0, z, dx, dy;  // float32 grid values, widened
    int nx, ny;
    double *e_strict;          // [nx*ny]
    double *e_flag;            // [nx*ny]
};

// Work buffers of the microphone stage: (segment, row) items of wide footprints,
// (segment, row, first column, last column) spans of long rows, and the overflow list
// of segments handled one wave each.
struct MicWork {
    int2 *rows;
    long long rows_cap;
    int4 *spans;
    long long spans_cap;
    int *general;      // segments for the general footprint path; capacity: the queue's
    int *big_list;     // capacity: the queue capacity
};

// Per-wave records of the statically partitioned kernels (wave w of a grid of W waves
// takes the batches w, w + W, ...), so that counts and offsets need no shared atomic:
//   trace:  children[w], stats (flagged, node visits, triangle tests) and power per wave,
//           turned into child offsets and per-generation totals by a one-block scan;
//   microphones: general[w] items found by wave w, stored in its own region.
constexpr int kBlocksPerCU = 8;
constexpr int kWavesPerBlock = 4;
struct WaveScratch {
    unsigned long long *children;  // [W]
    unsigned long long *offset;    // [W] exclusive scan of children
    unsigned long long *stats;     // [W][3] flagged, node visits, triangle tests
    double *power;                 // [W]
    unsigned int *general;         // [W] general-path items per wave (microphones)
    int n_waves;                   // W
};

struct TraceArgs {
    int gen;         // trace: the generation traced; microphones: first generation
    int gen_end;     // microphones: one past the last generation accumulated
    int max_depth;
    double t_min, delta, air_m, e_min;
    int *hit_out;
    uint8_t *flag_out;
    double *t_out;
};

// Kernel launchers (bt_kernels.hip); all enqueue on `s` and return hipGetLastError().
hipError_t launch_init_counters(DevCounters *ctr, long long n0, hipStream_t s);
hipError_t launch_emit(const double *base20, const float *src, const float *power, int n_src, int level,
                       DevQueue q, hipStream_t s);
hipError_t launch_trace(const DevMesh &m, DevQueue q, DevSegs segs, DevCounters *ctr, const TraceArgs &a,
                        WaveScratch ws, int n_cu, hipStream_t s);
hipError_t launch_mics(const DevMesh &m, DevQueue q, DevSegs segs, DevCounters *ctr, DevMics mics,
                       const TraceArgs &a, MicWork w, WaveScratch ws, int n_cu, hipStream_t s);
hipError_t launch_fill(double *p, long long n, double v, hipStream_t s);
hipError_t launch_levels(const double *es, const double *ef, double *level, long long n, hipStream_t s);

}  // namespace bt
