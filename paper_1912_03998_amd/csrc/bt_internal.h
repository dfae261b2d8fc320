// Internal layouts shared by the host code (bt_host.cpp) and the kernels (*.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bt.h"

namespace bt {

// ---------------------------------------------------------------------------------------
// Mesh in HBM
//
// Nodes: 4-wide BVH, one node = 128 B = 8 float4 (one cache line) holding the boxes of
// all four children, so a node fetch tests four boxes:
//   n[0] = lo.x of children 0..3     n[1] = hi.x of children 0..3
//   n[2] = lo.y                      n[3] = hi.y
//   n[4] = lo.z                      n[5] = hi.z
//   n[6] = (ref0, ref1, ref2, ref3) as int bits      n[7] = padding
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

constexpr int kStack = 32;          // traversal stack entries per lane (the builder bounds the
                                    // pushes of any root-leaf walk by it)
constexpr int kEmptyRoot = 0x7fffffff;  // empty tile
// Unused child slot of a node: an empty leaf (no triangle references) behind a box at
// 1e30 that no ray enters (its slab entry or exit is beyond every window: |1/c| >= 1 on
// each axis), so the traversal needs no test for it and an entry would be harmless.
constexpr int kEmptyChild = -1;

struct DevMesh {
    const float4 *nodes;      // 4-wide nodes, 8 float4 each: lo x, hi x, lo y, hi y, lo z,
                              // hi z of the four children, their references, padding
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

// Beam queue, structure of arrays with capacity `cap`.  Resident layout: all generations
// of a beam set stay in the queue, generation g occupying [start_g, start_g + count_g) with
// start_g = count_0 + ... + count_(g-1), so the capacity is n0 * (max_depth + 1) records.
// Two-slot layout (DevCounters::ring = S > 0): generation g occupies [(g mod 2) S, + count_g)
// and overwrites generation g - 2, so each generation must reach the microphones before the
// one after it is traced; the capacity is 2 S records with S >= n0.
//   dbl[k * cap + i], k = 0..18: A.xyz, d0.xyz, d1.xyz, d2.xyz, o.xyz, c.xyz, P
//   flt[k * cap + i], k = 0: K (W/sr)
// P is the beam's power K Omega in watts, kept in FP64 so that the energy-threshold
// decision (P (1 - alpha) > e_min) is taken in the same precision as the oracle's; K,
// which only scales the microphone contributions, is FP32.
//   ints[k * cap + i], k = 0..2: initial beam id, start triangle, meta
// meta: bits 0-7 depth, bit 8 near side is negative, bit 9 flagged (inherited); for beams
// of a multi-scenario set (batches, served requests) also bits 10-14 the scenario's
// max_depth and bits 16-31 its slot, inherited unchanged by children (zero otherwise)
enum { D_A = 0, D_D0 = 3, D_D1 = 6, D_D2 = 9, D_O = 12, D_C = 15, D_P = 18, D_N = 19 };
enum { F_K = 0, F_N = 1 };
enum { I_ID = 0, I_START = 1, I_META = 2, I_N = 3 };
constexpr int kMetaNegNear = 1 << 8;
constexpr int kMetaFlag = 1 << 9;
constexpr int kMetaMaxDepthShift = 10;
constexpr int kMetaSlotShift = 16;
constexpr int kMetaInherited = ~0x3ff;   // the scenario bits
constexpr int kMaxSlots = 1 << 16;

__host__ __device__ inline int scenario_meta(int slot, int max_depth)
{
    return (int)(((unsigned)slot << kMetaSlotShift) | ((unsigned)max_depth << kMetaMaxDepthShift));
}
__host__ __device__ inline int meta_slot(int meta) { return (int)((unsigned)meta >> kMetaSlotShift); }
__host__ __device__ inline int meta_max_depth(int meta) { return (meta >> kMetaMaxDepthShift) & 31; }

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

// Microphone statistics are spread over kStatSlots cache lines: wave w of a kernel adds
// its totals to line w mod kStatSlots, so that thousands of waves finishing together do
// not serialise on one address (one device-scope atomic per wave on a single counter
// cost a microphone pass about 0.15 ms).
constexpr int kStatSlots = 256;
constexpr int kStatStride = 16;   // 128 bytes per slot
enum { MS_TESTS = 0, MS_UPDATES = 1, MS_LAYERS = 2, MS_CLASSIFIED = 3, MS_LAYER_FALLBACK = 4 };

// Device-side counters of one beam set, zeroed at emission.
struct DevCounters {
    unsigned long long count[BT_MAX_DEPTH + 2];      // beams per generation
    unsigned long long flagged[BT_MAX_DEPTH + 2];
    double power[BT_MAX_DEPTH + 2];
    unsigned long long n_big[BT_MAX_DEPTH + 2];      // segments for the wave-per-segment fallback
    unsigned long long n_spans[BT_MAX_DEPTH + 2];    // (segment, row, columns) work items
    unsigned long long n_layers[BT_MAX_DEPTH + 2];   // volumetric: (segment, layer) items requested
                                                     // by the pass starting at this generation
    unsigned long long node_visits, tri_tests;
    unsigned long long ring;                         // two-slot layout: slot size (0 = resident)
    // microphone statistics per slot: MS_TESTS (segment, microphone) candidates tested,
    // MS_UPDATES contributions, MS_LAYERS volumetric (segment, layer) pairs examined,
    // MS_CLASSIFIED segments whose planar class was read from their record,
    // MS_LAYER_FALLBACK volumetric items done in place (their region of the buffer full)
    alignas(128) unsigned long long mic_stat[kStatSlots][kStatStride];
};
// Sum of one microphone statistic over the slots (host).
inline unsigned long long mic_stat_total(const DevCounters &h, int k)
{
    unsigned long long s = 0;
    for (int i = 0; i < kStatSlots; ++i) s += h.mic_stat[i][k];
    return s;
}

// Microphone (i, j, k) sits at (x0 + i dx, y0 + j dy, z + k dz) and has index
// (k ny + j) nx + i; a planar grid has nz = 1.  Work items name a microphone row by its
// global row k ny + j.
struct DevMics {
    double x0, y0, z, dx, dy;  // float32 grid values, widened
    int nx, ny;
    double *e_strict;          // [nx*ny*nz]
    double *e_flag;            // [nx*ny*nz]
    const unsigned *mask;      // scenario sets only (planar): bit (j nx + i) set for the
                               // microphones of the set's subset; NULL = every grid point
    double dz;                 // layer spacing (float32 value, widened); 0 when nz = 1
    int nz;                    // layers
    float fx0, fy0;            // volumetric fast path: x0, y0, 1/dx, 1/dy, nx - 1, ny - 1
    float fidx, fidy;          // in FP32, set with the grid
    float fnx1, fny1;
};

// Explicit microphone points with a uniform-bucket index in xy: the points sorted by
// bucket (row-major: bucket (i, j) is j nbx + i), so that a row of buckets is one
// contiguous index range.
struct DevPoints {
    const double *px, *py, *pz;   // sorted positions (float32 inputs, widened)
    const int *orig;              // original index of each sorted point (energy index)
    const int *cell;              // [nbx nby + 1] first sorted point of each bucket
    double bx0, by0, bh;          // bucket grid origin and bucket size
    int nbx, nby;
    double zlo, zhi;              // z range of the points
    long long n;
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
    int2 *layers;      // volumetric grids: (segment, layer) items of the general path, in
    long long layers_cap;  // kLayerRegions regions of layers_cap / kLayerRegions items
    unsigned *layer_cnt;   // [kLayerRegions][kLayerCntStride]: items requested per region in
                           // this pass (element 0 of each 128-byte line), zeroed per pass
};
// The volumetric pass's (segment, layer) items go to one of kLayerRegions regions of the
// item buffer, chosen by the producing wave's block, each with a reservation counter on a
// cache line of its own: thousands of waves reserving on one shared counter serialise on
// its address.
constexpr int kLayerRegions = 256;
constexpr int kLayerCntStride = 32;

// Per-wave records of the statically partitioned kernels (wave w of a grid of W waves
// takes the batches w, w + W, ...), so that counts and offsets need no shared atomic:
//   trace:  children[w], stats (flagged, node visits, triangle tests) and power per wave,
//           turned into child offsets and per-generation totals by a one-block scan;
//   microphones: general[w] items found by wave w, stored in its own region.
constexpr int kBlocksPerCU = 8;
constexpr int kWavesPerBlock = 4;
struct WaveScratch {
    unsigned long long *children;  // [W]
    // per block of kWavesPerBlock waves (k_tcount): children, flagged segments, node visits
    // and triangle tests ([W / kWavesPerBlock][4]), and power ([W / kWavesPerBlock])
    unsigned long long *block_rec;
    double *block_power;
    unsigned long long *stats;     // [W][3] flagged, node visits, triangle tests
    double *power;                 // [W]
    unsigned int *general;         // [W] general-path items per wave (microphones)
    unsigned int *rows_n;          // [W] (segment, row) items per wave, in its region of the
                                   // row buffer (rows_cap / W items each)
    int n_waves;                   // W
};

// Per-tile beam queues of one beam set (the trace's queued rounds).  Positions index the
// generation being traced (0 .. its size - 1, at most cap).  A round's items are produced
// by the waves of a W-wave grid, each into a region of its own (no shared cursor), counted
// per (tile, wave), and then ordered by tile with those counts (a counting sort without
// atomics: a scan over the waves of each tile, then a scatter).
//   stage / stage_n: each producer wave's items and their number
//   cnt:  [T][W] items per (tile, producer wave), cleared by the scan
//   off:  [T][W] exclusive scan of cnt over the waves of each tile
//   total, n_items: items per tile and in all of the round being sorted
//   list: the round's items ordered by tile (then by producer wave, then lane order)
//   lo, c1t, c2t, c1id: a handed-off ray's window start and flag candidates
constexpr int kMaxQueueTiles = 256;   // partitions with more tiles walk their tiles in-lane
constexpr int kMaxQueueRounds = 8;
constexpr int kXcds = 8;              // MI355X: 8 accelerator complex dies, each with its own L2
struct TileWork {
    int2 *stage;
    int *stage_n;
    int *cnt, *off, *total, *n_items;
    int2 *list;
    double *lo, *c1t, *c2t;
    int *c1id;
    long long cap;       // positions: the largest generation
    long long region;    // items per producer wave's region
    int n_waves;         // W: the producers' (and consumers') grid in waves
    int n_tiles;         // T of the mesh traced
    int rounds;          // queued rounds (>= 1); the last one finishes its rays in-lane
};

// A planar microphone grid that a beam set classifies its beams against as they are
// created (emission, reflection): cls[j], parallel to the queue, holds the planar fast
// path's decision for record j (plane_decide, encoded by plane_code), so that the
// microphone pass dismisses a beam without reading its frustum.  cls = NULL: none.
struct ClassGrid {
    double x0, y0, z, dx, dy;   // the grid's plane and lattice (float32 values, widened)
    int nx, ny;
    int2 *cls;
};
constexpr int kClassMaxDim = 1 << 26;   // grids this wide or wider are not classified

struct TraceArgs {
    int gen;         // trace: the generation traced; microphones: first generation
    int gen_end;     // microphones: one past the last generation accumulated
    int max_depth;   // single-scenario sets; a scenario set reads each beam's from its meta
    int scenarios;   // 1: a multi-scenario set (per-beam max_depth and slot in meta)
    const DevMics *slot_mics;  // scenario sets: microphone set of each slot
    double t_min, delta, air_m, e_min;
    double delta2;   // delta^2, formed on the host (a kernel argument, so no register holds it)
    int queue_rounds;  // trace: 0 = in-lane tile walk, k >= 1 = k rounds of per-tile queues
    ClassGrid cg;      // trace: classify the children against this grid (cg.cls = NULL: not)
    const int2 *mic_cls;  // microphones: the records' classes for this grid (NULL: decide
                          // from each frustum)
    int *hit_out;
    uint8_t *flag_out;
    double *t_out;
};

// Generation-0 beams of many scenarios, appended in one launch: source s emits the
// 20 4^level[s] beams [first[s], first[s + 1]) (relative to the append position) with
// the given meta and beam ids id0[s] + face.  The sizes are read from device memory so
// that a captured launch serves tables of any size up to the buffers' capacity.
struct EmitTable {
    const float *src;          // [n][3]
    const float *power;        // [n]
    const int *level;          // [n]
    const int *meta;           // [n]
    const int *id0;            // [n]
    const long long *first;    // [n + 1], first[n] = total beams
    const long long *dims;     // [0] total beams, [1] n (sources)
};

// Sizes of one batch chunk, read by its kernels from device memory.
struct BatchDesc {
    long long n_fill;          // energies to zero (strict then flag arrays)
    long long n_out;           // gathered outputs
    long long e_stride;        // offset of the flag energies from the strict ones
};

// Kernel launchers; all enqueue on `s` and return hipGetLastError().  The statically
// partitioned kernels run ws.n_waves waves (blocks of kWavesPerBlock waves).
// ring: the two-slot layout's slot size, 0 for the resident layout.
hipError_t launch_init_counters(DevCounters *ctr, long long n0, long long ring, hipStream_t s);
// The face table of an icosphere level (dirs: 12 nf doubles, om: nf doubles), and the
// emission of one beam set's generation 0 from it.
hipError_t launch_faces(const double *base20, int level, double *dirs, double *om, hipStream_t s);
// wt: NULL (omni) or [n_src][nf] face weights of directional sources, with norm a device
// double[n_src] filled here; cg.cls non-NULL: each beam's planar fast-path class is
// written there.
hipError_t launch_emit(const double *dirs, const double *om, const float *src, const float *power, const float *wt,
                       double *norm, int n_src, int level, DevQueue q, ClassGrid cg, hipStream_t s);
// Appends the table's beams to generation `gen` (after its current beams) and adds their
// number to count[gen].
hipError_t launch_emit_table(const double *base20, const EmitTable &t, long long max_total, DevQueue q,
                             DevCounters *ctr, int gen, hipStream_t s);
// Zero d->n_fill doubles at p; gather d->n_out outputs (e[i] + e[stride + i] and
// e[stride + i] for i = idx[k]).  max_n bounds the sizes (grid size).
hipError_t launch_fill_desc(double *p, const BatchDesc *d, long long max_n, hipStream_t s);
hipError_t launch_mics_points(const DevMesh &m, DevQueue q, DevSegs segs, DevCounters *ctr, DevMics mics,
                              DevPoints pts, const TraceArgs &a, int n_cu, hipStream_t s);
hipError_t launch_select(const double *es, const double *ef, const long long *sel, long long n, double *out_s,
                         double *out_f, double *out_level, hipStream_t s);
hipError_t launch_gather(const double *e, const long long *idx, const BatchDesc *d, long long max_n, double *out_e,
                         double *out_f, hipStream_t s);
// tw: NULL for the in-lane walk, else the beam set's tile queues (rounds from tw->rounds).
hipError_t launch_trace(const DevMesh &m, DevQueue q, DevSegs segs, DevCounters *ctr, const TraceArgs &a,
                        WaveScratch ws, const TileWork *tw, int n_cu, hipStream_t s);
hipError_t launch_zero_ints(int *p, long long n, hipStream_t s);
hipError_t launch_mics(const DevMesh &m, DevQueue q, DevSegs segs, DevCounters *ctr, DevMics mics,
                       const TraceArgs &a, MicWork w, WaveScratch ws, int n_cu, hipStream_t s);
hipError_t launch_fill(double *p, long long n, double v, hipStream_t s);

// Static work area of the allocation-free microphone pass (bt_accumulate_mics_static): a
// file-scope device array of kStaticScratchBytes per GPU, laid out as
//   [0, kStaticCountBytes)                per-wave general-path counts (<= kStaticMaxWaves)
//   rows:   kStaticRows int2              (segment, row) items (overflow: wave path)
//   spans:  kStaticSpans int4             (segment, row, columns) items (full: in place)
//   layers: kStaticLayers int2            volumetric (segment, layer) items (full: in place)
//   layer counters: kLayerRegions x kLayerCntStride unsigned
//   lists:  the rest, as ints             wave-path list (n) then general list (n + 64 (W + 1))
// Nothing in it needs to start at zero: every count lives in the beam set's counters.
constexpr size_t kStaticScratchBytes = 64ull << 20;
constexpr int kStaticMaxWaves = 16384;
constexpr size_t kStaticCountBytes = (size_t)kStaticMaxWaves * sizeof(unsigned);
constexpr long long kStaticRows = 1ll << 20;
constexpr long long kStaticSpans = 1ll << 19;
constexpr long long kStaticLayers = 1ll << 19;
constexpr size_t kStaticRowsOffset = kStaticCountBytes;
constexpr size_t kStaticSpansOffset = kStaticRowsOffset + (size_t)kStaticRows * 8;
constexpr size_t kStaticLayersOffset = kStaticSpansOffset + (size_t)kStaticSpans * 16;
constexpr size_t kStaticLayerCntOffset = kStaticLayersOffset + (size_t)kStaticLayers * 8;
constexpr size_t kStaticListsOffset = kStaticLayerCntOffset + (size_t)kLayerRegions * kLayerCntStride * 4;
constexpr long long kStaticListInts = (long long)((kStaticScratchBytes - kStaticListsOffset) / sizeof(int));
static_assert(kStaticListsOffset % 256 == 0, "static work area sections stay aligned");
// Device address of the calling thread's current device's static work area (looked up
// once per device; `device` must be current).
hipError_t static_scratch(int device, void **out);
hipError_t launch_levels(const double *es, const double *ef, double *level, long long n, hipStream_t s);

}  // namespace bt
