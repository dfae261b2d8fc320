// Host-side state of the C ABI handles and the helpers shared by the host sources
// (bt_host.cpp: contexts, meshes, single beam sets; bt_batch.cpp: scenario batches).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bt.h"
#include "bt_internal.h"

using namespace bt;

// Partitions of one beam set at most: a set emitted from several sources is split by
// source, and each partition is traced and accumulated on a stream of its own.
constexpr int kMaxParts = 4;

struct bt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int parts = 2;             // partitions of a beam set of two or more sources (bt_set_partitions)
    // the partitions' streams and the events that fork them from `stream` and join them
    // to it; all created together on first use
    hipStream_t part_stream[kMaxParts] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kMaxParts] = {};
    size_t budget = 0;
    size_t used = 0;
    int n_cu = 256;
    double *base20 = nullptr;  // device, 20 base faces x 9 doubles
    std::string err;
    std::mutex mtx;            // submit / poll / cancel
    uint64_t next_ticket = 1;
    std::map<uint64_t, struct Request *> requests;
    struct BatchWork *batch = nullptr;  // bt_batch_run's two workspaces ([2]), kept between calls
    double *face_dirs[BT_MAX_LEVEL + 1] = {};  // per icosphere level, built on first use
    double *face_om[BT_MAX_LEVEL + 1] = {};
    void *scratch = nullptr;   // this device's static work area (bt_accumulate_mics_static)
};

struct bt_mesh {
    bt_ctx *ctx = nullptr;
    DevMesh dev{};
    void *bufs[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    size_t sizes[6] = {0, 0, 0, 0, 0, 0};
    int64_t n_nodes = 0, n_refs = 0;
    int32_t max_depth = 0;
    double delta_cap = 0.0;   // largest edge_delta the box margins cover
    double r_eff = 0.0;       // largest |coordinate| of a ray origin the margins cover
};

struct bt_mics {
    bt_ctx *ctx = nullptr;
    DevMics dev{};
    double *level = nullptr;
    size_t bytes = 0;
    long long n_out = 0;          // values bt_levels returns
    // subset of a grid: the grid's energies, a membership bitmap and the output indices
    unsigned *mask = nullptr;
    size_t mask_bytes = 0;
    long long *sel = nullptr;     // [n_out] grid indices of the outputs
    double *sel_buf = nullptr;    // [3 n_out] strict, flag and level staging for bt_levels
    // explicit points
    bool points = false;
    DevPoints pts{};
    void *pts_buf = nullptr;
    size_t pts_bytes = 0;
};

struct bt_beams {
    bt_ctx *ctx = nullptr;
    long long cap = 0;
    DevQueue q{};             // every generation, contiguous (see DevQueue)
    DevSegs segs{};
    DevCounters *ctr = nullptr;
    WaveScratch ws{};         // per-wave records of the statically partitioned kernels
    void *ws_buf = nullptr;
    size_t ws_bytes = 0;
    int ws_cap_waves = 0;     // waves the per-wave arrays (and the lists sized per wave) hold;
                              // the grid in use, ws.n_waves, may be smaller
    int *big_list = nullptr;  // 2 * cap: wave-path overflow list, then the general-path list
    int2 *rows = nullptr;
    long long rows_cap = 0;
    int4 *spans = nullptr;
    long long spans_cap = 0;
    TileWork tw{};            // per-tile beam queues of the trace (cap = largest generation)
    void *tw_buf = nullptr;
    size_t tw_bytes = 0;
    int2 *layers = nullptr;   // volumetric grids: (segment, layer) items, allocated on first use
    long long layers_cap = 0;
    unsigned *layer_cnt = nullptr;  // their regions' reservation counters
    long long work_n0 = 0;    // generation-0 size the work buffers were sized for
    int acc_gen = 0;          // first generation not yet accumulated at the microphones
    int depth_hint = 0;       // max_depth of the previous run, to size the queue at emission
    float *src_dev = nullptr, *pow_dev = nullptr;
    double *norm_dev = nullptr;   // per source: sum of weight x solid angle (directional)
    int src_cap = 0;
    float *wt_dev = nullptr;      // directional sources' face weights
    long long wt_cap = 0;
    size_t bytes = 0;
    int gen = 0;              // generations traced
    int max_depth = -1;       // fixed by the first trace
    long long n0 = 0;
    long long ring = 0;       // two-slot layout's slot size (bt_run), 0 = every generation resident
    // planar microphone classification (bt_beams_bind_mics): while bound, emission and
    // reflection write each new record's fast-path class into cgrid.cls (cls_cap records);
    // bit g of class_gens: generation g's records hold classes for cgrid
    ClassGrid cgrid{};
    long long cls_cap = 0;
    bool bound = false;
    unsigned long long class_gens = 0;
    bt_stats prior{};         // statistics of the earlier source chunks of a bt_run
    double r_src = 0.0;
    // partitions of the last emission: partition 0 is this set, partition k >= 1 is
    // part[k - 1], a set of its own (its sources follow partition k - 1's); beam0 is the
    // partition's first beam in the emission, its first row of the parity outputs
    int n_parts = 1;
    bt_beams *part[kMaxParts - 1] = {};
    long long beam0 = 0;
    bool emitted = false;     // holds an emission (false when created, or after a failed one)
    const bt_mesh *mesh = nullptr;  // the mesh its emission is traced with (its hit ids index it)
};

struct Request {
    bt_request req{};
    std::vector<float> src, pw;
    bt_mics *mics = nullptr;
    bt_beams *beams = nullptr;
    hipEvent_t done = nullptr;
};

// ---------------------------------------------------------------------------------------
// errors and memory
// ---------------------------------------------------------------------------------------
bt_status fail(bt_ctx *ctx, bt_status s, const char *fmt, ...);
bt_status hip_fail(bt_ctx *ctx, hipError_t e, const char *what);

#define HIP_TRY(ctx, expr)                                  \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

// Device allocation counted against the context's budget, and its release.
bt_status dev_alloc(bt_ctx *ctx, void **p, size_t bytes);
void dev_free(bt_ctx *ctx, void *p, size_t bytes);

// Beam-set buffers: per-wave scratch for blocks_per_cu workgroups per CU, queue / segment
// / list capacity of n records (keeping the first `keep` records), microphone work items
// for n0 generation-0 beams, and their release.
size_t list_ints(long long n, int n_waves);
bt_status alloc_wave_scratch(bt_ctx *ctx, bt_beams *b, int blocks_per_cu);
void queue_free(bt_ctx *ctx, DevQueue &q);
void beams_release(bt_beams *b);
bt_status reserve_queue(bt_ctx *ctx, bt_beams *b, long long n, long long keep);
bt_status reserve_work(bt_ctx *ctx, bt_beams *b, long long n0);
// Tile-queue capacity for generations of up to n rays (allocated on first use).
bt_status reserve_tiles(bt_ctx *ctx, bt_beams *b, long long n);
// The tile queues a trace of generation sizes up to the reserved capacity uses (NULL for the
// in-lane walk).
const TileWork *trace_tiles(bt_beams *b, const bt_mesh *mesh, const TraceArgs &a);

bt_status check_params(bt_ctx *ctx, const bt_mesh *mesh, const bt_params *p);

// Host-only argument checks, shared by the entry points and the bt_validate_* calls:
// BT_OK, or BT_EINVAL with the reason in msg.  Nothing touches the device.
constexpr double kDeltaCap = 1e-3;   // largest edge_delta a mesh's box margins cover
bt_status check_mesh_args(const float *xyz, int64_t n_vert, const int32_t *tri, const float *absorption, int64_t n_tri,
                          int32_t tiles_x, int32_t tiles_y, std::string &msg);
bt_status check_source_args(const float *src_xyz, const float *src_power, const float *src_weight, int32_t n_src,
                            int32_t level, bool two_slot, std::string &msg);
bt_status check_grid_args(float x0, float y0, float z0, float dx, float dy, float dz, int32_t nx, int32_t ny,
                          int32_t nz, std::string &msg);
bt_status check_param_args(const bt_params *p, double delta_cap, std::string &msg);
TraceArgs make_args(const bt_params *p, int gen);

// Sizes of a scenario (a batch member or a served request), filled by validate_scenario,
// which checks it against the mesh (BT_EINVAL with a message naming scenario k).
struct ScenarioSize {
    long long n0;          // generation-0 beams
    long long records;     // n0 (max_depth + 1): queue records at most
    long long grid;        // grid microphones
    long long n_out;       // outputs
    long long mask_words;  // subset bitmap words (0 without a subset)
};
bt_status validate_scenario(bt_ctx *ctx, const bt_mesh *mesh, const bt_scenario &sc, int k, ScenarioSize &z);

// Point a microphone set at a new grid, reallocating only when it does not fit, and zero
// its energies (*m may be NULL: created).
bt_status mics_fit(bt_ctx *ctx, bt_mics **m, float x0, float y0, float z, float dx, float dy, int32_t nx, int32_t ny);

// Free bt_batch_run's cached workspace (bt_destroy, bt_batch_release).
void batch_work_free(bt_ctx *ctx);

// The context's partition streams (created together on first use, default priority).
hipError_t partition_streams(bt_ctx *ctx);
