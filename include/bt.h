/*
 * bt.h -- C ABI of the MI355X hybrid beam tracer.
 *
 * The library traces triangular-frustum sound beams from point sources through a
 * triangulated city model and accumulates, at microphones, the energy of every beam
 * whose frustum contains them (Gbikpi-Benissan & Magoules, "Beam-tracing domain
 * decomposition method for urban acoustic pollution", Section 2: the hybrid
 * beam/ray method).  Only a beam's guiding ray is intersected with the model, as in
 * ray tracing, so beams are never split; each hit spawns one specular child beam
 * that has lost energy at the surface.
 *
 * Conventions
 *   - Units: metres, watts, W/m^2; levels in dB re i0 = 1e-12 W/m^2.
 *   - Host input arrays are borrowed for the duration of the call only (copied).
 *   - Pointers documented as "device" must be device-accessible (hipMalloc or a
 *     torch CUDA tensor's data_ptr) and stay valid until the stream work finishes.
 *   - "host or device" output pointers are filled with hipMemcpyDefault.
 *   - All handles are created and freed by the library; the library never frees
 *     caller memory.
 *   - Every call returns a bt_status.  No exception or abort crosses the ABI.  On
 *     error bt_last_error(ctx) holds a message.
 *   - A bt_ctx is single-threaded except bt_submit / bt_poll / bt_cancel.
 *   - Work is enqueued on the context's stream; calls that return results to the
 *     host (bt_trace with n_next, bt_levels, bt_beams_stats, bt_poll) synchronise it.
 *     A call on a partitioned beam set (bt_set_partitions) also runs work on the
 *     library's own streams, forked from the context's stream at the call's start and
 *     joined to it before the call returns, so the ordering above holds.
 */
#ifndef BT_H
#define BT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BT_OK = 0,
    BT_PENDING = 1,      /* bt_poll: request not finished yet */
    BT_EINVAL = -1,      /* invalid argument (nothing was enqueued) */
    BT_ENOMEM = -2,      /* allocation failed or the context's HBM budget is exceeded */
    BT_EDEVICE = -3,     /* HIP runtime error; text in bt_last_error */
    BT_EOVERFLOW = -4,   /* an internal capacity was exceeded (e.g. BVH too deep) */
    BT_ENOTFOUND = -5,   /* unknown request ticket */
    BT_ESTATE = -6       /* call out of order (e.g. accumulate before any trace) */
} bt_status;

#define BT_MAX_LEVEL 9    /* icosphere level: 20 * 4^level beams per source */
#define BT_MAX_DEPTH 31   /* maximum reflections per beam */

typedef struct bt_ctx bt_ctx;
typedef struct bt_mesh bt_mesh;
typedef struct bt_mics bt_mics;
typedef struct bt_beams bt_beams;

/* Tracing parameters (paper Section 2: reflections lose energy; particle methods
 * also damp energy in air and delete it below a threshold). */
typedef struct {
    int32_t max_depth;    /* D: generations 0..D are traced; only depth < D reflects */
    double t_min;         /* hits at ray parameter t <= t_min are ignored (1e-3 m) */
    double edge_delta;    /* flag distance (1e-5 m): a segment whose hit point lies within
                             it of an edge, or with another triangle within it of the
                             ray near t*, is flagged; flags are inherited by children */
    double air_m;         /* air attenuation exp(-air_m * d); 0 = off */
    double e_min;         /* a child whose power K*Omega is <= e_min is dropped; 0 = off */
    int32_t queue_rounds; /* sub-domain hand-off (paper Section 3: a beam leaving a sub-domain
                             is passed to the one it enters): 0 = every guiding ray walks the
                             tiles it crosses in its own lane; k in 1..8 = per-tile beam queues,
                             each ray's first k tiles taken from the queue of the tile it is in
                             (a ray leaving a tile unresolved is handed to the queue of the tile
                             it enters) and any further tiles walked in its lane; partitions
                             of more than 256 tiles always walk in-lane.  Results are
                             identical either way. */
    int64_t run_records;  /* bt_run: beam records a source chunk may keep resident; when the
                             largest chunk's n_beams0 (max_depth + 1) fits, every chunk keeps
                             every generation and makes one microphone pass, else every chunk
                             keeps two generation slots and accumulates each generation as it
                             is traced; 0 = 64 Mi */
    /* optional per-(initial beam, generation) parity outputs, device pointers,
       row-major [n_beams0][max_depth + 1]; entries of untraced generations are
       left untouched (callers pre-fill them, e.g. with -2) */
    int32_t *hit_out;     /* hit triangle id, -1 = escaped */
    uint8_t *flag_out;    /* 1 = this segment or an ancestor is flagged */
    double *t_out;        /* hit parameter (metres along the guiding ray), inf on escape */
} bt_params;

/* Per-beam-set statistics, filled by bt_beams_stats (synchronises). */
typedef struct {
    int32_t generations;                 /* generations traced so far */
    int64_t count[BT_MAX_DEPTH + 1];     /* beams traced per generation */
    int64_t flagged[BT_MAX_DEPTH + 1];   /* of which flagged */
    double power[BT_MAX_DEPTH + 1];      /* sum of K * Omega over traced beams, watts */
    int64_t segments;                    /* beam segments (traced guiding rays) */
    int64_t node_visits;                 /* BVH interior nodes fetched */
    int64_t tri_tests;                   /* ray/triangle tests */
    int64_t mic_tests;                   /* (segment, microphone) candidates tested */
    int64_t mic_updates;                 /* (segment, microphone) pairs accumulated */
    int64_t mic_layer_visits;            /* volumetric grids: (segment, layer) pairs examined */
    int64_t mic_general;                 /* volumetric grids: of which on the clipped-footprint path */
    int64_t mic_fallback;                /* volumetric grids: of which done in place (item buffer full) */
    int64_t mic_classified;              /* segments whose planar class was taken from their
                                            creation (bt_beams_bind_mics) */
} bt_stats;

/* Defaults: max_depth 3, t_min 1e-3, edge_delta 1e-5, air_m 0, e_min 0, queue_rounds 0
 * (measured faster), run_records 0, no outputs. */
void bt_params_default(bt_params *p);

const char *bt_status_str(bt_status s);
const char *bt_last_error(const bt_ctx *ctx);

/* Host-only argument checks: the checks bt_build_mesh, bt_emit_beams(_directional),
 * bt_mics_grid3d and the tracing calls make before they touch the device, callable without
 * a context or a GPU (e.g. to validate inputs on a machine without one).  Return BT_OK,
 * or BT_EINVAL with the reason written to msg (msg_len bytes, NUL-terminated; msg may be
 * NULL).  Arguments as in the corresponding calls; src_weight may be NULL (omni sources);
 * bt_validate_params checks edge_delta against the largest flag distance any mesh's box
 * margins cover (1e-3 m). */
bt_status bt_validate_mesh(const float *xyz, int64_t n_vert, const int32_t *tri, const float *absorption,
                           int64_t n_tri, int32_t tiles_x, int32_t tiles_y, char *msg, size_t msg_len);
bt_status bt_validate_sources(const float *src_xyz, const float *src_power, const float *src_weight, int32_t n_src,
                              int32_t level, char *msg, size_t msg_len);
bt_status bt_validate_grid(float x0, float y0, float z0, float dx, float dy, float dz, int32_t nx, int32_t ny,
                           int32_t nz, char *msg, size_t msg_len);
bt_status bt_validate_params(const bt_params *params, char *msg, size_t msg_len);

/* Context on HIP device `device`.  hip_stream: a hipStream_t to enqueue on (e.g. a
 * torch stream's handle) or NULL for a library-owned stream.  hbm_budget_bytes caps
 * the device memory the context allocates (0 = unlimited). */
bt_status bt_create(int device, size_t hbm_budget_bytes, void *hip_stream, bt_ctx **out);
bt_status bt_destroy(bt_ctx *ctx);
/* Device bytes currently allocated through the context. */
bt_status bt_memory_used(const bt_ctx *ctx, size_t *bytes);

/* Partitions of a beam set (paper Section 3 shares the beams out among processors; on
 * one GPU the shares are streams).  A set emitted from n_src >= 2 sources is split by
 * source into min(k, n_src) partitions of contiguous sources (near-equal counts), each
 * with its own queue, counters and microphone work lists.  Every call on the set runs
 * partition j's kernels on stream j of the context's partition streams (created together
 * on first use, with default priority, so that the runtime gives them distinct hardware
 * queues).  A generation's last rays leave most compute units idle; the other
 * partitions' work fills them.  bt_trace joins the
 * streams after each generation; bt_trace_all and bt_run run a partition's generations
 * (and, in bt_run, its microphone passes) without waiting for the other partitions.
 * Results do not depend on k: hit ids, parameters and flags are identical, and
 * energies and power sums differ only in the order of FP64 additions.  k in
 * 1..4 (BT_EINVAL otherwise); default 2.  It applies to sets emitted afterwards. */
bt_status bt_set_partitions(bt_ctx *ctx, int32_t k);

/* Triangulated model (paper Section 4: a detailed district model; Section 3: the
 * model is split once and reused for many simulations).
 *   xyz        host float[n_vert][3]
 *   tri        host int32[n_tri][3], vertex indices
 *   absorption host float[n_tri], energy fraction lost per reflection, in [0, 1]
 *   tiles_x, tiles_y: on-device partition of the model's xy footprint into
 *     sub-domains (1..64 each); each has its own hierarchy, and a guiding ray hands
 *     over from one sub-domain to the next along its path.
 * Validates indices, finite coordinates, absorption range and non-zero areas
 * (BT_EINVAL), builds the hierarchy per sub-domain on the host and uploads it.
 * n_tri may be 0 (free field). */
bt_status bt_build_mesh(bt_ctx *ctx, const float *xyz, int64_t n_vert, const int32_t *tri,
                        const float *absorption, int64_t n_tri, int32_t tiles_x, int32_t tiles_y,
                        bt_mesh **out);
bt_status bt_mesh_free(bt_mesh *mesh);
/* Hierarchy facts: 4-wide nodes, depth of the binary SAH build they were collapsed
 * from, triangle references after duplication. */
bt_status bt_mesh_info(const bt_mesh *mesh, int64_t *n_nodes, int32_t *max_depth, int64_t *n_tri_refs);

/* Microphones on a regular planar grid (paper Section 4: microphones regularly
 * distributed on a grid): positions (x0 + i dx, y0 + j dy, z), i < nx, j < ny,
 * index j * nx + i.  Energies are owned by the set and start at zero. */
bt_status bt_mics_grid(bt_ctx *ctx, float x0, float y0, float z, float dx, float dy, int32_t nx, int32_t ny,
                       bt_mics **out);
/* Microphones on a regular volumetric grid (paper Section 4: the experiment fills the
 * model's bounding box with microphones, one every 4 m in each direction):
 * positions (x0 + i dx, y0 + j dy, z0 + k dz), i < nx, j < ny, k < nz, index
 * (k ny + j) nx + i; nx ny nz <= 2^31; when nz > 1, dz > 0, nx, ny < 2^24 and nz < 2^25.  nz = 1
 * is bt_mics_grid.
 * Energies (bt_levels returns nx ny nz values) are owned by the set and start at zero.
 * Usable with bt_accumulate_mics and bt_run; the scenario and serving interfaces take
 * planar grids. */
bt_status bt_mics_grid3d(bt_ctx *ctx, float x0, float y0, float z0, float dx, float dy, float dz, int32_t nx,
                         int32_t ny, int32_t nz, bt_mics **out);
/* Microphones at a chosen subset of a grid's points (paper Section 4's microphones are
 * grid points; a query may want only some of them): idx host int32[n], grid indices in
 * [0, nx ny nz), duplicates allowed; bt_levels returns the n points in idx order.  The set
 * owns its energies (a grid-sized array; contributions to points outside the subset are
 * skipped before accumulation) and copies idx.  `grid` must be a grid set (not a subset
 * or a point set) and is not referenced afterwards.  BT_EINVAL on an empty or
 * out-of-range idx. */
bt_status bt_mics_subset(bt_ctx *ctx, const bt_mics *grid, const int32_t *idx, int64_t n, bt_mics **out);
/* Microphones at explicit points (paper Section 2: every microphone inside a beam
 * receives its contribution; the points need not lie on a grid): xyz host float[n][3],
 * copied; 1 <= n < 2^31, finite coordinates (BT_EINVAL otherwise).  The library indexes
 * them by uniform buckets in xy; bt_levels returns n values in input order.  Usable with
 * bt_accumulate_mics and bt_run; the scenario and serving interfaces take grids. */
bt_status bt_mics_points(bt_ctx *ctx, const float *xyz, int64_t n, bt_mics **out);
bt_status bt_mics_reset(bt_ctx *ctx, bt_mics *mics);   /* zero the energies (kernel, no memset) */
bt_status bt_mics_free(bt_mics *mics);

/* Generation-0 beams (paper Section 2: a source's energy is shared between beams by
 * direction): for each source and each face of the
 * level-`level` icosphere, one frustum beam with apex at the source and intensity
 * constant K = W / (4 pi).  src_xyz host float[n_src][3]; src_power host float[n_src].
 * *inout: NULL to create a beam set, or an existing set to reuse (its capacity grows
 * if needed).  Resets the set's statistics. */
bt_status bt_emit_beams(bt_ctx *ctx, const float *src_xyz, const float *src_power, int32_t n_src,
                        int32_t level, bt_beams **inout);
/* Generation-0 beams of directional sources (paper Section 2: a source's power is shared
 * between beams by direction).  src_weight: host
 * float[n_src][20 4^level], the relative intensity of each source towards each face (in
 * emission order), finite and >= 0.  Beam b of source s gets K_b = W_s w_b /
 * sum_f(w_f Omega_f), so the beams' powers K_b Omega_b add up to W_s; equal weights give
 * the omni split of bt_emit_beams.  Otherwise as bt_emit_beams. */
bt_status bt_emit_beams_directional(bt_ctx *ctx, const float *src_xyz, const float *src_power,
                                    const float *src_weight, int32_t n_src, int32_t level, bt_beams **inout);
bt_status bt_beams_free(bt_beams *beams);
bt_status bt_beams_stats(bt_ctx *ctx, const bt_beams *beams, bt_stats *out);

/* Trace the current generation: closest hit of every guiding ray (paper Section 2:
 * intersections handled as in ray tracing, guiding ray only), hand-off between
 * sub-domains, then reflection of hits with depth < max_depth into the next
 * generation's queue (one child per hit, never split).  Every generation's segments
 * stay resident in device memory (n_beams0 * (max_depth + 1) records at most) until the
 * next emission.  n_next: NULL (no synchronisation) or host int64 receiving the next
 * generation's size (syncs).  Returns BT_ESTATE once max_depth + 1 generations have been
 * traced, or for a set that holds no emission (created by bt_beams_bind_mics and never
 * emitted, or whose last emission failed after its arguments were accepted, e.g. out of
 * memory: emit again); BT_EINVAL if n_beams0 * (max_depth + 1) exceeds 2^31 - 1, or if
 * the set's earlier generations were traced with another mesh (an emission's generations
 * and their accumulation all use one mesh). */
bt_status bt_trace(bt_ctx *ctx, const bt_mesh *mesh, bt_beams *beams, const bt_params *params,
                   int64_t *n_next);

/* Trace every remaining generation of the set, up to params->max_depth: the same work
 * and results as that many bt_trace calls, enqueued at once without synchronisation.  On a
 * partitioned set each partition's generations run on its own stream without waiting for
 * the others' (joined to the context's stream before the call returns).  BT_ESTATE when
 * every generation is already traced; otherwise as bt_trace. */
bt_status bt_trace_all(bt_ctx *ctx, const bt_mesh *mesh, bt_beams *beams, const bt_params *params);

/* Add the contributions of every segment traced since the previous call (all of them
 * after a first call) to the microphones, in one pass (paper Section 2: microphones sum
 * the contributions reaching them); a call with nothing new traced does nothing.
 * Returns BT_ESTATE before the first bt_trace.  A microphone inside
 * a segment's frustum (three side planes, the reflecting plane as near cap, the hit
 * plane as far cap) receives K exp(-air_m d) / d^2, d = distance to the beam's
 * (image) apex.  Contributions of flagged segments, and memberships decided within
 * edge_delta of a frustum plane, go to the set's flag energy, the others to its
 * strict energy; both are FP64.  A partitioned set's partitions make their passes on
 * their own streams at once (their contributions meet only in FP64 atomic additions). */
bt_status bt_accumulate_mics(bt_ctx *ctx, const bt_mesh *mesh, bt_beams *beams, const bt_params *params,
                             bt_mics *mics);

/* Classify a beam set's beams against a planar microphone grid as they are created
 * (paper Section 2: a beam contributes to the microphones inside its frustum, and most
 * beams hold none of a planar grid's microphones).  While bound, emission and every
 * trace's reflection decide for each new beam, from its frustum alone, whether it can
 * hold a microphone of the grid's plane, and which lattice box bounds the candidates; a
 * later bt_accumulate_mics (or _static) with that grid, or a subset of it, then reads
 * those decisions instead of every beam's frustum, for the generations created while
 * bound.  Results are identical with or without it.  *beams may be NULL: an empty set is
 * created (caller frees).  mics = NULL unbinds.  Costs 8 bytes of device memory per queue
 * record.  BT_EINVAL for explicit points, volumetric grids and grids of 2^26 or more
 * microphones per side.  bt_run binds its set to its microphones when they are planar. */
bt_status bt_beams_bind_mics(bt_ctx *ctx, bt_beams **beams, const bt_mics *mics);

/* bt_accumulate_mics for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments, kernels
 * and results as bt_accumulate_mics; it calls no hipMalloc, hipFree or allocating library
 * routine.  Its work lists live in a static device array of 64 MiB per GPU, which the
 * library holds from its first bt_create on that GPU until the process ends.  Limit: the
 * segments of the pass may number at most n_beams0 x (generations since the previous
 * accumulation) <= about 5.4 M (e.g. one generation of 64 level-6 sources); a larger pass
 * returns BT_EINVAL with nothing enqueued (accumulate after fewer generations).  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU (other contexts or
 * streams) race and must be serialised by the caller.  The partitions of a partitioned
 * set are accumulated one after another on the context's stream, and the limit applies
 * to each partition.  Explicit point sets use no work lists. */
bt_status bt_accumulate_mics_static(bt_ctx *ctx, const bt_mesh *mesh, bt_beams *beams, const bt_params *params,
                                    bt_mics *mics);

/* Copy results to caller-owned host or device buffers (any may be NULL), then
 * synchronise: strict_out / flag_out double[n_mic] energies (W/m^2), level_db_out
 * double[n_mic] = 10 log10((strict + flag) / 1e-12), -inf where no energy arrived. */
bt_status bt_levels(bt_ctx *ctx, const bt_mics *mics, double *strict_out, double *flag_out,
                    double *level_db_out);

/* Convenience: the whole method for a source set (paper Section 2), with memory bounded
 * whatever the number of sources, level or depth.  The sources are taken in chunks of at
 * most 16 Mi generation-0 beams (at least one source each).  When the largest chunk's
 * records, n_beams0 (max_depth + 1), fit params->run_records, every chunk keeps every
 * generation and makes one microphone pass at its end (the fast layout); otherwise every
 * chunk keeps two generation slots and each of its generations is accumulated as soon as
 * it is traced.  So n_src x 20 4^level may exceed 2^31, and a run holds at most
 * run_records (resident) or 2 x 16 Mi (two slots) beam records.  Parity outputs in
 * params keep their global rows [n_src 20 4^level][max_depth + 1].  bt_beams_stats on the
 * set afterwards reports the whole run (it synchronises once per extra chunk).  Each
 * chunk is emitted in partitions (bt_set_partitions), and each partition traces all its
 * generations and makes its microphone passes on its own stream, joined at the chunk's
 * end.  Reuses *beams when non-NULL (created otherwise; caller frees).  Does not
 * synchronise apart from those chunk boundaries. */
bt_status bt_run(bt_ctx *ctx, const bt_mesh *mesh, const float *src_xyz, const float *src_power,
                 int32_t n_src, int32_t level, const bt_params *params, bt_mics *mics, bt_beams **beams);

/* Request interface (paper Section 3: the model is prepared once for multiple
 * simulations).  A request is a source set, an icosphere level, a depth and the
 * microphone grid given at submission; its result is the grid's energies. */
typedef struct {
    const float *src_xyz;     /* host float[n_src][3] */
    const float *src_power;   /* host float[n_src] */
    int32_t n_src;
    int32_t level;
    int32_t max_depth;
    float mic_x0, mic_y0, mic_z, mic_dx, mic_dy;
    int32_t mic_nx, mic_ny;
} bt_request;

typedef struct {
    double *energy;           /* caller-owned host double[mic_nx * mic_ny] (strict + flag) */
    double *flag_energy;      /* caller-owned host double[...] or NULL */
    int64_t segments;         /* filled on completion */
    int64_t mic_updates;
} bt_result;

bt_status bt_submit(bt_ctx *ctx, const bt_mesh *mesh, const bt_request *req, uint64_t *ticket);
bt_status bt_poll(bt_ctx *ctx, uint64_t ticket, bt_result *out);
bt_status bt_cancel(bt_ctx *ctx, uint64_t ticket);

/* ------------------------------------------------------------------------------------
 * Batches of independent scenarios (paper Section 3: one model, many simulations; the
 * work of all of them is shared out over the same processors).  The beams of many
 * scenarios are traced together: each generation of every scenario in a chunk is one
 * set of kernel launches over a shared queue whose beams carry their scenario's slot and
 * depth limit, and each segment's contributions go to its own scenario's microphones.
 * Every scenario's result equals the one it has when run alone with bt_run (up to the
 * order of FP64 additions).
 * ------------------------------------------------------------------------------------ */
typedef struct {
    const float *src_xyz;       /* host float[n_src][3] */
    const float *src_power;     /* host float[n_src] */
    int32_t n_src;              /* >= 0 */
    int32_t level;              /* icosphere level of the scenario's sources, 0..BT_MAX_LEVEL */
    int32_t max_depth;          /* 0..BT_MAX_DEPTH */
    float mic_x0, mic_y0, mic_z, mic_dx, mic_dy;   /* microphone grid, as bt_mics_grid */
    int32_t mic_nx, mic_ny;
    const int32_t *mic_subset;  /* host int32[n_subset]: grid indices j * nx + i, in output
                                   order (repeats allowed); NULL = the whole grid */
    int64_t n_subset;
    double *energy_out;         /* caller-owned host double[n_out] (strict + flag), n_out =
                                   n_subset, or nx * ny without a subset */
    double *flag_out;           /* caller-owned host double[n_out] (flag part) or NULL */
} bt_scenario;

typedef struct {
    int64_t chunk_beams;        /* generation-0 beams traced together at most (a larger
                                   scenario forms a chunk of its own); 0 = 16 Mi */
    int32_t blocks_per_cu;      /* workgroups per compute unit of the statically partitioned
                                   trace and microphone kernels, 1..16; 0 = 8 */
    int32_t use_graph;          /* 1: a chunk's launches are captured once in a hipGraph and
                                   replayed for every chunk */
} bt_batch_opts;

typedef struct {
    int32_t chunks;
    int64_t beams0;             /* generation-0 beams */
    int64_t segments;           /* beam segments traced */
    int64_t mic_updates;
    double seconds;             /* wall time of the call after validation */
} bt_batch_stats;

/* Run n scenarios and write each one's microphone energies to its buffers; synchronises.
 * params: physics (t_min, edge_delta, air_m, e_min; NULL = defaults); its max_depth and
 * parity outputs are not used (each scenario has its own depth).  opts: NULL = defaults.
 * stats: NULL or filled (seconds: from the first upload to the last output, after the
 * workspace is in place).  Scenarios are taken in order into chunks.  BT_EINVAL on a bad
 * scenario (nothing is run), BT_ENOMEM when a chunk does not fit the budget. */
bt_status bt_batch_run(bt_ctx *ctx, const bt_mesh *mesh, const bt_scenario *scenarios, int32_t n,
                       const bt_params *params, const bt_batch_opts *opts, bt_batch_stats *stats);

/* bt_batch_run keeps its device workspace (queue, microphone arrays, staging, captured
 * graph) in the context between calls, grown to the largest chunk seen, so repeated
 * batches allocate nothing; this frees it (bt_destroy does too). */
bt_status bt_batch_release(bt_ctx *ctx);

/* ------------------------------------------------------------------------------------
 * Serving (paper Section 3: the model is built once and serves many simulations).  A
 * server owns a thread that admits requests as they arrive.  In the batched mode it runs
 * continuous batching: at every generation step, requests that fit the free queue
 * records and microphone memory join the shared multi-scenario beam set (their
 * generation-0 beams are appended to the generation being traced), every live request
 * advances by one generation in the same launches, and a request is finished once its
 * max_depth + 1 generations have been traced and accumulated.  In the plain mode it runs
 * one request at a time through bt_run (the baseline).  A request's result equals the
 * result of bt_run on it alone (up to the order of FP64 additions).
 * ------------------------------------------------------------------------------------ */
typedef struct bt_server bt_server;

#define BT_SERVE_BATCHED 0
#define BT_SERVE_PLAIN 1

typedef struct {
    int32_t mode;               /* BT_SERVE_BATCHED or BT_SERVE_PLAIN */
    int64_t max_records;        /* queue records of a batch session (sum over its requests of
                                   n_beams0 (max_depth + 1)); 0 = 32 Mi */
    int64_t arena_bytes;        /* device bytes per session for microphone energies and
                                   outputs; 0 = 1 GiB */
    int32_t blocks_per_cu;      /* 0 = 8 */
} bt_server_opts;

typedef struct {
    double t_submit;            /* seconds since the server started */
    double t_admit;             /* when its beams were first enqueued */
    double t_done;              /* when its outputs were written */
} bt_serve_result;

/* Start a server on (ctx, mesh); params as for bt_batch_run.  The server uses the
 * context's stream; other work on the same context must not run while it lives. */
bt_status bt_server_create(bt_ctx *ctx, const bt_mesh *mesh, const bt_params *params, const bt_server_opts *opts,
                           bt_server **out);
/* Queue a request (a scenario; its host inputs are copied).  Its output buffers must stay
 * valid until bt_server_poll reports it finished.  BT_EINVAL for a bad request, BT_ENOMEM
 * for one that can never fit a session. */
bt_status bt_server_submit(bt_server *s, const bt_scenario *req, uint64_t *ticket);
/* BT_PENDING while the request runs; BT_OK once its outputs are written (the ticket is
 * then released and out, if not NULL, filled); BT_ENOTFOUND for an unknown ticket. */
bt_status bt_server_poll(bt_server *s, uint64_t ticket, bt_serve_result *out);
/* Finish every queued request, stop the thread and free the server. */
bt_status bt_server_destroy(bt_server *s);

#define BT_TUNE_MAX_CANDIDATES 32

/* Choose bt_batch_opts for a workload by running a leading sample of it (about a quarter
 * of the generation-0 beams, at most 32 Mi) under each candidate chunk size and
 * workgroup count, with and without graphs, and keeping the fastest.  The sample's
 * scenarios have their output buffers written.  out receives the choice; seconds_out
 * (NULL or double[n_candidates]) the measured time of each candidate, n_candidates_out
 * (NULL or filled) their number. */
bt_status bt_batch_autotune(bt_ctx *ctx, const bt_mesh *mesh, const bt_scenario *scenarios, int32_t n,
                            const bt_params *params, bt_batch_opts *out, double *seconds_out,
                            int32_t *n_candidates_out);

#ifdef __cplusplus
}
#endif

#endif /* BT_H */
