// Batches of independent scenarios (bt_batch_run, bt_batch_autotune).
//
// The scenarios are taken in order into chunks.  A chunk's generation-0 beams of every
// scenario are emitted into one multi-scenario beam set (each beam's meta carries its
// scenario's slot and depth limit), every generation of the chunk is traced by one set of
// launches, one microphone pass sends each segment's contributions to its own scenario's
// grid arrays, and a gather kernel collects each scenario's outputs.  All sizes a chunk's
// kernels need are read from device memory, so one captured hipGraph serves every chunk.
// Two workspaces take the chunks in turn on two of the context's partition streams: while
// one chunk's last, sparse generations drain, the next chunk's tables are filled on the
// host and its launches run beside them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "bt_host.h"

namespace {

constexpr long long kDefaultChunkBeams = 16ll << 20;
constexpr long long kMaxChunkEnergies = 1ll << 28;   // strict doubles per chunk (2 GiB of both)
constexpr long long kIndexLimit = (1ll << 31) - 1;    // queue records and work items are int32

struct Chunk {
    int first = 0, end = 0;
    long long n0 = 0, records = 0, sources = 0, energy = 0, mask_words = 0, n_out = 0;
};

}  // namespace

// bt_batch_run's workspace, kept in the context between calls and grown when a batch
// needs more: the emission table, slot microphone sets, bitmaps, energies, gather
// indices and outputs (device, with pinned host mirrors), the shared beam set, and the
// captured launch graph (valid while the buffers, the depth and the physics stay).
struct BatchWork {
    bt_ctx *ctx = nullptr;
    long long cap_sources = 0, cap_slots = 0, cap_energy = 0, cap_mask = 0, cap_out = 0, cap_n0 = 0, cap_records = 0;
    int bpc = 0;
    // device
    float *src = nullptr, *power = nullptr;
    int *level = nullptr, *meta = nullptr, *id0 = nullptr;
    long long *first = nullptr, *dims = nullptr;
    DevMics *slots = nullptr;
    unsigned *mask = nullptr;
    double *energy = nullptr;      // per chunk: strict [E], then flag [E]
    long long *gidx = nullptr;
    double *out = nullptr;         // [2][cap_out]: strict + flag, flag
    BatchDesc *desc = nullptr;
    // pinned host
    float *h_src = nullptr, *h_power = nullptr;
    int *h_level = nullptr, *h_meta = nullptr, *h_id0 = nullptr;
    long long *h_first = nullptr, *h_dims = nullptr;
    DevMics *h_slots = nullptr;
    unsigned *h_mask = nullptr;
    long long *h_gidx = nullptr;
    double *h_out = nullptr;
    BatchDesc *h_desc = nullptr;
    DevCounters *h_ctr = nullptr;
    std::vector<std::pair<void *, size_t>> dev_bufs;
    std::vector<void *> host_bufs;
    bt_beams *beams = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_depth = -1;
    bt_params graph_params{};
    hipStream_t stream = nullptr;   // the stream of the chunk in flight (if any)
    hipEvent_t done = nullptr;      // recorded after the chunk's output copies
    int pending = -1;               // the chunk in flight, its outputs not yet unpacked

    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        graph_depth = -1;
    }
    void release()
    {
        if (ctx && ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        if (stream) (void)hipStreamSynchronize(stream);
        pending = -1;
        drop_graph();
        if (beams) bt_beams_free(beams);
        beams = nullptr;
        for (auto &d : dev_bufs) dev_free(ctx, d.first, d.second);
        for (void *h : host_bufs) (void)hipHostFree(h);
        dev_bufs.clear();
        host_bufs.clear();
        cap_sources = cap_slots = cap_energy = cap_mask = cap_out = cap_n0 = cap_records = 0;
        bpc = 0;
    }
    ~BatchWork()
    {
        release();
        if (done) (void)hipEventDestroy(done);
    }
    template <class T> bt_status dev(T **p, long long n)
    {
        const size_t bytes = (size_t)std::max(n, 1ll) * sizeof(T);
        bt_status s = dev_alloc(ctx, (void **)p, bytes);
        if (s == BT_OK) dev_bufs.push_back({(void *)*p, bytes});
        return s;
    }
    template <class T> bt_status host(T **p, long long n)
    {
        const size_t bytes = (size_t)std::max(n, 1ll) * sizeof(T);
        if (hipHostMalloc((void **)p, bytes, hipHostMallocDefault) != hipSuccess) {
            *p = nullptr;
            return fail(ctx, BT_ENOMEM, "pinned host allocation of %zu bytes failed", bytes);
        }
        host_bufs.push_back((void *)*p);
        return BT_OK;
    }
    // Capacity for chunks up to `need` (sources, slots, energy, mask words, outputs, n0,
    // records) with blocks_per_cu workgroups per CU; everything is reallocated (grown) if
    // anything is short.
    bt_status ensure(const Chunk &need, long long records, int blocks_per_cu)
    {
        if (bpc == blocks_per_cu && need.sources <= cap_sources && need.end - need.first <= cap_slots &&
            need.energy <= cap_energy && need.mask_words <= cap_mask && need.n_out <= cap_out && need.n0 <= cap_n0 &&
            records <= cap_records)
            return BT_OK;
        const long long s_ = std::max(need.sources, cap_sources), sl = std::max<long long>(need.end - need.first, cap_slots);
        const long long e_ = std::max(need.energy, cap_energy), m_ = std::max(need.mask_words, cap_mask);
        const long long o_ = std::max(need.n_out, cap_out), n0 = std::max(std::max(need.n0, cap_n0), 1ll);
        const long long r_ = std::max(std::max(records, cap_records), 1ll);
        release();
        bt_status st;
        if ((st = dev(&src, 3 * s_)) != BT_OK || (st = dev(&power, s_)) != BT_OK || (st = dev(&level, s_)) != BT_OK ||
            (st = dev(&meta, s_)) != BT_OK || (st = dev(&id0, s_)) != BT_OK || (st = dev(&first, s_ + 1)) != BT_OK ||
            (st = dev(&dims, 2)) != BT_OK || (st = dev(&slots, sl)) != BT_OK || (st = dev(&mask, m_)) != BT_OK ||
            (st = dev(&energy, 2 * e_)) != BT_OK || (st = dev(&gidx, o_)) != BT_OK || (st = dev(&out, 2 * o_)) != BT_OK ||
            (st = dev(&desc, 1)) != BT_OK)
            return st;
        if ((st = host(&h_src, 3 * s_)) != BT_OK || (st = host(&h_power, s_)) != BT_OK ||
            (st = host(&h_level, s_)) != BT_OK || (st = host(&h_meta, s_)) != BT_OK || (st = host(&h_id0, s_)) != BT_OK ||
            (st = host(&h_first, s_ + 1)) != BT_OK || (st = host(&h_dims, 2)) != BT_OK ||
            (st = host(&h_slots, sl)) != BT_OK || (st = host(&h_mask, m_)) != BT_OK || (st = host(&h_gidx, o_)) != BT_OK ||
            (st = host(&h_out, 2 * o_)) != BT_OK || (st = host(&h_desc, 1)) != BT_OK || (st = host(&h_ctr, 1)) != BT_OK)
            return st;
        // the shared beam set: every generation of the largest chunk resident
        beams = new bt_beams();
        beams->ctx = ctx;
        if ((st = dev_alloc(ctx, (void **)&beams->ctr, sizeof(DevCounters))) != BT_OK) return st;
        if ((st = alloc_wave_scratch(ctx, beams, blocks_per_cu)) != BT_OK) return st;
        if ((st = reserve_queue(ctx, beams, r_, 0)) != BT_OK) return st;
        if ((st = reserve_work(ctx, beams, n0)) != BT_OK) return st;
        if ((st = reserve_tiles(ctx, beams, n0)) != BT_OK) return st;
        cap_sources = s_;
        cap_slots = sl;
        cap_energy = e_;
        cap_mask = m_;
        cap_out = o_;
        cap_n0 = n0;
        cap_records = r_;
        bpc = blocks_per_cu;
        return BT_OK;
    }
};

void batch_work_free(bt_ctx *ctx)
{
    delete[] ctx->batch;
    ctx->batch = nullptr;
}

namespace {

// The chunk's launches: counters, emission, zeroed energies, every generation's trace,
// one microphone pass over all of them, the gather.  Grid sizes follow the capacities;
// the kernels read the chunk's own sizes from device memory.
bt_status enqueue_chunk(bt_ctx *ctx, const bt_mesh *mesh, BatchWork &w, const TraceArgs &base, int depth,
                        hipStream_t s)
{
    bt_beams *b = w.beams;
    const EmitTable t{w.src, w.power, w.level, w.meta, w.id0, w.first, w.dims};
    HIP_TRY(ctx, launch_init_counters(b->ctr, 0, 0, s));
    HIP_TRY(ctx, launch_emit_table(ctx->base20, t, w.cap_n0, b->q, b->ctr, 0, s));
    HIP_TRY(ctx, launch_fill_desc(w.energy, w.desc, 2 * w.cap_energy, s));
    for (int g = 0; g <= depth; ++g) {
        TraceArgs a = base;
        a.gen = g;
        HIP_TRY(ctx, launch_trace(mesh->dev, b->q, b->segs, b->ctr, a, b->ws, trace_tiles(b, mesh, a), ctx->n_cu, s));
    }
    TraceArgs a = base;
    a.gen = 0;
    a.gen_end = depth + 1;
    MicWork mw{b->rows, b->rows_cap, b->spans, b->spans_cap, b->big_list + b->cap, b->big_list};
    HIP_TRY(ctx, launch_mics(mesh->dev, b->q, b->segs, b->ctr, DevMics{}, a, mw, b->ws, ctx->n_cu, s));
    HIP_TRY(ctx, launch_gather(w.energy, w.gidx, w.desc, w.cap_out, w.out, w.out + w.cap_out, s));
    return BT_OK;
}

bool same_physics(const bt_params &a, const bt_params &b)
{
    return a.t_min == b.t_min && a.edge_delta == b.edge_delta && a.air_m == b.air_m && a.e_min == b.e_min;
}

bt_status run_batch(bt_ctx *ctx, const bt_mesh *mesh, const bt_scenario *sc, int n, const bt_params *params,
                    const bt_batch_opts &o, bt_batch_stats *stats)
{
    bt_params p;
    if (params) p = *params;
    else bt_params_default(&p);
    p.max_depth = 0;  // per scenario
    p.hit_out = nullptr;
    p.flag_out = nullptr;
    p.t_out = nullptr;
    bt_status st = check_params(ctx, mesh, &p);
    if (st != BT_OK) return st;
    std::vector<ScenarioSize> z((size_t)n);
    int depth = 0;
    for (int k = 0; k < n; ++k) {
        if ((st = validate_scenario(ctx, mesh, sc[k], k, z[k])) != BT_OK) return st;
        depth = std::max(depth, sc[k].max_depth);
    }
    // chunks, in scenario order
    std::vector<Chunk> chunks;
    Chunk c;
    for (int k = 0; k < n; ++k) {
        const bool fits = c.end == c.first ||
                          (c.n0 + z[k].n0 <= o.chunk_beams && c.records + z[k].records <= kIndexLimit &&
                           c.end - c.first + 1 < kMaxSlots && c.energy + z[k].grid <= kMaxChunkEnergies);
        if (!fits) {
            chunks.push_back(c);
            c = Chunk{};
            c.first = c.end = k;
        }
        c.end = k + 1;
        c.n0 += z[k].n0;
        c.records += z[k].records;
        c.sources += sc[k].n_src;
        c.energy += z[k].grid;
        c.mask_words += z[k].mask_words;
        c.n_out += z[k].n_out;
    }
    if (c.end > c.first) chunks.push_back(c);
    Chunk need;
    long long records = 1;
    for (const Chunk &ch : chunks) {
        need.sources = std::max(need.sources, ch.sources);
        need.end = std::max(need.end, ch.end - ch.first);
        need.energy = std::max(need.energy, ch.energy);
        need.mask_words = std::max(need.mask_words, ch.mask_words);
        need.n_out = std::max(need.n_out, ch.n_out);
        need.n0 = std::max(need.n0, ch.n0);
        records = std::max(records, ch.records);
    }
    if (!ctx->batch) {
        ctx->batch = new BatchWork[2];
        ctx->batch[0].ctx = ctx->batch[1].ctx = ctx;
    }
    BatchWork *W = ctx->batch;
    // two workspaces when there are two chunks or more (one if the second does not fit)
    int n_slots = chunks.size() > 1 ? 2 : 1;
    if ((st = W[0].ensure(need, records, o.blocks_per_cu)) != BT_OK) {
        W[0].release();
        return st;
    }
    if (n_slots == 2 && W[1].ensure(need, records, o.blocks_per_cu) != BT_OK) {
        W[1].release();
        n_slots = 1;
        ctx->err.clear();
    }
    hipStream_t streams[2] = {ctx->stream, ctx->stream};
    if (n_slots == 2) {
        HIP_TRY(ctx, partition_streams(ctx));
        // the slots' streams start after everything enqueued on the context's stream so far
        HIP_TRY(ctx, hipEventRecord(ctx->fork_ev, ctx->stream));
        for (int k = 0; k < 2; ++k) {
            streams[k] = ctx->part_stream[k];
            HIP_TRY(ctx, hipStreamWaitEvent(streams[k], ctx->fork_ev, 0));
        }
    }
    for (int k = 0; k < n_slots; ++k) {
        if (!W[k].done) HIP_TRY(ctx, hipEventCreateWithFlags(&W[k].done, hipEventDisableTiming));
        W[k].stream = streams[k];
        W[k].pending = -1;
    }
    TraceArgs base = make_args(&p, 0);
    base.max_depth = depth;
    base.scenarios = 1;
    const auto t0 = std::chrono::steady_clock::now();
    long long segments = 0, updates = 0, beams0 = 0;
    // a finished chunk's outputs to the scenarios' buffers, and its counts
    auto unpack = [&](BatchWork &w) -> bt_status {
        if (w.pending < 0) return BT_OK;
        HIP_TRY(ctx, hipEventSynchronize(w.done));
        const Chunk &ch = chunks[(size_t)w.pending];
        long long off = 0;
        for (int k = ch.first; k < ch.end; ++k) {
            std::memcpy(sc[k].energy_out, w.h_out + off, (size_t)z[k].n_out * sizeof(double));
            if (sc[k].flag_out)
                std::memcpy(sc[k].flag_out, w.h_out + w.cap_out + off, (size_t)z[k].n_out * sizeof(double));
            off += z[k].n_out;
        }
        for (int g = 0; g <= depth; ++g) segments += (long long)w.h_ctr->count[g];
        updates += (long long)mic_stat_total(*w.h_ctr, MS_UPDATES);
        beams0 += ch.n0;
        w.pending = -1;
        return BT_OK;
    };
    // on any early return, the slots' streams are drained (their host buffers stay valid)
    struct Drain {
        BatchWork *w;
        int n;
        ~Drain()
        {
            for (int k = 0; k < n; ++k)
                if (w[k].stream) (void)hipStreamSynchronize(w[k].stream);
        }
    } drain{W, n_slots};
    for (size_t ci = 0; ci < chunks.size(); ++ci) {
        const Chunk &ch = chunks[ci];
        BatchWork &w = W[ci % (size_t)n_slots];
        const hipStream_t s = w.stream;
        // the slot's previous chunk must be finished before its pinned tables are refilled
        if ((st = unpack(w)) != BT_OK) return st;
        if (w.exec && (w.graph_depth != depth || !same_physics(w.graph_params, p))) w.drop_graph();
        TraceArgs bw = base;
        bw.slot_mics = w.slots;
        // emission table, slot microphone sets, subset masks and gather indices; the flag
        // energies follow the chunk's E strict ones
        long long E = 0;
        for (int k = ch.first; k < ch.end; ++k) E += z[k].grid;
        long long ns = 0, beam = 0, eoff = 0, moff = 0, ooff = 0;
        for (int k = ch.first; k < ch.end; ++k) {
            const bt_scenario &q = sc[k];
            const int slot = k - ch.first;
            const long long nf = 20ll << (2 * q.level);
            for (int i = 0; i < q.n_src; ++i, ++ns) {
                std::memcpy(w.h_src + 3 * ns, q.src_xyz + 3 * i, 3 * sizeof(float));
                w.h_power[ns] = q.src_power[i];
                w.h_level[ns] = q.level;
                w.h_meta[ns] = scenario_meta(slot, q.max_depth);
                w.h_id0[ns] = (int)(i * nf);
                w.h_first[ns] = beam;
                beam += nf;
            }
            DevMics m{};
            m.x0 = q.mic_x0;
            m.y0 = q.mic_y0;
            m.z = q.mic_z;
            m.dx = q.mic_dx;
            m.dy = q.mic_dy;
            m.nx = q.mic_nx;
            m.ny = q.mic_ny;
            m.nz = 1;
            m.e_strict = w.energy + eoff;
            m.e_flag = w.energy + E + eoff;
            m.mask = nullptr;
            if (q.mic_subset) {
                unsigned *mk = w.h_mask + moff;
                std::memset(mk, 0, (size_t)z[k].mask_words * sizeof(unsigned));
                for (long long i = 0; i < q.n_subset; ++i) {
                    const long long g = q.mic_subset[i];
                    mk[g >> 5] |= 1u << (g & 31);
                    w.h_gidx[ooff + i] = eoff + g;
                }
                m.mask = w.mask + moff;
                moff += z[k].mask_words;
            } else {
                for (long long g = 0; g < z[k].grid; ++g) w.h_gidx[ooff + g] = eoff + g;
            }
            w.h_slots[slot] = m;
            eoff += z[k].grid;
            ooff += z[k].n_out;
        }
        w.h_first[ns] = beam;
        w.h_dims[0] = beam;
        w.h_dims[1] = ns;
        w.h_desc[0] = BatchDesc{2 * E, ooff, E};
        const size_t nsrc = (size_t)std::max(ns, 1ll);
        HIP_TRY(ctx, hipMemcpyAsync(w.src, w.h_src, 3 * nsrc * sizeof(float), hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(w.power, w.h_power, nsrc * sizeof(float), hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(w.level, w.h_level, nsrc * sizeof(int), hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(w.meta, w.h_meta, nsrc * sizeof(int), hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(w.id0, w.h_id0, nsrc * sizeof(int), hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(w.first, w.h_first, (nsrc + 1) * sizeof(long long), hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(w.dims, w.h_dims, 2 * sizeof(long long), hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(w.slots, w.h_slots, (size_t)(ch.end - ch.first) * sizeof(DevMics),
                                    hipMemcpyHostToDevice, s));
        if (moff > 0)
            HIP_TRY(ctx, hipMemcpyAsync(w.mask, w.h_mask, (size_t)moff * sizeof(unsigned), hipMemcpyHostToDevice, s));
        if (ooff > 0)
            HIP_TRY(ctx, hipMemcpyAsync(w.gidx, w.h_gidx, (size_t)ooff * sizeof(long long), hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(w.desc, w.h_desc, sizeof(BatchDesc), hipMemcpyHostToDevice, s));
        if (o.use_graph) {
            if (!w.exec) {
                HIP_TRY(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                bt_status cs = enqueue_chunk(ctx, mesh, w, bw, depth, s);
                hipGraph_t g = nullptr;
                const hipError_t ce = hipStreamEndCapture(s, &g);
                if (cs != BT_OK) {
                    if (g) (void)hipGraphDestroy(g);
                    return cs;
                }
                if (ce != hipSuccess) return hip_fail(ctx, ce, "hipStreamEndCapture");
                w.graph = g;
                HIP_TRY(ctx, hipGraphInstantiate(&w.exec, w.graph, nullptr, nullptr, 0));
                w.graph_depth = depth;
                w.graph_params = p;
            }
            HIP_TRY(ctx, hipGraphLaunch(w.exec, s));
        } else if ((st = enqueue_chunk(ctx, mesh, w, bw, depth, s)) != BT_OK) {
            return st;
        }
        if (ooff > 0) {
            HIP_TRY(ctx, hipMemcpyAsync(w.h_out, w.out, (size_t)ooff * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_TRY(ctx, hipMemcpyAsync(w.h_out + w.cap_out, w.out + w.cap_out, (size_t)ooff * sizeof(double),
                                        hipMemcpyDeviceToHost, s));
        }
        HIP_TRY(ctx, hipMemcpyAsync(w.h_ctr, w.beams->ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipEventRecord(w.done, s));
        w.pending = (int)ci;
    }
    for (int k = 0; k < n_slots; ++k)
        if ((st = unpack(W[k])) != BT_OK) return st;
    if (stats) {
        stats->chunks = (int32_t)chunks.size();
        stats->beams0 = beams0;
        stats->segments = segments;
        stats->mic_updates = updates;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return BT_OK;
}

bt_status resolve_opts(bt_ctx *ctx, const bt_batch_opts *opts, bt_batch_opts &o)
{
    o = bt_batch_opts{kDefaultChunkBeams, kBlocksPerCU, 0};
    if (opts) {
        if (opts->chunk_beams < 0) return fail(ctx, BT_EINVAL, "chunk_beams < 0");
        if (opts->blocks_per_cu < 0 || opts->blocks_per_cu > 16) return fail(ctx, BT_EINVAL, "blocks_per_cu not in 0..16");
        if (opts->chunk_beams > 0) o.chunk_beams = opts->chunk_beams;
        if (opts->blocks_per_cu > 0) o.blocks_per_cu = opts->blocks_per_cu;
        o.use_graph = opts->use_graph ? 1 : 0;
    }
    return BT_OK;
}

}  // namespace

bt_status validate_scenario(bt_ctx *ctx, const bt_mesh *mesh, const bt_scenario &sc, int k, ScenarioSize &z)
{
    if (sc.n_src < 0 || (sc.n_src > 0 && (!sc.src_xyz || !sc.src_power)))
        return fail(ctx, BT_EINVAL, "scenario %d: bad sources", k);
    if (sc.level < 0 || sc.level > BT_MAX_LEVEL) return fail(ctx, BT_EINVAL, "scenario %d: level %d", k, sc.level);
    if (sc.max_depth < 0 || sc.max_depth > BT_MAX_DEPTH)
        return fail(ctx, BT_EINVAL, "scenario %d: max_depth %d", k, sc.max_depth);
    for (int i = 0; i < sc.n_src; ++i) {
        for (int c = 0; c < 3; ++c) {
            const float v = sc.src_xyz[3 * i + c];
            if (!std::isfinite(v) || std::fabs((double)v) > mesh->r_eff)
                return fail(ctx, BT_EINVAL, "scenario %d: source %d outside the region the mesh margins cover", k, i);
        }
        if (!(sc.src_power[i] >= 0.f) || !std::isfinite(sc.src_power[i]))
            return fail(ctx, BT_EINVAL, "scenario %d: source %d power invalid", k, i);
    }
    if (sc.mic_nx < 1 || sc.mic_ny < 1 || (long long)sc.mic_nx * sc.mic_ny > kIndexLimit)
        return fail(ctx, BT_EINVAL, "scenario %d: bad microphone grid %d x %d", k, sc.mic_nx, sc.mic_ny);
    if (!std::isfinite(sc.mic_x0) || !std::isfinite(sc.mic_y0) || !std::isfinite(sc.mic_z) || !(sc.mic_dx > 0.f) ||
        !(sc.mic_dy > 0.f) || !std::isfinite(sc.mic_dx) || !std::isfinite(sc.mic_dy))
        return fail(ctx, BT_EINVAL, "scenario %d: bad microphone grid geometry", k);
    if (!sc.energy_out) return fail(ctx, BT_EINVAL, "scenario %d: energy_out is NULL", k);
    z.grid = (long long)sc.mic_nx * sc.mic_ny;
    if (sc.mic_subset) {
        if (sc.n_subset < 1 || sc.n_subset > kIndexLimit) return fail(ctx, BT_EINVAL, "scenario %d: n_subset", k);
        for (long long i = 0; i < sc.n_subset; ++i)
            if (sc.mic_subset[i] < 0 || (long long)sc.mic_subset[i] >= z.grid)
                return fail(ctx, BT_EINVAL, "scenario %d: subset index %lld out of the grid", k, i);
        z.n_out = sc.n_subset;
        z.mask_words = (z.grid + 31) / 32;
    } else {
        z.n_out = z.grid;
        z.mask_words = 0;
    }
    z.n0 = (long long)sc.n_src * (20ll << (2 * sc.level));
    z.records = z.n0 * (sc.max_depth + 1);
    if (z.records > kIndexLimit) return fail(ctx, BT_EINVAL, "scenario %d: too many beams", k);
    return BT_OK;
}

extern "C" bt_status bt_batch_run(bt_ctx *ctx, const bt_mesh *mesh, const bt_scenario *scenarios, int32_t n,
                                  const bt_params *params, const bt_batch_opts *opts, bt_batch_stats *stats)
{
    if (!ctx) return BT_EINVAL;
    if (!mesh || n < 0 || (n > 0 && !scenarios)) return fail(ctx, BT_EINVAL, "NULL mesh or scenarios, or n < 0");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n == 0) return BT_OK;
    bt_batch_opts o;
    bt_status s = resolve_opts(ctx, opts, o);
    if (s != BT_OK) return s;
    (void)hipSetDevice(ctx->device);
    return run_batch(ctx, mesh, scenarios, n, params, o, stats);
}

extern "C" bt_status bt_batch_release(bt_ctx *ctx)
{
    if (!ctx) return BT_EINVAL;
    (void)hipSetDevice(ctx->device);
    batch_work_free(ctx);
    return BT_OK;
}

extern "C" bt_status bt_batch_autotune(bt_ctx *ctx, const bt_mesh *mesh, const bt_scenario *scenarios, int32_t n,
                                       const bt_params *params, bt_batch_opts *out, double *seconds_out,
                                       int32_t *n_candidates_out)
{
    if (!ctx) return BT_EINVAL;
    if (!mesh || !out || n <= 0 || !scenarios) return fail(ctx, BT_EINVAL, "NULL mesh, out or scenarios, or n <= 0");
    (void)hipSetDevice(ctx->device);
    // the leading sample: about a quarter of the beams, at most 32 Mi, at least one scenario
    long long total = 0;
    for (int k = 0; k < n; ++k)
        total += (long long)std::max(scenarios[k].n_src, 0) * (20ll << (2 * std::min(std::max(scenarios[k].level, 0), BT_MAX_LEVEL)));
    const long long want = std::min(std::max(total / 4, 1ll), 32ll << 20);
    int m = 0;
    long long sample = 0;
    while (m < n && (m == 0 || sample < want)) {
        sample += (long long)std::max(scenarios[m].n_src, 0) *
                  (20ll << (2 * std::min(std::max(scenarios[m].level, 0), BT_MAX_LEVEL)));
        ++m;
    }
    // largest chunks first for each grid width, so the cached workspace is allocated once
    // per width rather than grown candidate by candidate
    std::vector<long long> sizes;
    for (long long cb : {4ll << 20, 8ll << 20, 16ll << 20, 32ll << 20}) {
        if (cb > 2 * sample && !sizes.empty()) break;
        sizes.push_back(cb);
    }
    std::vector<bt_batch_opts> cand;
    for (int bpc : {8, 4})
        for (auto it = sizes.rbegin(); it != sizes.rend(); ++it)
            for (int g : {0, 1}) cand.push_back(bt_batch_opts{*it, bpc, g});
    // an untimed first run pays for code loading and first-touch allocation
    bt_status s = bt_batch_run(ctx, mesh, scenarios, m, params, &cand[0], nullptr);
    if (s != BT_OK) return s;
    double best = INFINITY;
    for (size_t i = 0; i < cand.size(); ++i) {
        bt_batch_stats st{};
        if ((s = bt_batch_run(ctx, mesh, scenarios, m, params, &cand[i], &st)) != BT_OK) return s;
        if (seconds_out && i < BT_TUNE_MAX_CANDIDATES) seconds_out[i] = st.seconds;
        if (st.seconds < best) {
            best = st.seconds;
            *out = cand[i];
        }
    }
    if (n_candidates_out) *n_candidates_out = (int32_t)std::min<size_t>(cand.size(), BT_TUNE_MAX_CANDIDATES);
    return BT_OK;
}
