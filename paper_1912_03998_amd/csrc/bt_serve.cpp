// Request server (bt_server_*).
//
// Batched mode: continuous batching over two multi-scenario beam sets ("sessions").  The
// server thread runs steps; in each step every session that has requests in flight
// traces one generation, in one set of launches for all its requests; in a step that
// finishes a request, one microphone pass accumulates every generation traced since the
// previous pass into each request's own arrays (all generations stay resident).  Requests
// are admitted at step boundaries, in arrival order, into the open session while it has
// free queue records, arena memory, slots and generations: their generation-0 beams are
// appended to the generation the session traces next.  A request admitted at generation
// g with depth D is finished after the step that traces generation g + D; its outputs are
// gathered and copied back in that step.  When the open session cannot take the next
// request it is closed (it drains) and the other session, once empty, is reset and opened.
// At most two steps are in flight: the host prepares step k + 1 while the GPU runs step k.
//
// Plain mode: one request at a time through bt_run and bt_levels (the baseline).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "bt_host.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr long long kDefaultRecords = 32ll << 20;
constexpr long long kDefaultArena = 256ll << 20;
constexpr int kSessionSlots = 4096;   // requests per session at most
constexpr int kStepSources = 4096;    // sources emitted by one session in one step at most
constexpr int kLastGen = BT_MAX_DEPTH;

inline long long align256(long long n) { return (n + 255) & ~255ll; }

struct Req {
    uint64_t ticket = 0;
    bt_scenario sc{};
    std::vector<float> src, pw;
    std::vector<int32_t> subset;
    ScenarioSize z{};
    double t_submit = 0, t_admit = -1, t_done = -1;
    bool done = false;
    // batched mode: slot and generation of admission, device / pinned arena blocks
    int slot = -1, admit_gen = -1, session = -1;
    double *energy = nullptr;   // device: strict [grid], flag [grid]
    unsigned *mask = nullptr;   // device subset bitmap, or NULL
    long long *gidx = nullptr;  // device: output k -> energy index
    double *out = nullptr;      // device: [2][n_out] (strict + flag, flag)
    BatchDesc *desc = nullptr;  // device
    double *h_out = nullptr;    // pinned: [2][n_out]
    unsigned *h_mask = nullptr;
    long long *h_gidx = nullptr;
    BatchDesc *h_desc = nullptr;
};

// Device and pinned bytes a request takes from a session's arenas.
inline long long dev_need(const ScenarioSize &z)
{
    return align256(16 * z.grid) + align256(4 * z.mask_words) + align256(8 * z.n_out) + align256(16 * z.n_out) +
           align256(sizeof(BatchDesc));
}
inline long long host_need(const ScenarioSize &z)
{
    return align256(16 * z.n_out) + align256(4 * z.mask_words) + align256(8 * z.n_out) + align256(sizeof(BatchDesc));
}

struct Table {  // one step's emission table: device buffers and pinned staging
    float *src = nullptr, *pw = nullptr;
    int *level = nullptr, *meta = nullptr, *id0 = nullptr;
    long long *first = nullptr, *dims = nullptr;
};

struct Session {
    bt_beams *b = nullptr;
    DevMics *slots = nullptr, *h_slots = nullptr;
    Table dev, host[2];            // pinned staging alternates with the step parity
    char *arena = nullptr, *h_arena = nullptr;
    long long arena_used = 0, h_used = 0;
    long long records = 0;
    int n_slots = 0, gen = 0;
    int acc_gen = 0;               // first generation not yet accumulated at the microphones
    int unfinished = 0;            // admitted and not yet finalized
    bool open = false;
    std::vector<Req *> live, fresh;
    bool dirty = true;             // counters need zeroing before the next use
};

}  // namespace

struct bt_server {
    bt_ctx *ctx = nullptr;
    const bt_mesh *mesh = nullptr;
    bt_params params{};
    bt_server_opts opts{};
    Clock::time_point t0;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> pending;
    std::map<uint64_t, Req *> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    bt_status failed = BT_OK;
    // batched mode
    Session sess[2];
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<Req *> finishing[2];
    std::vector<std::pair<void *, size_t>> dev_bufs;
    std::vector<void *> host_bufs;
    // plain mode
    bt_beams *pb = nullptr;
    bt_mics *pm = nullptr;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
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
};

namespace {

bt_status alloc_table(bt_server *s, Table &t, bool pinned)
{
    const long long n = kStepSources;
    bt_status st;
    if (pinned) {
        if ((st = s->host(&t.src, 3 * n)) != BT_OK || (st = s->host(&t.pw, n)) != BT_OK ||
            (st = s->host(&t.level, n)) != BT_OK || (st = s->host(&t.meta, n)) != BT_OK ||
            (st = s->host(&t.id0, n)) != BT_OK || (st = s->host(&t.first, n + 1)) != BT_OK ||
            (st = s->host(&t.dims, 2)) != BT_OK)
            return st;
        return BT_OK;
    }
    if ((st = s->dev(&t.src, 3 * n)) != BT_OK || (st = s->dev(&t.pw, n)) != BT_OK ||
        (st = s->dev(&t.level, n)) != BT_OK || (st = s->dev(&t.meta, n)) != BT_OK ||
        (st = s->dev(&t.id0, n)) != BT_OK || (st = s->dev(&t.first, n + 1)) != BT_OK ||
        (st = s->dev(&t.dims, 2)) != BT_OK)
        return st;
    return BT_OK;
}

bt_status alloc_session(bt_server *s, Session &q)
{
    bt_ctx *ctx = s->ctx;
    bt_status st;
    q.b = new bt_beams();
    q.b->ctx = ctx;
    if ((st = dev_alloc(ctx, (void **)&q.b->ctr, sizeof(DevCounters))) != BT_OK) return st;
    if ((st = alloc_wave_scratch(ctx, q.b, s->opts.blocks_per_cu)) != BT_OK) return st;
    if ((st = reserve_queue(ctx, q.b, s->opts.max_records, 0)) != BT_OK) return st;
    if ((st = reserve_work(ctx, q.b, std::max<long long>(s->opts.max_records / 4, 1))) != BT_OK) return st;
    // a generation holds at most every record of the session
    if ((st = reserve_tiles(ctx, q.b, s->opts.max_records)) != BT_OK) return st;
    if ((st = s->dev(&q.slots, kSessionSlots)) != BT_OK || (st = s->host(&q.h_slots, kSessionSlots)) != BT_OK) return st;
    if ((st = alloc_table(s, q.dev, false)) != BT_OK || (st = alloc_table(s, q.host[0], true)) != BT_OK ||
        (st = alloc_table(s, q.host[1], true)) != BT_OK)
        return st;
    if ((st = s->dev(&q.arena, s->opts.arena_bytes)) != BT_OK || (st = s->host(&q.h_arena, s->opts.arena_bytes)) != BT_OK)
        return st;
    return BT_OK;
}

// Empty the session for new requests: counters zeroed on the stream, arenas rewound.
bt_status reset_session(bt_server *s, Session &q)
{
    if (q.dirty) HIP_TRY(s->ctx, launch_init_counters(q.b->ctr, 0, 0, s->ctx->stream));
    q.dirty = false;
    q.arena_used = q.h_used = 0;
    q.records = 0;
    q.n_slots = 0;
    q.gen = 0;
    q.acc_gen = 0;
    return BT_OK;
}

bool fits(const bt_server *s, const Session &q, const Req *r, int step_sources)
{
    return q.n_slots < kSessionSlots && q.records + r->z.records <= s->opts.max_records &&
           q.gen + r->sc.max_depth <= kLastGen && q.arena_used + dev_need(r->z) <= s->opts.arena_bytes &&
           q.h_used + host_need(r->z) <= s->opts.arena_bytes && step_sources + r->sc.n_src <= kStepSources;
}

// Admit r into q: slot, arena blocks, and its slot entry, bitmap, gather indices and
// descriptor staged in pinned memory (uploaded in the step that emits it).
void admit(bt_server *s, Session &q, int qi, Req *r)
{
    const ScenarioSize &z = r->z;
    char *d = q.arena + q.arena_used;
    r->energy = (double *)d;
    d += align256(16 * z.grid);
    r->mask = z.mask_words ? (unsigned *)d : nullptr;
    d += align256(4 * z.mask_words);
    r->gidx = (long long *)d;
    d += align256(8 * z.n_out);
    r->out = (double *)d;
    d += align256(16 * z.n_out);
    r->desc = (BatchDesc *)d;
    q.arena_used += dev_need(z);
    char *h = q.h_arena + q.h_used;
    r->h_out = (double *)h;
    h += align256(16 * z.n_out);
    r->h_mask = (unsigned *)h;
    h += align256(4 * z.mask_words);
    r->h_gidx = (long long *)h;
    h += align256(8 * z.n_out);
    r->h_desc = (BatchDesc *)h;
    q.h_used += host_need(z);
    if (z.mask_words) {
        std::memset(r->h_mask, 0, (size_t)z.mask_words * sizeof(unsigned));
        for (long long i = 0; i < z.n_out; ++i) {
            const long long g = r->subset[(size_t)i];
            r->h_mask[g >> 5] |= 1u << (g & 31);
            r->h_gidx[i] = g;
        }
    } else {
        for (long long g = 0; g < z.n_out; ++g) r->h_gidx[g] = g;
    }
    *r->h_desc = BatchDesc{2 * z.grid, z.n_out, z.grid};
    DevMics m{};
    m.x0 = r->sc.mic_x0;
    m.y0 = r->sc.mic_y0;
    m.z = r->sc.mic_z;
    m.dx = r->sc.mic_dx;
    m.dy = r->sc.mic_dy;
    m.nx = r->sc.mic_nx;
    m.ny = r->sc.mic_ny;
    m.nz = 1;
    m.e_strict = r->energy;
    m.e_flag = r->energy + z.grid;
    m.mask = r->mask;
    r->slot = q.n_slots++;
    q.h_slots[r->slot] = m;
    r->admit_gen = q.gen;
    r->session = qi;
    r->t_admit = s->now();
    q.records += z.records;
    q.unfinished++;
    q.fresh.push_back(r);
}

// One step of session q: emission of its fresh requests, the trace of its next
// generation, that generation's microphone pass, and the outputs of the requests it
// finishes.  `parity` selects the pinned staging not in use by the step in flight.
bt_status step_session(bt_server *s, Session &q, int parity, std::vector<Req *> &done_now)
{
    bt_ctx *ctx = s->ctx;
    hipStream_t st = ctx->stream;
    bt_beams *b = q.b;
    if (!q.fresh.empty()) {
        Table &h = q.host[parity];
        long long ns = 0, beam = 0;
        for (Req *r : q.fresh) {
            const long long nf = 20ll << (2 * r->sc.level);
            for (int i = 0; i < r->sc.n_src; ++i, ++ns) {
                std::memcpy(h.src + 3 * ns, r->src.data() + 3 * i, 3 * sizeof(float));
                h.pw[ns] = r->pw[(size_t)i];
                h.level[ns] = r->sc.level;
                h.meta[ns] = scenario_meta(r->slot, r->sc.max_depth);
                h.id0[ns] = (int)(i * nf);
                h.first[ns] = beam;
                beam += nf;
            }
            const ScenarioSize &z = r->z;
            HIP_TRY(ctx, hipMemcpyAsync(q.slots + r->slot, q.h_slots + r->slot, sizeof(DevMics), hipMemcpyHostToDevice, st));
            if (z.mask_words)
                HIP_TRY(ctx, hipMemcpyAsync(r->mask, r->h_mask, (size_t)z.mask_words * sizeof(unsigned),
                                            hipMemcpyHostToDevice, st));
            HIP_TRY(ctx, hipMemcpyAsync(r->gidx, r->h_gidx, (size_t)z.n_out * sizeof(long long), hipMemcpyHostToDevice, st));
            HIP_TRY(ctx, hipMemcpyAsync(r->desc, r->h_desc, sizeof(BatchDesc), hipMemcpyHostToDevice, st));
            HIP_TRY(ctx, launch_fill(r->energy, 2 * z.grid, 0.0, st));
        }
        h.first[ns] = beam;
        h.dims[0] = beam;
        h.dims[1] = ns;
        const size_t n1 = (size_t)std::max(ns, 1ll);
        HIP_TRY(ctx, hipMemcpyAsync(q.dev.src, h.src, 3 * n1 * sizeof(float), hipMemcpyHostToDevice, st));
        HIP_TRY(ctx, hipMemcpyAsync(q.dev.pw, h.pw, n1 * sizeof(float), hipMemcpyHostToDevice, st));
        HIP_TRY(ctx, hipMemcpyAsync(q.dev.level, h.level, n1 * sizeof(int), hipMemcpyHostToDevice, st));
        HIP_TRY(ctx, hipMemcpyAsync(q.dev.meta, h.meta, n1 * sizeof(int), hipMemcpyHostToDevice, st));
        HIP_TRY(ctx, hipMemcpyAsync(q.dev.id0, h.id0, n1 * sizeof(int), hipMemcpyHostToDevice, st));
        HIP_TRY(ctx, hipMemcpyAsync(q.dev.first, h.first, (n1 + 1) * sizeof(long long), hipMemcpyHostToDevice, st));
        HIP_TRY(ctx, hipMemcpyAsync(q.dev.dims, h.dims, 2 * sizeof(long long), hipMemcpyHostToDevice, st));
        const EmitTable t{q.dev.src, q.dev.pw, q.dev.level, q.dev.meta, q.dev.id0, q.dev.first, q.dev.dims};
        HIP_TRY(ctx, launch_emit_table(ctx->base20, t, beam, b->q, b->ctr, q.gen, st));
        q.live.insert(q.live.end(), q.fresh.begin(), q.fresh.end());
        q.fresh.clear();
    }
    TraceArgs a = make_args(&s->params, q.gen);
    a.max_depth = kLastGen;
    a.scenarios = 1;
    a.slot_mics = q.slots;
    HIP_TRY(ctx, launch_trace(s->mesh->dev, b->q, b->segs, b->ctr, a, b->ws, trace_tiles(b, s->mesh, a), ctx->n_cu,
                              st));
    q.dirty = true;
    // the microphone pass runs only in steps that finish a request, over every generation
    // traced since the previous pass (all stay resident in the session)
    bool finishing = false;
    for (Req *r : q.live) finishing = finishing || r->admit_gen + r->sc.max_depth == q.gen;
    if (finishing) {
        a.gen = q.acc_gen;
        a.gen_end = q.gen + 1;
        MicWork mw{b->rows, b->rows_cap, b->spans, b->spans_cap, b->big_list + b->cap, b->big_list};
        HIP_TRY(ctx, launch_mics(s->mesh->dev, b->q, b->segs, b->ctr, DevMics{}, a, mw, b->ws, ctx->n_cu, st));
        q.acc_gen = q.gen + 1;
    }
    std::vector<Req *> keep;
    for (Req *r : q.live) {
        if (r->admit_gen + r->sc.max_depth == q.gen) {
            const long long n = r->z.n_out;
            HIP_TRY(ctx, launch_gather(r->energy, r->gidx, r->desc, n, r->out, r->out + n, st));
            HIP_TRY(ctx, hipMemcpyAsync(r->h_out, r->out, (size_t)(2 * n) * sizeof(double), hipMemcpyDeviceToHost, st));
            done_now.push_back(r);
        } else {
            keep.push_back(r);
        }
    }
    q.live.swap(keep);
    q.gen++;
    return BT_OK;
}

// Outputs of requests whose last step has completed: copied to the caller's buffers.
void finalize(bt_server *s, std::vector<Req *> &list)
{
    if (list.empty()) return;
    std::lock_guard<std::mutex> lk(s->mu);
    for (Req *r : list) {
        const long long n = r->z.n_out;
        std::memcpy(r->sc.energy_out, r->h_out, (size_t)n * sizeof(double));
        if (r->sc.flag_out) std::memcpy(r->sc.flag_out, r->h_out + n, (size_t)n * sizeof(double));
        r->t_done = s->now();
        r->done = true;
        s->sess[r->session].unfinished--;
    }
    list.clear();
}

void set_failed(bt_server *s, bt_status st)
{
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed == BT_OK) s->failed = st;
    s->stop = true;
}

void run_batched(bt_server *s)
{
    int k = 0;          // step number
    bool inflight[2] = {false, false};
    int open = -1;
    while (true) {
        // admissions, in arrival order, at this step boundary
        int step_sources[2] = {0, 0};
        {
            std::unique_lock<std::mutex> lk(s->mu);
            const bool busy = !s->sess[0].live.empty() || !s->sess[1].live.empty() || inflight[0] || inflight[1];
            if (!busy) {
                if (s->stop && s->pending.empty()) break;
                s->cv.wait(lk, [&] { return s->stop || !s->pending.empty(); });
                if (s->stop && s->pending.empty()) break;
            }
            while (!s->pending.empty()) {
                Req *r = s->pending.front();
                if (open >= 0 && s->sess[open].unfinished == 0 && s->sess[open].gen > 0 &&
                    reset_session(s, s->sess[open]) != BT_OK) {
                    lk.unlock();
                    set_failed(s, BT_EDEVICE);
                    return;
                }
                if (open >= 0 && fits(s, s->sess[open], r, step_sources[open])) {
                    admit(s, s->sess[open], open, r);
                    step_sources[open] += r->sc.n_src;
                    s->pending.pop_front();
                    continue;
                }
                // the open session cannot take it: close it, open an empty one if any
                if (open >= 0 && s->sess[open].unfinished > 0) s->sess[open].open = false;
                int other = -1;
                for (int i = 0; i < 2; ++i)
                    if (i != open && s->sess[i].unfinished == 0) other = i;
                if (open >= 0 && s->sess[open].unfinished == 0) other = open;
                if (other < 0) {
                    open = -1;
                    break;  // both sessions drain: wait for one to empty
                }
                if (reset_session(s, s->sess[other]) != BT_OK) {
                    lk.unlock();
                    set_failed(s, BT_EDEVICE);
                    return;
                }
                s->sess[other].open = true;
                if (open >= 0 && open != other) s->sess[open].open = false;
                open = other;
                if (!fits(s, s->sess[open], r, step_sources[open])) {
                    // an empty session takes every request bt_server_submit accepts
                    lk.unlock();
                    set_failed(s, BT_EOVERFLOW);
                    return;
                }
            }
        }
        // one step of every session with requests in flight
        const int parity = k & 1;
        std::vector<Req *> &done_now = s->finishing[parity];
        bool any = false;
        for (int i = 0; i < 2; ++i) {
            Session &q = s->sess[i];
            if (q.live.empty() && q.fresh.empty()) continue;
            any = true;
            const bt_status st = step_session(s, q, parity, done_now);
            if (st != BT_OK) {
                set_failed(s, st);
                return;
            }
        }
        if (any) {
            if (hipEventRecord(s->ev[parity], s->ctx->stream) != hipSuccess) {
                set_failed(s, BT_EDEVICE);
                return;
            }
            inflight[parity] = true;
        }
        // wait for the previous step while this one runs, then finish its requests
        const int prev = parity ^ 1;
        if (inflight[prev]) {
            if (hipEventSynchronize(s->ev[prev]) != hipSuccess) {
                set_failed(s, BT_EDEVICE);
                return;
            }
            inflight[prev] = false;
            finalize(s, s->finishing[prev]);
        }
        if (!any && inflight[parity]) {
            // nothing new was enqueued: drain the step in flight
            if (hipEventSynchronize(s->ev[parity]) != hipSuccess) {
                set_failed(s, BT_EDEVICE);
                return;
            }
            inflight[parity] = false;
            finalize(s, s->finishing[parity]);
        }
        if (any) ++k;
    }
}

void run_plain(bt_server *s)
{
    std::vector<double> es, ef;
    while (true) {
        Req *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->pending.empty(); });
            if (s->pending.empty()) break;
            r = s->pending.front();
            s->pending.pop_front();
            r->t_admit = s->now();
        }
        bt_ctx *ctx = s->ctx;
        const bt_scenario &q = r->sc;
        bt_status st = mics_fit(ctx, &s->pm, q.mic_x0, q.mic_y0, q.mic_z, q.mic_dx, q.mic_dy, q.mic_nx, q.mic_ny);
        bt_params p = s->params;
        p.max_depth = q.max_depth;
        if (st == BT_OK)
            st = bt_run(ctx, s->mesh, r->src.data(), r->pw.data(), q.n_src, q.level, &p, s->pm, &s->pb);
        es.resize((size_t)r->z.grid);
        ef.resize((size_t)r->z.grid);
        if (st == BT_OK) st = bt_levels(ctx, s->pm, es.data(), ef.data(), nullptr);
        if (st != BT_OK) {
            set_failed(s, st);
            return;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        for (long long k = 0; k < r->z.n_out; ++k) {
            const size_t g = r->subset.empty() ? (size_t)k : (size_t)r->subset[(size_t)k];
            q.energy_out[k] = es[g] + ef[g];
            if (q.flag_out) q.flag_out[k] = ef[g];
        }
        r->t_done = s->now();
        r->done = true;
    }
}

void serve(bt_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    if (s->opts.mode == BT_SERVE_PLAIN) run_plain(s);
    else run_batched(s);
}

}  // namespace

extern "C" bt_status bt_server_create(bt_ctx *ctx, const bt_mesh *mesh, const bt_params *params,
                                      const bt_server_opts *opts, bt_server **out)
{
    if (!ctx) return BT_EINVAL;
    if (!mesh || !out) return fail(ctx, BT_EINVAL, "NULL mesh or out");
    *out = nullptr;
    bt_params p;
    if (params) p = *params;
    else bt_params_default(&p);
    p.max_depth = 0;
    p.hit_out = nullptr;
    p.flag_out = nullptr;
    p.t_out = nullptr;
    bt_status st = check_params(ctx, mesh, &p);
    if (st != BT_OK) return st;
    bt_server_opts o{BT_SERVE_BATCHED, kDefaultRecords, kDefaultArena, kBlocksPerCU};
    if (opts) {
        if (opts->mode != BT_SERVE_BATCHED && opts->mode != BT_SERVE_PLAIN) return fail(ctx, BT_EINVAL, "bad mode");
        if (opts->max_records < 0 || opts->max_records > (1ll << 31) - 1 || opts->arena_bytes < 0 ||
            opts->blocks_per_cu < 0 || opts->blocks_per_cu > 16)
            return fail(ctx, BT_EINVAL, "bad server options");
        o.mode = opts->mode;
        if (opts->max_records > 0) o.max_records = opts->max_records;
        if (opts->arena_bytes > 0) o.arena_bytes = opts->arena_bytes;
        if (opts->blocks_per_cu > 0) o.blocks_per_cu = opts->blocks_per_cu;
    }
    (void)hipSetDevice(ctx->device);
    bt_server *s = new bt_server();
    s->ctx = ctx;
    s->mesh = mesh;
    s->params = p;
    s->opts = o;
    s->t0 = Clock::now();
    if (o.mode == BT_SERVE_BATCHED) {
        for (int i = 0; i < 2 && st == BT_OK; ++i) st = alloc_session(s, s->sess[i]);
        for (int i = 0; i < 2 && st == BT_OK; ++i)
            if (hipEventCreateWithFlags(&s->ev[i], hipEventDisableTiming) != hipSuccess) st = BT_EDEVICE;
        if (st == BT_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = BT_EDEVICE;
        if (st != BT_OK) {
            s->stop = true;
            bt_server_destroy(s);
            return st;
        }
    }
    s->th = std::thread(serve, s);
    *out = s;
    return BT_OK;
}

extern "C" bt_status bt_server_submit(bt_server *s, const bt_scenario *req, uint64_t *ticket)
{
    if (!s || !req || !ticket) return BT_EINVAL;
    Req *r = new Req();
    r->sc = *req;
    bt_status st = validate_scenario(s->ctx, s->mesh, r->sc, 0, r->z);
    if (st != BT_OK) {
        delete r;
        return st;
    }
    if (s->opts.mode == BT_SERVE_BATCHED &&
        (r->z.records > s->opts.max_records || dev_need(r->z) > s->opts.arena_bytes ||
         host_need(r->z) > s->opts.arena_bytes || r->sc.n_src > kStepSources)) {
        delete r;
        return fail(s->ctx, BT_ENOMEM, "request larger than a server session");
    }
    r->src.assign(req->src_xyz, req->src_xyz + 3 * (size_t)req->n_src);
    r->pw.assign(req->src_power, req->src_power + (size_t)req->n_src);
    if (req->mic_subset) r->subset.assign(req->mic_subset, req->mic_subset + (size_t)req->n_subset);
    r->sc.src_xyz = r->src.data();
    r->sc.src_power = r->pw.data();
    r->sc.mic_subset = r->subset.empty() ? nullptr : r->subset.data();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->failed != BT_OK) {
            delete r;
            return s->failed;
        }
        r->ticket = s->next_ticket++;
        r->t_submit = s->now();
        s->reqs[r->ticket] = r;
        s->pending.push_back(r);
        *ticket = r->ticket;
    }
    s->cv.notify_one();
    return BT_OK;
}

extern "C" bt_status bt_server_poll(bt_server *s, uint64_t ticket, bt_serve_result *out)
{
    if (!s) return BT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return BT_ENOTFOUND;
    Req *r = it->second;
    if (!r->done) return s->failed != BT_OK ? s->failed : BT_PENDING;
    if (out) *out = bt_serve_result{r->t_submit, r->t_admit, r->t_done};
    s->reqs.erase(it);
    delete r;
    return BT_OK;
}

extern "C" bt_status bt_server_destroy(bt_server *s)
{
    if (!s) return BT_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    bt_ctx *ctx = s->ctx;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &kv : s->reqs) delete kv.second;
    for (int i = 0; i < 2; ++i) {
        if (s->sess[i].b) bt_beams_free(s->sess[i].b);
        if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
    }
    if (s->pb) bt_beams_free(s->pb);
    if (s->pm) bt_mics_free(s->pm);
    for (auto &d : s->dev_bufs) dev_free(ctx, d.first, d.second);
    for (void *h : s->host_bufs) (void)hipHostFree(h);
    const bt_status f = s->failed;
    delete s;
    return f == BT_OK ? BT_OK : f;
}
