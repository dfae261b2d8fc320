// Microphone accumulation: frustum footprints on the microphone plane, exact membership
// and FP64 accumulation.  Built with -ffp-contract=off: the tie rule on shared beam faces
// relies on exactly antisymmetric cross products.
#include <mutex>

#include "bt_device.h"

namespace bt {

// ---------------------------------------------------------------------------------------
// Microphones
//
// A segment's frustum meets the microphone plane z = zm in a convex polygon: three side
// half-planes through the (image) apex, the reflecting plane (outgoing side, strict) and
// the hit plane (incoming side, closed).  The kernels first bound the polygon's rows,
// then enumerate candidate microphones row by row (one column of slack on each side)
// and decide membership with the exact plane tests.
//   k_mics_plane:   one lane per segment (a set of its own): most segments are dismissed
//                   from their edge rays' crossings of the plane (or from the decision
//                   stored when the beam was created); boxed segments wait in an LDS ring
//                   until a round of them stages their frustums and their candidates
//                   are spread over the lanes; the rest go to the wave's region of the
//                   general list
//   k_mics:         the same fast path for multi-scenario sets, candidates in place
//   k_mics_general: one lane per listed segment (regions pooled over 64 waves): the
//                   clipped footprint's rows; up to kInlineRows rows are finished in
//                   place, wider footprints become (segment, row) work items in the
//                   wave's region of the row buffer
//   k_mic_rows:     one lane per (segment, row) work item (regions pooled over 64
//                   waves); rows longer than kSpan columns become (segment, row,
//                   columns) span items for k_mic_spans
//   k_mics_big:     one wave per segment, for segments whose rows did not fit the
//                   wave's region (overflow fallback)
// No kernel makes its waves meet on one shared counter: work lists live in per-wave
// regions, and statistics are spread over slots.
// A volumetric grid (Section 4's experiment fills the model's bounding box with
// microphones) is a stack of such planes: k_mics3d bounds the layers a segment's frustum
// can reach and runs the same footprint logic on each of them.  Explicit points
// (k_mics_points) are found through a bucket index in xy.
// ---------------------------------------------------------------------------------------
struct Frustum {
    V3 A;
    V3 n[3];
    double amb2[3];     // delta^2 |n_k|^2: |s| < delta |n| <=> s^2 < amb2
    bool has_near, has_far;
    V3 Nn, Pn;
    double near_sign, amb2_near;
    V3 Nf, Pf;
    double far_sign, amb2_far;
    float K;
    int flag;
};

struct HalfPlane {
    double a, b, k;  // a x + b y + k >= 0 on the microphone plane
};

__device__ __forceinline__ bool lex_positive(V3 n)
{
    if (n.x != 0.0) return n.x > 0.0;
    if (n.y != 0.0) return n.y > 0.0;
    return n.z > 0.0;
}

// Keep-side half-plane g . (p - P) >= 0 on z = zm, relaxed by eps * |g|_1 (>= eps |g|).
__device__ __forceinline__ HalfPlane make_hp(V3 g, V3 P, double z, double eps)
{
    HalfPlane h;
    h.a = g.x;
    h.b = g.y;
    h.k = g.z * (z - P.z) - g.x * P.x - g.y * P.y + eps * (fabs(g.x) + fabs(g.y) + fabs(g.z));
    return h;
}

__device__ void load_frustum(const DevMesh &M, const DevQueue &q, const DevSegs &segs, long long i, double delta,
                             Frustum &f)
{
    const long long cap = q.cap;
    const double d2 = delta * delta;
    f.A = ld3(q.dbl + D_A * cap, cap, i);
    V3 d[3] = {ld3(q.dbl + D_D0 * cap, cap, i), ld3(q.dbl + D_D1 * cap, cap, i), ld3(q.dbl + D_D2 * cap, cap, i)};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        f.n[k] = cross(d[k], d[(k + 1) % 3]);
        f.amb2[k] = d2 * dot(f.n[k], f.n[k]);
    }
    int meta = q.ints[I_META * cap + i];
    int start = q.ints[I_START * cap + i];
    int hit = segs.hit[i];
    f.K = q.flt[F_K * cap + i];
    f.flag = segs.flag[i];
    f.has_near = (meta & 0xff) > 0;
    if (f.has_near) {
        V3 v0, v1, v2;
        tri_vertices(M.tri_g, start, v0, v1, v2);
        f.Nn = cross(v1 - v0, v2 - v0);
        f.Pn = v0;
        f.near_sign = (meta & kMetaNegNear) ? -1.0 : 1.0;
        f.amb2_near = d2 * dot(f.Nn, f.Nn);
    }
    f.has_far = hit >= 0;
    if (f.has_far) {
        V3 v0, v1, v2;
        tri_vertices(M.tri_g, hit, v0, v1, v2);
        f.Nf = cross(v1 - v0, v2 - v0);
        f.Pf = v0;
        V3 c = ld3(q.dbl + D_C * cap, cap, i);
        f.far_sign = dot(c, f.Nf) > 0.0 ? 1.0 : -1.0;
        f.amb2_far = d2 * dot(f.Nf, f.Nf);
    }
}

// The frustum's half-planes on the microphone plane at height z, plus the grid rectangle
// (grown by half a cell) as 9 lines; unused slots are the always-true constraint
// 0 x + 0 y + 1 >= 0.
__device__ __forceinline__ void footprint_lines(const Frustum &f, const DevMics &mc, double z, HalfPlane *L)
{
    const double eps = 1e-6;
#pragma unroll
    for (int k = 0; k < 3; ++k) L[k] = make_hp(f.n[k], f.A, z, eps);
    L[3] = f.has_near ? make_hp(f.near_sign * f.Nn, f.Pn, z, eps) : HalfPlane{0.0, 0.0, 1.0};
    L[4] = f.has_far ? make_hp((-f.far_sign) * f.Nf, f.Pf, z, eps) : HalfPlane{0.0, 0.0, 1.0};
    double xlo = mc.x0 - 0.5 * mc.dx, xhi = mc.x0 + ((double)mc.nx - 0.5) * mc.dx;
    double ylo = mc.y0 - 0.5 * mc.dy, yhi = mc.y0 + ((double)mc.ny - 0.5) * mc.dy;
    L[5] = HalfPlane{1.0, 0.0, -xlo};
    L[6] = HalfPlane{-1.0, 0.0, xhi};
    L[7] = HalfPlane{0.0, 1.0, -ylo};
    L[8] = HalfPlane{0.0, -1.0, yhi};
}

// Row range of the footprint polygon: every constraint line is clipped by all the
// others (parametrically, comparing fractions without dividing); the endpoints of the
// surviving edges bound the polygon's y-extent.  One row of slack on each side.
__device__ bool footprint_rows(const HalfPlane *L, const DevMics &mc, int &j0, int &j1)
{
    double ymn = INFINITY, ymx = -INFINITY;
#pragma unroll
    for (int h = 0; h < 9; ++h) {
        const double a = L[h].a, b = L[h].b, k = L[h].k;
        const double nn = a * a + b * b;
        if (nn == 0.0) continue;
        const double px = -k * a / nn, py = -k * b / nn;  // point on the line
        const double dx = -b, dy = a;                     // direction along it
        // t >= lo_n / lo_d and t <= hi_n / hi_d with positive denominators
        double lo_n = -1.0, lo_d = 0.0, hi_n = 1.0, hi_d = 0.0;  // -inf, +inf
        bool empty = false;
#pragma unroll
        for (int g = 0; g < 9; ++g) {
            if (g == h) continue;
            const double den = L[g].a * dx + L[g].b * dy;
            const double num = -(L[g].a * px + L[g].b * py + L[g].k);  // need den * t >= num
            if (den > 0.0) {
                if (lo_d == 0.0 || num * lo_d > lo_n * den) { lo_n = num; lo_d = den; }
            } else if (den < 0.0) {
                if (hi_d == 0.0 || (-num) * hi_d < hi_n * (-den)) { hi_n = -num; hi_d = -den; }
            } else if (num > 0.0) {
                empty = true;
            }
        }
        if (empty || lo_d == 0.0 || hi_d == 0.0) continue;  // (bounded by the rectangle otherwise)
        const double tlo = lo_n / lo_d, thi = hi_n / hi_d;
        if (!(tlo <= thi)) continue;
        const double y0 = py + tlo * dy, y1 = py + thi * dy;
        ymn = fmin(ymn, fmin(y0, y1));
        ymx = fmax(ymx, fmax(y0, y1));
    }
    if (!(ymn <= ymx)) return false;
    double fj0 = ceil((ymn - mc.y0) / mc.dy) - 1.0, fj1 = floor((ymx - mc.y0) / mc.dy) + 1.0;
    fj0 = fmax(fj0, 0.0);
    fj1 = fmin(fj1, (double)(mc.ny - 1));
    if (!(fj0 <= fj1)) return false;
    j0 = (int)fj0;
    j1 = (int)fj1;
    return true;
}

// Column range of row j inside the relaxed frustum half-planes (one column of slack).
__device__ __forceinline__ bool row_cols(const HalfPlane *L, const DevMics &mc, int j, int &i0, int &i1)
{
    const double y = mc.y0 + (double)j * mc.dy;
    double lo = -INFINITY, hi = INFINITY;
#pragma unroll
    for (int h = 0; h < 5; ++h) {
        const double rest = L[h].b * y + L[h].k;
        if (L[h].a > 0.0) lo = fmax(lo, -rest / L[h].a);
        else if (L[h].a < 0.0) hi = fmin(hi, -rest / L[h].a);
        else if (rest < 0.0) return false;
    }
    if (!(lo <= hi)) return false;
    const double flo = (lo - mc.x0) / mc.dx, fhi = (hi - mc.x0) / mc.dx;
    if (flo > (double)mc.nx || fhi < -1.0) return false;
    const double a0 = fmax(ceil(flo) - 1.0, 0.0), a1 = fmin(floor(fhi) + 1.0, (double)(mc.nx - 1));
    if (!(a0 <= a1)) return false;
    i0 = (int)a0;
    i1 = (int)a1;
    return true;
}

// Membership of grid microphone (i, j) of layer k and its contribution; returns 1 if
// accumulated.  Ambiguous: every active test passes within -delta and one is within delta
// of its plane.
template <bool kSlots>
__device__ __forceinline__ int mic_apply(const Frustum &f, const DevMics &mc, int i, int j, int k, double air_m)
{
    const V3 m = {mc.x0 + (double)i * mc.dx, mc.y0 + (double)j * mc.dy, mc.z + (double)k * mc.dz};
    const V3 r = m - f.A;
    bool inside = true, far_out = false, near_any = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double s = dot(f.n[k], r);
        inside = inside && (s > 0.0 || (s == 0.0 && lex_positive(f.n[k])));
        const double s2 = s * s;
        far_out = far_out || (s < 0.0 && s2 >= f.amb2[k]);
        near_any = near_any || s2 < f.amb2[k];
    }
    if (f.has_near) {
        const double s = f.near_sign * dot(f.Nn, m - f.Pn);
        inside = inside && s > 0.0;
        const double s2 = s * s;
        far_out = far_out || (s < 0.0 && s2 >= f.amb2_near);
        near_any = near_any || s2 < f.amb2_near;
    }
    if (f.has_far) {
        const double s = -f.far_sign * dot(f.Nf, m - f.Pf);
        inside = inside && s >= 0.0;
        const double s2 = s * s;
        far_out = far_out || (s < 0.0 && s2 >= f.amb2_far);
        near_any = near_any || s2 < f.amb2_far;
    }
    if (!inside) return 0;
    const long long idx = ((long long)k * mc.ny + j) * mc.nx + i;
    if (mc.mask && !((mc.mask[idx >> 5] >> (idx & 31)) & 1u)) return 0;  // subsets
    const double d2 = dot(r, r);
    float e = f.K / (float)d2;
    if (air_m > 0.0) e *= expf(-(float)(air_m * sqrt(d2)));
    const bool amb = !far_out && near_any;
    atomicAdd((f.flag || amb) ? &mc.e_flag[idx] : &mc.e_strict[idx], (double)e);
    return 1;
}

constexpr int kInlineRows = 4;
constexpr int kSpan = 32;   // longest column run one lane processes in place

// Columns [c0, c1] of row j of layer k: processed here when short, else split into
// kSpan-column span items (processed here anyway if the span buffer is full).
template <bool kSlots>
__device__ __forceinline__ void process_row(const Frustum &f, const DevMics &mc, const MicWork &w, DevCounters *ctr,
                                            int gen, long long seg, int j, int k, int c0, int c1, double air_m,
                                            unsigned &tests, unsigned &updates)
{
    const int ncol = c1 - c0 + 1;
    if (ncol > kSpan) {
        const int nsp = (ncol + kSpan - 1) / kSpan;
        const unsigned long long b = atomicAdd(&ctr->n_spans[gen], (unsigned long long)nsp);
        if (b + (unsigned long long)nsp <= (unsigned long long)w.spans_cap) {
            for (int s = 0; s < nsp; ++s) {
                const int a0 = c0 + s * kSpan;
                w.spans[b + s] = make_int4((int)seg, k * mc.ny + j, a0, min(a0 + kSpan - 1, c1));
            }
            return;
        }
        for (unsigned long long r = b; r < (unsigned long long)w.spans_cap; ++r) w.spans[r] = make_int4(-1, 0, 0, -1);
    }
    for (int c = c0; c <= c1; ++c) {
        tests++;
        updates += mic_apply<kSlots>(f, mc, c, j, k, air_m);
    }
}

// The microphone set a segment contributes to: the set's own, or in a multi-scenario set
// the one of the segment's slot.
template <bool kSlots>
__device__ __forceinline__ DevMics seg_mics(const DevMics &mc, const TraceArgs &a, const DevQueue &q, long long i)
{
    if (!kSlots) return mc;
    return a.slot_mics[meta_slot(q.ints[I_META * q.cap + i])];
}

__device__ __forceinline__ void add_mic_stat(DevCounters *ctr, int k, unsigned long long v)
{
    // this wave's slot (statistics only: no result depends on them)
    const unsigned slot = (unsigned)(((unsigned long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6) % kStatSlots;
    if (v) atomicAdd(&ctr->mic_stat[slot][k], v);
}
__device__ __forceinline__ void flush_mic_counters(DevCounters *ctr, unsigned tests, unsigned updates)
{
    unsigned long long st = wave_sum_u64(tests), su = wave_sum_u64(updates);
    if (lane_id() == 0) {
        add_mic_stat(ctr, MS_TESTS, st);
        add_mic_stat(ctr, MS_UPDATES, su);
    }
}

// Planar fast path of segment i (plane_decide on its stored frustum): 0 = no microphone
// can be inside, 1 = the lattice box [i0, i1] x [j0, j1], 2 = the clipped footprint.
static_assert(kPlaneBox == kSpan, "a lattice box is at most one span of candidates");
__device__ __forceinline__ int plane_fast(const DevQueue &q, long long i, const DevMics &mc, int &i0, int &i1,
                                          int &j0, int &j1)
{
    const long long cap = q.cap;
    return plane_decide(ld3(q.dbl + D_A * cap, cap, i), ld3(q.dbl + D_D0 * cap, cap, i),
                        ld3(q.dbl + D_D1 * cap, cap, i), ld3(q.dbl + D_D2 * cap, cap, i), mc.x0, mc.y0, mc.z, mc.dx,
                        mc.dy, mc.nx, mc.ny, i0, i1, j0, j1);
}

// Fast path over all segments of generations [gen, gen_end) (contiguous in the queue):
// footprints that are a proper triangle on the microphone plane with at most kSpan
// lattice points in their bounding box are finished here (most have none); the others
// are appended to the general list.  k_mics_plane serves a set of its own; k_mics serves
// multi-scenario sets, whose segments send their contributions to different sets.
// Wave w's region of the general list: room for 64 items per batch it processes.
__device__ __forceinline__ unsigned long long general_region(unsigned long long n, int n_waves)
{
    const unsigned long long batches = (n + 63) / 64;
    return ((batches + (unsigned long long)n_waves - 1) / (unsigned long long)n_waves) * 64;
}

template <bool kSlots>
__global__ void __launch_bounds__(256, 4) k_mics(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr, DevMics mc0,
                                              TraceArgs a, MicWork w, WaveScratch ws)
{
    const unsigned long long s0 = gen_start(ctr, a.gen);
    const unsigned long long n = gen_count(ctr, a.gen, a.gen_end);
    const int lane = lane_id();
    const unsigned long long wave = wave_first_batch() >> 6;
    const unsigned long long region = wave * general_region(n, ws.n_waves);
    unsigned gcount = 0;
    unsigned tests = 0, updates = 0;
    for (unsigned long long base = wave_first_batch(); base < n; base += wave_batch_stride()) {
        const long long i = (long long)(s0 + base) + lane;
        bool general = false;
        if ((long long)base + lane < (long long)n) {
            const DevMics mc = seg_mics<kSlots>(mc0, a, q, i);
            int i0 = 0, i1 = -1, j0 = 0, j1 = -1;
            const int kind = plane_fast(q, i, mc, i0, i1, j0, j1);
            general = kind == 2;
            if (kind == 1) {
                Frustum f;
                load_frustum(M, q, segs, i, a.delta, f);
                for (int j = j0; j <= j1; ++j)
                    for (int c = i0; c <= i1; ++c) {
                        tests++;
                        updates += mic_apply<kSlots>(f, mc, c, j, 0, a.air_m);
                    }
            }
        }
        // general-path segments go to this wave's own region of the list (no atomics)
        const unsigned long long gm = __ballot(general);
        if (general) w.general[region + gcount + __popcll(gm & ((1ull << lane) - 1ull))] = (int)i;
        gcount += (unsigned)__popcll(gm);
    }
    if (lane == 0) ws.general[wave] = gcount;
    flush_mic_counters(ctr, tests, updates);
}

constexpr int kPoolWaves = 64;  // waves whose general-list regions k_mics_general pools

// General path, one lane per listed segment: the footprint's row range from the clipped
// polygon; up to kInlineRows rows are finished here, wider footprints become (segment,
// row) work items.
template <bool kSlots>
__global__ void __launch_bounds__(256, 3) k_mics_general(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr,
                                                      DevMics mc0, TraceArgs a, MicWork w, WaveScratch ws)
{
    // The items the fast-path kernel's waves put in their regions (same wave numbering),
    // pooled over kPoolWaves consecutive waves: the pool's waves take its concatenated
    // list 64 items at a time, so that no wave is left with a short region or a mostly
    // empty last batch of its own.
    const unsigned long long n_seg = gen_count(ctr, a.gen, a.gen_end);
    const int lane = lane_id();
    const unsigned long long wave = wave_first_batch() >> 6;
    const unsigned long long rsize = general_region(n_seg, ws.n_waves);
    const unsigned long long g0 = wave / kPoolWaves * kPoolWaves;  // the pool's first wave
    const int gi = (int)(wave - g0);
    const int pw = (int)min((unsigned long long)kPoolWaves, (unsigned long long)ws.n_waves - g0);
    // lane l: items of the pool's waves before wave g0 + l (the total for l >= pw)
    const int cnt = lane < pw ? (int)ws.general[g0 + lane] : 0;
    int pre = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(pre, off, 64);
        if (lane >= off) pre += u;
    }
    const int total = __shfl(pre, 63, 64);
    pre -= cnt;
    unsigned tests = 0, updates = 0;
    // this wave's region of the row buffer
    const long long rcap = w.rows_cap / ws.n_waves;
    const long long wave_row0 = (long long)wave * rcap;
    long long rn = 0;
    for (int t0 = 64 * gi; t0 < total; t0 += 64 * pw) {
        const int t = t0 + lane;
        const bool active = t < total;
        // the pool wave whose region holds item t: the largest l with pre[l] <= t
        int r = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            const int p = __shfl(pre, r + step < 64 ? r + step : 63, 64);
            if (r + step < 64 && p <= t) r += step;
        }
        const int pr = __shfl(pre, r, 64);
        const long long i = active ? w.general[(g0 + (unsigned long long)r) * rsize + (unsigned long long)(t - pr)] : 0;
        int nrows = 0, j0 = 0, j1 = -1;
        bool wide = false;
        if (active) {
            const DevMics mc = seg_mics<kSlots>(mc0, a, q, i);
            Frustum f;
            load_frustum(M, q, segs, i, a.delta, f);
            HalfPlane L[9];
            footprint_lines(f, mc, mc.z, L);
            if (footprint_rows(L, mc, j0, j1)) {
                nrows = j1 - j0 + 1;
                if (nrows <= kInlineRows) {
                    for (int j = j0; j <= j1; ++j) {
                        int c0, c1;
                        if (!row_cols(L, mc, j, c0, c1)) continue;
                        process_row<kSlots>(f, mc, w, ctr, a.gen, i, j, 0, c0, c1, a.air_m, tests, updates);
                    }
                } else {
                    wide = true;
                }
            }
        }
        // wide footprints: one work item per row, in this wave's region of the row buffer
        // (no shared counter); the lanes whose rows no longer fit go to the wave path
        const int want = wide ? nrows : 0;
        long long incl = want;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const long long v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        const bool fits = rn + incl <= rcap;   // a prefix of the lanes
        bool to_big = false;
        if (wide) {
            if (fits) {
                const long long first = wave_row0 + rn + (incl - want);
                for (int r = 0; r < want; ++r) w.rows[first + r] = make_int2((int)i, j0 + r);
            } else {
                to_big = true;
            }
        }
        const unsigned long long fm = __ballot(fits);
        if (fm) rn += __shfl(incl, 63 - __builtin_clzll(fm), 64);   // the last lane that fits
        const unsigned long long bm = __ballot(to_big);
        unsigned long long bbase = 0;
        if (lane == 0 && bm) bbase = atomicAdd(&ctr->n_big[a.gen], (unsigned long long)__popcll(bm));
        bbase = __shfl(bbase, 0, 64);
        if (to_big) w.big_list[bbase + __popcll(bm & ((1ull << lane) - 1ull))] = (int)i;
    }
    if (lane == 0) ws.rows_n[wave] = (unsigned)rn;
    flush_mic_counters(ctr, tests, updates);
}

// One lane per (segment, row) item: the items the general kernel's waves put in their
// regions of the row buffer, pooled over kPoolWaves consecutive waves as in
// k_mics_general (this grid has the same waves).
template <bool kSlots>
__global__ void __launch_bounds__(256) k_mic_rows(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr, DevMics mc0,
                                                  TraceArgs a, MicWork w, WaveScratch ws)
{
    const int lane = lane_id();
    const unsigned long long wave = wave_first_batch() >> 6;
    const long long rcap = w.rows_cap / ws.n_waves;
    const unsigned long long g0 = wave / kPoolWaves * kPoolWaves;
    const int gi = (int)(wave - g0);
    const int pw = (int)min((unsigned long long)kPoolWaves, (unsigned long long)ws.n_waves - g0);
    const int cnt = lane < pw ? (int)ws.rows_n[g0 + lane] : 0;
    int pre = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(pre, off, 64);
        if (lane >= off) pre += u;
    }
    const int total = __shfl(pre, 63, 64);
    pre -= cnt;
    unsigned tests = 0, updates = 0;
    for (int t0 = 64 * gi; t0 < total; t0 += 64 * pw) {
        const int t = t0 + lane;
        int r = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            const int p = __shfl(pre, r + step < 64 ? r + step : 63, 64);
            if (r + step < 64 && p <= t) r += step;
        }
        const int pr = __shfl(pre, r, 64);
        if (t < total) {
            const int2 it = w.rows[(long long)(g0 + (unsigned long long)r) * rcap + (t - pr)];
            const DevMics mc = seg_mics<kSlots>(mc0, a, q, it.x);
            const int j = it.y;
            Frustum f;
            load_frustum(M, q, segs, it.x, a.delta, f);
            HalfPlane L[9];
            footprint_lines(f, mc, mc.z, L);
            int c0, c1;
            if (row_cols(L, mc, j, c0, c1))
                process_row<kSlots>(f, mc, w, ctr, a.gen, it.x, j, 0, c0, c1, a.air_m, tests, updates);
        }
    }
    flush_mic_counters(ctr, tests, updates);
}

template <bool kSlots>
__global__ void __launch_bounds__(256) k_mic_spans(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr,
                                                   DevMics mc0, TraceArgs a, MicWork w)
{
    unsigned long long n = ctr->n_spans[a.gen];
    if (n > (unsigned long long)w.spans_cap) n = (unsigned long long)w.spans_cap;
    unsigned tests = 0, updates = 0;
    for (unsigned long long base = wave_first_batch(); base < n; base += wave_batch_stride()) {
        const unsigned long long r = base + (unsigned long long)lane_id();
        const int4 sp = r < n ? w.spans[r] : make_int4(-1, 0, 0, -1);
        if (sp.x >= 0) {
            const DevMics mc = seg_mics<kSlots>(mc0, a, q, sp.x);
            const int k = mc.nz > 1 ? sp.y / mc.ny : 0;  // global row k ny + j
            const int j = sp.y - k * mc.ny;
            Frustum f;
            load_frustum(M, q, segs, sp.x, a.delta, f);
            for (int c = sp.z; c <= sp.w; ++c) {
                tests++;
                updates += mic_apply<kSlots>(f, mc, c, j, k, a.air_m);
            }
        }
    }
    flush_mic_counters(ctr, tests, updates);
}

template <bool kSlots>
__global__ void __launch_bounds__(256) k_mics_big(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr,
                                                  DevMics mc0, TraceArgs a, MicWork w)
{
    const unsigned long long n = ctr->n_big[a.gen];
    const int lane = lane_id();
    const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int n_waves = (int)((gridDim.x * blockDim.x) >> 6);
    unsigned tests = 0, updates = 0;
    for (unsigned long long s = (unsigned long long)wave; s < n; s += (unsigned long long)n_waves) {
        const long long i = w.big_list[s];
        const DevMics mc = seg_mics<kSlots>(mc0, a, q, i);
        Frustum f;
        load_frustum(M, q, segs, i, a.delta, f);
        HalfPlane L[9];
        footprint_lines(f, mc, mc.z, L);
        int j0, j1;
        if (footprint_rows(L, mc, j0, j1)) {
            for (int j = j0 + lane; j <= j1; j += 64) {
                int c0, c1;
                if (!row_cols(L, mc, j, c0, c1)) continue;
                process_row<kSlots>(f, mc, w, ctr, a.gen, i, j, 0, c0, c1, a.air_m, tests, updates);
            }
        }
    }
    flush_mic_counters(ctr, tests, updates);
}

// ---------------------------------------------------------------------------------------
// Volumetric grids
//   k_mics3d:         one wave per 64 segments: the layers each frustum can reach, then
//                     the (segment, layer) pairs spread evenly over the lanes for the
//                     planar fast path, then the candidate microphones of the pairs'
//                     lattice boxes spread evenly over the lanes again, each lane reading
//                     its frustum from the wave's LDS staging.  Pairs that need the
//                     clipped footprint become (segment, layer) items (done in place when
//                     the item buffer is full).
//   k_mics3d_general: kVolSeg (segment, layer) items per wave: rows of the clipped
//                     footprints spread over the lanes, then their candidates
// A segment spans from one to every layer and a layer box from none to kSpan candidates,
// so a lane per segment would leave most lanes idle; the two even spreads keep them busy.
// ---------------------------------------------------------------------------------------

// Layers [k0, k1] a segment's frustum can reach, from its z-extent widened for rounding.
// When the apex is on the incoming side of the hit plane and all three edge rays cross
// that plane ahead of the apex, the frustum (cone cut by the hit plane) lies in the
// tetrahedron of the apex and the three crossing points; otherwise the cone of the edge
// directions is the bound (unbounded above if an edge rises, below if one falls).
__device__ __forceinline__ bool seg_layers(const DevMesh &M, const DevQueue &q, long long i, int hit, V3 A,
                                           const V3 *d, const DevMics &mc, int &k0, int &k1)
{
    double zlo = A.z, zhi = A.z, mag = fabs(A.z);
    bool cut = hit >= 0;
    bool up = false, down = false;
    V3 Nf = {0.0, 0.0, 0.0};
    double c0 = 0.0;
    if (cut) {
        V3 v0, v1, v2;
        tri_vertices(M.tri_g, hit, v0, v1, v2);
        const V3 c = ld3(q.dbl + D_C * q.cap, q.cap, i);
        Nf = cross(v1 - v0, v2 - v0);
        if (!(dot(c, Nf) > 0.0)) Nf = -1.0 * Nf;  // oriented along the guiding ray
        c0 = dot(Nf, v0 - A);
        cut = c0 > 0.0;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        up = up || d[k].z > 0.0;
        down = down || d[k].z < 0.0;
        const double g = dot(Nf, d[k]);  // rate of approach to the hit plane
        cut = cut && g > 0.0;
        if (cut && d[k].z != 0.0) {
            const double z = A.z + (c0 / g) * d[k].z;
            zlo = fmin(zlo, z);
            zhi = fmax(zhi, z);
            mag = fmax(mag, fabs(z));
        }
    }
    if (!cut) {
        zlo = down ? -INFINITY : A.z;
        zhi = up ? INFINITY : A.z;
    }
    const double slack = 1e-6 + 1e-9 * mag;
    const double fk0 = fmax(ceil((zlo - slack - mc.z) / mc.dz), 0.0);
    const double fk1 = fmin(floor((zhi + slack - mc.z) / mc.dz), (double)(mc.nz - 1));
    if (!(fk0 <= fk1)) return false;
    k0 = (int)fk0;
    k1 = (int)fk1;
    return true;
}

// Rows of the clipped footprint of layer k, done here (k_mics3d's fallback when the
// (segment, layer) item buffer is full).
__device__ __forceinline__ void layer_general(const Frustum &f, const DevMics &mc, const MicWork &w, DevCounters *ctr,
                                              const TraceArgs &a, long long seg, int k, unsigned &tests,
                                              unsigned &updates)
{
    HalfPlane L[9];
    footprint_lines(f, mc, mc.z + (double)k * mc.dz, L);
    int j0, j1;
    if (!footprint_rows(L, mc, j0, j1)) return;
    for (int j = j0; j <= j1; ++j) {
        int c0, c1;
        if (!row_cols(L, mc, j, c0, c1)) continue;
        process_row<false>(f, mc, w, ctr, a.gen, seg, j, k, c0, c1, a.air_m, tests, updates);
    }
}

// LDS staging of one wave of k_mics3d (structure of arrays: lanes reading the same
// segment share an address, lanes reading different ones mostly different banks).  A
// batch is kVolSeg segments (slots): half a wave, so that a CU holds 16 waves' staging.
constexpr int kVolF = 24;  // frustum doubles: A, n0, n1, n2, near N and P, far N and P
constexpr int kVolSeg = 32;
struct VolStage {
    double f[kVolF][kVolSeg];   // caps with their keep sides folded into N: near
                                // N.(m - P) > 0, far N.(m - P) >= 0
    double az[kVolSeg];         // apex height
    float ax[kVolSeg], ay[kVolSeg];  // apex x, y (FP32: the fast path only bounds candidates)
    float sxlo[kVolSeg], sxhi[kVolSeg];    // least and greatest edge slope dx/dz
    float sylo[kVolSeg], syhi[kVolSeg];    // the same for dy/dz
    float smag[kVolSeg];                   // largest |slope|
    float K[kVolSeg];
    int bits[kVolSeg];          // 1 has near cap, 2 has far cap, 4 flagged; every edge dz > 0:
                                // 8, every dz < 0: 16, no dz > 0: 32, no dz < 0: 64
    int k0[kVolSeg];
    alignas(16) int prefix[kVolSeg + 4];   // exclusive scan of the batch's pair counts
    alignas(16) int psk1[4];    // its search skips: prefix[8 (q+1)] at q,
    alignas(16) int psk2[16];   //   prefix[8q + 2 (t+1)] at 4q + t
    alignas(16) int cprefix[68];  // exclusive scan of the pair chunk's candidate counts
    alignas(16) int csk1[4];    // its search skips: cprefix[16 (q+1)] at q,
    alignas(16) int csk2[16];   //   cprefix[16q + 4 (t+1)] at 4q + t
    int4 box[64];               // pair chunk: (slot | layer << 6, i0, j0, columns)
};

__device__ __forceinline__ int wave_excl_scan(int v, int &total)
{
    const int lane = lane_id();
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(incl, off, 64);
        if (lane >= off) incl += u;
    }
    total = __shfl(incl, 63, 64);
    return incl - v;
}

// Largest l in [0, 4^3 s - 1] (s = 1: 64 entries, s = 1/2: 32) with pre[l] <= x, pre
// nondecreasing with pre[0] = 0 <= x: a 4-ary search, three dependent LDS reads.
// sk1[q] = pre[(q + 1) W], sk2[4q + t] = pre[qW + (t + 1) W/4] for W = 16 (64 entries)
// or W = 8 (32 entries); the last level reads pre itself.
__device__ __forceinline__ int owner64(const int *pre, const int *sk1, const int *sk2, int x)
{
    const int4 a = *reinterpret_cast<const int4 *>(sk1);
    const int q = (a.x <= x) + (a.y <= x) + (a.z <= x);
    const int4 b = *reinterpret_cast<const int4 *>(sk2 + 4 * q);
    const int base = 16 * q + 4 * ((b.x <= x) + (b.y <= x) + (b.z <= x));
    const int4 c = *reinterpret_cast<const int4 *>(pre + base);
    return base + (c.y <= x) + (c.z <= x) + (c.w <= x);
}
__device__ __forceinline__ int owner32(const int *pre, const int *sk1, const int *sk2, int x)
{
    const int4 a = *reinterpret_cast<const int4 *>(sk1);
    const int q = (a.x <= x) + (a.y <= x) + (a.z <= x);
    const int4 b = *reinterpret_cast<const int4 *>(sk2 + 4 * q);
    const int base = 8 * q + 2 * ((b.x <= x) + (b.y <= x) + (b.z <= x));
    const int2 c = *reinterpret_cast<const int2 *>(pre + base);
    return base + (c.y <= x);
}

// Writes lane l's prefix value into the search skips of owner64 (W = 16) or owner32 (W = 8).
template <int W>
__device__ __forceinline__ void write_skips(int *sk1, int *sk2, int l, int v)
{
    if (l > 0 && l % W == 0 && l / W <= 3) sk1[l / W - 1] = v;
    const int r = l % W;
    if (r > 0 && r % (W / 4) == 0) sk2[4 * (l / W) + r / (W / 4) - 1] = v;
}

template <class Stage>
__device__ __forceinline__ void stage_frustum(Stage &st, int l, const Frustum &f)
{
    const double v[kVolF] = {f.A.x, f.A.y, f.A.z,
                             f.n[0].x, f.n[0].y, f.n[0].z, f.n[1].x, f.n[1].y, f.n[1].z, f.n[2].x, f.n[2].y, f.n[2].z,
                             f.near_sign * f.Nn.x, f.near_sign * f.Nn.y, f.near_sign * f.Nn.z, f.Pn.x, f.Pn.y, f.Pn.z,
                             -f.far_sign * f.Nf.x, -f.far_sign * f.Nf.y, -f.far_sign * f.Nf.z, f.Pf.x, f.Pf.y, f.Pf.z};
#pragma unroll
    for (int c = 0; c < kVolF; ++c) st.f[c][l] = v[c];
}

// The staged frustum of slot l, as mic_apply takes it (cap signs folded into the
// normals: near_sign = 1, far_sign = -1; the same products and sums as load_frustum's).
__device__ __forceinline__ void unstage_frustum(const VolStage &st, int l, double delta, Frustum &f)
{
    const double d2 = delta * delta;
    f.A = {st.f[0][l], st.f[1][l], st.f[2][l]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        f.n[k] = {st.f[3 + 3 * k][l], st.f[4 + 3 * k][l], st.f[5 + 3 * k][l]};
        f.amb2[k] = d2 * dot(f.n[k], f.n[k]);
    }
    const int bits = st.bits[l];
    f.has_near = (bits & 1) != 0;
    f.has_far = (bits & 2) != 0;
    f.flag = (bits & 4) ? 1 : 0;
    f.K = st.K[l];
    f.Nn = {st.f[12][l], st.f[13][l], st.f[14][l]};
    f.Pn = {st.f[15][l], st.f[16][l], st.f[17][l]};
    f.near_sign = 1.0;
    f.amb2_near = d2 * dot(f.Nn, f.Nn);
    f.Nf = {st.f[18][l], st.f[19][l], st.f[20][l]};
    f.Pf = {st.f[21][l], st.f[22][l], st.f[23][l]};
    f.far_sign = -1.0;
    f.amb2_far = d2 * dot(f.Nf, f.Nf);
}

// Largest lattice box of a layer taken as candidates directly; larger footprints take the
// clipped-footprint path, whose rows bound the candidates tightly.
constexpr int kBox3 = 64;

// The planar fast path on layer k for staged segment l: 0 = no microphone can be inside,
// 1 = the candidates are the lattice box [i0, i1] x [j0, j1] (at most kBox3 points),
// 2 = the clipped footprint is needed.
__device__ __forceinline__ int layer_fast(const VolStage &st, int l, const DevMics &mc, int k, int &i0, int &i1,
                                          int &j0, int &j1)
{
    const double zr = (mc.z + (double)k * mc.dz) - st.az[l];
    const int bits = st.bits[l];
    const bool away = (zr > 1e-6 && (bits & 32)) || (zr < -1e-6 && (bits & 64));
    if (away) return 0;
    // all three edge rays cross the layer ahead of the apex: the frustum meets it inside
    // the triangle of the crossing points (the caps only cut it down)
    const bool proper = zr > 0.0 ? (bits & 8) != 0 : (zr < 0.0 && (bits & 16));
    if (!proper) return 2;
    // crossings in FP32: each coordinate within 6 x 2^-24 of `mag` (the largest magnitude
    // involved) of its exact value; the box is widened by 1e-5 mag and the exact FP64
    // membership test decides every candidate.  Rounding is monotone, so the extreme
    // crossings come from the extreme slopes (the least for zr > 0 giving the least x).
    const float zrf = (float)zr, axf = st.ax[l], ayf = st.ay[l];
    const bool up = zrf > 0.0f;
    const float xmn = axf + zrf * (up ? st.sxlo[l] : st.sxhi[l]);
    const float xmx = axf + zrf * (up ? st.sxhi[l] : st.sxlo[l]);
    const float ymn = ayf + zrf * (up ? st.sylo[l] : st.syhi[l]);
    const float ymx = ayf + zrf * (up ? st.syhi[l] : st.sylo[l]);
    const float mag = fmaxf(fmaxf(fabsf(axf), fabsf(ayf)), fabsf(zrf) * st.smag[l]);
    // FP32 overflow: the clipped footprint decides
    if (!(isfinite(xmn) && isfinite(xmx) && isfinite(ymn) && isfinite(ymx))) return 2;
    // lattice range in FP32 too: the grid values are FP32, and the index arithmetic
    // (two subtractions and a product) is within 2e-7 of |index| + 1e-4 cells of exact,
    // far inside the added 1e-6 |index| + 1e-3 cells
    const float relax = 1e-6f + 1e-5f * mag;
    const float gx = ((xmn - relax) - mc.fx0) * mc.fidx;
    const float hx = ((xmx + relax) - mc.fx0) * mc.fidx;
    const float gy = ((ymn - relax) - mc.fy0) * mc.fidy;
    const float hy = ((ymx + relax) - mc.fy0) * mc.fidy;
    const float fi0 = fmaxf(ceilf(gx - (1e-3f + 1e-6f * fabsf(gx))), 0.0f);
    const float fi1 = fminf(floorf(hx + (1e-3f + 1e-6f * fabsf(hx))), mc.fnx1);
    const float fj0 = fmaxf(ceilf(gy - (1e-3f + 1e-6f * fabsf(gy))), 0.0f);
    const float fj1 = fminf(floorf(hy + (1e-3f + 1e-6f * fabsf(hy))), mc.fny1);
    if (!(fi0 <= fi1 && fj0 <= fj1)) return 0;
    if ((fi1 - fi0 + 1.0f) * (fj1 - fj0 + 1.0f) > (float)kBox3) return 2;
    i0 = (int)fi0; i1 = (int)fi1; j0 = (int)fj0; j1 = (int)fj1;
    return 1;
}

// mic_apply for staged slot l, reading the staged frustum lazily: the side planes first
// (most candidates fail one of them), then the caps; the ambiguity distances only for
// microphones inside.  Same products, sums and decisions as mic_apply (for a microphone
// inside, no plane test is negative, so only `near_any` decides ambiguity).
template <class Stage>
__device__ __forceinline__ int staged_contribute(const Stage &st, int l, V3 m, long long idx, double *e_strict,
                                                 double *e_flag, const unsigned *mask, double d2, double air_m)
{
    const V3 A = {st.f[0][l], st.f[1][l], st.f[2][l]};
    const V3 r = m - A;
    double sd[3];
    V3 n[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        n[e] = {st.f[3 + 3 * e][l], st.f[4 + 3 * e][l], st.f[5 + 3 * e][l]};
        const double s = dot(n[e], r);
        if (!(s > 0.0 || (s == 0.0 && lex_positive(n[e])))) return 0;
        sd[e] = s;
    }
    const int bits = st.bits[l];
    double sn = 0.0, sf = 0.0;
    V3 Nn = {0.0, 0.0, 0.0}, Nf = {0.0, 0.0, 0.0};
    if (bits & 1) {
        Nn = {st.f[12][l], st.f[13][l], st.f[14][l]};
        sn = dot(Nn, m - V3{st.f[15][l], st.f[16][l], st.f[17][l]});
        if (!(sn > 0.0)) return 0;
    }
    if (bits & 2) {
        Nf = {st.f[18][l], st.f[19][l], st.f[20][l]};
        sf = dot(Nf, m - V3{st.f[21][l], st.f[22][l], st.f[23][l]});
        if (!(sf >= 0.0)) return 0;
    }
    bool near_any = false;
#pragma unroll
    for (int e = 0; e < 3; ++e) near_any = near_any || sd[e] * sd[e] < d2 * dot(n[e], n[e]);
    if (bits & 1) near_any = near_any || sn * sn < d2 * dot(Nn, Nn);
    if (bits & 2) near_any = near_any || sf * sf < d2 * dot(Nf, Nf);
    if (mask && !((mask[idx >> 5] >> (idx & 31)) & 1u)) return 0;
    const double dd = dot(r, r);
    float e = st.K[l] / (float)dd;
    if (air_m > 0.0) e *= expf(-(float)(air_m * sqrt(dd)));
    atomicAdd(((bits & 4) || near_any) ? &e_flag[idx] : &e_strict[idx], (double)e);
    return 1;
}

template <class Stage>
__device__ __forceinline__ int mic_apply_staged(const Stage &st, int l, const DevMics &mc, int i, int j, int k,
                                                double d2, double air_m)
{
    const V3 m = {mc.x0 + (double)i * mc.dx, mc.y0 + (double)j * mc.dy, mc.z + (double)k * mc.dz};
    return staged_contribute(st, l, m, ((long long)k * mc.ny + j) * mc.nx + i, mc.e_strict, mc.e_flag, mc.mask, d2,
                             air_m);
}

// LDS staging of one wave of k_mics_plane: up to kVolSeg segments with candidate boxes,
// and a ring of boxed segments waiting for a staging round.
constexpr int kPendRing = 128;   // > kVolSeg - 1 + 64: what one batch can leave waiting
struct PlaneStage {
    double f[kVolF][kVolSeg];   // frustum, as VolStage
    float K[kVolSeg];
    int bits[kVolSeg];          // 1 near cap, 2 far cap, 4 flagged
    alignas(16) int prefix[kVolSeg + 4];  // exclusive scan of the staged boxes' sizes
    alignas(16) int psk1[4];              // its owner32 search skips
    alignas(16) int psk2[16];
    int4 box[kVolSeg];          // (first column, first row, columns, -)
    int pend_seg[kPendRing];    // waiting boxed segments (queue index) ...
    int4 pend_box[kPendRing];   // ... and their boxes (first column, first row, columns, candidates)
};

// One staging round of k_mics_plane: the first nst (<= kVolSeg) waiting segments of the
// ring, from position head, stage their frustums (lane l < nst takes entry head + l), and
// their candidates are spread evenly over the lanes.  Every lane of the wave calls it.
__device__ __forceinline__ void plane_round(PlaneStage &st, const DevMesh &M, const DevQueue &q, const DevSegs &segs,
                                            const DevMics &mc, const TraceArgs &a, int head, int nst, unsigned &tests,
                                            unsigned &updates)
{
    const int lane = lane_id();
    const bool mine = lane < nst;
    int nc = 0;
    if (mine) {
        const int e = (head + lane) & (kPendRing - 1);
        const long long i = st.pend_seg[e];
        const int4 bx = st.pend_box[e];
        Frustum f{};  // caps the segment lacks are staged as zeros
        load_frustum(M, q, segs, i, a.delta, f);
        stage_frustum(st, lane, f);
        st.bits[lane] = (f.has_near ? 1 : 0) | (f.has_far ? 2 : 0) | (f.flag ? 4 : 0);
        st.K[lane] = f.K;
        st.box[lane] = make_int4(bx.x, bx.y, bx.z, 0);
        nc = bx.w;
    }
    int total;
    const int pre = wave_excl_scan(nc, total);
    // slots past the staged ones hold the total, so that no candidate maps to them
    if (lane < kVolSeg) {
        const int v = mine ? pre : total;
        st.prefix[lane] = v;
        write_skips<8>(st.psk1, st.psk2, lane, v);
    }
    __syncthreads();
    for (int cb = 0; cb < total; cb += 64) {
        const int c = cb + lane;
        if (c < total) {
            const int sl = owner32(st.prefix, st.psk1, st.psk2, c);
            const int o = c - st.prefix[sl];
            const int4 bx = st.box[sl];
            const int row = o / bx.z;
            tests++;
            updates += mic_apply_staged(st, sl, mc, bx.x + (o - row * bx.z), bx.y + row, 0, a.delta2, a.air_m);
        }
    }
    __syncthreads();
}

// k_mics for a planar grid of one microphone set: the same dismissal, lattice boxes and
// general-list regions (wave w of the grid is block w here), but the candidates of the
// boxes are not tested by their segment's lane.  Boxed segments wait in an LDS ring
// across batches; whenever kVolSeg of them wait, they stage their frustums and their
// candidates are spread evenly over the lanes, so that a staging round (dependent loads
// and two barriers) serves full slots rather than the few boxed segments of one batch.
__global__ void __launch_bounds__(64, 4) k_mics_plane(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr,
                                                      DevMics mc, TraceArgs a, MicWork w, WaveScratch ws)
{
    __shared__ PlaneStage st;
    const unsigned long long s0 = gen_start(ctr, a.gen);
    const unsigned long long n = gen_count(ctr, a.gen, a.gen_end);
    const int lane = lane_id();
    const unsigned long long wave = blockIdx.x;
    const unsigned long long region = wave * general_region(n, ws.n_waves);
    unsigned gcount = 0, tests = 0, updates = 0;
    int head = 0, waiting = 0;   // the ring's first entry and its length (wave-uniform)
    for (unsigned long long base = wave * 64; base < n; base += (unsigned long long)gridDim.x * 64) {
        const long long i = (long long)(s0 + base) + lane;
        bool general = false, boxed = false;
        int i0 = 0, j0 = 0, i1 = -1, j1 = -1;
        if (base + (unsigned long long)lane < n) {
            // the decision taken when the beam was created, if the set classified it
            const int kind = a.mic_cls ? plane_uncode(a.mic_cls[i], i0, i1, j0, j1)
                                       : plane_fast(q, i, mc, i0, i1, j0, j1);
            general = kind == 2;
            boxed = kind == 1;
        }
        const unsigned long long gm = __ballot(general);
        if (general) w.general[region + gcount + __popcll(gm & ((1ull << lane) - 1ull))] = (int)i;
        gcount += (unsigned)__popcll(gm);
        const unsigned long long bm = __ballot(boxed);
        if (boxed) {
            const int e = (head + waiting + __popcll(bm & ((1ull << lane) - 1ull))) & (kPendRing - 1);
            const int ncol = i1 - i0 + 1;
            st.pend_seg[e] = (int)i;
            st.pend_box[e] = make_int4(i0, j0, ncol, ncol * (j1 - j0 + 1));
        }
        waiting += __popcll(bm);
        __syncthreads();
        while (waiting >= kVolSeg) {
            plane_round(st, M, q, segs, mc, a, head, kVolSeg, tests, updates);
            head = (head + kVolSeg) & (kPendRing - 1);
            waiting -= kVolSeg;
        }
    }
    if (waiting > 0) plane_round(st, M, q, segs, mc, a, head, waiting, tests, updates);
    if (lane == 0) ws.general[wave] = gcount;
    flush_mic_counters(ctr, tests, updates);
    if (a.mic_cls && lane == 0 && wave * 64 < n) {
        // segments of this wave's batches: 64 per full batch
        const unsigned long long stride = (unsigned long long)gridDim.x * 64;
        const unsigned long long full = (n - wave * 64) / stride, rest = (n - wave * 64) % stride;
        add_mic_stat(ctr, MS_CLASSIFIED, 64 * full + (rest < 64 ? rest : 64));
    }
}

// One wave per block (the block's LDS is its staging), 4 waves per SIMD: at most 128 VGPRs.
__global__ void __launch_bounds__(64, 4) k_mics3d(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr,
                                                   DevMics mc, TraceArgs a, MicWork w)
{
    __shared__ VolStage st;
    const unsigned long long s0 = gen_start(ctr, a.gen);
    const unsigned long long n = gen_count(ctr, a.gen, a.gen_end);
    const int lane = lane_id();
    // this wave's region of the item buffer and its reservation counter
    const int region = (int)(blockIdx.x % kLayerRegions);
    const long long rcap = w.layers_cap / kLayerRegions;
    int2 *const items = w.layers + (long long)region * rcap;
    unsigned *const rcnt = w.layer_cnt + region * kLayerCntStride;
    unsigned tests = 0, updates = 0, visits = 0, in_place = 0;
    for (unsigned long long base = (unsigned long long)blockIdx.x * kVolSeg; base < n;
         base += (unsigned long long)gridDim.x * kVolSeg) {
        // stage the batch's segments (lanes 0..kVolSeg-1) and count their layers
        const long long i = (long long)(s0 + base) + lane;
        int cnt = 0, k0 = 0;
        if (lane < kVolSeg && base + (unsigned long long)lane < n) {
            const V3 A = ld3(q.dbl + D_A * q.cap, q.cap, i);
            V3 d[3];
            d[0] = ld3(q.dbl + D_D0 * q.cap, q.cap, i);
            d[1] = ld3(q.dbl + D_D1 * q.cap, q.cap, i);
            d[2] = ld3(q.dbl + D_D2 * q.cap, q.cap, i);
            int k1;
            if (seg_layers(M, q, i, segs.hit[i], A, d, mc, k0, k1)) {
                cnt = k1 - k0 + 1;
                Frustum f{};  // caps the segment lacks are staged as zeros
                load_frustum(M, q, segs, i, a.delta, f);
                stage_frustum(st, lane, f);
                int pos = 0, neg = 0;
                float sxlo = INFINITY, sxhi = -INFINITY, sylo = INFINITY, syhi = -INFINITY, smag = 0.0f;
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    pos += d[e].z > 0.0 ? 1 : 0;
                    neg += d[e].z < 0.0 ? 1 : 0;
                    const float sx = (float)(d[e].x / d[e].z), sy = (float)(d[e].y / d[e].z);
                    sxlo = fminf(sxlo, sx); sxhi = fmaxf(sxhi, sx);
                    sylo = fminf(sylo, sy); syhi = fmaxf(syhi, sy);
                    smag = fmaxf(smag, fmaxf(fabsf(sx), fabsf(sy)));
                }
                // the slopes are only read for layers every edge crosses (no dz = 0)
                st.sxlo[lane] = sxlo; st.sxhi[lane] = sxhi;
                st.sylo[lane] = sylo; st.syhi[lane] = syhi;
                st.smag[lane] = smag;
                st.bits[lane] = (f.has_near ? 1 : 0) | (f.has_far ? 2 : 0) | (f.flag ? 4 : 0) | (pos == 3 ? 8 : 0) |
                                (neg == 3 ? 16 : 0) | (pos == 0 ? 32 : 0) | (neg == 0 ? 64 : 0);
                st.K[lane] = f.K;
                st.az[lane] = A.z;
                st.ax[lane] = (float)A.x;
                st.ay[lane] = (float)A.y;
            }
        }
        visits += (unsigned)cnt;
        int total;
        const int pre = wave_excl_scan(cnt, total);
        if (lane < kVolSeg) {
            st.prefix[lane] = pre;
            st.k0[lane] = k0;
            write_skips<8>(st.psk1, st.psk2, lane, pre);
        }
        if (lane == 0) st.prefix[kVolSeg] = total;
        __syncthreads();
        // (segment, layer) pairs, 64 at a time
        for (int pb = 0; pb < total; pb += 64) {
            const int p = pb + lane;
            int kind = 0, slot = 0, k = 0, i0 = 0, i1 = -1, j0 = 0, j1 = -1;
            if (p < total) {
                slot = owner32(st.prefix, st.psk1, st.psk2, p);
                k = st.k0[slot] + (p - st.prefix[slot]);
                kind = layer_fast(st, slot, mc, k, i0, i1, j0, j1);
            }
            // clipped-footprint pairs become items of the wave's region (wave-aggregated
            // reservation on the region's counter)
            const bool gen_item = kind == 2;
            const unsigned long long gm = __ballot(gen_item);
            unsigned gb = 0;
            if (lane == 0 && gm) gb = atomicAdd(rcnt, (unsigned)__popcll(gm));
            gb = __shfl(gb, 0, 64);
            if (gen_item) {
                const unsigned below = __builtin_amdgcn_mbcnt_hi((unsigned)(gm >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((unsigned)gm, 0u));
                const long long e = (long long)gb + (long long)below;
                const long long seg = (long long)(s0 + base) + slot;
                if (e < rcap) {
                    items[e] = make_int2((int)seg, k);
                } else {
                    Frustum f;  // the region is full: done here
                    unstage_frustum(st, slot, a.delta, f);
                    layer_general(f, mc, w, ctr, a, seg, k, tests, updates);
                    in_place++;
                }
            }
            // candidates of the lattice boxes, 64 at a time
            const int nc = kind == 1 ? (i1 - i0 + 1) * (j1 - j0 + 1) : 0;
            int ctotal;
            const int cpre = wave_excl_scan(nc, ctotal);
            st.cprefix[lane] = cpre;
            write_skips<16>(st.csk1, st.csk2, lane, cpre);
            st.box[lane] = make_int4(slot | (k << 6), i0, j0, i1 - i0 + 1);
            if (lane == 0) st.cprefix[64] = ctotal;
            __syncthreads();
            for (int cb = 0; cb < ctotal; cb += 64) {
                const int c = cb + lane;
                if (c < ctotal) {
                    const int pl = owner64(st.cprefix, st.csk1, st.csk2, c);
                    const int o = c - st.cprefix[pl];
                    const int4 bx = st.box[pl];
                    const int row = o / bx.w;
                    tests++;
                    updates += mic_apply_staged(st, bx.x & 63, mc, bx.y + (o - row * bx.w), bx.z + row, bx.x >> 6,
                                                a.delta2, a.air_m);
                }
            }
            __syncthreads();
        }
        __syncthreads();
    }
    flush_mic_counters(ctr, tests, updates);
    const unsigned long long sv = wave_sum_u64(visits), sp = wave_sum_u64(in_place);
    if (lane == 0) {
        add_mic_stat(ctr, MS_LAYERS, sv);
        if (sp) add_mic_stat(ctr, MS_LAYER_FALLBACK, sp);
    }
}

// LDS staging of one wave of k_mics3d_general: kVolSeg (segment, layer) items with their
// frustums and the five frustum half-planes on the item's layer.
struct GenStage {
    double f[kVolF][kVolSeg];     // frustum, as VolStage
    double L[15][kVolSeg];        // half-planes 0..4 (a, b, k) on the item's layer
    float K[kVolSeg];
    int bits[kVolSeg];            // 1 near cap, 2 far cap, 4 flagged
    int k[kVolSeg];               // the item's layer
    int j0[kVolSeg];              // first row of its clipped footprint
    alignas(16) int prefix[kVolSeg + 4];  // exclusive scan of the items' row counts
    alignas(16) int psk1[4];
    alignas(16) int psk2[16];
    alignas(16) int cprefix[68];  // exclusive scan of the row chunk's column counts
    alignas(16) int csk1[4];
    alignas(16) int csk2[16];
    int4 row[64];                 // row chunk: (slot, row, first column, -)
};

// row_cols on staged half-planes (the same arithmetic as row_cols).
__device__ __forceinline__ bool row_cols_staged(const GenStage &st, int l, const DevMics &mc, int j, int &i0, int &i1)
{
    const double y = mc.y0 + (double)j * mc.dy;
    double lo = -INFINITY, hi = INFINITY;
#pragma unroll
    for (int h = 0; h < 5; ++h) {
        const double la = st.L[3 * h][l], lb = st.L[3 * h + 1][l], lk = st.L[3 * h + 2][l];
        const double rest = lb * y + lk;
        if (la > 0.0) lo = fmax(lo, -rest / la);
        else if (la < 0.0) hi = fmin(hi, -rest / la);
        else if (rest < 0.0) return false;
    }
    if (!(lo <= hi)) return false;
    const double flo = (lo - mc.x0) / mc.dx, fhi = (hi - mc.x0) / mc.dx;
    if (flo > (double)mc.nx || fhi < -1.0) return false;
    const double a0 = fmax(ceil(flo) - 1.0, 0.0), a1 = fmin(floor(fhi) + 1.0, (double)(mc.nx - 1));
    if (!(a0 <= a1)) return false;
    i0 = (int)a0;
    i1 = (int)a1;
    return true;
}

// The rows of the wave's staged footprints (slot l has nrows rows from st.j0[l] on layer
// st.k[l]; lane l < kVolSeg passes its slot's count), spread evenly over the lanes, each
// finding its row's column range; then the rows' candidate microphones spread evenly over
// the lanes and tested against the staged frustums.  Every lane of the wave calls it.
__device__ __forceinline__ void staged_rows(GenStage &st, const DevMics &mc, int nrows, const TraceArgs &a,
                                            unsigned &tests, unsigned &updates)
{
    const int lane = lane_id();
    int total;
    const int pre = wave_excl_scan(nrows, total);
    if (lane < kVolSeg) {
        st.prefix[lane] = pre;
        write_skips<8>(st.psk1, st.psk2, lane, pre);
    }
    __syncthreads();
    // rows, 64 at a time
    for (int rb = 0; rb < total; rb += 64) {
        const int r = rb + lane;
        int ncol = 0, slot = 0, j = 0, c0 = 0, c1 = -1;
        if (r < total) {
            slot = owner32(st.prefix, st.psk1, st.psk2, r);
            j = st.j0[slot] + (r - st.prefix[slot]);
            if (row_cols_staged(st, slot, mc, j, c0, c1)) ncol = c1 - c0 + 1;
        }
        int ctotal;
        const int cpre = wave_excl_scan(ncol, ctotal);
        st.cprefix[lane] = cpre;
        write_skips<16>(st.csk1, st.csk2, lane, cpre);
        st.row[lane] = make_int4(slot, j, c0, 0);
        __syncthreads();
        // candidate microphones, 64 at a time
        for (int cb = 0; cb < ctotal; cb += 64) {
            const int c = cb + lane;
            if (c < ctotal) {
                const int rl = owner64(st.cprefix, st.csk1, st.csk2, c);
                const int4 rw = st.row[rl];
                tests++;
                updates += mic_apply_staged(st, rw.x, mc, rw.z + (c - st.cprefix[rl]), rw.y, st.k[rw.x], a.delta2,
                                            a.air_m);
            }
        }
        __syncthreads();
    }
    __syncthreads();
}

// (segment, layer) items of the clipped-footprint path, kVolSeg per wave: each lane clips
// its item's footprint (its row range), then the rows are spread evenly over the lanes
// (each finds its column range), then the candidate microphones are spread evenly over
// the lanes and tested against the staged frustums.  One wave per block, 3 per SIMD.
__global__ void __launch_bounds__(64, 3) k_mics3d_general(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr,
                                                          DevMics mc, TraceArgs a, MicWork w)
{
    __shared__ GenStage st;
    // wave b takes region b mod kLayerRegions, with the other waves of that region (the
    // grid has at least kLayerRegions waves, one per block)
    const int region = (int)(blockIdx.x % kLayerRegions);
    const unsigned sub = blockIdx.x / kLayerRegions;
    const unsigned nsub = (gridDim.x - (unsigned)region + kLayerRegions - 1) / kLayerRegions;
    const long long rcap = w.layers_cap / kLayerRegions;
    const unsigned requested = w.layer_cnt[region * kLayerCntStride];
    const unsigned long long n = (long long)requested < rcap ? requested : (unsigned long long)rcap;
    const int2 *const items = w.layers + (long long)region * rcap;
    const int lane = lane_id();
    if (sub == 0 && lane == 0 && requested) atomicAdd(&ctr->n_layers[a.gen], (unsigned long long)requested);
    unsigned tests = 0, updates = 0;
    for (unsigned long long base = (unsigned long long)sub * kVolSeg; base < n;
         base += (unsigned long long)nsub * kVolSeg) {
        int nrows = 0;
        if (lane < kVolSeg && base + (unsigned long long)lane < n) {
            const int2 it = items[base + lane];
            Frustum f{};
            load_frustum(M, q, segs, it.x, a.delta, f);
            HalfPlane L[9];
            footprint_lines(f, mc, mc.z + (double)it.y * mc.dz, L);
            int j0, j1;
            if (footprint_rows(L, mc, j0, j1)) {
                nrows = j1 - j0 + 1;
                stage_frustum(st, lane, f);
                st.bits[lane] = (f.has_near ? 1 : 0) | (f.has_far ? 2 : 0) | (f.flag ? 4 : 0);
                st.K[lane] = f.K;
                st.k[lane] = it.y;
                st.j0[lane] = j0;
#pragma unroll
                for (int h = 0; h < 5; ++h) {
                    st.L[3 * h][lane] = L[h].a;
                    st.L[3 * h + 1][lane] = L[h].b;
                    st.L[3 * h + 2][lane] = L[h].k;
                }
            }
        }
        staged_rows(st, mc, nrows, a, tests, updates);
    }
    flush_mic_counters(ctr, tests, updates);
}

// ---------------------------------------------------------------------------------------
// Explicit microphone points
//   k_mics_points: one wave per kVolSeg segments: each lane bounds its frustum within the
//   points' z range in xy, the (segment, bucket row) pairs are spread evenly over the
//   lanes (a bucket row is one contiguous range of sorted points), then the points of the
//   ranges are spread evenly over the lanes and tested against the staged frustums.
// ---------------------------------------------------------------------------------------

// xy box of the part of a segment's frustum with z in [zlo, zhi], widened for rounding;
// false when empty.  The frustum lies in the tetrahedron of the apex and the edge rays'
// crossings of the hit plane (when all three cross it ahead of the apex), else in the cone
// of the edge directions.  The tetrahedron (or, when every edge rises or every edge falls,
// the cone) cut by the slab is the convex hull of its vertices inside the slab and its
// edges' crossings of the slab's planes; any other cone is unbounded in the slab.
__device__ bool seg_slab_box(const DevMesh &M, const DevQueue &q, long long i, int hit, V3 A, const V3 *d,
                             double zlo, double zhi, double &x0, double &x1, double &y0, double &y1, bool &all)
{
    V3 P[3];
    bool cut = hit >= 0;
    if (cut) {
        V3 v0, v1, v2;
        tri_vertices(M.tri_g, hit, v0, v1, v2);
        const V3 c = ld3(q.dbl + D_C * q.cap, q.cap, i);
        V3 Nf = cross(v1 - v0, v2 - v0);
        if (!(dot(c, Nf) > 0.0)) Nf = -1.0 * Nf;
        const double c0 = dot(Nf, v0 - A);
        cut = c0 > 0.0;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const double g = dot(Nf, d[e]);
            cut = cut && g > 0.0;
            P[e] = A + (c0 / g) * d[e];
        }
    }
    x0 = y0 = INFINITY;
    x1 = y1 = -INFINITY;
    double mag = fmax(fabs(A.x), fabs(A.y));
    auto take = [&](V3 p) {
        x0 = fmin(x0, p.x); x1 = fmax(x1, p.x);
        y0 = fmin(y0, p.y); y1 = fmax(y1, p.y);
        mag = fmax(mag, fmax(fabs(p.x), fabs(p.y)));
    };
    auto crossing = [&](V3 u, V3 v) {  // segment u-v against the two planes
        const double zc[2] = {zlo, zhi};
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if ((u.z - zc[h]) * (v.z - zc[h]) < 0.0) take(u + ((zc[h] - u.z) / (v.z - u.z)) * (v - u));
    };
    auto inside = [&](V3 p) { return p.z >= zlo && p.z <= zhi; };
    all = false;
    if (inside(A)) take(A);
    if (cut && isfinite(P[0].x + P[0].y + P[0].z + P[1].x + P[1].y + P[1].z + P[2].x + P[2].y + P[2].z)) {
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (inside(P[e])) take(P[e]);
            crossing(A, P[e]);
            crossing(P[e], P[(e + 1) % 3]);
        }
    } else {
        const bool up = d[0].z > 0.0 && d[1].z > 0.0 && d[2].z > 0.0;
        const bool down = d[0].z < 0.0 && d[1].z < 0.0 && d[2].z < 0.0;
        if (!up && !down) {
            all = true;   // horizontal directions in the cone: unbounded in the slab
            return true;
        }
        // every edge crosses each plane at most once, ahead of the apex when it lies on
        // its way: the crossings (t >= 0) and the apex bound the cut cone
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const double zc[2] = {zlo, zhi};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double t = (zc[h] - A.z) / d[e].z;
                if (t >= 0.0) take(A + t * d[e]);
            }
        }
    }
    if (!(x0 <= x1 && y0 <= y1)) return false;
    if (!isfinite(mag)) {
        all = true;
        return true;
    }
    const double slack = 1e-6 + 1e-9 * mag;
    x0 -= slack; x1 += slack; y0 -= slack; y1 += slack;
    return true;
}

// A convex polygon of at most kPolyMax vertices in xy.
constexpr int kPolyMax = 8;
struct Poly {
    double x[kPolyMax], y[kPolyMax];
    int n;
};

// Keeps the part of p with a x + b y + c >= 0 (Sutherland-Hodgman on a convex polygon).
__device__ __forceinline__ void clip_poly(Poly &p, double a, double b, double c)
{
    Poly o;
    o.n = 0;
    for (int k = 0; k < p.n; ++k) {
        const int l = k + 1 < p.n ? k + 1 : 0;
        const double sk = a * p.x[k] + b * p.y[k] + c, sl = a * p.x[l] + b * p.y[l] + c;
        if (sk >= 0.0 && o.n < kPolyMax) { o.x[o.n] = p.x[k]; o.y[o.n] = p.y[k]; o.n++; }
        if ((sk >= 0.0) != (sl >= 0.0) && o.n < kPolyMax) {
            const double t = sk / (sk - sl);
            o.x[o.n] = p.x[k] + t * (p.x[l] - p.x[k]);
            o.y[o.n] = p.y[k] + t * (p.y[l] - p.y[k]);
            o.n++;
        }
    }
    p = o;
}

// The wedge of xy directions a cone's edges span (their projections), as two half-planes
// through the apex's projection: false when the projections span half the plane or more
// (or nearly), the cone then being unbounded in every xy direction.
__device__ __forceinline__ bool cone_wedge(const V3 *d, double &ua, double &ub, double &va, double &vb)
{
    // the pair (u, v) with the third direction between them, counter-clockwise u -> v
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int e = k >> 1, f = (e + 1 + (k & 1)) % 3, g = 3 - e - f;
        const double uxv = d[e].x * d[f].y - d[e].y * d[f].x;
        const double uxw = d[e].x * d[g].y - d[e].y * d[g].x, wxv = d[g].x * d[f].y - d[g].y * d[f].x;
        const double lu = fabs(d[e].x) + fabs(d[e].y), lv = fabs(d[f].x) + fabs(d[f].y);
        // clearly less than half a turn (sine above 1e-6 of the L1 lengths), w inside
        if (uxv > 1e-6 * lu * lv && uxw >= 0.0 && wxv >= 0.0) {
            ua = d[e].x; ub = d[e].y; va = d[f].x; vb = d[f].y;
            return true;
        }
    }
    return false;
}

struct PtsStage {
    double f[kVolF][kVolSeg];     // frustum, as VolStage
    double px[kPolyMax][kVolSeg], py[kPolyMax][kVolSeg];   // its xy region in the points' slab
    int pn[kVolSeg];
    float K[kVolSeg];
    int bits[kVolSeg];            // 1 near cap, 2 far cap, 4 flagged
    int bj0[kVolSeg];             // first bucket row
    alignas(16) int prefix[kVolSeg + 4];  // exclusive scan of the segments' bucket rows
    alignas(16) int psk1[4];
    alignas(16) int psk2[16];
    alignas(16) int cprefix[68];  // exclusive scan of the row chunk's point counts
    alignas(16) int csk1[4];
    alignas(16) int csk2[16];
    int2 range[64];               // row chunk: (slot, first sorted point)
    double slack[kVolSeg];        // rounding allowance of the region
};

__global__ void __launch_bounds__(64, 3) k_mics_points(DevMesh M, DevQueue q, DevSegs segs, DevCounters *ctr,
                                                       DevMics mc, DevPoints pts, TraceArgs a)
{
    __shared__ PtsStage st;
    const unsigned long long s0 = gen_start(ctr, a.gen);
    const unsigned long long n = gen_count(ctr, a.gen, a.gen_end);
    const int lane = lane_id();
    unsigned tests = 0, updates = 0;
    for (unsigned long long base = (unsigned long long)blockIdx.x * kVolSeg; base < n;
         base += (unsigned long long)gridDim.x * kVolSeg) {
        int nrows = 0;
        if (lane < kVolSeg && base + (unsigned long long)lane < n) {
            const long long i = (long long)(s0 + base) + lane;
            const V3 A = ld3(q.dbl + D_A * q.cap, q.cap, i);
            V3 d[3];
            d[0] = ld3(q.dbl + D_D0 * q.cap, q.cap, i);
            d[1] = ld3(q.dbl + D_D1 * q.cap, q.cap, i);
            d[2] = ld3(q.dbl + D_D2 * q.cap, q.cap, i);
            double x0, x1, y0, y1;
            bool all;
            if (seg_slab_box(M, q, i, segs.hit[i], A, d, pts.zlo, pts.zhi, x0, x1, y0, y1, all)) {
                // the box (the points' extent when unbounded), cut by the cone's xy wedge
                const double gx0 = pts.bx0, gx1 = pts.bx0 + pts.nbx * pts.bh;
                const double gy0 = pts.by0, gy1 = pts.by0 + pts.nby * pts.bh;
                if (all) { x0 = gx0; x1 = gx1; y0 = gy0; y1 = gy1; }
                x0 = fmax(x0, gx0); x1 = fmin(x1, gx1); y0 = fmax(y0, gy0); y1 = fmin(y1, gy1);
                Poly pg;
                pg.n = 0;
                if (x0 <= x1 && y0 <= y1) {
                    pg.n = 4;
                    pg.x[0] = x0; pg.y[0] = y0; pg.x[1] = x1; pg.y[1] = y0;
                    pg.x[2] = x1; pg.y[2] = y1; pg.x[3] = x0; pg.y[3] = y1;
                    double ua, ub, va, vb;
                    if (cone_wedge(d, ua, ub, va, vb)) {
                        // cross(u, p - a) >= 0 and cross(p - a, v) >= 0, each relaxed
                        const double mg = fmax(fmax(fabs(A.x), fabs(A.y)), fmax(fmax(fabs(x0), fabs(x1)),
                                                                                fmax(fabs(y0), fabs(y1))));
                        const double lu = fabs(ua) + fabs(ub), lv = fabs(va) + fabs(vb);
                        clip_poly(pg, -ub, ua, ub * A.x - ua * A.y + (1e-6 + 1e-9 * mg) * lu);
                        clip_poly(pg, vb, -va, va * A.y - vb * A.x + (1e-6 + 1e-9 * mg) * lv);
                    }
                }
                double py0 = INFINITY, py1 = -INFINITY, mag = 1.0;
                for (int v = 0; v < pg.n; ++v) {
                    py0 = fmin(py0, pg.y[v]); py1 = fmax(py1, pg.y[v]);
                    mag = fmax(mag, fmax(fabs(pg.x[v]), fabs(pg.y[v])));
                }
                const double sl = 1e-6 + 1e-9 * mag;
                if (pg.n >= 3) {
                    const double fj0 = fmax(floor((py0 - sl - pts.by0) / pts.bh), 0.0);
                    const double fj1 = fmin(floor((py1 + sl - pts.by0) / pts.bh), (double)(pts.nby - 1));
                    if (fj0 <= fj1) {
                        nrows = (int)fj1 - (int)fj0 + 1;
                        Frustum f{};
                        load_frustum(M, q, segs, i, a.delta, f);
                        stage_frustum(st, lane, f);
                        st.bits[lane] = (f.has_near ? 1 : 0) | (f.has_far ? 2 : 0) | (f.flag ? 4 : 0);
                        st.K[lane] = f.K;
                        st.bj0[lane] = (int)fj0;
                        st.pn[lane] = pg.n;
                        st.slack[lane] = sl;
                        for (int v = 0; v < pg.n; ++v) {
                            st.px[v][lane] = pg.x[v];
                            st.py[v][lane] = pg.y[v];
                        }
                    }
                }
            }
        }
        int total;
        const int pre = wave_excl_scan(nrows, total);
        if (lane < kVolSeg) {
            st.prefix[lane] = pre;
            write_skips<8>(st.psk1, st.psk2, lane, pre);
        }
        __syncthreads();
        for (int rb = 0; rb < total; rb += 64) {
            const int r = rb + lane;
            int cnt = 0, slot = 0, first = 0;
            if (r < total) {
                slot = owner32(st.prefix, st.psk1, st.psk2, r);
                const int j = st.bj0[slot] + (r - st.prefix[slot]);
                // x extent of the region within the bucket row's strip (widened)
                const double sl = st.slack[slot];
                const double ya = pts.by0 + j * pts.bh - sl, yb = pts.by0 + (j + 1) * pts.bh + sl;
                const int np = st.pn[slot];
                double xa = INFINITY, xb = -INFINITY;
                for (int v = 0; v < np; ++v) {
                    const int w = v + 1 < np ? v + 1 : 0;
                    const double x1 = st.px[v][slot], y1 = st.py[v][slot];
                    const double x2 = st.px[w][slot], y2 = st.py[w][slot];
                    if (y1 >= ya && y1 <= yb) { xa = fmin(xa, x1); xb = fmax(xb, x1); }
                    const double yc[2] = {ya, yb};
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        if ((y1 - yc[h]) * (y2 - yc[h]) < 0.0) {
                            const double x = x1 + (yc[h] - y1) / (y2 - y1) * (x2 - x1);
                            xa = fmin(xa, x); xb = fmax(xb, x);
                        }
                }
                if (xa <= xb) {
                    const int bi0 = (int)fmax(floor((xa - sl - pts.bx0) / pts.bh), 0.0);
                    const int bi1 = (int)fmin(floor((xb + sl - pts.bx0) / pts.bh), (double)(pts.nbx - 1));
                    if (bi0 <= bi1) {
                        first = pts.cell[j * pts.nbx + bi0];
                        cnt = pts.cell[j * pts.nbx + bi1 + 1] - first;
                    }
                }
            }
            int ctotal;
            const int cpre = wave_excl_scan(cnt, ctotal);
            st.cprefix[lane] = cpre;
            write_skips<16>(st.csk1, st.csk2, lane, cpre);
            st.range[lane] = make_int2(slot, first);
            __syncthreads();
            for (int cb = 0; cb < ctotal; cb += 64) {
                const int c = cb + lane;
                if (c < ctotal) {
                    const int rl = owner64(st.cprefix, st.csk1, st.csk2, c);
                    const int2 rg = st.range[rl];
                    const int k = rg.y + (c - st.cprefix[rl]);
                    const V3 m = {pts.px[k], pts.py[k], pts.pz[k]};
                    tests++;
                    updates += staged_contribute(st, rg.x, m, (long long)pts.orig[k], mc.e_strict, mc.e_flag,
                                                 (const unsigned *)nullptr, a.delta2, a.air_m);
                }
            }
            __syncthreads();
        }
        __syncthreads();
    }
    flush_mic_counters(ctr, tests, updates);
}

hipError_t launch_mics_points(const DevMesh &m, DevQueue q, DevSegs segs, DevCounters *ctr, DevMics mics,
                              DevPoints pts, const TraceArgs &a, int n_cu, hipStream_t s)
{
    if (a.scenarios || pts.n <= 0 || pts.nbx <= 0 || pts.nby <= 0) return hipErrorInvalidValue;
    // eight times the resident waves, as the volumetric pass (100,000 district receivers:
    // 9.5 ms per pass at n_cu x 12 one-wave blocks, 8.0 at x 96)
    k_mics_points<<<n_cu * 96, 64, 0, s>>>(m, q, segs, ctr, mics, pts, a);
    return hipGetLastError();
}

template <bool kSlots>
static hipError_t launch_mics_t(const DevMesh &m, DevQueue q, DevSegs segs, DevCounters *ctr, DevMics mics,
                                const TraceArgs &a, MicWork w, WaveScratch ws, int n_cu, hipStream_t s)
{
    // k_mics and k_mics_general must use the same grid: wave w hands its region to wave w
    const int blocks = ws.n_waves / kWavesPerBlock;
    if (blocks <= 0 || blocks * kWavesPerBlock != ws.n_waves) return hipErrorInvalidValue;
    if constexpr (kSlots) {
        k_mics<true><<<blocks, 64 * kWavesPerBlock, 0, s>>>(m, q, segs, ctr, mics, a, w, ws);
    } else {
        // one wave per block: block w is wave w of k_mics_general's grid
        k_mics_plane<<<ws.n_waves, 64, 0, s>>>(m, q, segs, ctr, mics, a, w, ws);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_mics_general<kSlots><<<blocks, 64 * kWavesPerBlock, 0, s>>>(m, q, segs, ctr, mics, a, w, ws);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_mic_rows<kSlots><<<blocks, 64 * kWavesPerBlock, 0, s>>>(m, q, segs, ctr, mics, a, w, ws);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_mics_big<kSlots><<<n_cu * 4, 256, 0, s>>>(m, q, segs, ctr, mics, a, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_mic_spans<kSlots><<<n_cu * 8, 256, 0, s>>>(m, q, segs, ctr, mics, a, w);
    return hipGetLastError();
}

hipError_t launch_mics(const DevMesh &m, DevQueue q, DevSegs segs, DevCounters *ctr, DevMics mics,
                       const TraceArgs &a, MicWork w, WaveScratch ws, int n_cu, hipStream_t s)
{
    if (!a.scenarios && mics.nz > 1) {
        if (!(mics.dz > 0.0)) return hipErrorInvalidValue;
        if (!w.layers || w.layers_cap <= 0 || !w.layer_cnt) return hipErrorInvalidValue;
        // the regions' reservation counters start at zero in every pass
        hipError_t e = launch_zero_ints((int *)w.layer_cnt, (long long)kLayerRegions * kLayerCntStride, s);
        if (e != hipSuccess) return e;
        // one wave per block: a block's LDS is its wave's staging area.  A wave's batches
        // differ widely in work (layers per segment, candidates per layer), so the grid is
        // eight times what is resident at once: waves that finish early leave room for the
        // rest (tall district: 129 ms per step at n_cu x 16 one-wave blocks, 110 at x 128,
        // 111 at x 512)
        k_mics3d<<<n_cu * 128, 64, 0, s>>>(m, q, segs, ctr, mics, a, w);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_mics3d_general<<<std::max(n_cu * 96, kLayerRegions), 64, 0, s>>>(m, q, segs, ctr, mics, a, w);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_mic_spans<false><<<n_cu * 8, 256, 0, s>>>(m, q, segs, ctr, mics, a, w);
        return hipGetLastError();
    }
    if (a.scenarios) {
        if (!a.slot_mics) return hipErrorInvalidValue;
        return launch_mics_t<true>(m, q, segs, ctr, mics, a, w, ws, n_cu, s);
    }
    return launch_mics_t<false>(m, q, segs, ctr, mics, a, w, ws, n_cu, s);
}

// ---------------------------------------------------------------------------------------
// The static work area of bt_accumulate_mics_static (callers that cannot allocate): one
// array per GPU, held until the process ends.  Host code never names `scratch` in a kernel
// argument or copy (its host-side symbol is not a device address); it uses the address
// hipGetSymbolAddress returns, looked up once per device with that device current.
// ---------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mtx;
void *g_scratch_ptr[kScratchDevices] = {};
}  // namespace

hipError_t static_scratch(int device, void **out)
{
    if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mtx);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace bt
