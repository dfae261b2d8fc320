/*
 * Test driver (built only by tests/test_oracle_threads.py, with ThreadSanitizer): runs the
 * oracle's threaded trace on a small procedural scene (a ground quad and two boxes, one
 * source, a planar microphone grid) with 1 and with 6 worker threads and checks that the
 * two runs give the same counts and energies.  The workers' shared inputs are read-only
 * and every output has a per-thread copy reduced in thread order; ThreadSanitizer reports
 * any access that breaks this.  The oracle source is compiled into this file.
 */
#include "../oracle/bt_oracle.c"

#include <stdio.h>

static int add_vert(float *v, int n, float x, float y, float z)
{
    v[3 * n] = x; v[3 * n + 1] = y; v[3 * n + 2] = z;
    return n;
}

static int quad(int32_t *t, int nt, int a, int b, int c, int d)
{
    t[3 * nt] = a; t[3 * nt + 1] = b; t[3 * nt + 2] = c;
    t[3 * nt + 3] = a; t[3 * nt + 4] = c; t[3 * nt + 5] = d;
    return nt + 2;
}

int main(void)
{
    float v[3 * 20];
    int32_t t[3 * 24];
    float alpha[24];
    int nv = 0, nt = 0;
    /* ground 80 x 80 m */
    int g0 = nv; nv = add_vert(v, nv, -40, -40, 0) + 1; nv = add_vert(v, nv, 40, -40, 0) + 1;
    nv = add_vert(v, nv, 40, 40, 0) + 1; nv = add_vert(v, nv, -40, 40, 0) + 1;
    nt = quad(t, nt, g0, g0 + 1, g0 + 2, g0 + 3);
    /* two boxes (walls and roof) */
    const float box[2][4] = {{8, 8, 10, 12}, {-14, -6, 8, 20}};   /* cx, cy, half width, height */
    for (int b = 0; b < 2; ++b) {
        const float cx = box[b][0], cy = box[b][1], w = box[b][2], h = box[b][3];
        int k = nv;
        for (int z = 0; z < 2; ++z) {
            const float zz = z ? h : 0.0f;
            nv = add_vert(v, nv, cx - w, cy - w, zz) + 1; nv = add_vert(v, nv, cx + w, cy - w, zz) + 1;
            nv = add_vert(v, nv, cx + w, cy + w, zz) + 1; nv = add_vert(v, nv, cx - w, cy + w, zz) + 1;
        }
        for (int s = 0; s < 4; ++s) nt = quad(t, nt, k + s, k + (s + 1) % 4, k + 4 + (s + 1) % 4, k + 4 + s);
        nt = quad(t, nt, k + 4, k + 5, k + 6, k + 7);
    }
    for (int i = 0; i < nt; ++i) alpha[i] = 0.05f + 0.01f * (float)i;
    const float src[3] = {0.3f, -0.7f, 1.2f}, power[1] = {1.0f};
    orc_scene sc;
    memset(&sc, 0, sizeof sc);
    sc.xyz = v; sc.n_vert = nv; sc.tri = t; sc.n_tri = nt; sc.alpha = alpha;
    sc.src = src; sc.power = power; sc.n_src = 1;
    sc.mic_x0 = -38.0; sc.mic_y0 = -38.0; sc.mic_z = 1.5; sc.mic_dx = 2.0; sc.mic_dy = 2.0;
    sc.mic_nx = 39; sc.mic_ny = 39; sc.mic_dz = 4.0; sc.mic_nz = 2;
    const int level = 3, depth = 4;
    const int64_t nmic = 39 * 39 * 2;
    double *es[2], *ef[2];
    int64_t count[2][8];
    double pw[2][8];
    for (int run = 0; run < 2; ++run) {
        orc_params p;
        memset(&p, 0, sizeof p);
        p.level = level; p.depth = depth; p.t_min = 1e-3; p.delta = 1e-5;
        p.use_bvh = 1; p.mic_mode = 1; p.n_threads = run == 0 ? 1 : 6;
        p.beam_begin = 0; p.beam_end = -1;
        orc_result r;
        memset(&r, 0, sizeof r);
        int64_t flagged[8] = {0};
        memset(count[run], 0, sizeof count[run]);
        memset(pw[run], 0, sizeof pw[run]);
        es[run] = (double *)calloc((size_t)nmic, sizeof(double));
        ef[run] = (double *)calloc((size_t)nmic, sizeof(double));
        r.count = count[run]; r.flagged = flagged; r.power = pw[run]; r.e_strict = es[run]; r.e_flag = ef[run];
        if (orc_trace(&sc, &p, &r) != 0) { fprintf(stderr, "orc_trace failed\n"); return 2; }
        printf("threads %d: segments %lld, mic updates %lld\n", p.n_threads, (long long)r.counters[C_SEGMENTS],
               (long long)r.counters[C_MIC_UPDATES]);
    }
    double emax = 0.0, diff = 0.0;
    for (int64_t m = 0; m < nmic; ++m) {
        const double a = es[0][m] + ef[0][m], b = es[1][m] + ef[1][m];
        if (a > emax) emax = a;
        if (fabs(a - b) > diff) diff = fabs(a - b);
    }
    for (int g = 0; g <= depth; ++g)
        if (count[0][g] != count[1][g]) { fprintf(stderr, "count %d differs\n", g); return 3; }
    if (!(emax > 0.0) || diff > 1e-12 * emax) { fprintf(stderr, "energies differ (%g of %g)\n", diff, emax); return 4; }
    printf("ok: 1 and 6 threads agree (max difference %g of %g)\n", diff, emax);
    return 0;
}
