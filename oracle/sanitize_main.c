/*
 * Driver for a sanitized build of the oracle (test infrastructure, like
 * oracle.c): runs the oracle on a few small lattices built here with a
 * fixed integer generator and reads every output array, so that
 * AddressSanitizer and UndefinedBehaviorSanitizer see all of its code paths
 * (trimming, multi-arc seams, holes, free ends, high valence, the zipper).
 * Exit status 0 when every lattice ran; the sanitizers abort otherwise.
 *
 *   gcc -O1 -g -fsanitize=address,undefined -fno-omit-frame-pointer -pthread \
 *       oracle/oracle.c oracle/sanitize_main.c -lm -o oracle_sanitized
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct Ctx Ctx;
Ctx *orc_run(int64_t N, int64_t S, const float *x, const float *y, const float *z, const float *rad,
             const int32_t *sa, const int32_t *sb, int k, int threads);
void orc_free(Ctx *X);
void orc_sizes(const Ctx *X, int64_t *out);
void orc_nodes(const Ctx *X, int32_t *cnt, double *margin);
void orc_node_margins(const Ctx *X, double *out);
void orc_vertices(const Ctx *X, uint32_t *name, double *w, double *cond);
void orc_arcs(const Ctx *X, int32_t *iv, double *dv);
void orc_loops(const Ctx *X, int64_t *off, int32_t *arc, int32_t *dir);
void orc_adjacency(const Ctx *X, int64_t *off, int32_t *adj);
void orc_mesh(const Ctx *X, double *verts, int64_t *tris, int64_t *mesh_off, int64_t *band_off, int64_t *fan_off,
              double *strut_margin, int32_t *strut_status);

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static double urand(void)  /* xorshift64*, uniform in [0, 1) */
{
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return (double)((g_state * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0);
}

static int run_lattice(const char *name, int64_t N, int64_t S, const float *x, const float *y, const float *z,
                       const float *r, const int32_t *sa, const int32_t *sb, int k)
{
    Ctx *X = orc_run(N, S, x, y, z, r, sa, sb, k, 2);
    if (!X) {
        fprintf(stderr, "%s: oracle rejected the lattice\n", name);
        return 1;
    }
    int64_t sz[7];
    orc_sizes(X, sz);
    int32_t *cnt = malloc(sizeof(int32_t) * 8 * (N + 1));
    double *mg = malloc(sizeof(double) * (N + 1)), *kmg = malloc(sizeof(double) * 8 * (N + 1));
    orc_nodes(X, cnt, mg);
    orc_node_margins(X, kmg);
    uint32_t *vn = malloc(sizeof(uint32_t) * (sz[0] + 1));
    double *vw = malloc(sizeof(double) * 3 * (sz[0] + 1)), *vc = malloc(sizeof(double) * 2 * (sz[0] + 1));
    orc_vertices(X, vn, vw, vc);
    int32_t *ai = malloc(sizeof(int32_t) * 7 * (sz[1] + 1));
    double *ad = malloc(sizeof(double) * 11 * (sz[1] + 1));
    orc_arcs(X, ai, ad);
    int64_t *lo = malloc(sizeof(int64_t) * (2 * S + 1));
    int32_t *la = malloc(sizeof(int32_t) * (sz[6] + 1)), *ld = malloc(sizeof(int32_t) * (sz[6] + 1));
    orc_loops(X, lo, la, ld);
    int64_t *aoff = malloc(sizeof(int64_t) * (N + 1));
    int32_t *adj = malloc(sizeof(int32_t) * (2 * S + 1));
    orc_adjacency(X, aoff, adj);
    double *mesh = malloc(sizeof(double) * 3 * (sz[3] + 1)), *smg = malloc(sizeof(double) * (S + 1));
    int64_t *tris = malloc(sizeof(int64_t) * 3 * (sz[4] + sz[5] + 1));
    int64_t *moff = malloc(sizeof(int64_t) * (N + 1)), *boff = malloc(sizeof(int64_t) * (S + 1));
    int64_t *foff = malloc(sizeof(int64_t) * (N + 1));
    int32_t *sst = malloc(sizeof(int32_t) * (S + 1));
    orc_mesh(X, mesh, tris, moff, boff, foff, smg, sst);
    int64_t bad = 0;
    for (int64_t i = 0; i < N; ++i) bad += cnt[8 * i] != 0;
    int ok = 1;
    for (int64_t t = 0; t < 3 * (sz[4] + sz[5]); ++t) ok &= tris[t] >= 0 && tris[t] < sz[3];
    printf("%s: %lld nodes (%lld unmeshed), %lld struts, %lld vertices, %lld arcs, %lld mesh vertices, "
           "%lld triangles%s\n", name, (long long)N, (long long)bad, (long long)S, (long long)sz[0],
           (long long)sz[1], (long long)sz[3], (long long)(sz[4] + sz[5]), ok ? "" : " BAD INDEX");
    free(cnt); free(mg); free(kmg); free(vn); free(vw); free(vc); free(ai); free(ad); free(lo); free(la);
    free(ld); free(aoff); free(adj); free(mesh); free(smg); free(tris); free(moff); free(boff); free(foff);
    free(sst);
    orc_free(X);
    return ok ? 0 : 1;
}

int main(void)
{
    int fails = 0;
    /* jittered simple cubic 3^3 cells with node radii in [0.06, 0.14] */
    {
        const int m = 4;
        int64_t N = m * m * m, S = 3 * 3 * m * m, s = 0;
        float *x = malloc(sizeof(float) * N), *y = malloc(sizeof(float) * N), *z = malloc(sizeof(float) * N);
        float *r = malloc(sizeof(float) * N);
        int32_t *sa = malloc(sizeof(int32_t) * S), *sb = malloc(sizeof(int32_t) * S);
        for (int k = 0; k < m; ++k)
            for (int j = 0; j < m; ++j)
                for (int i = 0; i < m; ++i) {
                    const int id = i + m * (j + m * k);
                    x[id] = (float)(i + 0.04 * (2 * urand() - 1));
                    y[id] = (float)(j + 0.04 * (2 * urand() - 1));
                    z[id] = (float)(k + 0.04 * (2 * urand() - 1));
                    r[id] = (float)(0.06 + 0.08 * urand());
                    if (i + 1 < m) { sa[s] = id; sb[s++] = id + 1; }
                    if (j + 1 < m) { sa[s] = id; sb[s++] = id + m; }
                    if (k + 1 < m) { sa[s] = id; sb[s++] = id + m * m; }
                }
        fails += run_lattice("cubic3", N, s, x, y, z, r, sa, sb, 9);
        free(x); free(y); free(z); free(r); free(sa); free(sb);
    }
    /* stars: a centre node with v thin struts in jittered Fibonacci directions */
    for (int v = 2; v <= 40; v += 19) {
        int64_t N = v + 1, S = v;
        float *x = calloc(N, sizeof(float)), *y = calloc(N, sizeof(float)), *z = calloc(N, sizeof(float));
        float *r = malloc(sizeof(float) * N);
        int32_t *sa = malloc(sizeof(int32_t) * S), *sb = malloc(sizeof(int32_t) * S);
        r[0] = 0.08f;
        for (int i = 0; i < v; ++i) {
            const double f = (i + 0.5) / v, ph = acos(1 - 2 * f), th = 3.883222077450933 * i + 0.1 * sin(7.0 * i);
            x[i + 1] = (float)(cos(th) * sin(ph));
            y[i + 1] = (float)(sin(th) * sin(ph));
            z[i + 1] = (float)cos(ph);
            r[i + 1] = (float)(0.03 + 0.03 * urand());
            sa[i] = 0;
            sb[i] = i + 1;
        }
        char name[32];
        snprintf(name, sizeof name, "star%d", v);
        fails += run_lattice(name, N, S, x, y, z, r, sa, sb, 12);
        free(x); free(y); free(z); free(r); free(sa); free(sb);
    }
    /* a capsule (one strut) and an isolated node */
    {
        float x[3] = {0.f, 1.f, 5.f}, y[3] = {0.f, 0.f, 0.f}, z[3] = {0.f, 0.f, 0.f}, r[3] = {0.1f, 0.07f, 0.1f};
        int32_t sa[1] = {0}, sb[1] = {1};
        fails += run_lattice("capsule", 3, 1, x, y, z, r, sa, sb, 7);
    }
    return fails ? 1 : 0;
}
